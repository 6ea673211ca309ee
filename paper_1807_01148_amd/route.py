"""Iterative decaying re-routing (Sec. 6.3.1): argument marshalling over the
router entry points of include/trafficroute.h, and the iteration loop.

``Router(net)`` keeps the network, the trips' origins and destinations, the
link weights and the current routes on the GPU.  ``reroute(scen, masks)``
runs the loop of Sec. 6.3.1: plan every route on the initial estimates,
simulate, replace the estimates by the measured link times, plan again for
the trips selected by ``masks[k]`` (all, all, half, a quarter), simulate
again.  Routing, weights and simulation run in the library's kernels, and
the routes pass from the router to the simulation on the device.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import ALLOC_FN, FREE_FN, SIM_OK, Sim, SimError, SimNetwork, _TorchAllocator, _p, library

_BOUND = False


def _bind(lib):
    global _BOUND
    if _BOUND:
        return lib
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.rt_create.argtypes = [ctypes.POINTER(SimNetwork), P, ALLOC_FN, FREE_FN, P, ctypes.POINTER(P)]
    lib.rt_create.restype = ctypes.c_int
    lib.rt_set_trips.argtypes = [P, i32, P, i32, P, P]
    lib.rt_set_trips.restype = ctypes.c_int
    lib.rt_weights_initial.argtypes = [P]
    lib.rt_weights_initial.restype = ctypes.c_int
    lib.rt_weights_from_stats.argtypes = [P, P, P]
    lib.rt_weights_from_stats.restype = ctypes.c_int
    lib.rt_set_weights.argtypes = [P, P]
    lib.rt_set_weights.restype = ctypes.c_int
    lib.rt_read_weights.argtypes = [P, P]
    lib.rt_read_weights.restype = ctypes.c_int
    lib.rt_plan.argtypes = [P, P, ctypes.POINTER(ctypes.c_int64)]
    lib.rt_plan.restype = ctypes.c_int
    lib.rt_read_routes.argtypes = [P, P, P]
    lib.rt_read_routes.restype = ctypes.c_int
    lib.rt_route_views.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64)]
    lib.rt_route_views.restype = ctypes.c_int
    lib.rt_tree.argtypes = [P, i32, P, P]
    lib.rt_tree.restype = ctypes.c_int
    lib.rt_tree_static.argtypes = [P, i32, P, P]
    lib.rt_tree_static.restype = ctypes.c_int
    lib.rt_last_work.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32)]
    lib.rt_last_work.restype = ctypes.c_int
    lib.rt_set_batch.argtypes = [P, i32]
    lib.rt_set_batch.restype = ctypes.c_int
    lib.rt_set_delta.argtypes = [P, ctypes.c_int64]
    lib.rt_set_delta.restype = ctypes.c_int
    lib.rt_set_stream.argtypes = [P, P]
    lib.rt_set_stream.restype = ctypes.c_int
    lib.rt_last_error.argtypes = [P]
    lib.rt_last_error.restype = ctypes.c_char_p
    lib.rt_destroy.argtypes = [P]
    lib.rt_destroy.restype = None
    _BOUND = True
    return lib


class Router:
    """Route planner over ``net`` (a scenario network dict) on one GPU."""

    def __init__(self, net, device: int = 0, stream=None, torch_alloc: bool = True):
        import torch
        self.lib = _bind(library())
        self.h = None
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc = _TorchAllocator(device, self.stream) if torch_alloc else None
        self._keep = [np.ascontiguousarray(net[k], dt) for k, dt in
                      (("row_ptr", np.int32), ("col_idx", np.int32), ("lanes", np.int32),
                       ("length", np.float32), ("speed", np.float32))]
        rp, ci, ln, le, sp = self._keep
        self.num_nodes, self.num_edges = int(rp.size - 1), int(ci.size)
        self._net = SimNetwork(self.num_nodes, self.num_edges, _p(rp), _p(ci), _p(ln), _p(le), _p(sp), None)
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            rc = self.lib.rt_create(ctypes.byref(self._net), ctypes.c_void_p(self.stream.cuda_stream),
                                    self._alloc.alloc if self._alloc else ALLOC_FN(),
                                    self._alloc.free if self._alloc else FREE_FN(), None, ctypes.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, "rt_create failed")
        self.h = h
        self.num_trips = 0
        self.total = 0

    def _check(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, self.lib.rt_last_error(self.h).decode())

    def close(self):
        if self.h is not None:
            import torch
            with torch.cuda.device(self.device):
                self.lib.rt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def set_trips(self, src_nodes, trip_src, trip_dst):
        s = np.ascontiguousarray(src_nodes, np.int32)
        a = np.ascontiguousarray(trip_src, np.int32)
        b = np.ascontiguousarray(trip_dst, np.int32)
        self._check(self.lib.rt_set_trips(self.h, int(s.size), _p(s), int(a.size), _p(a), _p(b)))
        self.num_trips = int(a.size)

    def weights_initial(self):
        self._check(self.lib.rt_weights_initial(self.h))

    def weights_from_stats(self, count, tt_us):
        """count, tt_us: int64 torch tensors on the device (Sim.edge_stats_device)."""
        import torch
        with torch.cuda.stream(self.stream):
            self._check(self.lib.rt_weights_from_stats(self.h, ctypes.c_void_p(count.data_ptr()),
                                                       ctypes.c_void_p(tt_us.data_ptr())))

    def set_weights(self, w):
        w = np.ascontiguousarray(w, np.int64)
        self._check(self.lib.rt_set_weights(self.h, _p(w)))

    def weights(self) -> np.ndarray:
        w = np.empty(self.num_edges, np.int64)
        self._check(self.lib.rt_read_weights(self.h, _p(w)))
        return w

    def plan(self, select=None) -> int:
        sel = None if select is None else np.ascontiguousarray(select, np.uint8)
        tot = ctypes.c_int64(0)
        self._check(self.lib.rt_plan(self.h, _p(sel), ctypes.byref(tot)))
        self.total = int(tot.value)
        return self.total

    def routes(self):
        ptr = np.empty(self.num_trips + 1, np.int64)
        edges = np.empty(max(self.total, 1), np.int32)
        self._check(self.lib.rt_read_routes(self.h, _p(ptr), _p(edges)))
        return ptr, edges[:self.total]

    def route_views(self):
        """rt_route_views: DEVICE addresses of the current route table
        (route_ptr int64 [num_trips + 1], route_edges int32) and its length;
        valid until the next plan."""
        pa, ea, tot = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64(0)
        self._check(self.lib.rt_route_views(self.h, ctypes.byref(pa), ctypes.byref(ea), ctypes.byref(tot)))
        return int(pa.value or 0), int(ea.value or 0), int(tot.value)

    def tree(self, src_node: int):
        dist = np.empty(self.num_nodes, np.int64)
        pred = np.empty(self.num_nodes, np.int32)
        self._check(self.lib.rt_tree(self.h, int(src_node), _p(dist), _p(pred)))
        return dist, pred

    def tree_static(self, src_node: int, dist, pred):
        """rt_tree_static: the tree into the caller's DEVICE tensors dist
        (int64 [num_nodes]) and pred (int32 [num_nodes]); allocates nothing."""
        import torch
        for t, dt in ((dist, torch.int64), (pred, torch.int32)):
            if t is not None and (t.dtype != dt or not t.is_cuda or t.numel() != self.num_nodes or
                                  not t.is_contiguous()):
                raise ValueError("dist / pred must be contiguous %s device tensors of %d elements"
                                 % (dt, self.num_nodes))
        self.stream.synchronize()  # the tensors' memory is ready before the library's stream writes it
        with torch.cuda.device(self.device):
            self._check(self.lib.rt_tree_static(self.h, int(src_node),
                                                None if dist is None else ctypes.c_void_p(dist.data_ptr()),
                                                None if pred is None else ctypes.c_void_p(pred.data_ptr())))

    def last_work(self):
        r, s = ctypes.c_int64(0), ctypes.c_int32(0)
        self._check(self.lib.rt_last_work(self.h, ctypes.byref(r), ctypes.byref(s)))
        return int(r.value), int(s.value)

    def set_delta(self, delta_ms: int):
        self._check(self.lib.rt_set_delta(self.h, int(delta_ms)))

    def set_batch(self, n: int):
        self._check(self.lib.rt_set_batch(self.h, int(n)))


def with_routes(scen, route_ptr, route_edges):
    """The scenario with one route per trip (trip_route[i] = i)."""
    d = dict(scen["demand"])
    d["trip_route"] = np.arange(d["depart_step"].size, dtype=np.int32)
    d["route_ptr"] = route_ptr
    d["route_edges"] = route_edges
    out = dict(scen)
    out["demand"] = d
    return out


def reroute(scen, masks, iterations: int = 4, device: int = 0, on_iteration=None, handoff: str = "device"):
    """The loop of Sec. 6.3.1 on the GPU.  Returns one dict per iteration
    with the weights used, the link statistics and counters, and with
    handoff="host" the routes.  handoff="device": one simulation, its routes
    replaced on the device from the router's table each iteration (the demand
    starts again from its first step); "host": the routes are read out and a
    new simulation is loaded with them."""
    if handoff not in ("device", "host"):
        raise ValueError("handoff is 'device' or 'host'")
    d = scen["demand"]
    rt = Router(scen["net"], device)
    rt.set_trips(d["src_nodes"], d["trip_src"], d["trip_dst"])
    out = []
    sim = None
    for k in range(iterations):
        w = rt.weights()
        rt.plan(None if k == 0 else masks[k])
        ptr = edges = None
        if handoff == "device":
            if sim is None:
                sim = Sim(scen, device)
            sim.reload_routes(*rt.route_views())
        else:
            ptr, edges = rt.routes()
            sim = Sim(with_routes(scen, ptr, edges), device)
        sim.step(scen["steps"])
        st = sim.edge_stats_device()
        rt.weights_from_stats(st["count"], st["tt_us"])
        res = {"weights": w, "route_ptr": ptr, "route_edges": edges,
               "stats": {k2: v.cpu().numpy() for k2, v in st.items()}, "counters": sim.counters()}
        if on_iteration:
            on_iteration(k, res, rt, sim)
        out.append(res)
        if handoff == "host":
            sim.close()
    if sim is not None and handoff == "device":
        sim.close()
    rt.close()
    return out
