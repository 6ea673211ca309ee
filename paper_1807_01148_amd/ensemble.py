"""Batched ensembles of scenarios, graph-captured multi-step launches and the
launch-shape autotuner (argument marshalling over the C ABI only).

``Ensemble(scens)`` simulates several scenarios -- different networks, demand
and car-following parameters, one common time step -- as one simulation on
one GPU (sim_create_batch / sim_load_demand_batch).  Each scenario evolves
exactly as in its own simulation; ``scenario_*`` split the outputs back.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from . import (ALLOC_FN, FREE_FN, SIM_OK, Sim, SimError, SimNetwork, SimParams, _TorchAllocator, _p,
               library)

_BOUND = False


def _bind(lib):
    global _BOUND
    if _BOUND:
        return lib
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.sim_create_batch.argtypes = [i32, P, P, P, ALLOC_FN, FREE_FN, P, ctypes.POINTER(P)]
    lib.sim_create_batch.restype = ctypes.c_int
    lib.sim_load_demand_batch.argtypes = [P, i32, P, P, P, P, P, P]
    lib.sim_load_demand_batch.restype = ctypes.c_int
    lib.sim_set_launch.argtypes = [P, i32, i32]
    lib.sim_set_launch.restype = ctypes.c_int
    lib.sim_get_launch.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.sim_get_launch.restype = ctypes.c_int
    lib.sim_set_decide_shape.argtypes = [P, i32, i32]
    lib.sim_set_decide_shape.restype = ctypes.c_int
    lib.sim_get_decide_shape.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.sim_get_decide_shape.restype = ctypes.c_int
    lib.sim_step_graph.argtypes = [P, i32, i32]
    lib.sim_step_graph.restype = ctypes.c_int
    lib.sim_autotune.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    lib.sim_autotune.restype = ctypes.c_int
    _BOUND = True
    return lib


def vehicle_ids(depart_step):
    """Vehicle id of every trip: its rank by (departure step, trip index)."""
    dep = np.asarray(depart_step)
    order = np.lexsort((np.arange(dep.size), dep))
    vid = np.empty(dep.size, np.int64)
    vid[order] = np.arange(dep.size)
    return vid


def step_graph(sim: Sim, n: int, chunk: int = 60):
    """Advance ``n`` steps, replaying captured ``chunk``-step graphs."""
    lib = _bind(library())
    sim._check(lib.sim_step_graph(sim.h, int(n), int(chunk)))


def set_launch(sim: Sim, grid: int, grid_small: int):
    lib = _bind(library())
    sim._check(lib.sim_set_launch(sim.h, int(grid), int(grid_small)))


def get_launch(sim: Sim):
    lib = _bind(library())
    g, s = ctypes.c_int32(0), ctypes.c_int32(0)
    sim._check(lib.sim_get_launch(sim.h, ctypes.byref(g), ctypes.byref(s)))
    return g.value, s.value


def set_decide_shape(sim: Sim, block: int, per_thread: int):
    lib = _bind(library())
    sim._check(lib.sim_set_decide_shape(sim.h, int(block), int(per_thread)))


def get_decide_shape(sim: Sim):
    lib = _bind(library())
    b, r = ctypes.c_int32(0), ctypes.c_int32(0)
    sim._check(lib.sim_get_decide_shape(sim.h, ctypes.byref(b), ctypes.byref(r)))
    return b.value, r.value


def apply_shape(sim: Sim, shape: dict):
    """Set a launch shape as autotune returns it (grids, decide shape)."""
    set_launch(sim, shape["grid"], shape["grid_small"])
    if "decide_block" in shape:
        set_decide_shape(sim, shape["decide_block"], shape["decide_per_thread"])


def device_key(device: int = 0) -> str:
    """The GPU's architecture name (e.g. gfx950), the key of tuned launch
    shapes: stable across drivers and profilers, unlike the marketing name."""
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def autotune(sim: Sim, steps_per_trial: int = 60, cache_key: str | None = None, cache_path: str | None = None):
    """Pick the fastest launch shape from the current state (the state is
    restored).  With ``cache_key``, a result stored in the JSON cache (keyed by
    device name and ``cache_key``) is reused instead of timing again."""
    import torch
    lib = _bind(library())
    path = cache_path or os.path.join(os.path.expanduser("~"), ".cache", "trafficsim_autotune.json")
    key = None
    if cache_key is not None:
        key = "%s|%s" % (device_key(sim.device), cache_key)
        try:
            with open(path) as f:
                hit = json.load(f).get(key)
        except (OSError, ValueError):
            hit = None
        if hit:
            apply_shape(sim, hit)
            return dict(hit, cached=True)
    g, s, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0.0)
    sim._check(lib.sim_autotune(sim.h, int(steps_per_trial), ctypes.byref(g), ctypes.byref(s), ctypes.byref(ms)))
    db_, dr_ = get_decide_shape(sim)
    res = {"grid": g.value, "grid_small": s.value, "decide_block": db_, "decide_per_thread": dr_,
           "ms_per_step": ms.value}
    if key is not None:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            try:
                with open(path) as f:
                    db = json.load(f)
            except (OSError, ValueError):
                db = {}
            db[key] = res
            with open(path, "w") as f:
                json.dump(db, f, indent=1)
        except OSError:
            pass
    return dict(res, cached=False)


class Ensemble(Sim):
    """Several scenarios in one simulation (one batched launch per kernel)."""

    def __init__(self, scens, device: int = 0, stream=None, torch_alloc: bool = True):
        import torch
        self.lib = _bind(library())
        self.h = None
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._alloc = _TorchAllocator(device, stream) if torch_alloc else None
        n = len(scens)
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dt)
            keep.append(a)
            return _p(a)

        nets = (SimNetwork * n)()
        prms = (SimParams * n)()
        self.edge_off = [0]
        self.trip_off = [0]
        ncls = 0
        for q, sc in enumerate(scens):
            net, p = sc["net"], sc["params"]
            ne = int(net["col_idx"].size)
            cls = net.get("link_class")
            nets[q] = SimNetwork(int(net["row_ptr"].size - 1), ne, arr(net["row_ptr"], np.int32),
                                 arr(net["col_idx"], np.int32), arr(net["lanes"], np.int32),
                                 arr(net["length"], np.float32), arr(net["speed"], np.float32),
                                 None if cls is None else arr(cls, np.int32))
            k = int(p["num_classes"])
            prms[q] = SimParams(p["dt"], p["veh_length"], p["s0"], p["s_eps"], p["b_max"], k,
                                arr(np.asarray(p["idm"], np.float32).reshape(k, 4), np.float32), p["mobil_p"],
                                p["mobil_athr"], p["mobil_bsafe"], p["mand_dist"], int(p["lc_cooldown"]))
            ncls += k
            self.edge_off.append(self.edge_off[-1] + ne)
            self.trip_off.append(self.trip_off[-1] + int(sc["demand"]["depart_step"].size))
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            rc = self.lib.sim_create_batch(n, ctypes.cast(nets, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p),
                                           ctypes.c_void_p(stream.cuda_stream),
                                           self._alloc.alloc if self._alloc else ALLOC_FN(),
                                           self._alloc.free if self._alloc else FREE_FN(), None, ctypes.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, self.lib.sim_strerror(rc).decode())
        self.h = h
        self.num_scenarios = n
        self.num_edges = self.edge_off[-1]
        self.num_trips = self.trip_off[-1]
        self.num_classes = ncls
        if any(sc["net"].get("node_control") is not None for sc in scens):
            # one control array over the concatenated nodes; the timing parameters are shared
            keys = ("signal_green", "stop_dist", "stop_speed")
            ctl = [tuple(sc["params"].get(k, d) for k, d in zip(keys, (20, 3.0, 0.5))) for sc in scens]
            if len(set(ctl)) != 1:
                raise ValueError("ensemble members must share signal_green, stop_dist and stop_speed")
            ctrl = np.concatenate([np.asarray(sc["net"]["node_control"], np.int32)
                                   if sc["net"].get("node_control") is not None
                                   else np.zeros(sc["net"]["row_ptr"].size - 1, np.int32) for sc in scens])
            self.set_control(ctrl, *ctl[0])
        if any(sc["params"].get("vehicle_types") is not None or sc["demand"].get("trip_type") is not None
               for sc in scens):
            # one type table for the batch; trip types concatenated in scenario order
            tabs = [np.asarray(sc["params"].get("vehicle_types", [[sc["params"]["veh_length"], np.inf, np.inf]]),
                               np.float32) for sc in scens]
            if any(t.shape != tabs[0].shape or not np.array_equal(t, tabs[0]) for t in tabs):
                raise ValueError("ensemble members must share their vehicle types")
            tt = np.concatenate([np.asarray(sc["demand"]["trip_type"], np.uint8)
                                 if sc["demand"].get("trip_type") is not None
                                 else np.zeros(sc["demand"]["depart_step"].size, np.uint8) for sc in scens])
            self.set_vehicle_types(tabs[0], tt)
        PP = ctypes.c_void_p * n
        dem = [sc["demand"] for sc in scens]
        ntr = np.array([d["depart_step"].size for d in dem], np.int32)
        nro = np.array([d["route_ptr"].size - 1 for d in dem], np.int32)
        dep = PP(*[arr(d["depart_step"], np.int32) for d in dem])
        trr = PP(*[arr(d["trip_route"], np.int32) for d in dem])
        rpt = PP(*[arr(d["route_ptr"], np.int64) for d in dem])
        red = PP(*[arr(d["route_edges"], np.int32) for d in dem])
        with torch.cuda.device(device):
            rc = self.lib.sim_load_demand_batch(self.h, n, _p(ntr), ctypes.cast(dep, ctypes.c_void_p),
                                                ctypes.cast(trr, ctypes.c_void_p), _p(nro),
                                                ctypes.cast(rpt, ctypes.c_void_p), ctypes.cast(red, ctypes.c_void_p))
        self._check(rc)
        all_dep = np.concatenate([np.asarray(d["depart_step"], np.int64) for d in dem]) if n else np.zeros(0)
        self._vid_of_trip = vehicle_ids(all_dep)

    def scenario_edge_stats(self, q: int, stats=None):
        st = stats if stats is not None else self.edge_stats()
        a, b = self.edge_off[q], self.edge_off[q + 1]
        return {k: v[a:b] for k, v in st.items()}

    def scenario_trips(self, q: int, trips=None):
        """Per-trip outcomes of scenario q, indexed by the scenario's trip index."""
        tr = trips if trips is not None else self.trips()
        vids = self._vid_of_trip[self.trip_off[q]:self.trip_off[q + 1]]
        return {k: v[vids] for k, v in tr.items()}
