"""MI355X traffic microsimulation: Python binding of libtrafficsim.so.

Argument marshalling only.  Every step of the simulation runs in the HIP
kernels of ``csrc/trafficsim.hip`` behind the C ABI of
``include/trafficsim.h``; PyTorch supplies device memory (its caching
allocator, through the library's allocator hooks) and the HIP stream.  If the
library is not built, importing works but creating a simulation raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; TRAFFICSIM_LIB names another build of the same library
LIB_PATH = os.environ.get("TRAFFICSIM_LIB") or os.path.join(_HERE, "libtrafficsim.so")
_LIB = None

SIM_OK, SIM_EINVAL, SIM_EROUTE, SIM_ENOMEM, SIM_EHIP, SIM_ESTATE = 0, -1, -2, -3, -4, -5

EXPORTED = ("sim_create", "sim_load_demand", "sim_step", "sim_stats", "sim_read_vehicles",
            "sim_read_trips", "sim_set_idm", "sim_set_timing", "sim_read_timing", "sim_tape_begin",
            "sim_grad", "sim_read_emissions", "sim_set_sampler", "sim_read_samples", "sim_create_batch",
            "sim_load_demand_batch", "sim_set_launch", "sim_get_launch", "sim_step_graph", "sim_autotune",
            "sim_set_vehicle_types", "sim_set_control", "sim_state_bytes", "sim_get_state", "sim_set_state",
            "sim_set_stream", "sim_destroy", "sim_last_error", "sim_strerror", "sim_replay",
            "sim_set_decide_shape", "sim_get_decide_shape", "sim_step_persistent", "sim_reload_routes",
            "sim_check_state")
# the classes of sim_check_state, in the order of enum sim_check_class
CHECK_CLASSES = ("count", "key", "edge", "order", "position", "speed", "vid", "duplicate", "type", "route", "next",
                 "value", "arrived", "queue", "holder")
KERNELS = ("k_decide", "k_resolve", "k_scan", "k_scatter", "k_place", "k_lanes")


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "error"), code, msg))
        self.code = code


_ERRNAMES = {SIM_EINVAL: "SIM_EINVAL", SIM_EROUTE: "SIM_EROUTE", SIM_ENOMEM: "SIM_ENOMEM",
             SIM_EHIP: "SIM_EHIP", SIM_ESTATE: "SIM_ESTATE"}


class SimNetwork(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_int32), ("num_edges", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("lanes", ctypes.c_void_p),
                ("length_m", ctypes.c_void_p), ("speed_mps", ctypes.c_void_p), ("link_class", ctypes.c_void_p)]


class SimParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("veh_length", ctypes.c_float), ("s0", ctypes.c_float),
                ("s_eps", ctypes.c_float), ("b_max", ctypes.c_float), ("num_classes", ctypes.c_int32),
                ("idm", ctypes.c_void_p), ("mobil_p", ctypes.c_float), ("mobil_athr", ctypes.c_float),
                ("mobil_bsafe", ctypes.c_float), ("mand_dist", ctypes.c_float),
                ("lc_cooldown_steps", ctypes.c_int32)]


class SimStateView(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("num_vehicles", ctypes.c_int32)] + \
               [(n, ctypes.c_void_p) for n in ("key", "x", "v", "edge", "vid", "type")]


class SimStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("step", "loaded", "waiting", "en_route", "arrived", "departed",
                                              "vehicle_updates", "claims_lost", "clamps", "claims",
                                              "claims_departure", "lc_evaluated", "claims_lane_change")]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def library(path: str = LIB_PATH):
    """Load libtrafficsim.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch first: the library then binds to the HIP runtime torch loaded
        # (the same soname), whose device memory and streams it is handed
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise ImportError("libtrafficsim.so is not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(path)
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.sim_create.argtypes = [ctypes.POINTER(SimNetwork), ctypes.POINTER(SimParams), P, ALLOC_FN, FREE_FN,
                                   P, ctypes.POINTER(P)]
        lib.sim_create.restype = ctypes.c_int
        lib.sim_load_demand.argtypes = [P, i32, P, P, i32, P, P, P, P, P]
        lib.sim_load_demand.restype = ctypes.c_int
        lib.sim_step.argtypes = [P, i32]
        lib.sim_step.restype = ctypes.c_int
        lib.sim_step_persistent.argtypes = [P, i32]
        lib.sim_step_persistent.restype = ctypes.c_int
        lib.sim_reload_routes.argtypes = [P, P, P, ctypes.c_int64]
        lib.sim_reload_routes.restype = ctypes.c_int
        lib.sim_stats.argtypes = [P, ctypes.POINTER(SimStats), P, P, P]
        lib.sim_stats.restype = ctypes.c_int
        lib.sim_read_vehicles.argtypes = [P, i32, ctypes.POINTER(i32), P, P, P, P, P, P, P, P, P, P, P]
        lib.sim_read_vehicles.restype = ctypes.c_int
        lib.sim_read_trips.argtypes = [P, P, P]
        lib.sim_read_trips.restype = ctypes.c_int
        lib.sim_read_emissions.argtypes = [P, P, P]
        lib.sim_read_emissions.restype = ctypes.c_int
        lib.sim_set_sampler.argtypes = [P, i32, i32, i32]
        lib.sim_set_sampler.restype = ctypes.c_int
        lib.sim_read_samples.argtypes = [P, P, P]
        lib.sim_read_samples.restype = ctypes.c_int
        lib.sim_set_idm.argtypes = [P, P]
        lib.sim_set_idm.restype = ctypes.c_int
        lib.sim_set_timing.argtypes = [P, i32]
        lib.sim_set_timing.restype = ctypes.c_int
        lib.sim_read_timing.argtypes = [P, P, ctypes.POINTER(ctypes.c_int64)]
        lib.sim_read_timing.restype = ctypes.c_int
        lib.sim_tape_begin.argtypes = [P, i32]
        lib.sim_tape_begin.restype = ctypes.c_int
        lib.sim_grad.argtypes = [P, P, P]
        lib.sim_grad.restype = ctypes.c_int
        lib.sim_replay.argtypes = [P, P, i32, P]
        lib.sim_replay.restype = ctypes.c_int
        lib.sim_set_vehicle_types.argtypes = [P, i32, P, i32, P]
        lib.sim_set_vehicle_types.restype = ctypes.c_int
        lib.sim_set_control.argtypes = [P, P, i32, ctypes.c_float, ctypes.c_float]
        lib.sim_set_control.restype = ctypes.c_int
        lib.sim_state_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        lib.sim_state_bytes.restype = ctypes.c_int
        lib.sim_get_state.argtypes = [P, ctypes.POINTER(SimStateView), P]
        lib.sim_get_state.restype = ctypes.c_int
        lib.sim_set_state.argtypes = [P, P, ctypes.c_size_t]
        lib.sim_set_state.restype = ctypes.c_int
        lib.sim_check_state.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
        lib.sim_check_state.restype = ctypes.c_int
        lib.sim_set_stream.argtypes = [P, P]
        lib.sim_set_stream.restype = ctypes.c_int
        lib.sim_destroy.argtypes = [P]
        lib.sim_destroy.restype = None
        lib.sim_last_error.argtypes = [P]
        lib.sim_last_error.restype = ctypes.c_char_p
        lib.sim_strerror.argtypes = [ctypes.c_int]
        lib.sim_strerror.restype = ctypes.c_char_p
        _LIB = lib
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _TorchAllocator:
    """Allocator hooks backed by torch's caching allocator on one stream."""

    def __init__(self, device, stream):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, ctx, nbytes):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:  # noqa: BLE001 - reported to the library as NULL
            return None

    def _free(self, ctx, ptr):
        self.torch.cuda.caching_allocator_delete(ptr)


class Sim:
    """A simulation of one scenario dict (see ``scenarios``) on one GPU.

    ``stream``: a torch.cuda.Stream (default: the current stream of
    ``device``).  ``torch_alloc``: route device allocations through torch's
    caching allocator (otherwise the library calls hipMalloc)."""

    def __init__(self, scen, device: int = 0, stream=None, torch_alloc: bool = True):
        import torch
        self.lib = library()
        self.h = None
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._alloc = _TorchAllocator(device, stream) if torch_alloc else None
        net, p = scen["net"], scen["params"]
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dt)
            keep.append(a)
            return _p(a)

        self.num_edges = int(net["col_idx"].size)
        cls = net.get("link_class")
        self._net = SimNetwork(int(net["row_ptr"].size - 1), self.num_edges, arr(net["row_ptr"], np.int32),
                               arr(net["col_idx"], np.int32), arr(net["lanes"], np.int32),
                               arr(net["length"], np.float32), arr(net["speed"], np.float32),
                               None if cls is None else arr(cls, np.int32))
        self.num_classes = int(p["num_classes"])
        idm = np.ascontiguousarray(p["idm"], np.float32).reshape(self.num_classes, 4)
        self._params = SimParams(p["dt"], p["veh_length"], p["s0"], p["s_eps"], p["b_max"], self.num_classes,
                                 arr(idm, np.float32), p["mobil_p"], p["mobil_athr"], p["mobil_bsafe"],
                                 p["mand_dist"], int(p["lc_cooldown"]))
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            rc = self.lib.sim_create(ctypes.byref(self._net), ctypes.byref(self._params),
                                     ctypes.c_void_p(stream.cuda_stream),
                                     self._alloc.alloc if self._alloc else ALLOC_FN(),
                                     self._alloc.free if self._alloc else FREE_FN(), None, ctypes.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, self.lib.sim_strerror(rc).decode())
        self.h = h
        if net.get("node_control") is not None:
            self.set_control(net["node_control"], p.get("signal_green", 20), p.get("stop_dist", 3.0),
                             p.get("stop_speed", 0.5))
        d = scen["demand"]
        self.num_trips = int(d["depart_step"].size)
        if p.get("vehicle_types") is not None or d.get("trip_type") is not None:
            self.set_vehicle_types(p.get("vehicle_types", [[p["veh_length"], np.inf, np.inf]]), d.get("trip_type"))
        ix = d.get("init_x")
        with torch.cuda.device(device):
            rc = self.lib.sim_load_demand(
                self.h, self.num_trips, arr(d["depart_step"], np.int32), arr(d["trip_route"], np.int32),
                int(d["route_ptr"].size - 1), arr(d["route_ptr"], np.int64), arr(d["route_edges"], np.int32),
                None if ix is None else arr(ix, np.float32),
                None if d.get("init_v") is None else arr(d["init_v"], np.float32),
                None if d.get("init_lane") is None else arr(d["init_lane"], np.int32))
        self._check(rc)

    def set_vehicle_types(self, types, trip_type=None):
        """types: [[length, accel cap, speed cap], ...]; trip_type: per trip (input order)."""
        import torch
        vt = np.ascontiguousarray(types, np.float32).reshape(-1, 3)
        tt = None if trip_type is None else np.ascontiguousarray(trip_type, np.uint8)
        with torch.cuda.device(self.device):
            self._check(self.lib.sim_set_vehicle_types(self.h, int(vt.shape[0]), _p(vt), self.num_trips, _p(tt)))

    def set_control(self, node_control, signal_green=20, stop_dist=3.0, stop_speed=0.5):
        """Stop signs (1) and signals (2) per node, 0 = uncontrolled."""
        import torch
        ctrl = np.ascontiguousarray(node_control, np.int32)
        with torch.cuda.device(self.device):
            self._check(self.lib.sim_set_control(self.h, _p(ctrl), int(signal_green), float(stop_dist),
                                                 float(stop_speed)))

    def _check(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, self.lib.sim_last_error(self.h).decode())

    def close(self):
        if self.h is not None:
            import torch
            with torch.cuda.device(self.device):
                self.lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def step(self, n: int = 1):
        self._check(self.lib.sim_step(self.h, int(n)))

    def step_persistent(self, n: int = 1):
        """n steps in persistent launches (one cooperative launch per up to
        600 steps, device-wide barriers between the phases); synchronises."""
        self._check(self.lib.sim_step_persistent(self.h, int(n)))

    def counters(self) -> dict:
        st = SimStats()
        self._check(self.lib.sim_stats(self.h, ctypes.byref(st), None, None, None))
        return {n: int(getattr(st, n)) for n, _ in SimStats._fields_}

    def edge_stats_device(self):
        """Per-edge statistics as int64 torch tensors on the device."""
        import torch
        out = [torch.empty(self.num_edges, dtype=torch.int64, device="cuda:%d" % self.device) for _ in range(3)]
        with torch.cuda.stream(self.stream):
            self._check(self.lib.sim_stats(self.h, None, ctypes.c_void_p(out[0].data_ptr()),
                                           ctypes.c_void_p(out[1].data_ptr()), ctypes.c_void_p(out[2].data_ptr())))
        return {"count": out[0], "tt_steps": out[1], "tt_us": out[2]}

    def edge_stats(self) -> dict:
        d = self.edge_stats_device()
        self.stream.synchronize()
        return {k: v.cpu().numpy() for k, v in d.items()}

    def vehicles(self) -> dict:
        """Vehicles on the road, sorted by vehicle id (host arrays)."""
        n = ctypes.c_int32(0)
        cap = self.num_trips
        iv = {k: np.zeros(max(cap, 1), np.int32) for k in ("vid", "edge", "lane", "cursor", "lc", "kin")}
        fv = {k: np.zeros(max(cap, 1), np.float32) for k in ("x", "v", "phin", "fuel", "co")}
        self._check(self.lib.sim_read_vehicles(self.h, cap, ctypes.byref(n), _p(iv["vid"]), _p(iv["edge"]),
                                               _p(iv["lane"]), _p(iv["cursor"]), _p(iv["lc"]), _p(iv["kin"]),
                                               _p(fv["x"]), _p(fv["v"]), _p(fv["phin"]), _p(fv["fuel"]),
                                               _p(fv["co"])))
        m = n.value
        o = np.argsort(iv["vid"][:m], kind="stable")
        out = {k: a[:m][o] for k, a in iv.items()}
        out.update({k: a[:m][o] for k, a in fv.items()})
        return out

    def state_view(self) -> SimStateView:
        """Step, vehicle count and DEVICE pointers of the current vehicle arrays."""
        v = SimStateView()
        self._check(self.lib.sim_get_state(self.h, ctypes.byref(v), None))
        return v

    def save_state(self):
        """The whole dynamic state as a uint8 tensor on the device (a checkpoint)."""
        import torch
        nb = ctypes.c_size_t(0)
        self._check(self.lib.sim_state_bytes(self.h, ctypes.byref(nb)))
        img = torch.empty(nb.value, dtype=torch.uint8, device="cuda:%d" % self.device)
        self.stream.synchronize()  # the tensor's memory is ready before the library's stream writes it
        v = SimStateView()
        self._check(self.lib.sim_get_state(self.h, ctypes.byref(v), ctypes.c_void_p(img.data_ptr())))
        return img

    def load_state(self, img):
        """Continue from a checkpoint written by save_state (this simulation or
        another one with the same network, parameters, types and demand)."""
        self.stream.synchronize()
        self._check(self.lib.sim_set_state(self.h, ctypes.c_void_p(img.data_ptr()), img.numel()))

    def check_state(self):
        """sim_check_state: violations per class of the current state (all 0
        for a valid one) and the lowest offending entry of each class (None
        where there is none)."""
        n = len(CHECK_CLASSES)
        counts = (ctypes.c_int64 * n)()
        first = (ctypes.c_int32 * n)()
        self._check(self.lib.sim_check_state(self.h, counts, first))
        return ({c: int(counts[k]) for k, c in enumerate(CHECK_CLASSES)},
                {c: (None if first[k] == 2**31 - 1 else int(first[k])) for k, c in enumerate(CHECK_CLASSES)})

    def reload_routes(self, route_ptr, route_edges, total=None):
        """sim_reload_routes: new routes for the same trips from DEVICE memory
        (torch tensors on this GPU, int64 [num_trips + 1] and int32, or raw
        device addresses with `total`), and the demand started again from
        its first step."""
        if hasattr(route_ptr, "data_ptr"):
            import torch
            if route_ptr.dtype != torch.int64 or route_edges.dtype != torch.int32 or not route_ptr.is_cuda \
                    or not route_edges.is_cuda or route_ptr.numel() != self.num_trips + 1:
                raise ValueError("route_ptr: int64 [num_trips + 1] and route_edges: int32, both on the GPU")
            route_ptr, route_edges = route_ptr.contiguous(), route_edges.contiguous()
            total = route_edges.numel()
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            pa, ea = route_ptr.data_ptr(), route_edges.data_ptr()
        else:
            if total is None:
                raise ValueError("raw device addresses need the total number of route edges")
            pa, ea = int(route_ptr), int(route_edges)
        self._check(self.lib.sim_reload_routes(self.h, ctypes.c_void_p(pa), ctypes.c_void_p(ea or None),
                                               int(total)))

    def trips(self) -> dict:
        da = np.zeros(self.num_trips, np.int32)
        ar = np.zeros(self.num_trips, np.int32)
        self._check(self.lib.sim_read_trips(self.h, _p(da), _p(ar)))
        return {"depart_actual": da, "arrive_step": ar}

    def emissions(self) -> dict:
        """Fuel (mL) and CO (g) of every vehicle id over its trip (0 before arrival)."""
        f = np.zeros(self.num_trips, np.float32)
        c = np.zeros(self.num_trips, np.float32)
        self._check(self.lib.sim_read_emissions(self.h, _p(f), _p(c)))
        return {"fuel": f, "co": c}

    def set_sampler(self, every: int = 120, group: int = 6, max_groups: int = 32):
        """Sample link utilization and speed every ``every`` steps, in groups."""
        self._check(self.lib.sim_set_sampler(self.h, int(every), int(group), int(max_groups)))
        self._samp = (int(max_groups), int(group))

    def samples(self) -> dict:
        g = self._samp[0]
        cnt = np.zeros((g, self.num_edges), np.int64)
        spd = np.zeros((g, self.num_edges), np.int64)
        self._check(self.lib.sim_read_samples(self.h, _p(cnt), _p(spd)))
        return {"count": cnt, "speed_um": spd}

    def set_timing(self, every: int):
        """Sample per-kernel HIP-event timings on every ``every``-th step."""
        self._check(self.lib.sim_set_timing(self.h, int(every)))

    def read_timing(self):
        """(sum of ms per kernel over sampled steps, number of sampled steps)."""
        # room for more kernels than this binding names (a newer library)
        ms = np.zeros(max(32, len(KERNELS)), np.float64)
        n = ctypes.c_int64(0)
        self._check(self.lib.sim_read_timing(self.h, _p(ms), ctypes.byref(n)))
        return dict(zip(KERNELS, ms[:len(KERNELS)].tolist())), int(n.value)

    def tape_begin(self, checkpoint_every: int = 60):
        """Start a differentiation window at the current step."""
        self._check(self.lib.sim_tape_begin(self.h, int(checkpoint_every)))

    def mean_travel_times(self):
        """Mean crossing-interpolated travel time per link in seconds (torch
        float32 on the device; 0 where no traversal was completed) and the
        traversal counts."""
        import torch
        st = self.edge_stats_device()
        cnt = st["count"]
        with torch.cuda.stream(self.stream):
            tbar = torch.where(cnt > 0, st["tt_us"].double() / cnt.clamp(min=1).double() / 1e6,
                               torch.zeros((), dtype=torch.float64, device=cnt.device)).float()
        return tbar, cnt

    def grad(self, dL_dmeanTT):
        """dLoss/dtheta [num_classes, 4] (torch float32, device) for the window
        since tape_begin, given dLoss/d(mean link travel time) [num_edges]."""
        import torch
        g = dL_dmeanTT.detach().to(device="cuda:%d" % self.device, dtype=torch.float32).contiguous()
        out = torch.empty(self.num_classes * 4, dtype=torch.float32, device=g.device)
        with torch.cuda.stream(self.stream):
            self._check(self.lib.sim_grad(self.h, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out.view(self.num_classes, 4)

    def replay(self, idm, fp64: bool = False) -> np.ndarray:
        """Frozen-event replay of the differentiation window at ``idm``
        [num_classes, 4], in float or double: per link, the sum over the
        window's completed traversals of (exit fraction - entry fraction),
        float64 [num_edges]."""
        idm = np.ascontiguousarray(idm, np.float64).reshape(self.num_classes, 4)
        out = np.zeros(self.num_edges, np.float64)
        self.stream.synchronize()
        self._check(self.lib.sim_replay(self.h, _p(idm), 1 if fp64 else 0, _p(out)))
        return out

    def set_idm(self, idm):
        idm = np.ascontiguousarray(idm, np.float32).reshape(self.num_classes, 4)
        self._check(self.lib.sim_set_idm(self.h, _p(idm)))
