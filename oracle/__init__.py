"""CPU oracle for the traffic microsimulation step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

``oracle.c`` is one plain C source compiled twice (FP32 and FP64, -O2
-ffp-contract=off -fno-fast-math); ``brute.py`` is an independent pure-Python
FP64 implementation with O(N^2) neighbour searches and pairwise claim checks,
used to pin the C oracle on tiny networks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}

FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC"]


def build(force: bool = False):
    """Compile liboracle_f32.so, liboracle_f64.so, libadjoint.so and
    liboracle_route.so with gcc."""
    outs = []
    # f32omp: the FP32 oracle with its per-vehicle decision loop split over
    # threads (OpenMP); the same source, the same results
    for prec, defs, name in (("f32", [], "oracle.c"), ("f64", ["-DORACLE_F64"], "oracle.c"),
                             ("f32omp", ["-fopenmp"], "oracle.c"),
                             ("adj", [], "adjoint.c"), ("route", [], "routing.c")):
        src = os.path.join(_HERE, name)
        out = os.path.join(_HERE, "liboracle_%s.so" % prec if prec != "adj" else "libadjoint.so")
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
            tmp = out + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc"] + FLAGS + defs + ["-o", tmp, src, "-lm"])
            os.replace(tmp, out)
        outs.append(out)
    return outs


def _path(key, default):
    """The library to load: a sanitizer build named by ORACLE_LIB_<KEY> (the
    sanitizer test's child process), else the one build() writes."""
    return os.environ.get("ORACLE_LIB_" + key, os.path.join(_HERE, default))


def _adjlib():
    if "adj" not in _LIBS:
        build()
        lib = ctypes.CDLL(_path("ADJ", "libadjoint.so"))
        P = ctypes.c_void_p
        lib.adj_eval.argtypes = [ctypes.c_int64] + [P] * 8 + [ctypes.c_int32, ctypes.c_int32, P, P, P,
                                                            ctypes.c_int32] + [P] * 9 + [ctypes.c_int32] * 2 + [P] * 2
        lib.adj_eval.restype = ctypes.c_int
        _LIBS["adj"] = lib
    return _LIBS["adj"]


def _lib(prec):
    if prec not in _LIBS:
        build()
        lib = ctypes.CDLL(_path(prec.upper(), "liboracle_%s.so" % prec))
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        lib.or_create.argtypes = [i32, i32, P, P, P, P, P, P, i32, P, P, i32, P]
        lib.or_create.restype = P
        lib.or_destroy.argtypes = [P]
        lib.or_load_demand.argtypes = [P, i32, P, P, i32, P, P, P, P, P]
        lib.or_load_demand.restype = ctypes.c_int
        lib.or_step.argtypes = [P, i32]
        lib.or_step.restype = ctypes.c_int
        lib.or_counters.argtypes = [P, P]
        lib.or_get_vehicles.argtypes = [P, P, P]
        lib.or_get_vehicles.restype = i32
        lib.or_get_trips.argtypes = [P, P, P]
        lib.or_get_edge_stats.argtypes = [P, P, P, P]
        lib.or_num_active.argtypes = [P]
        lib.or_num_active.restype = i32
        lib.or_num_pending.argtypes = [P]
        lib.or_num_pending.restype = i32
        lib.or_set_vehicle_types.argtypes = [P, i32, P, i32, P]
        lib.or_set_vehicle_types.restype = ctypes.c_int
        lib.or_set_control.argtypes = [P, P, i32, ctypes.c_float, ctypes.c_float]
        lib.or_set_control.restype = ctypes.c_int
        lib.or_get_emissions.argtypes = [P, P, P]
        lib.or_set_sampler.argtypes = [P, i32, i32, i32]
        lib.or_set_sampler.restype = ctypes.c_int
        lib.or_get_samples.argtypes = [P, P, P]
        lib.or_tape_enable.argtypes = [P, i32]
        lib.or_tape_size.argtypes = [P]
        lib.or_tape_size.restype = ctypes.c_int64
        lib.or_tape_get.argtypes = [P] + [P] * 8
        lib.or_set_state.argtypes = [P, i32, i32] + [P] * 10
        lib.or_set_state.restype = ctypes.c_int
        _LIBS[prec] = lib
    return _LIBS[prec]


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def fparams(p):
    """The float parameter block shared by both implementations' entry points."""
    return np.array([p["dt"], p["veh_length"], p["s0"], p["s_eps"], p["b_max"],
                     p["mobil_p"], p["mobil_athr"], p["mobil_bsafe"], p["mand_dist"]], np.float32)


COUNTERS = ("step", "loaded", "waiting", "en_route", "arrived", "departed",
            "vehicle_updates", "claims_lost", "clamps", "claims", "claims_departure",
            "lc_evaluated", "claims_lane_change")


class OracleError(RuntimeError):
    pass


TAPE_INT = ("step", "vid", "mode", "lead", "flags", "edge")
TAPE_F64 = ("x0", "v0")


def replay(tape, scen, theta, target, mask, grad=True, at_tape_states=False):
    """Frozen-event FP64 replay of ``tape`` at parameters ``theta``
    [num_classes, 4] = (v0_scale, T, a, b): returns (loss, gradient or None,
    mean link travel times [E], final x [V], final v [V]).  With
    ``at_tape_states`` the states are taken from the tape instead of being
    replayed (linearization along the recording forward's trajectory)."""
    lib = _adjlib()
    net, p = scen["net"], scen["params"]
    ne = int(net["col_idx"].size)
    nveh = int(scen["demand"]["depart_step"].size)
    # the network and constants enter as the float32 values the simulators use
    length = np.asarray(net["length"], np.float32).astype(np.float64)
    speed = np.asarray(net["speed"], np.float32).astype(np.float64)
    cls = np.ascontiguousarray(net.get("link_class", np.zeros(ne)), np.int32)
    th = np.ascontiguousarray(theta, np.float64).reshape(-1, 4)
    fp = np.array([np.float32(p[k]) for k in ("dt", "veh_length", "s0", "s_eps", "b_max")], np.float64)
    tgt = np.ascontiguousarray(target, np.float64)
    msk = np.ascontiguousarray(mask, np.uint8)
    loss = ctypes.c_double(0.0)
    g = np.zeros(th.size, np.float64) if grad else None
    tbar = np.zeros(ne, np.float64)
    xf = np.zeros(max(nveh, 1), np.float64)
    vf = np.zeros(max(nveh, 1), np.float64)
    tp = {k: np.ascontiguousarray(tape[k]) for k in TAPE_INT + TAPE_F64}
    # vehicle types (Sec. 6.3.5): the table as float32 inputs, the type of each vehicle id
    types = np.ascontiguousarray(np.asarray(p.get("vehicle_types", [[p["veh_length"], np.inf, np.inf]]),
                                            np.float32).astype(np.float64).reshape(-1, 3))
    tt = scen["demand"].get("trip_type")
    dep = np.asarray(scen["demand"]["depart_step"])
    order = np.lexsort((np.arange(dep.size), dep))  # vehicle id -> trip
    vtype = np.zeros(max(nveh, 1), np.int32)
    if tt is not None:
        vtype[:nveh] = np.asarray(tt, np.int32)[order]
    rc = lib.adj_eval(int(tp["step"].size), *[_p(tp[k]) for k in TAPE_INT + TAPE_F64], nveh, ne,
                      _p(length), _p(speed), _p(cls), int(th.shape[0]), _p(th), _p(fp), _p(tgt), _p(msk),
                      ctypes.byref(loss), _p(g), _p(tbar), _p(xf), _p(vf), 1 if at_tape_states else 0,
                      int(types.shape[0]), _p(types), _p(vtype))
    if rc != 0:
        raise OracleError("adj_eval failed: %d" % rc)
    return loss.value, (None if g is None else g.reshape(th.shape)), tbar, xf[:nveh], vf[:nveh]


class Oracle:
    """One oracle simulation of a scenario dict (see ``scenarios``)."""

    def __init__(self, scen, precision: str = "f32", tape: bool = False):
        self.lib = _lib(precision)
        self.precision = precision
        net, p = scen["net"], scen["params"]
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dt)
            self._keep.append(a)
            return a

        self.ne = int(net["col_idx"].size)
        err = ctypes.c_int32(0)
        idm = arr(p["idm"], np.float32)
        self.h = self.lib.or_create(
            int(net["row_ptr"].size - 1), self.ne, _p(arr(net["row_ptr"], np.int32)),
            _p(arr(net["col_idx"], np.int32)), _p(arr(net["lanes"], np.int32)),
            _p(arr(net["length"], np.float32)), _p(arr(net["speed"], np.float32)),
            _p(arr(net.get("link_class", np.zeros(self.ne)), np.int32)), int(p["num_classes"]),
            _p(idm), _p(arr(fparams(p), np.float32)), int(p["lc_cooldown"]), ctypes.byref(err))
        if not self.h:
            raise OracleError("or_create failed: %d" % err.value)
        if net.get("node_control") is not None:
            ctrl = arr(net["node_control"], np.int32)
            if self.lib.or_set_control(self.h, _p(ctrl), int(p.get("signal_green", 20)),
                                       float(p.get("stop_dist", 3.0)), float(p.get("stop_speed", 0.5))) != 0:
                self.lib.or_destroy(self.h)
                self.h = None
                raise OracleError("or_set_control failed")
        d = scen["demand"]
        self.ntrips = int(d["depart_step"].size)
        if p.get("vehicle_types") is not None or d.get("trip_type") is not None:
            vt = arr(p.get("vehicle_types", [[p["veh_length"], np.inf, np.inf]]), np.float32)
            tt = None if d.get("trip_type") is None else arr(d["trip_type"], np.uint8)
            if self.lib.or_set_vehicle_types(self.h, int(vt.size // 3), _p(vt), self.ntrips, _p(tt)) != 0:
                self.lib.or_destroy(self.h)
                self.h = None
                raise OracleError("or_set_vehicle_types failed")
        ix = d.get("init_x")
        if tape:
            self.lib.or_tape_enable(self.h, 1)
        rc = self.lib.or_load_demand(
            self.h, self.ntrips, _p(arr(d["depart_step"], np.int32)), _p(arr(d["trip_route"], np.int32)),
            int(d["route_ptr"].size - 1), _p(arr(d["route_ptr"], np.int64)), _p(arr(d["route_edges"], np.int32)),
            _p(None if ix is None else arr(ix, np.float32)),
            _p(None if d.get("init_v") is None else arr(d["init_v"], np.float32)),
            _p(None if d.get("init_lane") is None else arr(d["init_lane"], np.int32)))
        self._keep = []
        if rc != 0:
            self.lib.or_destroy(self.h)
            self.h = None
            raise OracleError("or_load_demand failed: %d" % rc)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or_destroy(self.h)
            self.h = None

    def step(self, n: int = 1):
        rc = self.lib.or_step(self.h, int(n))
        if rc != 0:
            raise OracleError("or_step failed: %d" % rc)

    def counters(self) -> dict:
        out = np.zeros(len(COUNTERS), np.int64)
        self.lib.or_counters(self.h, _p(out))
        return dict(zip(COUNTERS, out.tolist()))

    def vehicles(self) -> dict:
        n = self.lib.or_num_active(self.h)
        iv = np.zeros((max(n, 1), 6), np.int32)
        rv = np.zeros((max(n, 1), 5), np.float64)
        n = self.lib.or_get_vehicles(self.h, _p(iv), _p(rv))
        iv, rv = iv[:n], rv[:n]
        dt = np.float32 if self.precision != "f64" else np.float64
        return {"vid": iv[:, 0].copy(), "edge": iv[:, 1].copy(), "lane": iv[:, 2].copy(),
                "cursor": iv[:, 3].copy(), "lc": iv[:, 4].copy(), "kin": iv[:, 5].copy(),
                "x": rv[:, 0].astype(dt), "v": rv[:, 1].astype(dt), "phin": rv[:, 2].astype(dt),
                "fuel": rv[:, 3].astype(dt), "co": rv[:, 4].astype(dt)}

    def emissions(self) -> dict:
        """Fuel (mL) and CO (g) of every vehicle id at its arrival (0 before)."""
        f = np.zeros(self.ntrips, np.float64)
        c = np.zeros(self.ntrips, np.float64)
        self.lib.or_get_emissions(self.h, _p(f), _p(c))
        dt = np.float32 if self.precision != "f64" else np.float64
        return {"fuel": f.astype(dt), "co": c.astype(dt)}

    def set_control(self, node_control, signal_green: int = 20, stop_dist: float = 3.0, stop_speed: float = 0.5):
        """Change intersection control between steps; every stop node starts free."""
        ctrl = np.ascontiguousarray(node_control, np.int32)
        self._keep.append(ctrl)
        if self.lib.or_set_control(self.h, _p(ctrl), int(signal_green), float(stop_dist), float(stop_speed)) != 0:
            raise OracleError("or_set_control failed")

    def set_sampler(self, every: int = 120, group: int = 6, max_groups: int = 32):
        if self.lib.or_set_sampler(self.h, int(every), int(group), int(max_groups)) != 0:
            raise OracleError("or_set_sampler failed")
        self._samp = int(max_groups)

    def samples(self) -> dict:
        cnt = np.zeros((self._samp, self.ne), np.int64)
        spd = np.zeros((self._samp, self.ne), np.int64)
        self.lib.or_get_samples(self.h, _p(cnt), _p(spd))
        return {"count": cnt, "speed_um": spd}

    def trips(self) -> dict:
        da = np.zeros(self.ntrips, np.int32)
        ar = np.zeros(self.ntrips, np.int32)
        self.lib.or_get_trips(self.h, _p(da), _p(ar))
        return {"depart_actual": da, "arrive_step": ar}

    def enable_tape(self, on: bool = True):
        """Record the discrete events of the following steps."""
        self.lib.or_tape_enable(self.h, 1 if on else 0)

    def tape(self) -> dict:
        n = int(self.lib.or_tape_size(self.h))
        t = {k: np.zeros(max(n, 1), np.int32) for k in TAPE_INT}
        t.update({k: np.zeros(max(n, 1), np.float64) for k in TAPE_F64})
        self.lib.or_tape_get(self.h, *[_p(t[k]) for k in TAPE_INT + TAPE_F64])
        return {k: a[:n] for k, a in t.items()}

    def set_state(self, step, veh, trips, emissions, edge_stats, counters):
        """Continue from another simulation's state at ``step`` (before any
        step of this one; no intersection control): ``veh`` = vehicles on the
        road as returned by ``vehicles()`` (any order), ``trips`` and
        ``emissions`` per vehicle id, ``edge_stats`` per link, ``counters``
        as returned by ``counters()``."""
        n = int(veh["vid"].size)
        iv = np.ascontiguousarray(np.stack([veh[k] for k in ("vid", "edge", "lane", "cursor", "lc", "kin")],
                                           axis=1), np.int32)
        rv = np.ascontiguousarray(np.stack([veh[k] for k in ("x", "v", "phin", "fuel", "co")], axis=1),
                                  np.float64)
        arrs = [np.ascontiguousarray(trips["depart_actual"], np.int32),
                np.ascontiguousarray(trips["arrive_step"], np.int32),
                np.ascontiguousarray(emissions["fuel"], np.float64), np.ascontiguousarray(emissions["co"], np.float64),
                np.ascontiguousarray(edge_stats["count"], np.int64), np.ascontiguousarray(edge_stats["tt_steps"], np.int64),
                np.ascontiguousarray(edge_stats["tt_us"], np.int64),
                np.ascontiguousarray([counters[k] for k in COUNTERS], np.int64)]
        rc = self.lib.or_set_state(self.h, int(step), n, _p(iv), _p(rv), *[_p(a) for a in arrs])
        if rc != 0:
            raise OracleError("or_set_state failed: %d" % rc)

    def edge_stats(self) -> dict:
        c = np.zeros(self.ne, np.int64)
        s = np.zeros(self.ne, np.int64)
        u = np.zeros(self.ne, np.int64)
        self.lib.or_get_edge_stats(self.h, _p(c), _p(s), _p(u))
        return {"count": c, "tt_steps": s, "tt_us": u}
