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
    """Compile liboracle_f32.so and liboracle_f64.so with gcc."""
    src = os.path.join(_HERE, "oracle.c")
    outs = []
    for prec, defs in (("f32", []), ("f64", ["-DORACLE_F64"])):
        out = os.path.join(_HERE, "liboracle_%s.so" % prec)
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
            tmp = out + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc"] + FLAGS + defs + ["-o", tmp, src, "-lm"])
            os.replace(tmp, out)
        outs.append(out)
    return outs


def _lib(prec):
    if prec not in _LIBS:
        build()
        lib = ctypes.CDLL(os.path.join(_HERE, "liboracle_%s.so" % prec))
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
        _LIBS[prec] = lib
    return _LIBS[prec]


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def fparams(p):
    """The float parameter block shared by both implementations' entry points."""
    return np.array([p["dt"], p["veh_length"], p["s0"], p["s_eps"], p["b_max"],
                     p["mobil_p"], p["mobil_athr"], p["mobil_bsafe"], p["mand_dist"]], np.float32)


COUNTERS = ("step", "loaded", "waiting", "en_route", "arrived", "departed",
            "vehicle_updates", "claims_lost", "clamps")


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle simulation of a scenario dict (see ``scenarios``)."""

    def __init__(self, scen, precision: str = "f32"):
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
        d = scen["demand"]
        self.ntrips = int(d["depart_step"].size)
        ix = d.get("init_x")
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
        rv = np.zeros((max(n, 1), 3), np.float64)
        n = self.lib.or_get_vehicles(self.h, _p(iv), _p(rv))
        iv, rv = iv[:n], rv[:n]
        dt = np.float32 if self.precision == "f32" else np.float64
        return {"vid": iv[:, 0].copy(), "edge": iv[:, 1].copy(), "lane": iv[:, 2].copy(),
                "cursor": iv[:, 3].copy(), "lc": iv[:, 4].copy(), "kin": iv[:, 5].copy(),
                "x": rv[:, 0].astype(dt), "v": rv[:, 1].astype(dt), "phin": rv[:, 2].astype(dt)}

    def trips(self) -> dict:
        da = np.zeros(self.ntrips, np.int32)
        ar = np.zeros(self.ntrips, np.int32)
        self.lib.or_get_trips(self.h, _p(da), _p(ar))
        return {"depart_actual": da, "arrive_step": ar}

    def edge_stats(self) -> dict:
        c = np.zeros(self.ne, np.int64)
        s = np.zeros(self.ne, np.int64)
        u = np.zeros(self.ne, np.int64)
        self.lib.or_get_edge_stats(self.h, _p(c), _p(s), _p(u))
        return {"count": c, "tt_steps": s, "tt_us": u}
