"""Oracle of iterative decaying re-routing (Sec. 6.3.1) -- TEST INFRASTRUCTURE
ONLY (see the package docstring).

Sec. 6.3.1 plans routes on estimated link travel times, runs the simulation,
replaces the estimates by the measured times, and plans again for a shrinking
random subset of the vehicles: all of them in the first two iterations, then
half, then a quarter.

Readings (the paper gives no units or rounding):
  * weights are integer milliseconds, at least 1;
  * initial estimate of link e: sqrt(lanes_e) * length_e / speed_e, rounded to
    the nearest millisecond (halves up), evaluated in double precision from
    the float32 link attributes;
  * measured estimate: the mean traversal time of the link's completed
    traversals, (tt_us + 500 count) // (1000 count); a link nobody finished
    keeps its previous weight;
  * the shortest route is made unique by the rule in routing.c (last edge into
    each node = the lowest-numbered tight edge);
  * which vehicles are re-planned is a random draw passed in as a mask.
"""
import ctypes
import os

import numpy as np

from . import build, _p

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
INF = np.iinfo(np.int64).max

# share of the vehicles whose routes are planned again, per iteration
DECAY = (1.0, 1.0, 0.5, 0.25)


def _lib():
    global _LIB
    if _LIB is None:
        build()
        lib = ctypes.CDLL(os.environ.get("ORACLE_LIB_ROUTE", os.path.join(_HERE, "liboracle_route.so")))
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.or_sssp.argtypes = [i32, i32, P, P, P, i32, P, P]
        lib.or_sssp.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def sssp(net, w, src):
    """(dist int64[nn] with INF where unreachable, pred int32[nn]) from node src."""
    nn = int(net["row_ptr"].size - 1)
    ne = int(net["col_idx"].size)
    rp = np.ascontiguousarray(net["row_ptr"], np.int32)
    ci = np.ascontiguousarray(net["col_idx"], np.int32)
    ww = np.ascontiguousarray(w, np.int64)
    dist = np.empty(nn, np.int64)
    pred = np.empty(nn, np.int32)
    rc = _lib().or_sssp(nn, ne, _p(rp), _p(ci), _p(ww), int(src), _p(dist), _p(pred))
    if rc != 0:
        raise ValueError("or_sssp failed: %d" % rc)
    return dist, pred


def initial_weights(net):
    lanes = np.asarray(net["lanes"], np.float64)
    length = np.asarray(net["length"], np.float32).astype(np.float64)
    speed = np.asarray(net["speed"], np.float32).astype(np.float64)
    ms = np.sqrt(lanes) * length / speed * 1000.0
    return np.maximum(np.floor(ms + 0.5), 1.0).astype(np.int64)


def weights_from_stats(prev, count, tt_us):
    count = np.asarray(count, np.int64)
    tt_us = np.asarray(tt_us, np.int64)
    out = np.array(prev, np.int64, copy=True)
    m = count > 0
    out[m] = (tt_us[m] + 500 * count[m]) // (1000 * count[m])
    return np.maximum(out, 1)


def tails(net):
    rp = np.asarray(net["row_ptr"], np.int64)
    return np.repeat(np.arange(rp.size - 1, dtype=np.int32), np.diff(rp))


def walk(pred, tail, src, dst):
    """Edges of the route src -> dst, in driving order."""
    out = []
    v = int(dst)
    while v != src:
        e = int(pred[v])
        if e < 0:
            raise ValueError("node %d unreachable from %d" % (dst, src))
        out.append(e)
        v = int(tail[e])
    out.reverse()
    return out


def plan(net, w, src_nodes, trip_src, trip_dst, select=None, old=None):
    """Per-trip routes (route_ptr int64[ntrips+1], route_edges int32): trips
    with select[i] (all when select is None) get the shortest route under w,
    the others keep theirs from old = (route_ptr, route_edges)."""
    tail = tails(net)
    n = int(np.asarray(trip_src).size)
    sel = np.ones(n, bool) if select is None else np.asarray(select, bool)
    routes = [None] * n
    for s in np.unique(np.asarray(trip_src)[sel]):
        _, pred = sssp(net, w, int(src_nodes[s]))
        for i in np.flatnonzero(sel & (np.asarray(trip_src) == s)):
            routes[i] = walk(pred, tail, int(src_nodes[s]), int(trip_dst[i]))
    for i in np.flatnonzero(~sel):
        routes[i] = list(old[1][old[0][i]:old[0][i + 1]])
    lens = np.array([len(r) for r in routes], np.int64)
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum(lens)
    edges = np.array([e for r in routes for e in r], np.int32)
    return ptr, edges


def od_demand(scen, route_ptr, route_edges):
    """The scenario's demand with one route per trip."""
    d = dict(scen["demand"])
    n = int(d["depart_step"].size)
    d["trip_route"] = np.arange(n, dtype=np.int32)
    d["route_ptr"] = np.asarray(route_ptr, np.int64)
    d["route_edges"] = np.asarray(route_edges, np.int32)
    out = dict(scen)
    out["demand"] = d
    return out


def reroute(scen, masks, iterations=len(DECAY), precision="f32"):
    """Run the re-routing loop on the oracle simulator.  scen["demand"] holds
    "src_nodes", "trip_src" (index into src_nodes) and "trip_dst"; masks[k]
    (bool per trip) selects the trips planned again before iteration k >= 1.
    Returns one dict per iteration: the weights used, the routes, the link
    statistics and the counters at the end of the run."""
    from . import Oracle
    d = scen["demand"]
    w = initial_weights(scen["net"])
    routes = None
    out = []
    for k in range(iterations):
        sel = None if k == 0 else masks[k]
        routes = plan(scen["net"], w, d["src_nodes"], d["trip_src"], d["trip_dst"], sel, routes)
        o = Oracle(od_demand(scen, *routes), precision)
        o.step(scen["steps"])
        st = o.edge_stats()
        out.append({"weights": w, "route_ptr": routes[0], "route_edges": routes[1], "stats": st,
                    "counters": o.counters()})
        w = weights_from_stats(w, st["count"], st["tt_us"])
    return out
