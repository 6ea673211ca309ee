"""Seeded synthetic scenarios for the traffic microsimulation step.

This module only builds INPUTS: road networks in CSR form, trips with
departure steps and edge-list routes, and parameter sets.  It holds none of
the simulated dynamics, and both the CPU oracle and the HIP library consume
exactly the arrays it returns.

The paper's inputs (its Bay Area road graph, ActivitySim origin/destination
demand, Sec. 6.2) are not available; the generators below stand in for them
with the shapes the workloads need:

* ``grid``      -- square grid of intersections, bidirectional links.
* ``ring``      -- one self-loop link (closed ring road).
* ``metro``     -- random planar graph: Delaunay triangulation of uniform
                   points thinned to a spanning tree plus random extra edges.
* ``demand_*``  -- trips with departure steps and free-flow shortest-path
                   routes.  Departure times follow the paper's histogram
                   method (pick a bucket by frequency, then a uniform offset
                   inside it; Sec. 6.4, departure-time item).

A scenario is a plain dict::

    {"name": str, "net": {...}, "params": {...}, "demand": {...}, "steps": int}
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SPEED_CLASSES = (11.0, 15.0, 20.0, 29.0)


# ---------------------------------------------------------------------------
# native routing helper
# ---------------------------------------------------------------------------
def build_routing_lib(force: bool = False) -> str:
    """Compile ``_routing.c`` into ``_routing.so`` (gcc, -O2)."""
    src = os.path.join(_HERE, "_routing.c")
    out = os.path.join(_HERE, "_routing.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_routing_lib())
        P = ctypes.c_void_p
        lib.ts_dijkstra.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int32, P, P, P, ctypes.c_int32]
        lib.ts_dijkstra.restype = ctypes.c_int
        lib.ts_paths.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, P, P, P]
        lib.ts_paths.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
def default_params(num_classes: int = 1, *, v0_scale=1.0, T=1.5, a=1.0, b=1.5,
                   dt: float = 0.5) -> dict:
    """Model constants.  IDM values per class are (v0_scale, T, a, b); the
    desired speed of a link is v0_scale[class] * speed limit (Sec. 6.3.2)."""
    idm = np.zeros((num_classes, 4), np.float32)
    idm[:, 0] = v0_scale
    idm[:, 1] = T
    idm[:, 2] = a
    idm[:, 3] = b
    return {
        "dt": float(dt),
        "veh_length": 5.0,
        "s0": 2.0,
        "s_eps": 0.1,
        "b_max": 9.0,
        "num_classes": int(num_classes),
        "idm": idm,
        "mobil_p": 0.2,
        "mobil_athr": 0.1,
        "mobil_bsafe": 4.0,
        # mandatory-change distance D*sqrt(ln(1/theta)), D = 100 m, theta = 0.5
        "mand_dist": float(100.0 * math.sqrt(math.log(2.0))),
        "lc_cooldown": 4,
        # intersection control (used where the network has "node_control"):
        # green time of each signal movement, and the stop-sign waiting zone
        "signal_green": 20,
        "stop_dist": 3.0,
        "stop_speed": 0.5,
    }


# ---------------------------------------------------------------------------
# networks
# ---------------------------------------------------------------------------
def _csr_from_directed(n_nodes, tails, heads, attrs):
    order = np.lexsort((heads, tails))
    tails = tails[order]
    heads = heads[order]
    row_ptr = np.zeros(n_nodes + 1, np.int64)
    np.add.at(row_ptr, tails + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    net = {"row_ptr": row_ptr, "col_idx": heads.astype(np.int32)}
    for k, v in attrs.items():
        net[k] = v[order]
    return net


def _undirected_to_net(n_nodes, u, v, lanes, length, speed, cls):
    tails = np.concatenate([u, v]).astype(np.int64)
    heads = np.concatenate([v, u]).astype(np.int64)
    attrs = {
        "lanes": np.concatenate([lanes, lanes]).astype(np.int32),
        "length": np.concatenate([length, length]).astype(np.float32),
        "speed": np.concatenate([speed, speed]).astype(np.float32),
        "link_class": np.concatenate([cls, cls]).astype(np.int32),
    }
    return _csr_from_directed(n_nodes, tails, heads, attrs)


def grid(side: int, *, seed: int = 0, link_len=100.0, lanes=2, speed=15.0,
         lane_probs=None, lognormal=None, num_classes: int = 1, min_len: float = 20.0):
    """Square grid with ``side x side`` intersections, links in both directions.

    ``lane_probs`` (p1, p2, ...) draws 1.. lanes per undirected link;
    ``lognormal=(median, sigma)`` draws link lengths; ``num_classes`` > 1 draws
    a link class uniformly.  Attributes are shared by both directions."""
    rng = np.random.default_rng(seed)
    r, c = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    nid = (r * side + c).ravel()
    right = nid[(c < side - 1).ravel()]
    down = nid[(r < side - 1).ravel()]
    u = np.concatenate([right, down])
    v = np.concatenate([right + 1, down + side])
    m = u.size
    if lane_probs is not None:
        ln = rng.choice(np.arange(1, len(lane_probs) + 1), size=m, p=np.asarray(lane_probs) / np.sum(lane_probs))
    else:
        ln = np.full(m, lanes)
    if lognormal is not None:
        med, sig = lognormal
        length = np.maximum(min_len, med * np.exp(sig * rng.standard_normal(m)))
    else:
        length = np.full(m, float(link_len))
    cls = rng.integers(0, num_classes, m) if num_classes > 1 else np.zeros(m, np.int64)
    net = _undirected_to_net(side * side, u, v, ln, length, np.full(m, float(speed)), cls)
    net["xy"] = np.stack([c.ravel() * 100.0, r.ravel() * 100.0], 1).astype(np.float64)
    return net


def ring(length: float = 1000.0, speed: float = 15.0, lanes: int = 1):
    """One node with one self-loop link: a closed ring road."""
    return {
        "row_ptr": np.array([0, 1], np.int32),
        "col_idx": np.array([0], np.int32),
        "lanes": np.array([lanes], np.int32),
        "length": np.array([length], np.float32),
        "speed": np.array([speed], np.float32),
        "link_class": np.array([0], np.int32),
    }


def metro(n_nodes: int = 1_000_000, n_edges: int = 2_500_000, *, seed: int = 1810,
          spacing: float = 111.0, median_len: float = 120.0, sigma: float = 0.4,
          class_probs=(0.5, 0.3, 0.15, 0.05), min_len: float = 20.0):
    """Random planar road graph: Delaunay triangulation of uniform points,
    thinned to its Euclidean minimum spanning tree plus random extra Delaunay
    edges until ``n_edges`` directed edges (both directions of each).  Road
    class k ~ class_probs gives lanes k+1 and speed limit SPEED_CLASSES[k];
    lengths are lognormal and independent of the geometry."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    side = math.sqrt(n_nodes) * spacing
    pts = rng.uniform(0.0, side, (n_nodes, 2))
    # spatial ordering of node ids (1 km strips, then x) for memory locality
    order = np.lexsort((pts[:, 0], np.floor(pts[:, 1] / 1000.0)))
    pts = pts[order]
    tri = Delaunay(pts)
    s = tri.simplices.astype(np.int64)
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e.sort(axis=1)
    key = np.unique(e[:, 0] * n_nodes + e[:, 1])
    a, b = key // n_nodes, key % n_nodes
    d = np.hypot(pts[a, 0] - pts[b, 0], pts[a, 1] - pts[b, 1])
    g = coo_matrix((d, (a, b)), shape=(n_nodes, n_nodes)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    mkey = np.minimum(mst.row, mst.col).astype(np.int64) * n_nodes + np.maximum(mst.row, mst.col)
    in_mst = np.isin(key, mkey)
    n_und = n_edges // 2
    extra_pool = np.flatnonzero(~in_mst)
    n_extra = max(0, n_und - int(in_mst.sum()))
    extra = rng.choice(extra_pool, size=n_extra, replace=False)
    keep = np.concatenate([np.flatnonzero(in_mst), np.sort(extra)])
    u, v = a[keep], b[keep]
    m = u.size
    k = rng.choice(len(class_probs), size=m, p=np.asarray(class_probs) / np.sum(class_probs))
    lanes = k + 1
    speed = np.asarray(SPEED_CLASSES, np.float64)[k]
    length = np.maximum(min_len, median_len * np.exp(sigma * rng.standard_normal(m)))
    net = _undirected_to_net(n_nodes, u, v, lanes, length, speed, np.zeros(m, np.int64))
    net["xy"] = pts
    return net


def random_control(net, seed, p_stop=0.3, p_signal=0.3):
    """Node control drawn per node: 0 none, 1 stop sign, 2 traffic signal."""
    rng = np.random.default_rng(seed)
    n = net["row_ptr"].size - 1
    u = rng.uniform(0.0, 1.0, n)
    return np.where(u < p_stop, 1, np.where(u < p_stop + p_signal, 2, 0)).astype(np.int32)


def tails_of(net) -> np.ndarray:
    rp = net["row_ptr"]
    return np.repeat(np.arange(rp.size - 1, dtype=np.int32), np.diff(rp))


# ---------------------------------------------------------------------------
# demand
# ---------------------------------------------------------------------------
def histogram_departures(rng, n, bucket_s, weights):
    """The paper's departure sampler: choose a bucket with probability
    proportional to its frequency, then add a uniform offset within it."""
    w = np.asarray(weights, np.float64)
    b = rng.choice(w.size, size=n, p=w / w.sum())
    return (b + rng.uniform(0.0, 1.0, n)) * bucket_s


def mixture_weights(minutes, comps):
    """Per-minute bucket mass of a truncated Gaussian mixture.
    comps = [(weight, mean_min, sd_min), ...]."""
    from scipy.stats import norm
    edges = np.arange(minutes + 1, dtype=np.float64)
    w = np.zeros(minutes)
    for wt, mu, sd in comps:
        w += wt * np.diff(norm.cdf(edges, mu, sd))
    return w


def free_flow_weights(net):
    return net["length"].astype(np.float64) / net["speed"].astype(np.float64)


def routes_for_pairs(net, orig, dest, *, threads=None):
    """Free-flow shortest-path routes for trips (orig[i] -> dest[i]).

    Returns (trip_route, route_ptr, route_edges): one route per distinct
    (origin, destination) pair, shared by all trips of that pair."""
    lib = _lib()
    n = int(net["row_ptr"].size - 1)
    row_ptr = np.ascontiguousarray(net["row_ptr"], np.int32)
    col_idx = np.ascontiguousarray(net["col_idx"], np.int32)
    w = np.ascontiguousarray(free_flow_weights(net))
    tail = np.ascontiguousarray(tails_of(net))
    orig = np.asarray(orig, np.int64)
    dest = np.asarray(dest, np.int64)
    pair = orig * n + dest
    upair, trip_route = np.unique(pair, return_inverse=True)
    po, pd = upair // n, upair % n
    uo, ostart = np.unique(po, return_index=True)
    ostart = np.append(ostart, po.size)

    def work(k):
        src = int(uo[k])
        dst = np.ascontiguousarray(pd[ostart[k]:ostart[k + 1]], np.int32)
        need = np.zeros(n, np.uint8)
        need[dst] = 1
        dist = np.empty(n, np.float64)
        pred = np.empty(n, np.int32)
        rc = lib.ts_dijkstra(n, _ptr(row_ptr), _ptr(col_idx), _ptr(w), src, _ptr(dist), _ptr(pred),
                             _ptr(need), int(np.count_nonzero(need)))
        if rc != 0:
            raise MemoryError("dijkstra")
        lens = np.empty(dst.size, np.int64)
        if lib.ts_paths(src, _ptr(pred), _ptr(tail), dst.size, _ptr(dst), _ptr(lens), None, None) != 0:
            raise ValueError("unreachable destination from node %d" % src)
        off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        out = np.empty(int(lens.sum()), np.int32)
        lib.ts_paths(src, _ptr(pred), _ptr(tail), dst.size, _ptr(dst), None, _ptr(off), _ptr(out))
        return lens, out

    nthreads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        res = list(ex.map(work, range(uo.size)))
    lens = np.concatenate([r[0] for r in res])
    route_edges = np.concatenate([r[1] for r in res]).astype(np.int32)
    route_ptr = np.zeros(lens.size + 1, np.int64)
    route_ptr[1:] = np.cumsum(lens)
    return trip_route.astype(np.int32), route_ptr, route_edges


def uniform_od(rng, n_nodes, n_trips):
    o = rng.integers(0, n_nodes, n_trips)
    d = rng.integers(0, n_nodes, n_trips)
    bad = o == d
    while bad.any():
        d[bad] = rng.integers(0, n_nodes, int(bad.sum()))
        bad = o == d
    return o, d


def make_demand(net, orig, dest, depart_s, dt):
    trip_route, route_ptr, route_edges = routes_for_pairs(net, orig, dest)
    src_nodes, trip_src = np.unique(np.asarray(orig, np.int64), return_inverse=True)
    return {
        "depart_step": np.floor(np.asarray(depart_s) / dt).astype(np.int32),
        "trip_route": trip_route,
        "route_ptr": route_ptr,
        "route_edges": route_edges,
        # the O/D pairs, for planning routes again: distinct origins, and per
        # trip the index of its origin and its destination node
        "src_nodes": src_nodes.astype(np.int32),
        "trip_src": trip_src.astype(np.int32),
        "trip_dst": np.asarray(dest, np.int32),
    }


def reroute_masks(seed: int, n_trips: int, shares=(1.0, 1.0, 0.5, 0.25)):
    """Per iteration, which trips plan their route again: a uniform random
    subset of exactly round(share * n) trips (all of them for share 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for sh in shares:
        m = np.zeros(n_trips, bool)
        k = int(round(sh * n_trips))
        m[rng.choice(n_trips, k, replace=False)] = True
        out.append(m)
    return out


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def small_grid(seed: int = 1807, n_trips: int = 2000, steps: int = 3600):
    """10x10 grid, 100 m links, 2 lanes each way, 15 m/s; uniform random O/D
    nodes; departures uniform over 600 s; 3,600 steps of 0.5 s."""
    rng = np.random.default_rng(seed)
    net = grid(10, seed=seed, link_len=100.0, lanes=2, speed=15.0)
    p = default_params()
    o, d = uniform_od(rng, 100, n_trips)
    dep = rng.uniform(0.0, 600.0, n_trips)
    return {"name": "grid10_2k", "net": net, "params": p,
            "demand": make_demand(net, o, d, dep, p["dt"]), "steps": steps}


def ring_road(seed: int = 1808, n_veh: int = 40, length: float = 1000.0, steps: int = 14400,
              speed: float = 15.0, jitter: float = 1.0, v_init=None, laps: int = 200):
    """Single-lane ring of ``length`` m with ``n_veh`` vehicles at uniform
    spacing plus a seeded +-``jitter`` m perturbation."""
    rng = np.random.default_rng(seed)
    net = ring(length, speed)
    p = default_params()
    spacing = length / n_veh
    x = (np.arange(n_veh) * spacing + p["veh_length"] + rng.uniform(-jitter, jitter, n_veh)).astype(np.float32)
    v = np.full(n_veh, 0.0 if v_init is None else v_init, np.float32)
    demand = {
        "depart_step": np.zeros(n_veh, np.int32),
        "trip_route": np.zeros(n_veh, np.int32),
        "route_ptr": np.array([0, laps], np.int64),
        "route_edges": np.zeros(laps, np.int32),
        "init_x": x, "init_v": v, "init_lane": np.zeros(n_veh, np.int32),
    }
    return {"name": "ring%d" % n_veh, "net": net, "params": p, "demand": demand, "steps": steps}


def mid_grid(seed: int = 1809, side: int = 50, n_trips: int = 100_000, steps: int = 14400,
             num_classes: int = 1, depart_mode: str = "double_peak"):
    """50x50 grid, 1-3 lanes (p = .5/.35/.15), lognormal lengths (median 120 m,
    sigma 0.4), 15 m/s; 100k uniform O/D trips; departures from a 2-hour
    double-peak mixture by the histogram method."""
    rng = np.random.default_rng(seed)
    net = grid(side, seed=seed, lane_probs=(0.5, 0.35, 0.15), lognormal=(120.0, 0.4), speed=15.0,
               num_classes=num_classes)
    p = default_params(num_classes)
    o, d = uniform_od(rng, side * side, n_trips)
    if depart_mode == "double_peak":
        w = mixture_weights(120, [(0.5, 40.0, 15.0), (0.5, 80.0, 15.0)])
        dep = histogram_departures(rng, n_trips, 60.0, w)
    else:
        dep = rng.uniform(0.0, 600.0, n_trips)
    return {"name": "grid%d_%dk" % (side, n_trips // 1000), "net": net, "params": p,
            "demand": make_demand(net, o, d, dep, p["dt"]), "steps": steps}


def metro_scenario(seed: int = 1810, n_nodes: int = 1_000_000, n_edges: int = 2_500_000,
                   n_trips: int = 4_000_000, n_zones: int = 2000, steps: int = 21600,
                   decay_m: float = 8000.0):
    """Metro-scale workload: random planar graph (see ``metro``), gravity-model
    origin/destination demand over k-means zones (zone node = node nearest
    the zone centroid), departures from a 3-hour two-peak mixture."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed + 1)
    net = metro(n_nodes, n_edges, seed=seed)
    pts = net["xy"]
    # k-means zones (a few Lloyd iterations)
    cent = pts[rng.choice(n_nodes, n_zones, replace=False)]
    for _ in range(6):
        lab = cKDTree(cent).query(pts)[1]
        cnt = np.bincount(lab, minlength=n_zones).astype(np.float64)
        ok = cnt > 0
        cent[ok, 0] = np.bincount(lab, pts[:, 0], n_zones)[ok] / cnt[ok]
        cent[ok, 1] = np.bincount(lab, pts[:, 1], n_zones)[ok] / cnt[ok]
    znode = cKDTree(pts).query(cent)[1]
    znode = np.unique(znode)
    nz = znode.size
    zp = pts[znode]
    P = np.exp(0.5 * rng.standard_normal(nz))
    A = np.exp(0.5 * rng.standard_normal(nz))
    dij = np.hypot(zp[:, None, 0] - zp[None, :, 0], zp[:, None, 1] - zp[None, :, 1])
    T = P[:, None] * A[None, :] * np.exp(-dij / decay_m)
    np.fill_diagonal(T, 0.0)
    flat = rng.choice(nz * nz, size=n_trips, p=(T / T.sum()).ravel())
    o, d = znode[flat // nz], znode[flat % nz]
    w = mixture_weights(180, [(0.6, 60.0, 20.0), (0.4, 120.0, 25.0)])
    dep = histogram_departures(rng, n_trips, 60.0, w)
    p = default_params()
    net.pop("xy")
    return {"name": "metro1M", "net": net, "params": p,
            "demand": make_demand(net, o, d, dep, p["dt"]), "steps": steps}


def sorted_trip_order(depart_step):
    """Vehicle ids: trips ranked by (departure step, trip index)."""
    return np.lexsort((np.arange(depart_step.size), depart_step))


def placed_snapshot(net, n_veh: int, *, seed: int = 7, route_len: int = 3, spacing=(8.0, 40.0),
                    platoon=(1, 6), params=None, name="snapshot"):
    """A synthetic mid-simulation snapshot on ``net``: about ``n_veh`` vehicles
    placed in platoons on randomly chosen lanes (weighted by lane length),
    consecutive vehicles of a platoon ``spacing`` metres apart (front to
    front), speeds uniform below the speed limit, each with a random
    ``route_len``-edge route that starts on its edge.  All trips depart at
    step 0 as placed trips."""
    rng = np.random.default_rng(seed)
    E = int(net["col_idx"].size)
    lanes = net["lanes"].astype(np.int64)
    length = net["length"].astype(np.float64)
    lane_edge = np.repeat(np.arange(E), lanes)
    lane_no = np.arange(lane_edge.size) - np.repeat(np.concatenate([[0], np.cumsum(lanes)[:-1]]), lanes)
    w = length[lane_edge]
    mean_pl = 0.5 * (platoon[0] + platoon[1])
    n_lanes = min(lane_edge.size, max(1, int(n_veh / mean_pl)))
    chosen = rng.choice(lane_edge.size, size=n_lanes, replace=False, p=w / w.sum())
    k = rng.integers(platoon[0], platoon[1] + 1, n_lanes)
    e_of = np.repeat(lane_edge[chosen], k)
    l_of = np.repeat(lane_no[chosen], k)
    first = np.repeat(np.concatenate([[0], np.cumsum(k)[:-1]]), k)
    rank = np.arange(e_of.size) - first
    gaps = rng.uniform(spacing[0], spacing[1], e_of.size)
    gaps[rank == 0] = 0.0
    offs = np.cumsum(gaps)
    offs -= np.repeat(offs[first[rank == 0]], k)
    start = np.repeat(rng.uniform(0.0, 1.0, n_lanes), k) * length[e_of]
    x = start + offs
    keep = x < length[e_of] - 0.01
    e_of, l_of, x = e_of[keep], l_of[keep], x[keep]
    n = e_of.size
    v = rng.uniform(0.0, 1.0, n) * net["speed"][e_of]
    # random contiguous routes
    rp = net["row_ptr"].astype(np.int64)
    head = net["col_idx"].astype(np.int64)
    route = np.empty((n, route_len), np.int64)
    route[:, 0] = e_of
    for j in range(1, route_len):
        h = head[route[:, j - 1]]
        deg = rp[h + 1] - rp[h]
        route[:, j] = rp[h] + np.floor(rng.uniform(0.0, 1.0, n) * deg).astype(np.int64)
    p = params if params is not None else default_params(int(net.get("link_class", np.zeros(1)).max()) + 1)
    demand = {
        "depart_step": np.zeros(n, np.int32),
        "trip_route": np.arange(n, dtype=np.int32),
        "route_ptr": np.arange(0, n * route_len + 1, route_len, dtype=np.int64),
        "route_edges": route.ravel().astype(np.int32),
        "init_x": x.astype(np.float32), "init_v": v.astype(np.float32), "init_lane": l_of.astype(np.int32),
    }
    return {"name": name, "net": net, "params": p, "demand": demand, "steps": 1}


def draw_idm(rng, num_classes):
    """IDM parameters (v0_scale, T, a, b) per class, drawn v0 x U(0.8, 1.2),
    T ~ U(1, 2), a ~ U(0.7, 1.5), b ~ U(1, 2.5)."""
    idm = np.zeros((num_classes, 4), np.float32)
    idm[:, 0] = rng.uniform(0.8, 1.2, num_classes)
    idm[:, 1] = rng.uniform(1.0, 2.0, num_classes)
    idm[:, 2] = rng.uniform(0.7, 1.5, num_classes)
    idm[:, 3] = rng.uniform(1.0, 2.5, num_classes)
    return idm


def ensemble_scenarios(seed: int = 1811, n: int = 64, steps: int = 3600):
    """The batched-ensemble workload: uneven grid scenarios, side U{20..120},
    trips log-uniform in [1e4, 3e5], IDM parameters per scenario
    (v0 x U(0.8,1.2), T U(1,2), a U(0.7,1.5), b U(1,2.5)), 100 m links,
    2 lanes, 15 m/s, departures U(0, 1800 s)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        side = int(rng.integers(20, 121))
        ntr = int(np.exp(rng.uniform(np.log(1e4), np.log(3e5))))
        net = grid(side, seed=seed * 1000 + q, link_len=100.0, lanes=2, speed=15.0)
        p = default_params()
        p["idm"] = draw_idm(rng, 1)
        o, d = uniform_od(rng, side * side, ntr)
        dep = rng.uniform(0.0, 1800.0, ntr)
        out.append({"name": "ens%d" % q, "net": net, "params": p,
                    "demand": make_demand(net, o, d, dep, p["dt"]), "steps": steps})
    return out


def diff_scenario(seed: int = 1812, side: int = 50, n_trips: int = 100_000, steps: int = 1800,
                  depart_s: float = 600.0, num_classes: int = 4):
    """Differentiation workload: the 50x50 grid network with link classes drawn
    uniformly over ``num_classes``, uniform O/D trips departing U(0, 600 s),
    1,800 steps.  ``hidden_idm`` holds the parameters that generate the target
    travel times; ``params['idm']`` starts at the default values."""
    rng = np.random.default_rng(seed)
    net = grid(side, seed=seed, lane_probs=(0.5, 0.35, 0.15), lognormal=(120.0, 0.4), speed=15.0,
               num_classes=num_classes)
    p = default_params(num_classes)
    o, d = uniform_od(rng, side * side, n_trips)
    dep = rng.uniform(0.0, depart_s, n_trips)
    return {"name": "diff%d_%d" % (side, n_trips), "net": net, "params": p,
            "demand": make_demand(net, o, d, dep, p["dt"]), "steps": steps,
            "hidden_idm": draw_idm(np.random.default_rng(seed + 1), num_classes)}
