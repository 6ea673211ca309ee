"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

* free road from rest: the IDM ODE with no vehicle ahead has a closed-form
  solution; the discrete trajectory converges to it at first order in dt;
* ring road: a uniform platoon settles at the equilibrium speed that solves
  1 - (v/v0)^4 - ((s0 + v T)/s)^2 = 0 for the ring's gap s;
* IDM special cases: standing start behind a stopped vehicle (a(1-(s0/s)^2))
  and the "intelligent braking" relation acc = a - b_kin^2/b with
  b_kin = v^2/(2 s) when s0 and T vanish and v0 is huge;
* invariants: vehicle conservation, no overlap within a lane, every traversal
  accounted for;
* an independent brute-force implementation agrees bit for bit on tiny
  networks, and exhaustively on small placements.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import scenarios as S
from oracle.brute import Brute

from tiny import chain_net, tiny_grid


def one_link(length, speed, n_lanes=1):
    return {"row_ptr": np.array([0, 1, 1], np.int32), "col_idx": np.array([1], np.int32),
            "lanes": np.array([n_lanes], np.int32), "length": np.array([length], np.float32),
            "speed": np.array([speed], np.float32), "link_class": np.array([0], np.int32)}


def placed(net, params, xs, vs, lanes=None, route=(0,), steps=1):
    n = len(xs)
    return {"name": "placed", "net": net, "params": params, "steps": steps,
            "demand": {"depart_step": np.zeros(n, np.int32), "trip_route": np.zeros(n, np.int32),
                       "route_ptr": np.array([0, len(route)], np.int64),
                       "route_edges": np.array(route, np.int32),
                       "init_x": np.array(xs, np.float32), "init_v": np.array(vs, np.float32),
                       "init_lane": np.zeros(n, np.int32) if lanes is None else np.array(lanes, np.int32)}}


# ---------------------------------------------------------------------------
# free road from rest
# ---------------------------------------------------------------------------
def _time_to_fraction(dt, U=0.9, v0=15.0, a=1.0):
    p = S.default_params(a=a, dt=dt)
    scen = placed(one_link(20000.0, v0), p, [0.0], [0.0])
    o = oracle.Oracle(scen, "f64")
    prev_v, prev_x = 0.0, 0.0
    for k in range(1, 100000):
        o.step()
        V = o.vehicles()
        v, x = float(V["v"][0]), float(V["x"][0])
        if v >= U * v0:
            w = (U * v0 - prev_v) / (v - prev_v)
            return (k - 1 + w) * dt, prev_x + w * (x - prev_x)
        prev_v, prev_x = v, x
    raise AssertionError("never reached")


def test_free_road_converges_to_closed_form():
    v0, a, U = 15.0, 1.0, 0.9
    t_exact = v0 / (2 * a) * (math.atanh(U) + math.atan(U))
    x_exact = v0 ** 2 / (2 * a) * math.atanh(U ** 2)
    assert abs(t_exact - 16.538) < 1e-3 and abs(x_exact - 126.79) < 1e-2
    errs = []
    for dt in (0.5, 0.25, 0.125, 0.0625):
        t, x = _time_to_fraction(dt)
        errs.append((abs(t - t_exact), abs(x - x_exact)))
    # first-order convergence: halving dt roughly halves the error
    for (et0, ex0), (et1, ex1) in zip(errs, errs[1:]):
        assert 1.5 < et0 / et1 < 2.6, errs
        assert 1.5 < ex0 / ex1 < 2.6, errs
    assert errs[-1][0] < 0.1 and errs[-1][1] < 1.5


def test_free_road_speed_monotone_below_v0():
    p = S.default_params()
    o = oracle.Oracle(placed(one_link(20000.0, 15.0), p, [0.0], [0.0]), "f32")
    prev = -1.0
    for _ in range(600):
        o.step()
        v = float(o.vehicles()["v"][0])
        assert prev < v < 15.0 or (v == prev and v < 15.0)
        prev = v
    assert 15.0 - prev < 1e-3


# ---------------------------------------------------------------------------
# ring-road equilibrium
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,L,T,a,b", [(40, 1000.0, 1.5, 1.0, 1.5), (30, 1000.0, 1.5, 1.0, 1.5),
                                       (40, 1000.0, 1.0, 1.5, 2.0), (25, 600.0, 1.5, 1.0, 1.5)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ring_equilibrium(n, L, T, a, b, prec):
    scen = S.ring_road(n_veh=n, length=L)
    scen["params"]["idm"][0] = [1.0, T, a, b]
    o = oracle.Oracle(scen, prec)
    o.step(14400)
    V = o.vehicles()
    gap = L / n - 5.0
    ve = brentq(lambda v: 1 - (v / 15.0) ** 4 - ((2.0 + T * v) / gap) ** 2, 0.0, 15.0)
    if (n, L, T) == (40, 1000.0, 1.5):
        assert abs(ve - 10.37512396) < 1e-7
    x = np.sort(V["x"].astype(np.float64))
    g = np.diff(np.concatenate([x, [x[0] + L]])) - 5.0
    assert np.all(np.abs(V["v"].astype(np.float64) - ve) < 1e-4)
    assert np.all(np.abs(g - gap) < 1e-3)
    c = o.counters()
    assert c["en_route"] == n and c["arrived"] == 0


# ---------------------------------------------------------------------------
# IDM special cases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("s", [3.0, 6.0, 20.0])
def test_standing_start_behind_stopped_vehicle(s):
    p = S.default_params(a=1.3)
    scen = placed(one_link(500.0, 15.0), p, [10.0, 10.0 + 5.0 + s], [0.0, 0.0])
    o = oracle.Oracle(scen, "f64")
    o.step()
    V = o.vehicles()
    follower = int(np.argmin(V["x"]))
    acc = float(V["v"][follower]) / 0.5
    a = float(np.float32(1.3))  # the parameter travels as float32
    assert abs(acc - a * (1 - (2.0 / s) ** 2)) < 1e-12


@pytest.mark.parametrize("v,kin_ratio,a,b", [(10.0, 3.0, 1.0, 1.5), (20.0, 2.0, 0.8, 2.0), (8.0, 4.0, 1.5, 1.0)])
def test_intelligent_braking(v, kin_ratio, a, b):
    # s0 -> 0, T = 0, v0 huge: acc = a - b_kin^2 / b with b_kin = v^2 / (2 s)
    p = S.default_params(T=0.0, a=a, b=b)
    p["s0"] = 1e-4
    p["b_max"] = 1000.0
    bkin = kin_ratio * b
    s = v * v / (2 * bkin)
    scen = placed(one_link(2000.0, 1e5), p, [0.0, s + 5.0], [v, 0.0])
    o = oracle.Oracle(scen, "f64")
    o.step()
    V = o.vehicles()
    follower = int(np.argmin(V["x"]))
    acc = (float(V["v"][follower]) - v) / 0.5
    expect = a - bkin ** 2 / b
    assert abs(acc - expect) < 2e-3 * abs(expect)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
def check_invariants(o, scen, ntrips):
    c = o.counters()
    assert c["loaded"] == ntrips
    assert c["loaded"] == c["waiting"] + c["en_route"] + c["arrived"]
    assert c["departed"] == c["en_route"] + c["arrived"]
    V = o.vehicles()
    net, lveh = scen["net"], scen["params"]["veh_length"]
    L = net["length"][V["edge"]]
    assert np.all(V["x"] >= 0) and np.all(V["x"] <= L)
    assert np.all((V["lane"] >= 0) & (V["lane"] < net["lanes"][V["edge"]]))
    key = V["edge"].astype(np.int64) * 16 + V["lane"]
    order = np.lexsort((V["x"], key))
    k, x = key[order], V["x"][order].astype(np.float64)
    same = k[1:] == k[:-1]
    gaps = (x[1:] - lveh) - x[:-1]
    # within a lane, consecutive vehicles never overlap (up to float rounding
    # of the clamped position, far below a millimetre)
    assert np.all(gaps[same] >= -1e-4), gaps[same].min()
    # every completed link traversal is accounted for
    d = scen["demand"]
    rl = np.diff(d["route_ptr"])[d["trip_route"]][S.sorted_trip_order(d["depart_step"])]
    tr = o.trips()
    arrived = tr["arrive_step"] >= 0
    assert o.edge_stats()["count"].sum() == rl[arrived].sum() + V["cursor"].sum()
    return c


def test_invariants_small_grid():
    scen = S.small_grid()
    o = oracle.Oracle(scen, "f32")
    for _ in range(360):
        o.step(10)
        c = check_invariants(o, scen, 2000)
    assert c["arrived"] == 2000


def test_invariants_mid_grid_prefix():
    scen = S.mid_grid(n_trips=20000)
    o = oracle.Oracle(scen, "f32")
    for _ in range(20):
        o.step(100)
        check_invariants(o, scen, 20000)


def test_fp32_fp64_link_times_agree():
    scen = S.small_grid()
    a, b = oracle.Oracle(scen, "f32"), oracle.Oracle(scen, "f64")
    a.step(3600)
    b.step(3600)
    ea, eb = a.edge_stats(), b.edge_stats()
    m = eb["count"] >= 20
    ta = ea["tt_us"][m] / ea["count"][m]
    tb = eb["tt_us"][m] / eb["count"][m]
    assert np.sum(np.abs(ta - tb) * eb["count"][m]) / np.sum(tb * eb["count"][m]) < 0.005
    net_a = ea["tt_us"].sum() / ea["count"].sum()
    net_b = eb["tt_us"].sum() / eb["count"].sum()
    assert abs(net_a - net_b) / net_b < 0.005


# ---------------------------------------------------------------------------
# brute force
# ---------------------------------------------------------------------------
def same_state(o, b):
    A, B = o.vehicles(), b.vehicles()
    for k in B:  # the brute force models the dynamics, not the emission accumulators
        if A[k].shape != B[k].shape or not np.array_equal(A[k].astype(np.float64), B[k].astype(np.float64)):
            return k
    return None


@pytest.mark.parametrize("seed", range(10))
def test_brute_force_tiny_grids(seed):
    scen = tiny_grid(seed, n_trips=60, horizon=30)
    o, b = oracle.Oracle(scen, "f64"), Brute(scen)
    lane_changes = 0
    for st in range(300):
        prev = o.vehicles()
        o.step()
        b.step()
        bad = same_state(o, b)
        assert bad is None, (seed, st, bad)
        V = o.vehicles()
        common, ia, ib = np.intersect1d(prev["vid"], V["vid"], return_indices=True)
        lane_changes += int(np.sum((prev["edge"][ia] == V["edge"][ib]) & (prev["lane"][ia] != V["lane"][ib])))
        check_invariants(o, scen, 60)
    for k, v in o.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k])
    assert np.array_equal(o.trips()["arrive_step"], np.array(b.arrive_step))
    assert lane_changes > 0


def test_brute_force_multilane_ring():
    scen = S.ring_road(n_veh=24, length=400.0, jitter=3.0)
    scen["net"]["lanes"][:] = 3
    scen["demand"]["init_lane"] = (np.arange(24) % 3).astype(np.int32)
    scen["demand"]["init_x"] = (np.arange(24) // 3 * 50.0 + 5.0 + np.arange(24) % 3 * 7.0).astype(np.float32)
    o, b = oracle.Oracle(scen, "f64"), Brute(scen)
    for st in range(400):
        o.step()
        b.step()
        assert same_state(o, b) is None, st


def test_exhaustive_small_placements():
    """Every placement of 1-3 vehicles on a two-link, two-lane chain (6 m grid
    of positions, three speeds): one brute-force step equals one oracle step."""
    net, tails, heads = chain_net(n_edges=2, length=30.0, lanes=2)
    p = S.default_params()
    p["mand_dist"] = 20.0
    p["lc_cooldown"] = 0
    main = [int(np.flatnonzero((tails == k) & (heads == k + 1))[0]) for k in range(2)]
    slots = [(e, l, x) for e in main for l in (0, 1) for x in (0.0, 6.0, 12.0, 18.0, 24.0)]
    cases = 0
    rng = np.random.default_rng(5)
    for n in (1, 2, 3):
        for combo in itertools.combinations(slots, n):
            edges = [c[0] for c in combo]
            if n == 3 and rng.random() > 0.7:
                continue
            # vehicles on the second link follow a 1-link route, others 2 links
            xs = [c[2] for c in combo]
            lanes = [c[1] for c in combo]
            ok = True
            for i, j in itertools.permutations(range(n), 2):
                if edges[i] == edges[j] and lanes[i] == lanes[j] and 0 <= xs[j] - xs[i] < 5.0:
                    ok = False
            if not ok:
                continue
            speeds = rng.choice([0.0, 6.0, 12.0], size=n)
            routes = {main[0]: [main[0], main[1]], main[1]: [main[1]]}
            rp, re, tr = [0], [], []
            for e in edges:
                re += routes[e]
                rp.append(len(re))
                tr.append(len(rp) - 2)
            scen = {"name": "ex", "net": net, "params": p, "steps": 3, "demand": {
                "depart_step": np.zeros(n, np.int32), "trip_route": np.array(tr, np.int32),
                "route_ptr": np.array(rp, np.int64), "route_edges": np.array(re, np.int32),
                "init_x": np.array(xs, np.float32), "init_v": speeds.astype(np.float32),
                "init_lane": np.array(lanes, np.int32)}}
            o, b = oracle.Oracle(scen, "f64"), Brute(scen)
            for st in range(3):
                o.step()
                b.step()
                assert same_state(o, b) is None, (combo, st)
            cases += 1
    assert cases > 800


# ---------------------------------------------------------------------------
# input validation
# ---------------------------------------------------------------------------
def test_rejects_noncontiguous_route():
    scen = S.small_grid(n_trips=10)
    d = scen["demand"]
    d["route_edges"] = d["route_edges"].copy()
    d["route_edges"][1] = d["route_edges"][0]  # edge followed by itself: not contiguous
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(scen, "f32")


def test_rejects_overlapping_placement():
    p = S.default_params()
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(placed(one_link(100.0, 15.0), p, [10.0, 13.0], [0.0, 0.0]), "f32")
