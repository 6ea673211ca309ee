"""Pins of the second vehicle type (Sec. 6.3.5: trucks differ from cars in
size, acceleration and maximum speed), checked on the oracle:

* brute force: the independent Python implementation, with per-vehicle
  lengths and per-type caps, agrees bit for bit with the FP64 C oracle on
  tiny grids with a mix of cars and trucks;
* lengths: a single-lane ring of 20 cars (5 m) and 10 trucks (12 m) settles
  at the equilibrium of the car-following equation with the gap
  (L - sum of lengths) / n, the same for every vehicle;
* caps: a truck from rest accelerates at exactly its cap in the first step,
  never exceeds its speed cap, and its discrete run converges to the free-road
  closed form with a = cap_a, v0 = cap_v;
* entry: a truck enters at x = 12 m, and no vehicle ever overlaps the rear of
  a truck ahead of it in the same lane;
* adjoint: with caps active, the reverse-mode gradient still equals central
  differences of the replay (the capped parameter drops out for trucks).
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import scenarios as S
from oracle.brute import Brute

from test_oracle_adjoint import fd_grad, small_diff
from test_oracle_pins import one_link, placed, same_state
from tiny import tiny_grid

CAR = (5.0, math.inf, math.inf)
TRUCK = (12.0, 0.8, 12.0)


def with_trucks(scen, share=0.3, seed=0, types=(CAR, TRUCK)):
    scen["params"]["vehicle_types"] = np.array(types, np.float32)
    n = scen["demand"]["depart_step"].size
    scen["demand"]["trip_type"] = (np.random.default_rng(seed).random(n) < share).astype(np.uint8)
    return scen


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_with_trucks(seed):
    scen = with_trucks(tiny_grid(seed, n_trips=60, horizon=30), 0.35, seed)
    o, b = oracle.Oracle(scen, "f64"), Brute(scen)
    for st in range(300):
        o.step()
        b.step()
        assert same_state(o, b) is None, (seed, st)
    for k, v in o.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_ring_equilibrium(prec):
    n, L = 30, 1000.0
    scen = S.ring_road(n_veh=n, length=L)
    types = np.array([5.0, 12.0] * 15, np.float32)[:n]
    scen["params"]["vehicle_types"] = np.array([CAR, (12.0, math.inf, math.inf)], np.float32)
    scen["demand"]["trip_type"] = (types == 12.0).astype(np.uint8)
    o = oracle.Oracle(scen, prec)
    o.step(14400)
    V = o.vehicles()
    gap = (L - types.sum()) / n
    ve = brentq(lambda v: 1 - (v / 15.0) ** 4 - ((2.0 + 1.5 * v) / gap) ** 2, 0.0, 15.0)
    order = np.argsort(V["x"])
    x = V["x"][order].astype(np.float64)
    lead_len = types[V["vid"][order]]  # trip order = vehicle id order here (all depart at 0)
    g = np.diff(np.concatenate([x, [x[0] + L]])) - np.roll(lead_len, -1)
    assert np.all(np.abs(V["v"].astype(np.float64) - ve) < 1e-4)
    assert np.all(np.abs(g - gap) < 1e-3)


def truck_alone(dt=0.5, length=20000.0):
    p = S.default_params(dt=dt)
    p["vehicle_types"] = np.array([CAR, TRUCK], np.float32)
    scen = placed(one_link(length, 15.0), p, [12.0], [0.0])
    scen["demand"]["trip_type"] = np.array([1], np.uint8)
    return scen


def test_truck_caps_acceleration_and_speed():
    o = oracle.Oracle(truck_alone(), "f64")
    o.step(1)
    assert float(o.vehicles()["v"][0]) == np.float32(0.8) * 0.5  # a = min(1.0, 0.8) from rest
    top = 0.0
    for _ in range(2000):
        o.step()
        top = max(top, float(o.vehicles()["v"][0]))
    assert top < 12.0 and 12.0 - top < 1e-3  # v0 = min(15, 12)


def test_truck_free_road_closed_form():
    v0, a, U, dt = 12.0, float(np.float32(0.8)), 0.9, 0.0625
    t_exact = v0 / (2 * a) * (math.atanh(U) + math.atan(U))
    o = oracle.Oracle(truck_alone(dt), "f64")
    prev = 0.0
    for k in range(1, 200000):
        o.step()
        v = float(o.vehicles()["v"][0])
        if v >= U * v0:
            t = (k - 1 + (U * v0 - prev) / (v - prev)) * dt
            break
        prev = v
    assert abs(t - t_exact) < 0.1, (t, t_exact)


def test_trucks_enter_at_their_length_and_never_overlap():
    scen = with_trucks(S.small_grid(n_trips=1500, steps=1800), 0.3, 4)
    o = oracle.Oracle(scen, "f32")
    tlen = np.array([5.0, 12.0])
    dep = scen["demand"]["depart_step"]
    order = np.lexsort((np.arange(dep.size), dep))
    vtype = scen["demand"]["trip_type"][order]  # by vehicle id
    seen = set()
    for _ in range(1800):
        o.step()
        V = o.vehicles()
        for vid, kin, x, cur in zip(V["vid"], V["kin"], V["x"], V["cursor"]):
            if vid not in seen and cur == 0 and kin == o.counters()["step"]:
                assert x == np.float32(tlen[vtype[vid]])  # front at its own length on entry
            seen.add(int(vid))
        key = V["edge"].astype(np.int64) * 8 + V["lane"]
        srt = np.lexsort((V["x"], key))
        k, x, ty = key[srt], V["x"][srt].astype(np.float64), vtype[V["vid"][srt]]
        same = k[1:] == k[:-1]
        rear_ahead = x[1:] - tlen[ty[1:]]
        assert np.all(rear_ahead[same] - x[:-1][same] > -1e-4)
    assert o.counters()["arrived"] > 0 and vtype.sum() > 0


@pytest.mark.parametrize("seed", [5, 6])
def test_adjoint_with_capped_trucks_matches_central_differences(seed):
    scen = with_trucks(small_diff(seed=seed), 0.4, seed)
    o = oracle.Oracle(scen, "f32", tape=True)
    o.step(scen["steps"])
    tape, es = o.tape(), o.edge_stats()
    mask = es["count"] > 0
    th = scen["params"]["idm"].astype(np.float64)
    ref = np.where(mask, es["tt_us"] / np.maximum(es["count"], 1) / 1e6, 0.0)
    tgt = ref * np.random.default_rng(seed).uniform(0.8, 1.2, ref.size)
    _, g, _, _, _ = oracle.replay(tape, scen, th, tgt, mask)
    scale = np.abs(g).max()
    err6 = np.abs(fd_grad(tape, scen, th, tgt, mask, 1e-6) - g).max() / scale
    assert err6 < 1e-5, err6


def test_replay_reproduces_fp64_forward_with_trucks():
    scen = with_trucks(small_diff(), 0.4, 3)
    o = oracle.Oracle(scen, "f64", tape=True)
    o.step(scen["steps"])
    es, V = o.edge_stats(), o.vehicles()
    mask = es["count"] > 0
    th = scen["params"]["idm"].astype(np.float64)
    _, _, tbar, xf, vf = oracle.replay(o.tape(), scen, th, np.zeros(mask.size), mask, grad=False)
    assert V["vid"].size > 0
    assert np.array_equal(xf[V["vid"]], V["x"]) and np.array_equal(vf[V["vid"]], V["v"])
    ref = es["tt_us"][mask] / es["count"][mask] / 1e6
    assert np.abs(tbar[mask] - ref).max() <= 1e-6
