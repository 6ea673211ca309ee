"""Pins of the FP64 differentiation oracle (frozen-event replay + adjoint).

* the replay of a tape recorded by the FP64 forward reproduces that forward
  exactly (positions and speeds bit for bit, link times to the microsecond);
* the reverse-mode gradient equals central finite differences of the replay
  itself (a different computation: two more forward evaluations per
  parameter), converging as h shrinks;
* on single-vehicle and two-vehicle chains (free road, following, crossings,
  arrival) the agreement is to 1e-8.
"""
import numpy as np
import pytest

import oracle
import scenarios as S

from tiny import chain_net


def small_diff(seed=5, side=8, n_trips=400, steps=260):
    scen = S.diff_scenario(seed=seed, side=side, n_trips=n_trips, steps=steps, depart_s=100.0)
    scen["net"]["length"] = np.maximum(scen["net"]["length"] * 0.6, 20.0).astype(np.float32)
    return scen


def run_taped(scen, prec="f64"):
    o = oracle.Oracle(scen, prec, tape=True)
    o.step(scen["steps"])
    return o


def fd_grad(tape, scen, th, tgt, mask, h):
    g = np.zeros_like(th)
    for c in range(th.shape[0]):
        for j in range(4):
            a, b = th.copy(), th.copy()
            a[c, j] += h
            b[c, j] -= h
            g[c, j] = (oracle.replay(tape, scen, a, tgt, mask, grad=False)[0]
                       - oracle.replay(tape, scen, b, tgt, mask, grad=False)[0]) / (2 * h)
    return g


def test_replay_reproduces_fp64_forward():
    scen = small_diff()
    o = run_taped(scen, "f64")
    es, V = o.edge_stats(), o.vehicles()
    mask = es["count"] > 0
    th = scen["params"]["idm"].astype(np.float64)
    _, _, tbar, xf, vf = oracle.replay(o.tape(), scen, th, np.zeros(mask.size), mask, grad=False)
    assert V["vid"].size > 0
    assert np.array_equal(xf[V["vid"]], V["x"]) and np.array_equal(vf[V["vid"]], V["v"])
    ref = es["tt_us"][mask] / es["count"][mask] / 1e6
    assert np.abs(tbar[mask] - ref).max() <= 1e-6


def test_replay_close_to_fp32_forward():
    scen = small_diff()
    o = run_taped(scen, "f32")
    V = o.vehicles()
    es = o.edge_stats()
    mask = es["count"] > 0
    th = scen["params"]["idm"].astype(np.float64)
    _, _, tbar, xf, vf = oracle.replay(o.tape(), scen, th, np.zeros(mask.size), mask, grad=False)
    assert np.abs(xf[V["vid"]] - V["x"]).max() < 1e-3
    assert np.abs(vf[V["vid"]] - V["v"]).max() < 1e-4


@pytest.mark.parametrize("seed", [5, 6])
def test_adjoint_matches_central_differences(seed):
    scen = small_diff(seed=seed)
    o = run_taped(scen, "f32")
    tape, es = o.tape(), o.edge_stats()
    mask = es["count"] > 0
    th = scen["params"]["idm"].astype(np.float64)
    ref = np.where(mask, es["tt_us"] / np.maximum(es["count"], 1) / 1e6, 0.0)
    tgt = ref * np.random.default_rng(seed).uniform(0.8, 1.2, ref.size)
    _, g, _, _, _ = oracle.replay(tape, scen, th, tgt, mask)
    scale = np.abs(g).max()
    err6 = np.abs(fd_grad(tape, scen, th, tgt, mask, 1e-6) - g).max() / scale
    err5 = np.abs(fd_grad(tape, scen, th, tgt, mask, 1e-5) - g).max() / scale
    assert err6 < 1e-5, err6
    assert err5 < 1e-3, err5


@pytest.mark.parametrize("n", [1, 2, 3])
def test_adjoint_chain_exact(n):
    net, _, _ = chain_net(n_edges=4, length=60.0, lanes=1, branch=False)
    p = S.default_params()
    scen = {"name": "chain", "net": net, "params": p, "steps": 200, "demand": {
        "depart_step": (np.arange(n) * 8).astype(np.int32), "trip_route": np.zeros(n, np.int32),
        "route_ptr": np.array([0, 4], np.int64), "route_edges": np.arange(4, dtype=np.int32)}}
    o = run_taped(scen, "f64")
    es = o.edge_stats()
    mask = es["count"] > 0
    th = p["idm"].astype(np.float64)
    tgt = np.where(mask, es["tt_us"] / np.maximum(es["count"], 1) / 1e6 * 0.9, 0.0)
    _, g, _, _, _ = oracle.replay(o.tape(), scen, th, tgt, mask)
    fd = fd_grad(o.tape(), scen, th, tgt, mask, 1e-5)
    assert np.abs(fd - g).max() <= 1e-8 * max(1.0, np.abs(g).max())
    assert abs(g[0, 2]) > 0.1  # the acceleration matters


def test_tape_states_equal_replay_on_fp64_tape():
    """Linearizing at the recorded states is the same computation as replaying
    them when the tape comes from the FP64 forward (whose states the replay
    reproduces exactly)."""
    scen = small_diff(seed=7)
    o = run_taped(scen, "f64")
    es = o.edge_stats()
    mask = es["count"] > 0
    th = scen["params"]["idm"].astype(np.float64)
    tgt = np.where(mask, es["tt_us"] / np.maximum(es["count"], 1) / 1e6 * 1.1, 0.0)
    a = oracle.replay(o.tape(), scen, th, tgt, mask)
    b = oracle.replay(o.tape(), scen, th, tgt, mask, at_tape_states=True)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
