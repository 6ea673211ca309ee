"""GPU adjoint (sim_grad, IDMTravelTime) against the FP64 CPU adjoint.

The FP32 GPU forward equals the FP32 oracle bit for bit, so both record the
same discrete events.  Two FP64 CPU references differentiate the FP32 oracle's
event tape (the adjoint oracle is pinned by central differences):
  * linearized at the recorded FP32 states -- the same trajectory the GPU
    adjoint linearizes at: agreement to 1e-5 of the largest component;
  * with the states replayed in FP64 -- differs from the FP32 trajectory by
    rounding that the traffic dynamics amplify (the events are the same):
    agreement to 1.5e-3 (measured: 1.03e-3 on this workload, which is also
    the gap between the two CPU references themselves).
"""
import numpy as np
import pytest

import oracle
import scenarios as S

pytestmark = pytest.mark.gpu


def diff_small(seed=21, side=10, n_trips=1500, steps=600):
    return S.diff_scenario(seed=seed, side=side, n_trips=n_trips, steps=steps, depart_s=200.0)


def targets(scen):
    """Mean link travel times at the hidden parameters (FP32 oracle run)."""
    sc = dict(scen)
    sc["params"] = dict(scen["params"])
    sc["params"]["idm"] = scen["hidden_idm"]
    o = oracle.Oracle(sc, "f32")
    o.step(scen["steps"])
    es = o.edge_stats()
    return np.where(es["count"] > 0, es["tt_us"] / np.maximum(es["count"], 1) / 1e6, 0.0)


def cpu_reference(scen, target, at_tape_states=True):
    o = oracle.Oracle(scen, "f32", tape=True)
    o.step(scen["steps"])
    es = o.edge_stats()
    mask = es["count"] > 0
    loss, g, tbar, _, _ = oracle.replay(o.tape(), scen, scen["params"]["idm"].astype(np.float64), target, mask,
                                        at_tape_states=at_tape_states)
    return loss, g, mask


def gpu_grad(scen, target, every):
    import torch

    import paper_1807_01148_amd as P
    sim = P.Sim(scen)
    sim.tape_begin(every)
    sim.step(scen["steps"])
    tbar, cnt = sim.mean_travel_times()
    t = torch.tensor(target, dtype=torch.float32, device=tbar.device)
    m = cnt > 0
    nm = int(m.sum())
    dL = torch.where(m, 2.0 * (tbar - t) / nm, torch.zeros_like(tbar))
    g = sim.grad(dL).cpu().numpy().astype(np.float64)
    loss = float(((tbar - t)[m] ** 2).mean())
    return sim, g, loss


@pytest.mark.parametrize("every", [60, 17])
def test_gpu_adjoint_matches_fp64_cpu_adjoint(every):
    scen = diff_small()
    tgt = targets(scen)
    loss_c, g_c, _ = cpu_reference(scen, tgt, at_tape_states=True)
    _, g_g, loss_g = gpu_grad(scen, tgt, every)
    assert abs(loss_g - loss_c) <= 1e-5 * loss_c
    err = np.abs(g_g - g_c).max() / np.abs(g_c).max()
    assert err < 1e-5, (err, g_g, g_c)
    _, g_r, _ = cpu_reference(scen, tgt, at_tape_states=False)
    err_r = np.abs(g_g - g_r).max() / np.abs(g_r).max()
    print("adjoint vs FP64 at the FP32 states: %.3g; vs the FP64-replayed states: %.3g" % (err, err_r))
    assert err_r < 1.5e-3, err_r


def test_gpu_adjoint_independent_of_checkpoint_interval_and_deterministic():
    scen = diff_small(seed=22)
    tgt = targets(scen)
    _, g60, _ = gpu_grad(scen, tgt, 60)
    _, g60b, _ = gpu_grad(scen, tgt, 60)
    _, g7, _ = gpu_grad(scen, tgt, 7)
    assert np.array_equal(g60, g60b)
    assert np.array_equal(g60, g7)


def test_grad_leaves_live_state_untouched():
    scen = diff_small(seed=23, steps=300)
    tgt = targets(scen)
    import paper_1807_01148_amd as P
    sim = P.Sim(scen)
    sim.tape_begin(60)
    sim.step(scen["steps"])
    before_v, before_c, before_s = sim.vehicles(), sim.counters(), sim.edge_stats()
    import torch
    sim.grad(torch.ones(sim.num_edges, device="cuda"))
    after_v, after_c, after_s = sim.vehicles(), sim.counters(), sim.edge_stats()
    for k in before_v:
        assert np.array_equal(before_v[k], after_v[k])
    assert before_c == after_c
    for k in before_s:
        assert np.array_equal(before_s[k], after_s[k])
    # and the simulation continues exactly like the oracle
    o = oracle.Oracle(scen, "f32")
    o.step(scen["steps"] + 100)
    sim.step(100)
    V, O = sim.vehicles(), o.vehicles()
    for k in ("vid", "edge", "lane", "x", "v"):
        assert np.array_equal(V[k], O[k])


def test_autograd_function():
    import torch

    from paper_1807_01148_amd.diff import IDMTravelTime, travel_time_loss
    scen = diff_small(seed=24)
    tgt = targets(scen)
    theta = torch.tensor(scen["params"]["idm"], dtype=torch.float32, requires_grad=True)
    tbar, cnt = IDMTravelTime.apply(theta, scen, scen["steps"], 60)
    loss = travel_time_loss(tbar, cnt, torch.tensor(tgt, dtype=torch.float32, device=tbar.device))
    loss.backward()
    _, g_c, _ = cpu_reference(scen, tgt)
    err = np.abs(theta.grad.numpy().astype(np.float64) - g_c).max() / np.abs(g_c).max()
    assert err < 1e-5, err
