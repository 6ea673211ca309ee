"""GPU intersection control (Sec. 6.3.2: stop signs and signals) against the
FP32 oracle, bit for bit, through the C ABI: every step on tiny controlled
grids, the 10x10 grid with a third of its nodes signalled and a third
stop-controlled, a batch of controlled and uncontrolled scenarios against
the same scenarios run alone, the adjoint across held movements, and the
entry point's error codes.
"""
import numpy as np
import pytest

import oracle
import scenarios as S

from test_gpu_ensemble import per_trip
from test_gpu_parity import assert_same, assert_same_outputs, lockstep
from tiny import tiny_grid

pytestmark = pytest.mark.gpu


def controlled(scen, seed, p_stop=0.35, p_signal=0.35, green=6):
    scen["net"]["node_control"] = S.random_control(scen["net"], seed, p_stop, p_signal)
    scen["params"]["signal_green"] = green
    return scen


@pytest.mark.parametrize("seed", range(6))
def test_tiny_controlled_grids_every_step(seed):
    scen = controlled(tiny_grid(seed, n_trips=60, horizon=30), seed + 100)
    g, o = lockstep(scen, 400, 1, "ctl%d" % seed)
    assert o.counters()["arrived"] > 0


def test_grid10_controlled_full_run():
    scen = controlled(S.small_grid(), 7, 0.3, 0.3, green=20)
    g, o = lockstep(scen, 3600, 100, "grid10ctl")
    assert o.counters()["arrived"] > 0


def test_control_set_after_load_equals_oracle():
    """Control switched on mid-run (every stop node starts free)."""
    import paper_1807_01148_amd as P
    scen = S.small_grid(n_trips=600, steps=900)
    g = P.Sim(scen)
    g.step(300)
    ctrl = S.random_control(scen["net"], 3, 0.4, 0.4)
    g.set_control(ctrl, 10, 3.0, 0.5)
    g.step(600)
    scen2 = dict(scen)
    scen2["net"] = dict(scen["net"])
    o = oracle.Oracle(scen2, "f32")
    o.step(300)
    o.set_control(ctrl, 10, 3.0, 0.5)
    o.step(600)
    assert_same(g, o, "late control")
    assert_same_outputs(g, o, "late control")


def test_ensemble_with_control_equals_separate_runs():
    from paper_1807_01148_amd.ensemble import Ensemble
    scens = [controlled(tiny_grid(40 + q, n_trips=60, horizon=30), 200 + q) for q in range(3)]
    scens.append(tiny_grid(50, n_trips=60, horizon=30))
    for sc in scens:
        sc["params"]["signal_green"] = 6
    ens = Ensemble(scens)
    ens.step(400)
    st, tr = ens.edge_stats(), ens.trips()
    for q, sc in enumerate(scens):
        o = oracle.Oracle(sc, "f32")
        o.step(400)
        es = ens.scenario_edge_stats(q, st)
        for k, v in o.edge_stats().items():
            assert np.array_equal(es[k], v), (q, k)
        ts, to = ens.scenario_trips(q, tr), per_trip(o, sc["demand"]["depart_step"])
        for k, v in to.items():
            assert np.array_equal(ts[k], v), (q, k)


def test_adjoint_across_held_movements():
    from test_gpu_adjoint import cpu_reference, gpu_grad, targets
    scen = S.diff_scenario(seed=23, side=10, n_trips=1500, steps=600, depart_s=200.0)
    controlled(scen, 9, 0.3, 0.3, green=20)
    tgt = targets(scen)
    loss_c, g_c, _ = cpu_reference(scen, tgt, at_tape_states=True)
    _, g_g, loss_g = gpu_grad(scen, tgt, 60)
    assert abs(loss_g - loss_c) <= 1e-5 * loss_c
    err = np.abs(g_g - g_c).max() / np.abs(g_c).max()
    assert err < 1e-5, (err, g_g, g_c)


def test_set_control_errors():
    import paper_1807_01148_amd as P
    scen = tiny_grid(1, n_trips=20, horizon=10)
    g = P.Sim(scen)
    nn = scen["net"]["row_ptr"].size - 1
    bad = np.zeros(nn, np.int32)
    bad[0] = 3
    with pytest.raises(P.SimError) as e:
        g.set_control(bad)
    assert e.value.code == P.SIM_EINVAL
    with pytest.raises(P.SimError):
        g.set_control(np.zeros(nn, np.int32), 0)
    with pytest.raises(P.SimError):
        g.set_control(np.zeros(nn, np.int32), 5, 0.0)
    g.tape_begin(10)
    with pytest.raises(P.SimError) as e:
        g.set_control(np.zeros(nn, np.int32))
    assert e.value.code == P.SIM_ESTATE
