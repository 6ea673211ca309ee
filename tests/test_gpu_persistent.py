"""The persistent step (sim_step_persistent): the step's phases in one
cooperative launch with device-wide barriers between them, several steps per
launch.  It must give exactly what the six launches give (which equal the
FP32 oracle): every vehicle field, the counters, the link statistics and the
per-trip outcomes, bit for bit."""
import numpy as np
import pytest

import oracle
import scenarios as S
from test_gpu_control import controlled

pytestmark = pytest.mark.gpu


def assert_equal_runs(a, b, what):
    assert a.counters() == b.counters(), what
    Va, Vb = a.vehicles(), b.vehicles()
    for k in Va:
        assert np.array_equal(Va[k], Vb[k]), (what, k)
    for k, v in a.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k]), (what, k)
    for k, v in a.trips().items():
        assert np.array_equal(v, b.trips()[k]), (what, k)


def test_small_grid_persistent_equals_plain_and_oracle():
    import paper_1807_01148_amd as P
    sc = S.small_grid()
    a, b = P.Sim(sc), P.Sim(sc)
    for k in range(6):
        a.step(600)
        b.step_persistent(600)
        assert_equal_runs(a, b, "grid10 at %d" % (600 * (k + 1)))
    o = oracle.Oracle(sc, "f32")
    o.step(3600)
    assert o.counters()["vehicle_updates"] == b.counters()["vehicle_updates"]
    for k, v in o.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k]), k


@pytest.mark.parametrize("dshape", [(256, 1), (256, 2)])
def test_mid_grid_persistent_equals_plain(dshape):
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import set_decide_shape
    sc = S.mid_grid(n_trips=20000)
    a, b = P.Sim(sc), P.Sim(sc)
    set_decide_shape(b, *dshape)
    a.step(1)
    b.step(1)  # an odd start: the persistent launch begins on the second buffer
    for k in range(3):
        a.step(700)
        b.step_persistent(700)  # two launches each (600 + 100 steps)
        assert_equal_runs(a, b, "grid50 %s at %d" % (dshape, 1 + 700 * (k + 1)))


def test_controlled_grid_persistent_equals_plain():
    import paper_1807_01148_amd as P
    sc = controlled(S.small_grid(), 7, 0.3, 0.3, green=20)
    a, b = P.Sim(sc), P.Sim(sc)
    a.step(1800)
    b.step_persistent(1800)
    assert_equal_runs(a, b, "grid10 with stop signs and signals")


def test_ensemble_persistent_equals_graph_steps():
    from paper_1807_01148_amd.ensemble import Ensemble, step_graph
    scens = [S.small_grid(seed=300 + q, n_trips=500 + 300 * q, steps=900) for q in range(4)]
    a, b = Ensemble(scens), Ensemble(scens)
    step_graph(a, 900, 60)
    b.step_persistent(900)
    assert_equal_runs(a, b, "ensemble")


def test_persistent_falls_back_inside_a_differentiation_window_and_checks_the_shape():
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import SIM_EINVAL, SimError
    from paper_1807_01148_amd.ensemble import set_decide_shape
    sc = S.small_grid(n_trips=400, steps=600)
    a, b = P.Sim(sc), P.Sim(sc)
    b.tape_begin(60)
    a.step(300)
    b.step_persistent(300)  # per-step checkpoints: plain launches
    assert_equal_runs(a, b, "tape window")
    c = P.Sim(sc)
    set_decide_shape(c, 128, 1)
    with pytest.raises(SimError) as ei:
        c.step_persistent(10)
    assert ei.value.code == SIM_EINVAL
