"""GPU: batched ensembles, graph-captured steps, launch shapes and the autotuner.

Every one of these must leave the simulated results bit-identical:
  * a batch of scenarios equals the scenarios run one by one;
  * graph-captured chunks equal plain launches;
  * any launch shape gives the same results; the autotuner restores the state.
"""
import numpy as np
import pytest

import scenarios as S

pytestmark = pytest.mark.gpu


def small_scenarios(n=5, seed=40):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        side = int(rng.integers(4, 9))
        net = S.grid(side, seed=seed + q, link_len=60.0, lanes=2, speed=15.0)
        p = S.default_params()
        p["idm"] = S.draw_idm(rng, 1)
        ntr = int(rng.integers(100, 400))
        o, d = S.uniform_od(rng, side * side, ntr)
        dep = rng.uniform(0.0, 120.0, ntr)
        out.append({"name": "e%d" % q, "net": net, "params": p,
                    "demand": S.make_demand(net, o, d, dep, p["dt"]), "steps": 500})
    return out


def per_trip(sim, dep):
    from paper_1807_01148_amd.ensemble import vehicle_ids
    tr = sim.trips()
    v = vehicle_ids(dep)
    return {k: a[v] for k, a in tr.items()}


def oracle_trips(o, dep):
    from paper_1807_01148_amd.ensemble import vehicle_ids
    tr = o.trips()
    v = vehicle_ids(dep)
    return {k: a[v] for k, a in tr.items()}


def test_batch_equals_separate_runs_and_the_oracle():
    """Every member of a batch equals its own simulation and the FP32 oracle
    run of that scenario alone: link statistics and per-trip outcomes."""
    import oracle
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import Ensemble
    scens = small_scenarios()
    ens = Ensemble(scens)
    ens.step(500)
    est, etr = ens.edge_stats(), ens.trips()
    total = 0
    for q, sc in enumerate(scens):
        one = P.Sim(sc)
        one.step(500)
        o = oracle.Oracle(sc, "f32")
        o.step(500)
        a = ens.scenario_edge_stats(q, est)
        for b in (one.edge_stats(), o.edge_stats()):
            for k in b:
                assert np.array_equal(a[k], b[k]), (q, k)
        ta = ens.scenario_trips(q, etr)
        for tb in (per_trip(one, sc["demand"]["depart_step"]), oracle_trips(o, sc["demand"]["depart_step"])):
            for k in tb:
                assert np.array_equal(ta[k], tb[k]), (q, k)
        total += one.counters()["vehicle_updates"]
        assert one.counters()["vehicle_updates"] == o.counters()["vehicle_updates"]
    assert ens.counters()["vehicle_updates"] == total


def test_graph_chunks_equal_plain_steps():
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import step_graph
    sc = S.small_grid()
    a, b = P.Sim(sc), P.Sim(sc)
    a.step(3600)
    step_graph(b, 3600, 60)
    step_graph(b, 0, 60)
    Va, Vb = a.vehicles(), b.vehicles()
    for k in Va:
        assert np.array_equal(Va[k], Vb[k])
    assert a.counters() == b.counters()
    for k, v in a.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k])
    # odd start parity and a remainder
    c, d = P.Sim(sc), P.Sim(sc)
    c.step(1001)
    d.step(1)
    step_graph(d, 1000, 60)
    assert c.counters() == d.counters()
    for k, v in c.vehicles().items():
        assert np.array_equal(v, d.vehicles()[k])


@pytest.mark.parametrize("shape", [(1, 1), (3, 1), (64, 8), (4096, 512)])
def test_launch_shape_does_not_change_results(shape):
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import set_launch
    sc = S.mid_grid(n_trips=20000)
    ref, alt = P.Sim(sc), P.Sim(sc)
    set_launch(alt, *shape)
    ref.step(1500)
    alt.step(1500)
    assert ref.counters() == alt.counters()
    for k, v in ref.vehicles().items():
        assert np.array_equal(v, alt.vehicles()[k])


@pytest.mark.parametrize("dshape", [(256, 2), (128, 1), (128, 2), (512, 1), (256, 4)])
def test_decide_shape_does_not_change_results(dshape):
    """Every decide-kernel shape (threads per block, entries per thread: the
    tile of sorted entries staged in LDS) gives the default shape's results,
    with a small grid too (tiles looped over per block)."""
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import get_decide_shape, set_decide_shape, set_launch
    sc = S.mid_grid(n_trips=20000)
    ref, alt, few = P.Sim(sc), P.Sim(sc), P.Sim(sc)
    set_decide_shape(alt, *dshape)
    set_decide_shape(few, *dshape)
    set_launch(few, 16, 2)
    assert get_decide_shape(alt) == dshape
    ref.step(1500)
    alt.step(1500)
    few.step(1500)
    assert ref.counters() == alt.counters() == few.counters()
    for k, v in ref.vehicles().items():
        assert np.array_equal(v, alt.vehicles()[k]), k
        assert np.array_equal(v, few.vehicles()[k]), k
    for k, v in ref.edge_stats().items():
        assert np.array_equal(v, alt.edge_stats()[k]), k


def test_decide_shape_errors():
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import SIM_EINVAL, SimError
    from paper_1807_01148_amd.ensemble import set_decide_shape
    sim = P.Sim(S.small_grid(n_trips=50, steps=10))
    with pytest.raises(SimError) as ei:
        set_decide_shape(sim, 192, 1)
    assert ei.value.code == SIM_EINVAL


def test_autotune_restores_state():
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import autotune, get_launch
    sc = S.mid_grid(n_trips=20000)
    ref, tun = P.Sim(sc), P.Sim(sc)
    ref.step(600)
    tun.step(600)
    before = tun.counters()
    res = autotune(tun, steps_per_trial=30)
    assert tun.counters() == before
    assert get_launch(tun) == (res["grid"], res["grid_small"])
    from paper_1807_01148_amd.ensemble import get_decide_shape
    assert get_decide_shape(tun) == (res["decide_block"], res["decide_per_thread"])
    ref.step(900)
    tun.step(900)
    assert ref.counters() == tun.counters()
    for k, v in ref.vehicles().items():
        assert np.array_equal(v, tun.vehicles()[k])
    for k, v in ref.trips().items():
        assert np.array_equal(v, tun.trips()[k])


def test_batched_ensemble_workload_at_full_size():
    """The batched-ensemble workload at full size (64 grid scenarios, side
    20-120, 1e4-3e5 trips each, per-scenario IDM parameters) as one simulation
    with graph-captured 60-step chunks and a tuned launch shape, over 1,800
    steps: every member's link statistics and trip outcomes equal its own
    simulation's, and the three smallest members equal the FP32 oracle."""
    import oracle
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import Ensemble, autotune, step_graph
    steps = 1800
    scens = S.ensemble_scenarios(n=64, steps=steps)
    ens = Ensemble(scens)
    step_graph(ens, 60, 60)
    autotune(ens, steps_per_trial=20)
    step_graph(ens, steps - 60, 60)
    est, etr = ens.edge_stats(), ens.trips()
    upd = 0
    for q, sc in enumerate(scens):
        one = P.Sim(sc)
        one.step(steps)
        for k, v in one.edge_stats().items():
            assert np.array_equal(ens.scenario_edge_stats(q, est)[k], v), (q, k)
        ts, to = ens.scenario_trips(q, etr), per_trip(one, sc["demand"]["depart_step"])
        for k, v in to.items():
            assert np.array_equal(ts[k], v), (q, k)
        upd += one.counters()["vehicle_updates"]
        one.close()
    assert ens.counters()["vehicle_updates"] == upd
    small = sorted(range(len(scens)), key=lambda q: scens[q]["demand"]["depart_step"].size)[:3]
    for q in small:
        o = oracle.Oracle(scens[q], "f32")
        o.step(steps)
        for k, v in o.edge_stats().items():
            assert np.array_equal(ens.scenario_edge_stats(q, est)[k], v), (q, k)
        ts, to = ens.scenario_trips(q, etr), oracle_trips(o, scens[q]["demand"]["depart_step"])
        for k, v in to.items():
            assert np.array_equal(ts[k], v), (q, k)
