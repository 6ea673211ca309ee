"""GPU vehicle types (Sec. 6.3.5: trucks with their own length, acceleration
cap and speed cap) against the FP32 oracle, bit for bit, through the C ABI:
every step on tiny grids with a mix of cars and trucks, the 10x10 grid with a
third trucks, a mixed single-lane ring, a batch of scenarios against the same
scenarios run alone, the adjoint with capped trucks, and the error codes.
"""
import numpy as np
import pytest

import oracle
import scenarios as S

from test_gpu_ensemble import per_trip
from test_gpu_parity import lockstep
from test_oracle_trucks import CAR, TRUCK, with_trucks
from tiny import tiny_grid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", range(6))
def test_tiny_grids_with_trucks_every_step(seed):
    scen = with_trucks(tiny_grid(seed, n_trips=60, horizon=30), 0.35, seed)
    lockstep(scen, 300, 1, "trucks%d" % seed)


def test_grid10_with_trucks_full_run():
    scen = with_trucks(S.small_grid(), 0.3, 7)
    g, o = lockstep(scen, 3600, 100, "grid10trucks")
    assert o.counters()["arrived"] > 0


def test_mixed_ring():
    scen = S.ring_road(n_veh=30, length=1000.0, steps=3600)
    scen["params"]["vehicle_types"] = np.array([CAR, (12.0, 0.9, 14.0)], np.float32)
    scen["demand"]["trip_type"] = (np.arange(30) % 2).astype(np.uint8)
    lockstep(scen, 3600, 600, "ring-mixed")


def test_ensemble_with_trucks_equals_separate_runs():
    from paper_1807_01148_amd.ensemble import Ensemble
    scens = [with_trucks(tiny_grid(60 + q, n_trips=60, horizon=30), 0.3 * q, q) for q in range(3)]
    ens = Ensemble(scens)
    ens.step(300)
    st, tr = ens.edge_stats(), ens.trips()
    for q, sc in enumerate(scens):
        o = oracle.Oracle(sc, "f32")
        o.step(300)
        es = ens.scenario_edge_stats(q, st)
        for k, v in o.edge_stats().items():
            assert np.array_equal(es[k], v), (q, k)
        ts, to = ens.scenario_trips(q, tr), per_trip(o, sc["demand"]["depart_step"])
        for k, v in to.items():
            assert np.array_equal(ts[k], v), (q, k)


def test_adjoint_with_capped_trucks():
    from test_gpu_adjoint import cpu_reference, gpu_grad, targets
    scen = with_trucks(S.diff_scenario(seed=24, side=10, n_trips=1500, steps=600, depart_s=200.0), 0.3, 24)
    tgt = targets(scen)
    loss_c, g_c, _ = cpu_reference(scen, tgt, at_tape_states=True)
    _, g_g, loss_g = gpu_grad(scen, tgt, 60)
    assert abs(loss_g - loss_c) <= 1e-5 * loss_c
    err = np.abs(g_g - g_c).max() / np.abs(g_c).max()
    assert err < 1e-5, (err, g_g, g_c)


def test_vehicle_type_errors():
    import paper_1807_01148_amd as P
    scen = tiny_grid(2, n_trips=20, horizon=10)
    g = P.Sim(scen)
    with pytest.raises(P.SimError) as e:
        g.set_vehicle_types([CAR, TRUCK])  # demand already loaded
    assert e.value.code == P.SIM_ESTATE
    sc = with_trucks(tiny_grid(2, n_trips=20, horizon=10), 0.5, 2, types=(CAR, (60.0, 1.0, 10.0)))
    with pytest.raises(P.SimError) as e:
        P.Sim(sc)  # longer than the shortest link
    assert e.value.code == P.SIM_EINVAL
    sc = with_trucks(tiny_grid(2, n_trips=20, horizon=10), 0.5, 2)
    sc["demand"]["trip_type"][0] = 2
    with pytest.raises(P.SimError) as e:
        P.Sim(sc)
    assert e.value.code == P.SIM_EINVAL
