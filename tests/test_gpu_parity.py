"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar (from the method's definition of the step, FP32 state):
  * HIP vs FP32 oracle: bit-exact -- every discrete outcome (edge, lane,
    route cursor, lane-change step, entry step, arrival step) and every float
    (position, speed, entry fraction), every link statistic, every counter;
  * HIP vs FP64 oracle from an identical placed state: discrete outcomes equal
    except where the FP64 decision margin is within FP32 rounding; positions
    within 1e-5 * max(|x|, link length), speeds within 1e-5 * max(|v|, 1 m/s);
  * full runs: traversal-weighted mean link travel time within 0.5% of the
    FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import scenarios as S

from fp64check import link_time_gap, one_step_vs_fp64
from tiny import tiny_grid

pytestmark = pytest.mark.gpu

KEYS = ("vid", "edge", "lane", "cursor", "lc", "kin", "x", "v", "phin", "fuel", "co")


def sim(scen):
    import paper_1807_01148_amd as P
    return P.Sim(scen)


def assert_same(g, o, tag):
    G, O = g.vehicles(), o.vehicles()
    assert G["vid"].size == O["vid"].size, (tag, G["vid"].size, O["vid"].size)
    for k in KEYS:
        if not np.array_equal(G[k], O[k]):
            bad = np.flatnonzero(G[k] != O[k])[:5]
            raise AssertionError("%s: %s differs at vids %s: gpu %s oracle %s"
                                 % (tag, k, G["vid"][bad], G[k][bad], O[k][bad]))


def assert_same_outputs(g, o, tag):
    cg, co = g.counters(), o.counters()
    assert {k: cg[k] for k in co} == co, (tag, cg, co)
    eg, eo = g.edge_stats(), o.edge_stats()
    for k in eo:
        assert np.array_equal(eg[k], eo[k]), (tag, k)
    tg, to = g.trips(), o.trips()
    for k in to:
        assert np.array_equal(tg[k], to[k]), (tag, k)
    eg, eo = g.emissions(), o.emissions()
    for k in eo:
        assert np.array_equal(eg[k], eo[k]), (tag, k)


def lockstep(scen, steps, every, tag):
    g, o = sim(scen), oracle.Oracle(scen, "f32")
    assert_same(g, o, tag + " t=0")
    t = 0
    while t < steps:
        n = min(every, steps - t)
        g.step(n)
        o.step(n)
        t += n
        assert_same(g, o, "%s t=%d" % (tag, t))
    assert_same_outputs(g, o, tag)
    return g, o


def test_ring_bit_exact_and_equilibrium():
    g, o = lockstep(S.ring_road(), 14400, 1800, "ring40")
    V = g.vehicles()
    assert np.all(np.abs(V["v"].astype(np.float64) - 10.37512396) < 1e-4)


@pytest.mark.parametrize("seed", range(8))
def test_tiny_grids_every_step(seed):
    lockstep(tiny_grid(seed, n_trips=60, horizon=30), 300, 1, "tiny%d" % seed)


def test_multilane_ring_every_step():
    scen = S.ring_road(n_veh=24, length=400.0, jitter=3.0)
    scen["net"]["lanes"][:] = 3
    scen["demand"]["init_lane"] = (np.arange(24) % 3).astype(np.int32)
    scen["demand"]["init_x"] = (np.arange(24) // 3 * 50.0 + 5.0 + np.arange(24) % 3 * 7.0).astype(np.float32)
    lockstep(scen, 400, 1, "ring3lane")


def test_small_grid_full_run():
    """10x10 grid, 2,000 trips, 3,600 steps: state compared every 100 steps."""
    g, o = lockstep(S.small_grid(), 3600, 100, "grid10")
    assert g.counters()["arrived"] == 2000


@pytest.mark.timeout(600)
def test_mid_grid_full_run():
    """50x50 grid, 100k trips, 14,400 steps, compared every 1,800 steps."""
    lockstep(S.mid_grid(), 14400, 1800, "grid50")


@pytest.mark.timeout(600)
def test_metro_snapshot_bit_exact():
    """Full metro-size network (1M nodes, 2.5M directed edges) with a
    synthetic snapshot of ~1M placed vehicles: three steps in lockstep."""
    net = S.metro()
    net.pop("xy", None)
    scen = S.placed_snapshot(net, 1_000_000, seed=11)
    lockstep(scen, 3, 1, "metro-snapshot")


def test_sampler_and_emissions_grid50():
    """Utilization/speed sampler sums and per-trip fuel/CO on the 50x50 grid
    (first 3,600 steps): identical to the FP32 oracle."""
    scen = S.mid_grid(n_trips=40000)
    g, o = sim(scen), oracle.Oracle(scen, "f32")
    g.set_sampler(120, 6, 8)
    o.set_sampler(120, 6, 8)
    g.step(3600)
    o.step(3600)
    assert_same(g, o, "grid50 sampler")
    assert_same_outputs(g, o, "grid50 sampler")
    sg, so = g.samples(), o.samples()
    for k in so:
        assert np.array_equal(sg[k], so[k]), k
    assert so["count"].sum() > 0


@pytest.mark.timeout(600)
def test_snapshot_vs_fp64_one_step():
    """HIP (FP32) against the FP64 oracle from identical states -- placed
    snapshots on a 50x50 grid, and the 50x50 grid workload's own state at
    steps 3,600 and 7,200 (queues, platoons, lane changes in progress): every
    discrete mismatch is listed and must be a decision whose FP64 margin lies
    within FP32 rounding (an input change of a few float32 ulps flips the
    FP64 decision to the GPU's); positions and speeds within 1e-5."""
    net = S.grid(50, seed=3, lane_probs=(0.5, 0.35, 0.15), lognormal=(120.0, 0.4))
    for seed in range(3):
        scen = S.placed_snapshot(net, 20000, seed=seed)
        one_step_vs_fp64(scen, sim(scen), "snapshot %d" % seed)
    scen = S.mid_grid()
    g = sim(scen)
    for t in (3600, 7200):
        g.step(t - g.counters()["step"])
        one_step_vs_fp64(scen, g, "grid50 t=%d" % t)


def test_small_grid_link_times_vs_fp64():
    scen = S.small_grid()
    g, o = sim(scen), oracle.Oracle(scen, "f64")
    g.step(3600)
    o.step(3600)
    eg, eo = g.edge_stats(), o.edge_stats()
    m = eo["count"] >= 20
    tg = eg["tt_us"][m] / eg["count"][m]
    to = eo["tt_us"][m] / eo["count"][m]
    assert np.sum(np.abs(tg - to) * eo["count"][m]) / np.sum(to * eo["count"][m]) < 0.005
    assert abs(eg["tt_us"].sum() / eg["count"].sum() - eo["tt_us"].sum() / eo["count"].sum()) \
        / (eo["tt_us"].sum() / eo["count"].sum()) < 0.005


@pytest.mark.timeout(600)
def test_mid_grid_link_times_vs_fp64_before_gridlock():
    """50x50 grid workload, its first 3,600 steps (before its centre locks
    up): traversal-weighted mean link travel time and network-wide mean
    travel time within 0.5% of the FP64 oracle.  Later the uncontrolled
    merges gridlock the centre and FP32 and FP64 runs take different
    discrete paths (a chaotic regime; reported, not gated)."""
    scen = S.mid_grid()
    g, o = sim(scen), oracle.Oracle(scen, "f64")
    g.step(3600)
    o.step(3600)
    weighted, network, nlinks = link_time_gap(g.edge_stats(), o.edge_stats())
    print("grid50 3,600 steps: %d links, weighted %.3g, network %.3g" % (nlinks, weighted, network))
    assert nlinks > 3000 and weighted < 0.005 and network < 0.005


def test_determinism_two_runs():
    scen = tiny_grid(3, n_trips=80, horizon=20)
    a, b = sim(scen), sim(scen)
    a.step(400)
    b.step(400)
    A, B = a.vehicles(), b.vehicles()
    for k in KEYS:
        assert np.array_equal(A[k], B[k])
    assert a.counters() == b.counters()
    for k, v in a.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k])


def test_empty_demand_and_zero_steps():
    scen = S.small_grid(n_trips=10)
    d = scen["demand"]
    d["depart_step"] = d["depart_step"][:0]
    d["trip_route"] = d["trip_route"][:0]
    g = sim(scen)
    g.step(0)
    g.step(5)
    c = g.counters()
    assert c["step"] == 5 and c["en_route"] == 0 and c["vehicle_updates"] == 0


def test_errors_are_reported_not_fatal():
    import paper_1807_01148_amd as P
    scen = S.small_grid(n_trips=10)
    bad = dict(scen)
    bad["demand"] = dict(scen["demand"])
    re_ = scen["demand"]["route_edges"].copy()
    re_[1] = re_[0]
    bad["demand"]["route_edges"] = re_
    with pytest.raises(P.SimError) as ei:
        P.Sim(bad)
    assert ei.value.code == P.SIM_EROUTE
    bad = dict(scen)
    bad["net"] = dict(scen["net"])
    bad["net"]["length"] = scen["net"]["length"].copy()
    bad["net"]["length"][3] = 1.0
    with pytest.raises(P.SimError) as ei:
        P.Sim(bad)
    assert ei.value.code == P.SIM_EINVAL


@pytest.mark.parametrize("seed", range(3))
def test_widest_links_and_four_vehicle_types_every_step(seed):
    """The largest values the step packs into its records: links of 1 to 8
    lanes (8 being the maximum) and four vehicle types of different lengths
    and caps, compared with the oracle at every step."""
    probs = np.full(8, 1.0 / 8)
    scen = tiny_grid(40 + seed, side=4, n_trips=160, horizon=40, lane_probs=tuple(probs), lognormal=(60.0, 0.3))
    scen["params"]["vehicle_types"] = np.array([(5.0, np.inf, np.inf), (12.0, 0.8, 12.0), (7.5, 1.2, 20.0),
                                               (3.0, np.inf, 9.0)], np.float32)
    n = scen["demand"]["depart_step"].size
    scen["demand"]["trip_type"] = np.random.default_rng(seed).integers(0, 4, n).astype(np.uint8)
    assert scen["net"]["lanes"].max() == 8
    g, o = lockstep(scen, 400, 1, "wide%d" % seed)
    assert o.counters()["claims_lane_change"] > 0
