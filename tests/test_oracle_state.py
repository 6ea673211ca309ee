"""The oracle's state import (used to time it, and to compare with the GPU, on
a state the GPU reached) and its all-cores build.

* An oracle that takes over another oracle's state at step t continues
  exactly as the one that wrote it: every vehicle, counter, trip outcome and
  link statistic equal after further steps (10x10 grid, mid-run, with
  waiting trips, lane changes and crossings in flight).
* The all-cores build (decision loop split over threads) gives the same
  results as the single-threaded one, bit for bit.
"""
import numpy as np
import pytest

import oracle
import scenarios as S


def snapshot(o):
    return o.vehicles(), o.trips(), o.emissions(), o.edge_stats(), o.counters()


def assert_same(a, b):
    va, ta, ea, sa, ca = snapshot(a)
    vb, tb, eb, sb, cb = snapshot(b)
    assert ca == cb
    for pa, pb in ((va, vb), (ta, tb), (ea, eb), (sa, sb)):
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_state_import_continues_exactly(prec):
    scen = S.small_grid(n_trips=1500, steps=1200)
    a = oracle.Oracle(scen, prec)
    a.step(400)
    c = a.counters()
    assert c["waiting"] > 0 and c["en_route"] > 50 and c["arrived"] > 0
    v, t, e, s, c = snapshot(a)
    b = oracle.Oracle(scen, prec)
    b.set_state(c["step"], v, t, e, s, c)
    assert_same(a, b)
    a.step(300)
    b.step(300)
    assert_same(a, b)
    assert b.counters()["claims_lane_change"] > 0


def test_state_import_rejects_a_foreign_state():
    scen = S.small_grid(n_trips=300, steps=600)
    a = oracle.Oracle(scen, "f32")
    a.step(200)
    v, t, e, s, c = snapshot(a)
    b = oracle.Oracle(scen, "f32")
    bad = dict(v)
    bad["edge"] = (v["edge"] + 1) % scen["net"]["col_idx"].size  # not where their routes are
    with pytest.raises(oracle.OracleError):
        b.set_state(c["step"], bad, t, e, s, c)


def test_all_cores_build_equals_single_thread():
    scen = S.small_grid(n_trips=2000, steps=900)
    a = oracle.Oracle(scen, "f32")
    b = oracle.Oracle(scen, "f32omp")
    for _ in range(3):
        a.step(300)
        b.step(300)
        assert_same(a, b)


def test_fp32_oracle_vs_fp64_one_step_from_identical_states():
    """The FP32 oracle against the FP64 oracle from the same state (the 50x50
    grid workload at steps 2,400 and 4,800): discrete outcomes equal except
    where FP32 rounding explains them, positions and speeds within 1e-5."""
    from fp64check import one_step_vs_fp64
    scen = S.mid_grid(n_trips=60000)
    a = oracle.Oracle(scen, "f32")
    for t in (2400, 4800):
        a.step(t - a.counters()["step"])
        one_step_vs_fp64(scen, a, "grid50 (60k trips) t=%d" % t)


def test_fp32_oracle_link_times_vs_fp64_before_gridlock():
    """The 50x50 grid workload's first 3,600 steps: FP32 and FP64 oracles
    agree on link travel times within 0.5% (traversal-weighted and
    network-wide; measured 0.32% and 2e-5)."""
    from fp64check import link_time_gap
    scen = S.mid_grid()
    a, b = oracle.Oracle(scen, "f32"), oracle.Oracle(scen, "f64")
    a.step(3600)
    b.step(3600)
    weighted, network, nlinks = link_time_gap(a.edge_stats(), b.edge_stats())
    assert nlinks > 3000 and weighted < 0.005 and network < 0.005
