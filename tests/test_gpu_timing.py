"""Per-kernel timing through the C ABI (sim_set_timing, sim_read_timing): the
sampled steps launch each kernel with its own start and stop events, and

* change nothing in the simulation (plain and graph-replayed runs with timing
  equal the run without, which equals the FP32 oracle);
* count exactly the sampled steps, one in every `every`, in plain steps and
  in graph replays (a sampled step runs outside the graphs);
* give every kernel a positive time, and the kernels of the sampled steps
  take less time than the steps did on the wall clock;
* reject a negative period; reading releases the samples.
"""
import time

import numpy as np
import pytest

import oracle
import scenarios as S

from test_gpu_parity import assert_same_outputs

pytestmark = pytest.mark.gpu


def snapshot(g):
    return {"v": g.vehicles(), "c": g.counters(), "e": g.edge_stats(), "t": g.trips(), "m": g.emissions()}


def same(a, b):
    assert a["c"] == b["c"]
    for part in ("v", "e", "t", "m"):
        for k in a[part]:
            assert np.array_equal(a[part][k], b[part][k]), (part, k)


def test_timing_changes_nothing_and_counts_the_sampled_steps():
    import torch
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import ensemble as E
    scen = S.small_grid(n_trips=1500, steps=1800)
    steps = 900
    ref = P.Sim(scen)
    ref.step(steps)
    o = oracle.Oracle(scen, "f32")
    o.step(steps)
    assert_same_outputs(ref, o, "untimed")
    want = snapshot(ref)

    a = P.Sim(scen)
    a.set_timing(7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.step(steps)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    kms, n = a.read_timing()
    assert n == len(range(0, steps, 7))
    assert list(kms) == list(P.KERNELS)
    assert all(v > 0.0 for v in kms.values()), kms
    assert sum(kms.values()) < wall_ms
    same(snapshot(a), want)
    # reading released the samples
    kms2, n2 = a.read_timing()
    assert n2 == 0 and all(v == 0.0 for v in kms2.values())

    b = P.Sim(scen)
    b.set_timing(50)
    E.step_graph(b, steps, 60)
    kms, n = b.read_timing()
    assert n == len(range(0, steps, 50))
    assert all(v > 0.0 for v in kms.values()), kms
    same(snapshot(b), want)

    # timing off again: no new samples
    b.set_timing(0)
    b.step(10)
    assert b.read_timing()[1] == 0
    with pytest.raises(P.SimError) as e:
        b.set_timing(-1)
    assert e.value.code == P.SIM_EINVAL
