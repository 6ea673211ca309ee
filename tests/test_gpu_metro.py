"""The metro1M workload at full size, in the launch configuration the
benchmark times (60-step HIP graphs, the autotuned launch shape read from
the cache), against the configuration the parity tests use (plain steps,
default shape): the two runs are bit-identical after 7,200 steps (the busy
part of the run, ~760,000 vehicles on the road), and the state satisfies the
invariants of the step at that size:

* trips: loaded = waiting + en_route + arrived, departed = en_route + arrived;
* every vehicle on a lane of its link, 0 <= x <= length, 0 <= v;
* no overlap: within a lane the rear of every vehicle is at or ahead of the
  front of the one behind it (to float rounding);
* link statistics: every completed traversal took at least one step, and
  the traversal counts add up to the crossings and arrivals seen.
"""
import json
import os

import numpy as np
import pytest

import scenarios as S

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def metro():
    scen = S.metro_scenario()
    return scen


def cached_shape():
    """The launch shape the benchmark takes from the tuned-shape cache."""
    from paper_1807_01148_amd import ensemble as E
    with open(os.path.join(ROOT, "paper_1807_01148_amd", "autotune_cache.json")) as f:
        db = json.load(f)
    hit = db.get("%s|metro" % E.device_key(0))
    return hit or {"grid": 1536, "grid_small": 192, "decide_block": 256, "decide_per_thread": 1}


def test_benchmark_configuration_equals_plain_steps_at_full_size(metro):
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import ensemble as E
    steps = 7200
    bench = P.Sim(metro)
    E.apply_shape(bench, cached_shape())
    E.step_graph(bench, steps, 60)
    vb, cb, eb, tb = bench.vehicles(), bench.counters(), bench.edge_stats(), bench.trips()
    bench.close()
    plain = P.Sim(metro)
    plain.step(steps)
    vp, cp, ep, tp = plain.vehicles(), plain.counters(), plain.edge_stats(), plain.trips()
    plain.close()
    assert cb == cp
    for part_b, part_p in ((vb, vp), (eb, ep), (tb, tp)):
        for k in part_p:
            assert np.array_equal(part_b[k], part_p[k]), k

    net, d = metro["net"], metro["demand"]
    c = cb
    assert c["en_route"] > 500_000
    assert c["loaded"] == c["waiting"] + c["en_route"] + c["arrived"]
    assert c["departed"] == c["en_route"] + c["arrived"]
    e, lane, x, v = vb["edge"], vb["lane"], vb["x"].astype(np.float64), vb["v"]
    length = net["length"].astype(np.float64)
    assert np.all((lane >= 0) & (lane < net["lanes"][e]))
    assert np.all((x >= 0) & (x <= length[e])) and np.all(v >= 0)
    key = np.concatenate([[0], np.cumsum(net["lanes"])])[e] + lane
    o = np.lexsort((x, key))
    same = key[o][1:] == key[o][:-1]
    veh_len = float(metro["params"]["veh_length"])
    assert np.all((x[o][1:] - veh_len - x[o][:-1])[same] > -1e-3)
    # every crossing and every arrival completes one traversal of a link: the
    # vehicles on the road have completed `cursor` links of their routes, the
    # arrived trips all of theirs
    cnt, steps_sum = eb["count"], eb["tt_steps"]
    assert np.all(steps_sum >= cnt)
    trip_of_vid = S.sorted_trip_order(d["depart_step"])
    rlen = np.diff(d["route_ptr"])[d["trip_route"][trip_of_vid]]
    arrived = tb["arrive_step"] >= 0
    assert arrived.sum() == c["arrived"]
    assert cnt.sum() == vb["cursor"].astype(np.int64).sum() + rlen[arrived].sum()
