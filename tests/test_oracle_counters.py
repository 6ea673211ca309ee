"""Pins of the oracle's event counters, from the vehicle states alone:

* every winning claim is an event visible in consecutive states: a vehicle
  on the next link of its route (crossing), a vehicle in another lane of the
  same link (lane change) or a new vehicle on the road (departure), so
  claims - claims_lost equals the number of those events, and each kind of
  claim is at least as frequent as its visible winners (Sec. 6.2.2, 6.3.2);
* on a long multi-lane link that nobody leaves, the vehicles evaluated for a
  lane change are exactly those past the cool-down and fully on the link at
  the start of each step.
"""
import numpy as np
import pytest

import oracle
import scenarios as S

from test_oracle_pins import one_link, placed
from tiny import tiny_grid


def snapshot(o):
    V = o.vehicles()
    return {int(v): (int(e), int(l), int(c)) for v, e, l, c in zip(V["vid"], V["edge"], V["lane"], V["cursor"])}


@pytest.mark.parametrize("seed", range(4))
def test_winning_claims_are_the_visible_events(seed):
    o = oracle.Oracle(tiny_grid(seed, n_trips=80, horizon=40), "f64")
    prev = snapshot(o)
    crossings = changes = entries = 0
    for _ in range(300):
        o.step()
        cur = snapshot(o)
        for vid, (e, l, c) in cur.items():
            if vid not in prev:
                entries += 1
            elif c != prev[vid][2]:
                crossings += 1
            elif l != prev[vid][1]:
                changes += 1
        prev = cur
    c = o.counters()
    assert c["claims"] - c["claims_lost"] == crossings + changes + entries
    assert entries == c["departed"] and c["claims_departure"] >= entries
    assert c["claims_lane_change"] >= changes > 0
    assert c["claims"] - c["claims_departure"] - c["claims_lane_change"] >= crossings > 0
    assert c["lc_evaluated"] >= c["claims_lane_change"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lane_change_evaluations_on_a_long_link(prec):
    rng = np.random.default_rng(5)
    n = 18
    k = np.arange(n)
    xs = (3.0 + 7.0 * k + rng.uniform(0.0, 1.0, n)).astype(np.float32)  # 21 m apart per lane; the first
    lanes = k % 3                                                         # starts shorter than a car
    vs = rng.uniform(3.0, 12.0, n).astype(np.float32)
    p = S.default_params()
    scen = placed(one_link(8000.0, 15.0, n_lanes=3), p, xs, vs, lanes=lanes)
    o = oracle.Oracle(scen, prec)
    cool = int(p["lc_cooldown"])
    expect = 0
    for _ in range(120):
        t = o.counters()["step"]
        V = o.vehicles()
        expect += int(np.sum(((t - V["lc"].astype(np.int64)) >= cool) & (V["x"] >= 5.0)))
        o.step()
    c = o.counters()
    assert c["en_route"] == n and c["arrived"] == 0
    assert c["lc_evaluated"] == expect
    assert 0 < c["claims_lane_change"] <= expect
