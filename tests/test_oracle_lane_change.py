"""Pins of the oracle's lane-change decision (Sec. 6.3.2: mandatory or
discretionary changes, each behind gap acceptance), from constructed
placements whose outcome is derived by hand from the published MOBIL rule
(Kesting, Treiber and Helbing 2007, the reading this build takes for the
discretionary criterion and the safety test):

    change to lane L' iff
      safety:    the new follower's acceleration after the change >= -b_safe
      incentive: (a~_c - a_c) + p * ((a~_n - a_n) + (a~_o - a_o)) > a_thr
    (c = the changing vehicle, n = its new follower, o = its old follower;
     ~ = after the change), ties between the two sides to the lower lane;
    mandatory (outside the lane band of the next turn within d_mand of the
    link end): toward the band, safety only.

Each case is built so that exactly one term of that rule decides, and a
mistake in that term (a dropped term, a flipped sign, a_n in place of a~_n,
the wrong threshold, the wrong side of d_mand) flips the outcome.  The
accelerations are the IDM's, whose form is pinned by the free-road, ring and
intelligent-braking pins; the numbers quoted in the comments are its FP64
values at the defaults (v0 = 15 m/s, T = 1.5 s, a = 1, b = 1.5, s0 = 2 m,
length 5 m, p = 0.2, a_thr = 0.1, b_safe = 4).

Also the queue pins: vehicles at rest queued behind a stopped obstacle (a
stop line held red) close up to the minimum gap s0; from above when the IDM's
linearization there is overdamped, with a small overshoot when it is not.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import scenarios as S
from oracle.brute import Brute

from test_oracle_pins import one_link, placed
from tiny import chain_net

PRECS = ["f32", "f64", "brute"]


def idm(v, s=None, vl=0.0, v0=15.0, T=1.5, a=1.0, b=1.5, s0=2.0):
    """IDM acceleration (FP64) behind a leader at bumper gap s (None: free road)."""
    acc = 1.0 - (v / v0) ** 4
    if s is not None:
        star = s0 + max(0.0, v * T + v * (v - vl) / (2.0 * math.sqrt(a * b)))
        acc -= (star / s) ** 2
    return max(a * acc, -9.0)


def run_one_step(scen, prec):
    o = Brute(scen) if prec == "brute" else oracle.Oracle(scen, prec)
    o.step(1)
    v = o.vehicles()
    return dict(zip(v["vid"].tolist(), v["lane"].tolist()))


def scenario(xs, vs, lanes, n_lanes=2, length=1000.0, p=None, route=(0,), net=None):
    prm = S.default_params()
    if p is not None:
        prm["mobil_p"] = p
    if net is None:
        net = one_link(length, 15.0, n_lanes)
    return placed(net, prm, xs, vs, lanes, route=route)


# vehicle ids are the trips' ranks by (departure step, index): all depart
# now, so vid = position in the lists below


@pytest.mark.parametrize("prec", PRECS)
def test_lane_with_faster_leader_is_taken(prec):
    # A (vid 0) at x=200, v=10 in lane 0, 10 m behind a stopped B (vid 1):
    # a_c is the floor -9.  In lane 1, C (vid 2) at x=214 drives at 15 m/s:
    # a~_c = 0.802 - 0.049 = 0.753 (its desired gap is s0 only, C recedes),
    # so the own gain alone is 9.75 > a_thr.  B cannot go to lane 1 (C's rear
    # is 4 m ahead of B's front) and C cannot go to lane 0 (B overlaps it).
    assert idm(10.0, 10.0, 0.0) == -9.0 and abs(idm(10.0, 9.0, 15.0) - 0.753) < 1e-3
    lanes = run_one_step(scenario([200.0, 215.0, 214.0], [10.0, 0.0, 15.0], [0, 0, 1]), prec)
    assert lanes == {0: 1, 1: 0, 2: 1}


@pytest.mark.parametrize("prec", PRECS)
def test_lane_with_a_leader_as_slow_is_not_taken(prec):
    # as above with C stopped: a~_c = a_c = -9 (both floored), no follower
    # anywhere: incentive 0 < a_thr
    assert idm(10.0, 9.0, 0.0) == -9.0
    lanes = run_one_step(scenario([200.0, 215.0, 214.0], [10.0, 0.0, 0.0], [0, 0, 1]), prec)
    assert lanes == {0: 0, 1: 0, 2: 1}


@pytest.mark.parametrize("prec", PRECS)
def test_empty_lane_taken_and_blocker_yields_out_of_politeness(prec):
    # lane 1 empty.  A's own gain 0.802 + 9 > a_thr.  The stopped B gains
    # nothing itself (free road both ways, 1 m/s^2), but its old follower A
    # does: a~_o - a_o = 0.802 + 9, times p = 1.96 > a_thr, so B moves over as
    # well; their claims (cells 198..205 and 208..215) do not overlap.
    lanes = run_one_step(scenario([200.0, 215.0], [10.0, 0.0], [0, 0]), prec)
    assert lanes == {0: 1, 1: 1}


@pytest.mark.parametrize("prec", PRECS)
def test_tie_between_sides_goes_to_the_lower_lane(prec):
    # three lanes, A and B in the middle one, lanes 0 and 2 empty: equal
    # incentives on both sides, the lower lane wins (for B too)
    lanes = run_one_step(scenario([200.0, 215.0], [10.0, 0.0], [1, 1], n_lanes=3), prec)
    assert lanes == {0: 0, 1: 0}


def _new_follower_speed_at(acc_target, gap=9.0, vl=10.0):
    return brentq(lambda v: idm(v, gap, vl) - acc_target, 10.0, 30.0)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("side", [-1, 1])
def test_safety_uses_new_followers_acceleration_after_the_change(prec, side):
    # A blocked in lane 0 as above; lane 1 holds only F (vid 2) at x=186,
    # 9 m behind A's rear once A is there.  F's acceleration behind A,
    # a~_n, crosses -b_safe = -4 at a speed v*; 0.4 m/s below v* the change
    # is safe, 0.4 m/s above it is not.  Everything else passes at both
    # speeds: F's current acceleration a_n (free road) is >= -0.6, its
    # free-road displacement (< 8 m) fits in the 14 m it has, and the
    # incentive is >= 9.8 + 0.2 * (-4.4 - 1) > a_thr.
    vstar = _new_follower_speed_at(-4.0)
    vf = vstar + 0.4 * side
    assert (idm(vf, 9.0, 10.0) < -4.0) == (side > 0)
    assert idm(vf) > -0.6 and vf * 0.5 + idm(vf) * 0.125 < 14.0
    lanes = run_one_step(scenario([200.0, 215.0, 186.0], [10.0, 0.0, vf], [0, 0, 1]), prec)
    assert lanes[0] == (0 if side > 0 else 1)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [0.2, 0.0])
def test_old_followers_gain_counts_with_politeness(prec, p):
    # A at x=200, v=10 follows B (x=281, v=10) at a 76 m gap: a_c = 0.7524,
    # free road in lane 1: a~_c = 0.8025, own gain 0.050 < a_thr.  O at
    # x=192, v=12 is 3 m behind A (floored at -9); with A gone it follows B
    # at 84 m: 0.4645.  Incentive 0.050 + p * 9.46: 1.94 with p = 0.2 (A
    # changes), 0.050 with p = 0 (A stays).  O wants lane 1 in both cases
    # (its own gain is large); with p = 0.2 its claim (cells 191..198) meets
    # A's (198..205) in cell 198 and A, the lower id, wins it: O stays.
    assert abs((idm(10.0) - idm(10.0, 76.0, 10.0)) - 0.050) < 1e-3
    assert abs(idm(12.0, 84.0, 10.0) - 0.4645) < 1e-3 and idm(12.0, 3.0, 10.0) == -9.0
    lanes = run_one_step(scenario([200.0, 281.0, 192.0], [10.0, 10.0, 12.0], [0, 0, 0], p=p), prec)
    assert lanes[0] == (1 if p > 0 else 0)
    assert lanes[1] == 0 and lanes[2] == (0 if p > 0 else 1)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("far", [False, True])
def test_new_followers_loss_counts_against_the_change(prec, far):
    # A at x=200, v=10 follows B (x=236, v=10) at 31 m: own gain in the empty
    # lane ahead 0.300 > a_thr.  In lane 1, F (v=12) behind: at a 20.6 m gap
    # behind A its acceleration drops from 0.590 (free) to -1.50, a loss of
    # 2.09 (still safe): 0.300 + 0.2 * (-2.09) = -0.118 < a_thr, A stays.
    # With F 100 m back the loss is 0.089: 0.282 > a_thr, A changes.
    g = 100.0 if far else 20.6
    gain = idm(10.0) - idm(10.0, 31.0, 10.0)
    loss = idm(12.0, g, 10.0) - idm(12.0)
    assert abs(gain - 0.300) < 2e-3
    assert (gain + 0.2 * loss > 0.1) == far and idm(12.0, g, 10.0) > -4.0
    xf = 195.0 - g
    lanes = run_one_step(scenario([200.0, 236.0, xf], [10.0, 10.0, 12.0], [0, 0, 1]), prec)
    assert lanes[0] == (1 if far else 0)
    assert lanes[1] == 0 and lanes[2] == 1


def _turn_scenario(x, lane, xs_extra=(), vs_extra=(), lanes_extra=()):
    # link 0 (200 m, 2 lanes) ends at node 1, whose out-links are link 1
    # (rank 0: band lane 0) and link 2 (rank 1: band lane 1); every vehicle
    # turns onto link 2
    net, _, _ = chain_net(n_edges=2, length=200.0, lanes=2, branch=True)
    return scenario([x] + list(xs_extra), [10.0] + list(vs_extra), [lane] + list(lanes_extra),
                    route=(0, 2), net=net)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d", [83.2, 83.3, 120.0])
def test_mandatory_change_toward_the_band_only_within_d_mand(prec, d):
    # alone in lane 0, outside the band of its turn (lane 1): within
    # d_mand = 100 sqrt(ln 2) = 83.26 m of the link end the change is
    # mandatory (no incentive needed); farther out it is discretionary and
    # an empty road gives no incentive
    dmand = S.default_params()["mand_dist"]
    assert (d <= dmand) == (d == 83.2)
    lanes = run_one_step(_turn_scenario(200.0 - d, 0), prec)
    assert lanes[0] == (1 if d <= dmand else 0)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d", [50.0, 150.0])
def test_in_band_vehicle_keeps_its_band_near_the_turn(prec, d):
    # in lane 1 (its band) behind a stopped vehicle 10 m ahead, lane 0 with
    # a fast vehicle beside the blocker (as in the first test): far from the
    # link end it changes to lane 0; within d_mand it may not leave its band
    x = 200.0 - d
    lanes = run_one_step(_turn_scenario(x, 1, [x + 15.0, x + 14.0], [0.0, 15.0], [1, 0]), prec)
    assert lanes[0] == (0 if d > 83.26 else 1)


def _queue(prec, T, dt=0.5, n_veh=6, gap0=10.0, seconds=2000.0):
    """A standing queue: n_veh vehicles at rest, gap0 apart, on a one-lane
    link (300 m) into node 1, all turning onto the side link; node 1 is a
    signal whose green for that movement comes only after 10^8 steps, so the
    movement stays held: a stopped "vehicle" with its rear at the end of
    link 0.  Yields the gaps (to the vehicle ahead, the first to the line)
    and the top speed after every step."""
    net, _, _ = chain_net(n_edges=2, length=300.0, lanes=1, branch=True)
    net["node_control"] = np.array([0, 2, 0, 0], np.int32)
    prm = S.default_params(T=T, dt=dt)
    prm["signal_green"] = 10 ** 8
    xs = [300.0 - gap0 - (n_veh - 1 - k) * (5.0 + gap0) for k in range(n_veh)]
    o = oracle.Oracle(placed(net, prm, xs, [0.0] * n_veh, [0] * n_veh, route=(0, 2)), prec)
    for _ in range(int(seconds / dt)):
        o.step(1)
        v = o.vehicles()
        x = np.sort(v["x"].astype(np.float64))
        yield np.append((x[1:] - 5.0) - x[:-1], 300.0 - x[-1]), float(v["v"].max())


# Near rest at gap s = s0 + e the IDM reads e'' = -(2a/s0) e - (2aT/s0) e':
# a damped oscillator with damping ratio zeta = T sqrt(a/(2 s0)).  With
# zeta >= 1 (T >= 2 at a = 1, s0 = 2) a queue released from rest closes up
# to s0 from above, never below it; with the defaults (T = 1.5, zeta = 0.75)
# the approach overshoots and the queue stops a little short of s0.
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("T", [2.5, 3.0])
@pytest.mark.parametrize("dt", [0.5, 0.25])
def test_overdamped_standing_queue_closes_to_s0_from_above(prec, T, dt):
    tol = 1e-12 if prec == "f64" else 1e-4  # rounding of positions near 300 m
    prev = None
    for gaps, vmax in _queue(prec, T, dt):
        assert np.all(gaps >= 2.0 - tol), gaps
        if prev is not None:
            assert np.all(gaps <= prev + tol)  # every gap only closes
        prev = gaps
    assert np.all(gaps - 2.0 < 1e-3) and vmax < 1e-3


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_underdamped_standing_queue_stops_near_s0(prec):
    for gaps, vmax in _queue(prec, 1.5):
        assert np.all(gaps > 2.0 - 0.05)
    assert vmax == 0.0 and np.all(np.abs(gaps - 2.0) < 0.05) and gaps.min() < 2.0
