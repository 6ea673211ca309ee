"""Pins of intersection control (Sec. 6.3.2, last paragraph), checked from the
outside on the oracle's trajectories:

* stop sign: every vehicle that passes a stop node has first come to rest at
  its line (speed <= stop_speed within stop_dist of the link end), and the
  node lets vehicles through one at a time (never two crossings in one step);
* traffic signal: with n inbound and m outbound links, the n*m movements get
  the green in turn, `signal_green` steps each; every crossing happens while
  its own movement is green;
* the brute-force implementation agrees bit for bit.
"""
import numpy as np
import pytest

import oracle
import scenarios as S
from oracle.brute import Brute

from test_oracle_pins import same_state
from tiny import tiny_grid


def controlled(seed, p_stop=0.4, p_signal=0.4, green=6):
    scen = tiny_grid(seed, n_trips=60, horizon=30)
    scen["net"]["node_control"] = S.random_control(scen["net"], seed + 100, p_stop, p_signal)
    scen["params"]["signal_green"] = green
    return scen


def movements(net):
    rp, head = net["row_ptr"], net["col_idx"]
    tails = S.tails_of(net)
    out = {}
    for h in range(rp.size - 1):
        inbound = [e for e in range(head.size) if head[e] == h]
        outs = list(range(rp[h], rp[h + 1]))
        out[h] = [(i, o) for i in inbound for o in outs]
    return out, tails


@pytest.mark.parametrize("seed", range(6))
def test_stop_and_signal_rules(seed):
    scen = controlled(seed)
    net, p = scen["net"], scen["params"]
    ctrl = net["node_control"]
    mv, _ = movements(net)
    o = oracle.Oracle(scen, "f64")
    prev = o.vehicles()
    stopped_at_line = set()  # (vid, edge)
    crossings_stop = crossings_signal = 0
    for t in range(400):
        for vid, e, x, v in zip(prev["vid"], prev["edge"], prev["x"], prev["v"]):
            if net["length"][e] - x <= p["stop_dist"] and v <= p["stop_speed"]:
                stopped_at_line.add((int(vid), int(e)))
        o.step()
        cur = o.vehicles()
        common, ia, ib = np.intersect1d(prev["vid"], cur["vid"], return_indices=True)
        moved = prev["edge"][ia] != cur["edge"][ib]
        per_node = {}
        for vid, e0, e1 in zip(common[moved], prev["edge"][ia][moved], cur["edge"][ib][moved]):
            h = int(net["col_idx"][e0])
            if ctrl[h] == 1:
                assert (int(vid), int(e0)) in stopped_at_line, (t, vid)
                per_node[h] = per_node.get(h, 0) + 1
                crossings_stop += 1
            elif ctrl[h] == 2:
                phase = (t // p["signal_green"]) % len(mv[h])
                assert mv[h][phase] == (int(e0), int(e1)), (t, vid)
                crossings_signal += 1
        assert all(c == 1 for c in per_node.values())
        prev = cur
    assert crossings_stop > 0 and crossings_signal > 0


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_with_control(seed):
    scen = controlled(seed, 0.35, 0.35)
    o, b = oracle.Oracle(scen, "f64"), Brute(scen)
    for st in range(400):
        o.step()
        b.step()
        assert same_state(o, b) is None, (seed, st)
    for k, v in o.edge_stats().items():
        assert np.array_equal(v, b.edge_stats()[k])


def test_single_stop_sign_comes_to_rest():
    from tiny import chain_net
    net, tails, heads = chain_net(n_edges=2, length=120.0, lanes=1, branch=False)
    net["node_control"] = np.array([0, 1, 0], np.int32)
    p = S.default_params()
    scen = {"name": "stop", "net": net, "params": p, "steps": 200, "demand": {
        "depart_step": np.array([0], np.int32), "trip_route": np.array([0], np.int32),
        "route_ptr": np.array([0, 2], np.int64), "route_edges": np.array([0, 1], np.int32)}}
    o = oracle.Oracle(scen, "f64")
    vmin_near_line = 1e9
    for _ in range(200):
        o.step()
        V = o.vehicles()
        if V["vid"].size and V["edge"][0] == 0 and 120.0 - V["x"][0] <= p["stop_dist"]:
            vmin_near_line = min(vmin_near_line, float(V["v"][0]))
    assert vmin_near_line <= p["stop_speed"]
    assert o.trips()["arrive_step"][0] > 0
