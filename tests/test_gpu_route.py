"""GPU route planning for re-routing (Sec. 6.3.1) against the CPU oracle,
through the C ABI (include/trafficroute.h).

Bar: bit-exact.  Weights are integers, so distances are exact, and the route
rule (lowest tight edge into every node) makes every route unique:
  * shortest-path trees (distance and predecessor of every node) equal the
    oracle's Dijkstra on random digraphs with many equal-length paths, on the
    10x10 grid, and from sampled origins of the 1M-node metro network;
  * planned routes equal the oracle's for full and partial plans, for any
    number of origins searched at once;
  * the whole loop (plan, simulate, measured weights, partial re-plans) equals
    the oracle's loop on the 10x10 grid, iteration by iteration;
  * error codes for unreachable destinations and bad calls.
"""
import numpy as np
import pytest

import scenarios as S
from oracle import routing as R

from test_oracle_routing import diamond, random_digraph
from tiny import tiny_grid

pytestmark = pytest.mark.gpu


def router(net):
    from paper_1807_01148_amd.route import Router
    return Router(net)


def as_net(g):
    ne = g["col_idx"].size
    return dict(g, lanes=np.ones(ne, np.int32), length=np.full(ne, 50.0, np.float32),
                speed=np.full(ne, 10.0, np.float32))


@pytest.mark.parametrize("seed", range(8))
def test_trees_match_dijkstra_on_random_digraphs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    g, _, w = random_digraph(rng, n, p=min(0.5, 4.0 / n), wmax=3)
    if g["col_idx"].size == 0:
        return
    net = as_net(g)
    rt = router(net)
    rt.set_weights(w)
    for s in range(n):
        dg, pg = rt.tree(s)
        do, po = R.sssp(net, w, s)
        assert np.array_equal(dg, do), s
        assert np.array_equal(pg, po), s


def test_trees_match_dijkstra_on_grid_with_random_weights():
    scen = S.small_grid()
    net = scen["net"]
    rng = np.random.default_rng(3)
    rt = router(net)
    for wmax in (1, 3, 100000):
        w = rng.integers(1, wmax + 1, net["col_idx"].size).astype(np.int64)
        rt.set_weights(w)
        for s in (0, 17, 55, 99):
            dg, pg = rt.tree(s)
            do, po = R.sssp(net, w, s)
            assert np.array_equal(dg, do), (wmax, s)
            assert np.array_equal(pg, po), (wmax, s)


def test_initial_weights_equal_the_oracle():
    scen = tiny_grid(5, n_trips=20)
    rt = router(scen["net"])
    assert np.array_equal(rt.weights(), R.initial_weights(scen["net"]))


@pytest.mark.parametrize("batch", [0, 1, 7])
def test_full_and_partial_plans_equal_the_oracle(batch):
    scen = S.small_grid()
    net, d = scen["net"], scen["demand"]
    rt = router(net)
    if batch:
        rt.set_batch(batch)
    rt.set_trips(d["src_nodes"], d["trip_src"], d["trip_dst"])
    w0 = R.initial_weights(net)
    rt.plan()
    ptr, edges = rt.routes()
    optr, oedges = R.plan(net, w0, d["src_nodes"], d["trip_src"], d["trip_dst"])
    assert np.array_equal(ptr, optr) and np.array_equal(edges, oedges)
    rng = np.random.default_rng(11)
    w1 = rng.integers(5000, 20000, net["col_idx"].size).astype(np.int64)
    rt.set_weights(w1)
    mask = S.reroute_masks(2, d["trip_src"].size)[2]
    rt.plan(mask)
    ptr2, edges2 = rt.routes()
    optr2, oedges2 = R.plan(net, w1, d["src_nodes"], d["trip_src"], d["trip_dst"], mask, (optr, oedges))
    assert np.array_equal(ptr2, optr2) and np.array_equal(edges2, oedges2)
    relax, nsrc = rt.last_work()
    assert nsrc == np.unique(d["trip_src"][mask]).size and relax >= nsrc


def test_reroute_loop_equals_the_oracle_loop():
    from paper_1807_01148_amd.route import reroute
    scen = S.small_grid(n_trips=2000, steps=3600)
    masks = S.reroute_masks(5, 2000)
    g = reroute(scen, masks)
    o = R.reroute(scen, masks)
    for k, (a, b) in enumerate(zip(g, o)):
        assert np.array_equal(a["weights"], b["weights"]), k
        assert np.array_equal(a["route_ptr"], b["route_ptr"]), k
        assert np.array_equal(a["route_edges"], b["route_edges"]), k
        for key in b["stats"]:
            assert np.array_equal(a["stats"][key], b["stats"][key]), (k, key)
        assert {x: a["counters"][x] for x in b["counters"]} == b["counters"], k


def test_diamond_loop_equals_the_oracle_loop():
    from paper_1807_01148_amd.route import reroute
    scen = diamond()
    masks = S.reroute_masks(1, 300)
    g, o = reroute(scen, masks), R.reroute(scen, masks)
    for a, b in zip(g, o):
        assert np.array_equal(a["route_edges"], b["route_edges"])
        assert np.array_equal(a["weights"], b["weights"])


def test_metro_trees_from_sampled_origins():
    net = S.metro(seed=1810)
    net.pop("xy", None)
    rt = router(net)
    w = R.initial_weights(net)
    assert np.array_equal(rt.weights(), w)
    rng = np.random.default_rng(8)
    for s in rng.choice(net["row_ptr"].size - 1, 3, replace=False):
        dg, pg = rt.tree(int(s))
        do, po = R.sssp(net, w, int(s))
        assert np.array_equal(dg, do), s
        assert np.array_equal(pg, po), s


def test_errors():
    import paper_1807_01148_amd as P
    scen = diamond()
    net, d = scen["net"], scen["demand"]
    rt = router(net)
    with pytest.raises(P.SimError) as e:
        rt.plan()
    assert e.value.code == P.SIM_ESTATE
    with pytest.raises(P.SimError) as e:
        rt.set_trips([0], [0], [0])  # destination is the origin
    assert e.value.code == P.SIM_EINVAL
    rt.set_trips([3], [0], [0])  # node 3 has no way out
    with pytest.raises(P.SimError) as e:
        rt.plan()
    assert e.value.code == P.SIM_EROUTE
    rt.set_trips(d["src_nodes"], d["trip_src"], d["trip_dst"])
    with pytest.raises(P.SimError) as e:
        rt.plan(np.ones(d["trip_src"].size, np.uint8))  # partial plan before any routes
    assert e.value.code == P.SIM_ESTATE
    with pytest.raises(P.SimError) as e:
        rt.set_weights(np.zeros(net["col_idx"].size, np.int64))
    assert e.value.code == P.SIM_EINVAL
    assert rt.plan() == 2 * d["trip_src"].size


@pytest.mark.parametrize("delta", [500, 20000, 10 ** 9])
def test_band_width_changes_work_not_result(delta):
    scen = S.small_grid()
    net, d = scen["net"], scen["demand"]
    rng = np.random.default_rng(12)
    w = rng.integers(1000, 60000, net["col_idx"].size).astype(np.int64)
    rt = router(net)
    rt.set_weights(w)
    rt.set_delta(delta)
    rt.set_trips(d["src_nodes"], d["trip_src"], d["trip_dst"])
    rt.plan()
    ptr, edges = rt.routes()
    optr, oedges = R.plan(net, w, d["src_nodes"], d["trip_src"], d["trip_dst"])
    assert np.array_equal(ptr, optr) and np.array_equal(edges, oedges)
    for s in (0, 42):
        dg, pg = rt.tree(s)
        do, po = R.sssp(net, w, s)
        assert np.array_equal(dg, do) and np.array_equal(pg, po)
