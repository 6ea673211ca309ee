"""Pins of the re-routing oracle (Sec. 6.3.1), against things it does not
compute itself:

* distances: Floyd-Warshall in Python integers on small random digraphs with
  weights 1..4 (many equal-length paths);
* the route: brute-force enumeration of every simple path on tiny graphs;
  the oracle's route must be a shortest one and, among all shortest ones, the
  one whose edge list read backwards (last edge first) is smallest;
* the weight readings: worked values of sqrt(lanes) * length / speed in ms,
  and of the rounded mean of measured traversal times;
* the loop: trips outside the re-planning mask keep their routes exactly,
  every route runs from its origin to its destination, and on two equal
  parallel paths the traffic that all starts on one (the tie rule) spreads
  onto the other once its measured time is higher.
"""
import numpy as np
import pytest

import scenarios as S
from oracle import routing as R
from tiny import tiny_grid


def random_digraph(rng, n, p=0.35, wmax=4):
    edges = [(u, v) for u in range(n) for v in range(n) if u != v and rng.random() < p]
    edges.sort()
    rp = np.zeros(n + 1, np.int32)
    for u, _ in edges:
        rp[u + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    net = {"row_ptr": rp, "col_idx": np.array([v for _, v in edges], np.int32)}
    w = rng.integers(1, wmax + 1, len(edges)).astype(np.int64)
    return net, edges, w


def floyd(n, edges, w):
    INF = float("inf")
    D = [[0 if i == j else INF for j in range(n)] for i in range(n)]
    for (u, v), c in zip(edges, w):
        D[u][v] = min(D[u][v], int(c))
    for k in range(n):
        for i in range(n):
            for j in range(n):
                if D[i][k] + D[k][j] < D[i][j]:
                    D[i][j] = D[i][k] + D[k][j]
    return D


@pytest.mark.parametrize("seed", range(20))
def test_distances_match_floyd_warshall(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 12))
    net, edges, w = random_digraph(rng, n)
    D = floyd(n, edges, w)
    for s in range(n):
        dist, pred = R.sssp(net, w, s)
        for v in range(n):
            want = D[s][v]
            assert (dist[v] == R.INF) if want == float("inf") else dist[v] == want, (s, v)
            assert (pred[v] < 0) == (v == s or want == float("inf"))


def all_simple_paths(edges, src, dst, n):
    out = []

    def dfs(v, seen, path):
        if v == dst:
            out.append(list(path))
            return
        for e, (a, b) in enumerate(edges):
            if a == v and b not in seen:
                seen.add(b)
                path.append(e)
                dfs(b, seen, path)
                path.pop()
                seen.discard(b)

    dfs(src, {src}, [])
    return out


def test_route_is_the_backward_smallest_shortest_path():
    ties = 0
    for seed in range(12):
        ties += check_backward_smallest(seed)
    assert ties >= 20  # pairs with more than one shortest path


def check_backward_smallest(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(4, 8))
    net, edges, w = random_digraph(rng, n, p=0.5, wmax=2)
    tail = R.tails(net)
    checked = 0
    for s in range(n):
        _, pred = R.sssp(net, w, s)
        for d in range(n):
            if d == s:
                continue
            paths = all_simple_paths(edges, s, d, n)
            if not paths:
                continue
            cost = [int(sum(w[e] for e in p)) for p in paths]
            best = min(cost)
            shortest = [p for p, c in zip(paths, cost) if c == best]
            want = min(shortest, key=lambda p: tuple(reversed(p)))
            got = R.walk(pred, tail, s, d)
            assert got == want, (s, d, got, shortest)
            checked += len(shortest) > 1
    return checked


def test_initial_weight_worked_values():
    net = {"lanes": np.array([1, 2, 4, 3]), "length": np.array([100.0, 100.0, 250.0, 0.0005], np.float32),
           "speed": np.array([15.0, 10.0, 20.0, 10.0], np.float32)}
    # 6666.67 -> 6667; sqrt(2) 10 s = 14142.14 -> 14142; 2 * 12.5 s = 25000; 0.09 ms -> floor at 1
    assert list(R.initial_weights(net)) == [6667, 14142, 25000, 1]


def test_measured_weights_round_the_mean_and_keep_unvisited_links():
    prev = np.array([7, 7, 7, 7], np.int64)
    count = np.array([3, 2, 0, 1], np.int64)
    tt_us = np.array([10_000_500, 3_000, 0, 400], np.int64)
    # 3333.5 ms -> 3334; 1.5 ms -> 2; unvisited -> 7; 0.4 ms -> 0 -> floor at 1
    assert list(R.weights_from_stats(prev, count, tt_us)) == [3334, 2, 7, 1]


def check_routes(net, scen, ptr, edges):
    tail = R.tails(net)
    d = scen["demand"]
    for i in range(ptr.size - 1):
        r = edges[ptr[i]:ptr[i + 1]]
        assert r.size > 0
        assert tail[r[0]] == d["src_nodes"][d["trip_src"][i]]
        assert net["col_idx"][r[-1]] == d["trip_dst"][i]
        assert np.all(net["col_idx"][r[:-1]] == tail[r[1:]])


def test_loop_keeps_unselected_routes_and_routes_connect():
    scen = S.small_grid(n_trips=800, steps=1800)
    masks = S.reroute_masks(3, 800)
    res = R.reroute(scen, masks)
    for k, r in enumerate(res):
        check_routes(scen["net"], scen, r["route_ptr"], r["route_edges"])
        if k == 0:
            continue
        prev = res[k - 1]
        for i in np.flatnonzero(~masks[k]):
            a = r["route_edges"][r["route_ptr"][i]:r["route_ptr"][i + 1]]
            b = prev["route_edges"][prev["route_ptr"][i]:prev["route_ptr"][i + 1]]
            assert np.array_equal(a, b)
    assert [int(m.sum()) for m in masks] == [800, 800, 400, 200]
    # the weights of iteration k+1 are the measured times of iteration k
    for k in range(1, len(res)):
        st = res[k - 1]["stats"]
        assert np.array_equal(res[k]["weights"], R.weights_from_stats(res[k - 1]["weights"], st["count"],
                                                                      st["tt_us"]))


def diamond(n_trips=300):
    """Node 0 -> {1, 2} -> 3, every link 200 m, one lane, 15 m/s: two equal
    routes 0-1-3 (edges 0, 2) and 0-2-3 (edges 1, 3)."""
    tails = np.array([0, 0, 1, 2])
    heads = np.array([1, 2, 3, 3])
    net = {"row_ptr": np.array([0, 2, 3, 4, 4], np.int32), "col_idx": heads.astype(np.int32),
           "lanes": np.ones(4, np.int32), "length": np.full(4, 200.0, np.float32),
           "speed": np.full(4, 15.0, np.float32), "link_class": np.zeros(4, np.int32)}
    assert np.array_equal(R.tails(net), tails)
    p = S.default_params()
    rng = np.random.default_rng(4)
    dep = np.sort(rng.uniform(0, 300, n_trips))
    demand = {"depart_step": np.floor(dep / p["dt"]).astype(np.int32),
              "trip_route": np.zeros(n_trips, np.int32), "route_ptr": np.array([0, 2], np.int64),
              "route_edges": np.array([0, 2], np.int32), "src_nodes": np.array([0], np.int32),
              "trip_src": np.zeros(n_trips, np.int32), "trip_dst": np.full(n_trips, 3, np.int32)}
    return {"name": "diamond", "net": net, "params": p, "demand": demand, "steps": 1800}


def test_equal_parallel_routes_spread_after_measurement():
    scen = diamond()
    res = R.reroute(scen, S.reroute_masks(1, 300), iterations=2)
    first = res[0]["route_edges"].reshape(-1, 2)
    assert np.all(first[:, 0] == 0)  # the tie goes to the lower edge id
    assert res[1]["weights"][0] > res[1]["weights"][1]  # upper path measured slower, lower unused
    second = res[1]["route_edges"].reshape(-1, 2)
    assert np.all(second[:, 0] == 1)  # everyone moves (share 1 in the second iteration)


def test_tiny_grid_loop_is_deterministic():
    scen = tiny_grid(3, n_trips=60, horizon=30)
    d = scen["demand"]
    assert "src_nodes" in d
    masks = S.reroute_masks(9, d["depart_step"].size)
    a = R.reroute(scen, masks)
    b = R.reroute(scen, masks)
    for x, y in zip(a, b):
        assert np.array_equal(x["route_edges"], y["route_edges"])
