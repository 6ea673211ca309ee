"""Tiny seeded scenarios for brute-force and exhaustive checks."""
import numpy as np

import scenarios as S


def tiny_grid(seed, side=3, n_trips=10, horizon=40, lane_probs=(0.3, 0.4, 0.3), lognormal=(30.0, 0.3),
              num_classes=2, min_len=20.0):
    rng = np.random.default_rng(seed)
    net = S.grid(side, seed=seed, lane_probs=lane_probs, lognormal=lognormal, speed=12.0,
                 num_classes=num_classes, min_len=min_len)
    p = S.default_params(num_classes)
    p["idm"][:, 0] = rng.uniform(0.8, 1.2, num_classes)
    p["idm"][:, 1] = rng.uniform(1.0, 2.0, num_classes)
    p["idm"][:, 2] = rng.uniform(0.7, 1.5, num_classes)
    p["idm"][:, 3] = rng.uniform(1.0, 2.5, num_classes)
    p["mand_dist"] = 15.0
    o, d = S.uniform_od(rng, side * side, n_trips)
    dep = rng.integers(0, horizon, n_trips) * p["dt"]
    return {"name": "tiny%d" % seed, "net": net, "params": p,
            "demand": S.make_demand(net, o, d, dep, p["dt"]), "steps": 400}


def chain_net(n_edges=2, length=30.0, lanes=2, branch=True, speed=12.0):
    """Node chain 0 -> 1 -> ... with, at every inner node, an extra side
    link (so turn bands split the lanes)."""
    tails, heads = [], []
    n_nodes = n_edges + 1
    for k in range(n_edges):
        tails.append(k)
        heads.append(k + 1)
    if branch:
        for k in range(1, n_edges):
            tails.append(k)
            heads.append(n_nodes)
            n_nodes += 1
    tails = np.array(tails)
    heads = np.array(heads)
    order = np.lexsort((heads, tails))
    tails, heads = tails[order], heads[order]
    row_ptr = np.zeros(n_nodes + 1, np.int32)
    np.add.at(row_ptr, tails + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    m = tails.size
    return {"row_ptr": row_ptr, "col_idx": heads.astype(np.int32),
            "lanes": np.full(m, lanes, np.int32), "length": np.full(m, length, np.float32),
            "speed": np.full(m, speed, np.float32), "link_class": np.zeros(m, np.int32)}, tails, heads
