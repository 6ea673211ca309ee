"""The allocation-free shortest-path tree (rt_tree_static, include/
trafficroute.h), through the C ABI, against the allocating rt_tree on the same
router: distances and predecessors bit for bit.  Two networks in a row, the
second smaller than the first, so the second call runs on what the first left
in the shared static scratch; a network too large for the scratch is refused
with SIM_EINVAL before anything runs."""
import numpy as np
import pytest

import scenarios as S

pytestmark = pytest.mark.gpu


def _router(net, w):
    from paper_1807_01148_amd.route import Router
    rt = Router(net)
    rt.set_weights(w)
    return rt


def _static_tree(rt, src):
    import torch
    dist = torch.full((rt.num_nodes,), -7, dtype=torch.int64, device="cuda:0")
    pred = torch.full((rt.num_nodes,), -7, dtype=torch.int32, device="cuda:0")
    rt.tree_static(src, dist, pred)
    return dist.cpu().numpy(), pred.cpu().numpy()


def test_static_tree_equals_tree_on_two_networks_in_a_row():
    rng = np.random.default_rng(21)
    big = S.grid(40, seed=5)
    small = S.grid(9, seed=6)
    cases = []
    for net, srcs in ((big, (0, 777, 1599)), (small, (0, 40, 80))):
        w = rng.integers(1, 4, net["col_idx"].size).astype(np.int64)  # many ties: the route rule decides
        cases.append((net, w, srcs))
    for net, w, srcs in cases:
        rt = _router(net, w)
        for s in srcs:
            da, pa = rt.tree(s)
            ds, ps = _static_tree(rt, s)
            assert np.array_equal(ds, da), s
            assert np.array_equal(ps, pa), s
            assert ps[s] == -1 and ds[s] == 0
        rt.close()


def test_static_tree_refuses_a_network_beyond_the_scratch():
    import torch
    from paper_1807_01148_amd import SimError, SIM_EINVAL
    # a path of nodes larger than the static scratch holds (32 B per node, 48 MiB)
    n = 1_700_000
    tails = np.arange(n - 1, dtype=np.int32)
    net = {"row_ptr": np.concatenate([np.arange(n, dtype=np.int32), [n - 1]]).astype(np.int32),
           "col_idx": (tails + 1).astype(np.int32), "lanes": np.ones(n - 1, np.int32),
           "length": np.full(n - 1, 10.0, np.float32), "speed": np.full(n - 1, 10.0, np.float32)}
    rt = _router(net, np.ones(n - 1, np.int64))
    d = torch.empty(n, dtype=torch.int64, device="cuda:0")
    with pytest.raises(SimError) as ei:
        rt.tree_static(0, d, None)
    assert ei.value.code == SIM_EINVAL and "static buffer" in str(ei.value)
    rt.close()
