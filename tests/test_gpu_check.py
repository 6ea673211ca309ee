"""State validation through the C ABI (sim_check_state, and sim_set_state,
which validates an image before it copies anything in):

* every state the step produces passes every class: the 10x10 grid with lane
  changes, lost claims and arrivals (plain steps and graph replays), a grid
  with trucks, stop signs and signals, a multi-lane ring of placed vehicles,
  and a batch of scenarios;
* an image with one planted violation of each class is refused with
  SIM_EINVAL, the class named in the message, and the simulation it was
  offered to continues exactly as before.
"""
import numpy as np
import pytest

import scenarios as S

from test_gpu_state import controlled_trucks, snapshot, same
from tiny import tiny_grid

pytestmark = pytest.mark.gpu

COUNTERS_BYTES = 96  # int t, n, n_next; unsigned scan_tile, epoch_next; nine 64-bit counters


def assert_clean(counts, first, what):
    bad = {k: (c, first[k]) for k, c in counts.items() if c}
    assert not bad, (what, bad)


def image_layout(img):
    """Offsets of the arrays of a state image, from its header (magic, step,
    capacity, queues, nodes, links, trips, bytes), each array starting on a
    256-byte boundary after a 256-byte header."""
    hdr = np.frombuffer(img[:64].tobytes(), np.int64)
    cap, nq, nn, ne = (int(a) for a in hdr[2:6])
    off, o = {}, 256

    def take(name, nbytes):
        nonlocal o
        off[name] = o
        o = (o + nbytes + 255) // 256 * 256
    for f in ("key", "x", "v", "edge", "rcur", "next", "lc", "kin", "phin", "vid", "fuel", "co"):
        take(f, 4 * cap)
    take("ty", cap)
    take("q", 8 * nq)
    take("ctr", COUNTERS_BYTES)
    take("hold", 4 * nn)
    for f in ("depart", "arrive", "fuel_total", "co_total"):
        take(f, 4 * cap)
    for f in ("st_cnt", "st_steps", "st_us"):
        take(f, 8 * ne)
    assert o == int(hdr[7]) == img.size  # the layout is the library's
    return off, dict(cap=cap, nq=nq, nn=nn, ne=ne, ntrips=int(hdr[6]))


class Image:
    """A host copy of a state image with typed views of its arrays."""

    def __init__(self, dev_img):
        self.b = dev_img.cpu().numpy().copy()
        self.off, self.dims = image_layout(self.b)
        self.n = int(self.arr("ctr", np.int32, 2)[1])

    def arr(self, name, dt, count=None):
        count = self.dims["cap"] if count is None else count
        return np.frombuffer(self.b, dt, count, self.off[name])

    def field(self, name):
        dt = {"x": np.float32, "v": np.float32, "phin": np.float32, "fuel": np.float32, "co": np.float32,
              "ty": np.uint8}.get(name, np.int32)
        return self.arr(name, dt)

    def device(self):
        import torch
        return torch.from_numpy(self.b).cuda()


def run_grid():
    import paper_1807_01148_amd as P
    g = P.Sim(S.small_grid(n_trips=1500, steps=1800))
    g.step(700)
    return g


@pytest.mark.parametrize("make", [lambda: S.small_grid(n_trips=2000, steps=3600), controlled_trucks],
                         ids=["grid10", "grid10-trucks-control"])
def test_states_the_step_produces_pass(make):
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import step_graph
    scen = make()
    g = P.Sim(scen)
    for k in range(6):
        if k % 2:
            step_graph(g, 300, 60)
        else:
            g.step(300)
        counts, first = g.check_state()
        assert_clean(counts, first, k)
    c = g.counters()
    assert c["claims_lost"] > 0 and c["arrived"] > 0 and c["claims_lane_change"] > 0, c


def test_placed_ring_and_batch_pass():
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd.ensemble import Ensemble
    scen = S.ring_road(n_veh=24, length=400.0, jitter=3.0)
    scen["net"]["lanes"][:] = 3
    scen["demand"]["init_lane"] = (np.arange(24) % 3).astype(np.int32)
    scen["demand"]["init_x"] = (np.arange(24) // 3 * 50.0 + 5.0 + np.arange(24) % 3 * 7.0).astype(np.float32)
    g = P.Sim(scen)
    for _ in range(4):
        counts, first = g.check_state()
        assert_clean(counts, first, "ring")
        g.step(100)
    ens = Ensemble([tiny_grid(70 + q, n_trips=60, horizon=30) for q in range(3)])
    for _ in range(3):
        ens.step(100)
        counts, first = ens.check_state()
        assert_clean(counts, first, "batch")
    assert ens.counters()["arrived"] > 0


def plant(img, cls):
    """One violation of class cls in the host image img (a vehicle entry of
    the sorted arrays, its trip state, a queue or a node)."""
    key, x, v, edge = img.field("key"), img.field("x"), img.field("v"), img.field("edge")
    vid, nxt, ty = img.field("vid"), img.field("next"), img.field("ty")
    n = img.n
    same_lane = np.flatnonzero((key[:n - 1] == key[1:n]) & (x[:n - 1] < x[1:n]))
    first_of_lane = np.flatnonzero(np.r_[True, key[1:n] != key[:n - 1]])
    i = int(same_lane[0])
    if cls == "count":
        img.arr("ctr", np.int32, 2)[1] = img.dims["cap"] + 1
    elif cls == "key":
        key[n - 1] = 1 << 30
    elif cls == "edge":
        edge[i] = (edge[i] + 1) % img.dims["ne"]
    elif cls == "order":
        x[i], x[i + 1] = x[i + 1], x[i]
    elif cls == "position":
        x[int(first_of_lane[0])] = -1.0
    elif cls == "speed":
        v[i] = np.nan
    elif cls == "vid":
        vid[i] = img.dims["ntrips"]
    elif cls == "duplicate":
        vid[i + 1] = vid[i]
    elif cls == "type":
        ty[i] = 3
    elif cls == "route":
        img.field("rcur")[vid[i]] = -5
    elif cls == "next":
        nxt[i] = (nxt[i] + 2) % img.dims["ne"] if nxt[i] >= 0 else 0
    elif cls == "value":
        img.field("phin")[vid[i]] = 2.0
    elif cls == "arrived":
        img.arr("arrive", np.int32)[vid[i]] = 5
    elif cls == "queue":
        q = img.arr("q", np.int32, 2 * img.dims["nq"])
        q[0] = q[img.dims["nq"]] + 1
    elif cls == "holder":
        img.arr("hold", np.int32, img.dims["nn"])[0] = img.dims["ntrips"] + 7
    else:
        raise AssertionError(cls)


def test_images_with_a_planted_violation_are_refused():
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import CHECK_CLASSES
    g = run_grid()
    good = g.save_state().clone()
    ref_img = Image(good)
    # the unchanged image passes the same path, and is byte-identical through the host
    g.load_state(ref_img.device())
    names = {"count": "vehicle count or step", "key": "lane key", "edge": "link of the lane key",
             "order": "order by (lane, position)", "position": "position", "speed": "speed",
             "vid": "vehicle id", "duplicate": "duplicate vehicle id", "type": "vehicle type",
             "route": "route cursor", "next": "next link", "value": "entry fraction, fuel or CO",
             "arrived": "arrived vehicle on the road", "queue": "departure queue", "holder": "stop-node holder"}
    assert set(names) == set(CHECK_CLASSES)
    for cls in CHECK_CLASSES:
        img = Image(good)
        plant(img, cls)
        with pytest.raises(P.SimError) as e:
            g.load_state(img.device())
        assert e.value.code == P.SIM_EINVAL, cls
        assert "fails validation: " + names[cls] + " (" in str(e.value), (cls, str(e.value))
    # nothing was copied in: the simulation continues as the uninterrupted run
    g.step(400)
    b = run_grid()
    b.step(400)
    same(snapshot(g), snapshot(b))
    counts, first = g.check_state()
    assert_clean(counts, first, "after refusals")
