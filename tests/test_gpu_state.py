"""State views, checkpoint and resume through the C ABI (sim_get_state,
sim_set_state, sim_state_bytes):

* a simulation resumed from an image in a new handle, and the same handle
  rewound to an image, continue exactly as the uninterrupted run, which itself
  equals the FP32 oracle (vehicles, counters, link statistics, trips,
  emissions), also with trucks and intersection control;
* the device views hold the vehicles that sim_read_vehicles reports;
* errors: an image of another simulation, a wrong size, inside a
  differentiation window.
"""
import ctypes

import numpy as np
import pytest

import oracle
import scenarios as S

from test_gpu_parity import assert_same_outputs
from test_oracle_trucks import with_trucks
from tiny import tiny_grid

pytestmark = pytest.mark.gpu


def snapshot(g):
    return {"v": g.vehicles(), "c": g.counters(), "e": g.edge_stats(), "t": g.trips(), "m": g.emissions()}


def same(a, b):
    assert a["c"] == b["c"]
    for part in ("v", "e", "t", "m"):
        for k in a[part]:
            assert np.array_equal(a[part][k], b[part][k]), (part, k)


def controlled_trucks():
    scen = with_trucks(S.small_grid(n_trips=1500, steps=1800), 0.3, 9)
    scen["net"]["node_control"] = S.random_control(scen["net"], 9)
    return scen


@pytest.mark.parametrize("make", [lambda: S.small_grid(n_trips=1500, steps=1800), controlled_trucks],
                         ids=["grid10", "grid10-trucks-control"])
def test_resume_and_rewind_continue_exactly(make):
    import paper_1807_01148_amd as P
    scen = make()
    a = P.Sim(scen)
    a.step(700)
    img = a.save_state().clone()
    a.step(600)
    ref = snapshot(a)
    # the uninterrupted run is the oracle's
    o = oracle.Oracle(scen, "f32")
    o.step(1300)
    assert_same_outputs(a, o, "uninterrupted")
    # a new handle resumed from the image
    b = P.Sim(scen)
    b.load_state(img)
    assert b.counters()["step"] == 700
    b.step(600)
    same(snapshot(b), ref)
    # the first handle rewound to the image
    a.load_state(img)
    a.step(600)
    same(snapshot(a), ref)


def test_views_hold_the_vehicles_on_the_road():
    import paper_1807_01148_amd as P
    scen = tiny_grid(3, n_trips=80, horizon=30)
    g = P.Sim(scen)
    g.step(60)
    v = g.state_view()
    n = v.num_vehicles
    assert v.step == 60 and n == g.counters()["en_route"] > 0
    # the HIP runtime this process already uses (the one the library and torch share)
    path = next(ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64.so" in ln)
    hip = ctypes.CDLL(path)
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]

    def fetch(ptr, dt):
        a = np.zeros(n, dt)
        assert hip.hipMemcpy(a.ctypes.data_as(ctypes.c_void_p), ptr, a.nbytes, 2) == 0  # device to host
        return a
    vid, edge = fetch(v.vid, np.int32), fetch(v.edge, np.int32)
    x, sp, key = fetch(v.x, np.float32), fetch(v.v, np.float32), fetch(v.key, np.int32)
    ref = g.vehicles()
    o = np.argsort(vid)
    assert np.array_equal(vid[o], ref["vid"]) and np.array_equal(edge[o], ref["edge"])
    assert np.array_equal(x[o], ref["x"]) and np.array_equal(sp[o], ref["v"])
    lane_base = np.concatenate([[0], np.cumsum(scen["net"]["lanes"])])
    assert np.array_equal((key - lane_base[edge])[o], ref["lane"])
    assert np.all(np.diff(key) >= 0)  # sorted by lane, then position
    same_lane = np.diff(key) == 0
    assert np.all(np.diff(x)[same_lane] >= 0)


def test_state_errors():
    import paper_1807_01148_amd as P
    g = P.Sim(tiny_grid(4, n_trips=40, horizon=20))
    g.step(10)
    img = g.save_state()
    other = P.Sim(tiny_grid(5, n_trips=41, horizon=20))
    with pytest.raises(P.SimError) as e:
        other.load_state(img)  # another simulation
    assert e.value.code == P.SIM_EINVAL
    with pytest.raises(P.SimError) as e:
        g.load_state(img[:-256])  # wrong size
    assert e.value.code == P.SIM_EINVAL
    g.tape_begin(10)
    with pytest.raises(P.SimError) as e:
        g.load_state(img)  # inside a differentiation window
    assert e.value.code == P.SIM_ESTATE
