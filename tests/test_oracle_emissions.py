"""Pins of the oracle's fuel, CO and utilization/speed sampler (Sec. 6.3.4, 6.4).

* a jammed ring (every vehicle at rest with exactly the minimum gap, so the
  IDM acceleration is exactly zero): fuel grows at the idle rate 0.666 mL/s
  and CO at -0.064 + 0.00026 * 50^2 = 0.586 g/s; utilization is exactly 1;
* a vehicle cruising at its desired speed: the two printed equations
  evaluated at that speed (acceleration ~ 0);
* hard braking: the fuel bracket is floored, so the rate is the idle rate;
* the sampler counts every vehicle on the road at every sampling step.
"""
import numpy as np
import pytest

import oracle
import scenarios as S

from test_oracle_pins import one_link, placed


def jammed_ring(n=20, gap=2.0):
    length = n * (5.0 + gap)
    scen = S.ring_road(n_veh=n, length=length, jitter=0.0, steps=200)
    scen["demand"]["init_x"] = (5.0 + np.arange(n) * (5.0 + gap)).astype(np.float32)
    scen["demand"]["init_v"] = np.zeros(n, np.float32)
    return scen


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_idle_fuel_and_co_on_jammed_ring(prec):
    scen = jammed_ring()
    o = oracle.Oracle(scen, prec)
    o.set_sampler(every=120, group=6, max_groups=2)
    steps = 240
    o.step(steps)
    V = o.vehicles()
    assert np.all(V["v"] == 0) and np.all(np.diff(np.sort(V["x"])) == 7.0)
    t = steps * 0.5
    rtol = 1e-12 if prec == "f64" else 1e-5
    np.testing.assert_allclose(V["fuel"].astype(np.float64), 0.666 * t, rtol=rtol)
    np.testing.assert_allclose(V["co"].astype(np.float64), (-0.064 + 0.00026 * 50.0 ** 2) * t, rtol=rtol)
    smp = o.samples()
    # samples at steps 0 and 120 fall in group 0: utilization = count / (6 cap), cap = len*lanes/(l + s0)
    cap = 140.0 * 1 / 7.0
    assert smp["count"][0, 0] == 2 * 20 and smp["count"][1, 0] == 0
    assert smp["count"][0, 0] / (2 * cap) == 1.0
    assert smp["speed_um"][0, 0] == 0


def fuel_rate(v, a):
    pea = 0.79296 * a * a * v if a > 0 else 0.0
    return 0.666 + 0.072 * max(0.0, 0.269 * v + 0.0171 * v ** 2 + 0.000672 * v ** 3 + 1.680 * a * v + pea)


def co_rate(v):
    vm = v / 0.44704
    return -0.064 + 0.0056 * vm + 0.00026 * (vm - 50.0) ** 2


def test_cruising_rates_match_the_printed_equations():
    p = S.default_params()
    o = oracle.Oracle(placed(one_link(30000.0, 15.0), p, [0.0], [0.0]), "f64")
    o.step(1200)  # reach the desired speed
    V0 = o.vehicles()
    o.step(200)
    V1 = o.vehicles()
    v = float(V0["v"][0])
    assert abs(v - 15.0) < 1e-3
    dt = 200 * 0.5
    assert abs((V1["fuel"][0] - V0["fuel"][0]) / dt - fuel_rate(v, 0.0)) < 1e-4
    assert abs((V1["co"][0] - V0["co"][0]) / dt - co_rate(v)) < 1e-4
    # at 15 m/s: 0.666 + 0.072 (4.035 + 3.8475 + 2.268) = 1.39684 mL/s
    assert abs(fuel_rate(15.0, 0.0) - 1.396836) < 1e-6


def test_accelerating_step_uses_realized_acceleration():
    p = S.default_params()
    o = oracle.Oracle(placed(one_link(1000.0, 15.0), p, [0.0], [5.0]), "f64")
    o.step(1)
    V = o.vehicles()
    v1 = float(V["v"][0])
    a = (v1 - 5.0) / 0.5
    assert a > 0.5
    assert abs(V["fuel"][0] - fuel_rate(5.0, a) * 0.5) < 1e-12
    assert abs(V["co"][0] - co_rate(5.0) * 0.5) < 1e-12


def test_hard_braking_is_idle_fuel():
    p = S.default_params()
    # fast vehicle 6 m behind a stopped one: brakes at -b_max
    o = oracle.Oracle(placed(one_link(1000.0, 15.0), p, [0.0, 11.0], [14.0, 0.0]), "f64")
    o.step(1)
    V = o.vehicles()
    k = int(np.argmin(V["x"]))
    assert V["v"][k] < 14.0 - 3.0
    assert abs(V["fuel"][k] - 0.666 * 0.5) < 1e-12


def test_sampler_counts_every_vehicle_on_the_road():
    scen = S.small_grid()
    o = oracle.Oracle(scen, "f32")
    o.set_sampler(every=120, group=6, max_groups=8)
    on_road = 0
    for t in range(3600):
        if t % 120 == 0:
            on_road += o.counters()["en_route"]
        o.step(1)
    smp = o.samples()
    assert smp["count"].sum() == on_road > 0
    es = o.emissions()
    tr = o.trips()
    assert np.all(es["fuel"][tr["arrive_step"] >= 0] > 0)
