"""FP32 against FP64 from one identical state: the check shared by the GPU
parity tests (the HIP library's state) and the oracle's own pins (the FP32
oracle's state).  The state is handed to the FP64 oracle through its state
import; every vehicle whose discrete outcome (link, lane, route cursor) after
one step differs is listed and must be explained by FP32 rounding."""
import numpy as np

import oracle


def gpu_state(g):
    """A simulation's state on the host (the HIP library's or an oracle's), as
    the oracle's state import takes it."""
    return {"veh": g.vehicles(), "trips": g.trips(), "emissions": g.emissions(), "edge_stats": g.edge_stats(),
            "counters": g.counters()}


def oracle_at(scen, st, prec="f64", nudge=None):
    """An oracle continuing from state st; nudge = (vid, "x" or "v", k) moves
    that vehicle's position or speed by k float32 ulps first."""
    veh = st["veh"]
    if nudge is not None:
        vid, field, k = nudge
        veh = dict(veh)
        a = veh[field].astype(np.float32).copy()
        i = int(np.flatnonzero(veh["vid"] == vid)[0])
        for _ in range(abs(k)):
            a[i] = np.nextafter(a[i], np.float32(np.inf if k > 0 else -np.inf))
        veh[field] = a
    o = oracle.Oracle(scen, prec)
    c = st["counters"]
    o.set_state(c["step"], veh, st["trips"], st["emissions"], st["edge_stats"], c)
    return o


def _outcome(o):
    V = o.vehicles()
    return {int(v): (int(e), int(l), int(c)) for v, e, l, c in zip(V["vid"], V["edge"], V["lane"], V["cursor"])}


def explain_by_rounding(scen, st, gpu_out, bad, max_ulp=8):
    """For every vehicle whose discrete outcome differs between the GPU (FP32)
    and the FP64 oracle from the same state st, find an input perturbation of
    FP32-rounding size that turns the FP64 oracle's outcome for it into the
    GPU's: the position or the speed of that vehicle, or of another
    mismatching one (one decision can cost another its claim), moved by at
    most max_ulp float32 ulps.  Returns the vehicles left unexplained (their
    FP64 decision margin is not within FP32 rounding)."""
    left = []
    for vid in bad:
        found = False
        for who in [vid] + [w for w in bad if w != vid]:
            for field in ("x", "v"):
                for k in (1, -1, 2, -2, 4, -4, max_ulp, -max_ulp):
                    o = oracle_at(scen, st, "f64", (who, field, k))
                    o.step(1)
                    if _outcome(o).get(vid) == gpu_out.get(vid):
                        found = True
                        break
                if found:
                    break
            if found:
                break
        if not found:
            left.append(vid)
    return left


def one_step_vs_fp64(scen, g, tag):
    """One step of the GPU and of the FP64 oracle from the GPU's current
    state: mismatching discrete outcomes listed and each explained by FP32
    rounding; positions and speeds of the others within 1e-5."""
    st = gpu_state(g)
    o = oracle_at(scen, st, "f64")
    g.step(1)
    o.step(1)
    G, O = g.vehicles(), o.vehicles()
    assert np.array_equal(G["vid"], O["vid"]), tag
    disc = np.ones(G["vid"].size, bool)
    for k in ("edge", "lane", "cursor"):
        disc &= G[k] == O[k]
    bad = [int(v) for v in G["vid"][~disc]]
    print("%s: %d discrete mismatches of %d vehicles: vids %s" % (tag, len(bad), disc.size, bad))
    left = explain_by_rounding(scen, st, _outcome(g), bad)
    assert not left, ("mismatches not within FP32 rounding", tag, left)
    L = scen["net"]["length"][G["edge"]].astype(np.float64)
    x64, v64 = O["x"].astype(np.float64), O["v"].astype(np.float64)
    ex = np.abs(G["x"].astype(np.float64) - x64) / np.maximum(np.abs(x64), L)
    ev = np.abs(G["v"].astype(np.float64) - v64) / np.maximum(np.abs(v64), 1.0)
    assert ex[disc].max() <= 1e-5 and ev[disc].max() <= 1e-5, (tag, ex[disc].max(), ev[disc].max())
    return len(bad), disc.size


def link_time_gap(eg, eo, min_count=20):
    """Traversal-weighted mean |T_e - T64_e| / T64_e over links with at least
    min_count traversals (in the FP64 run), and the relative gap of the
    network-wide mean travel time; eg, eo = link statistics of the run under
    test and of the FP64 oracle."""
    m = eo["count"] >= min_count
    tg = eg["tt_us"][m] / np.maximum(eg["count"][m], 1)
    to = eo["tt_us"][m] / eo["count"][m]
    weighted = np.sum(np.abs(tg - to) * eo["count"][m]) / np.sum(to * eo["count"][m])
    mean_g = eg["tt_us"].sum() / eg["count"].sum()
    mean_o = eo["tt_us"].sum() / eo["count"].sum()
    return float(weighted), float(abs(mean_g - mean_o) / mean_o), int(m.sum())
