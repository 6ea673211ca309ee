#!/usr/bin/env python
"""Benchmark of the traffic microsimulation step on one MI355X.

A "step" is one synchronous simulation step (dt = 0.5 s) of the whole hot
path: leader search, IDM, lane changes, claims, crossings/arrivals/insertions
and the re-sort of the vehicle arrays.  The default workload is the
metro-scale configuration: random planar road graph with 1M nodes and 2.5M
directed links, 4M gravity-model trips with departures over a 3-hour two-peak
mixture, 21,600 steps.  The timed window starts at the step where the
workload carries its most vehicles (``--start-step``, default the workload's
load peak: 1.78M vehicles on the road for metro at step 18,300).  The run is
advanced there untimed (graph replays), or loaded from a state image written
by an earlier run (``--state-file``).  ``--warmup W`` steps then run untimed
from that state (graph capture, caches), the state is put back, and exactly
``--steps K`` steps are timed from the window start (HIP events on the
stream, graph replays, inputs resident in HBM).  The same K steps are then
replayed from the saved state with every kernel launched between its own
start and stop events, for the per-kernel times and the roofline; the FP32
oracle is timed on the host from the same state.

value = vehicle-updates per second over the timed steps (a vehicle-update is
one vehicle on the road advanced by one step).  Prints ONE JSON line on stdout;
progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vehicle-updates/sec at 1 GPU + % HBM roofline; adjoint & ensemble vs plain"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of k_decide: x and v read and written once per
# vehicle-update (16 B), plus one 64-byte record per claim
B_PER_VEH = 16.0
B_PER_EVENT = 64.0


# Step near which each workload carries its most vehicles (measured on one
# MI355X, vehicles on the road every 300 steps (120 for grid10): the first
# step within 1% of the maximum).  metro: 1.78M vehicles at step 18,300
# (maximum 1.79M at 19,500; 777k at 7,200, the peak of the departures);
# grid50: 58k at 13,200; grid10: 214 at 600.
PEAK_STEP = {"metro": 18300, "grid50": 13200, "grid10": 600}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_1807_01148_amd/csrc/common.h", "paper_1807_01148_amd/csrc/step_kernels.h")
TRAFFIC_SUMMARY = "profiles/step_traffic_metro1M.md"
STEP_KERNELS = ("k_decide", "k_resolve", "k_scan", "k_scatter", "k_place", "k_lanes")


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload="metro", start_step=None, launch=None):
    """HBM bytes per launch of every step kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration), as
    {kernel: (fetch, write)}, or None when there is none, the kernel sources
    changed since it was taken, or it was taken on another workload, window
    (its first step) or launch shape (grid, small grid, decide block, decide
    entries per thread)."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_SUMMARY)) as f:
            kv = dict(line.strip()[2:].split(": ", 1) for line in f if line.startswith("- ") and ": " in line)
        if kv.get("kernel_sources_sha256") != kernel_sources_sha():
            return None
        if kv.get("workload") != workload or (start_step is not None and
                                              int(kv.get("window_start_step", -1)) != start_step):
            return None
        if launch is not None and tuple(int(v) for v in kv.get("launch", "").split(",")) != tuple(launch):
            return None
        out = {}
        for k in STEP_KERNELS:
            if k + "_fetch_bytes_per_launch" in kv:
                out[k] = (float(kv[k + "_fetch_bytes_per_launch"]), float(kv[k + "_write_bytes_per_launch"]))
        return out or None
    except (OSError, KeyError, ValueError):
        return None


def workload(name):
    import scenarios as S
    if name == "metro":
        s = S.metro_scenario()
        desc = ("metro1M: random planar road graph (Delaunay-thinned), 1,000,000 nodes, 2,500,000 directed "
                "links, lanes 1-4, speed classes 11/15/20/29 m/s, lognormal lengths (median 120 m); "
                "4,000,000 gravity-model trips over 2,000 zones, 3-hour two-peak departures; "
                "dt 0.5 s, 21,600 steps, FP32 state")
    elif name == "grid50":
        s = S.mid_grid()
        desc = "grid50: 50x50 grid, 1-3 lanes, lognormal lengths, 100,000 trips, 2-hour double peak, 14,400 steps"
    elif name == "grid10":
        s = S.small_grid()
        desc = "grid10: 10x10 grid, 100 m links, 2 lanes, 2,000 trips, 3,600 steps"
    else:
        raise SystemExit("unknown workload " + name)
    return s, desc


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "available_cores": len(os.sched_getaffinity(0))}


def gpu_state_for_oracle(sim):
    """The simulation's dynamic state on the host, in the form the oracle's
    state import takes (vehicles, trip outcomes, emissions, link statistics,
    counters)."""
    return {"veh": sim.vehicles(), "trips": sim.trips(), "emissions": sim.emissions(),
            "edge_stats": sim.edge_stats(), "counters": sim.counters()}


def _time_oracle(scen, state, precision, seconds_budget, max_steps):
    import oracle
    o = oracle.Oracle(scen, precision)
    c = state["counters"]
    o.set_state(c["step"], state["veh"], state["trips"], state["emissions"], state["edge_stats"], c)
    u0 = o.counters()["vehicle_updates"]
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        o.step(1)
        steps += 1
        if time.perf_counter() - t0 > seconds_budget:
            break
    el = time.perf_counter() - t0
    c1 = o.counters()
    del o
    return (c1["vehicle_updates"] - u0) / el, steps, el, c1


def cpu_baseline(scen, state, seconds_budget=20.0):
    """The FP32 oracle from the GPU's own state at the start of the timed
    window (same network, demand and step), stepped for about seconds_budget
    of CPU work: single-threaded, then the all-cores build (the per-vehicle
    decision loop split over OpenMP threads) for the same number of steps,
    whose counters must equal the single-threaded run's."""
    cores = len(os.sched_getaffinity(0))
    v1, steps, el1, c1 = _time_oracle(scen, state, "f32", seconds_budget, 2000)
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    threads = int(os.environ["OMP_NUM_THREADS"])
    vn, _, eln, cn = _time_oracle(scen, state, "f32omp", 1e30, steps)
    c = state["counters"]
    sample = ("FP32 C oracle from the GPU state at step %d (%d vehicles on the road, %d waiting), %d steps: "
              "%.1f s on 1 thread, %.1f s on %d threads" % (c["step"], c["en_route"], c["waiting"], steps, el1, eln,
                                                          threads))
    return {"value": vn, "unit": "vehicle-updates/s", "cores": threads, "kind": "oracle", "sample": sample,
            "single_thread": {"value": v1, "cores": 1}, "threads_agree": c1 == cn, "host": host_cpu()}


def ensemble_scenarios(seed=1811, n=64, steps=3600):
    import scenarios as S
    return S.ensemble_scenarios(seed=seed, n=n, steps=steps)


def ensemble_speedup(args, n=64, log_prefix="[ensemble]"):
    """Batched ensemble (one simulation of all scenarios, graph-captured
    chunks, tuned launch shape) against the per-scenario GPU loops (each
    scenario its own simulation, same steps): once with plain launches and
    once with the same graph-captured chunks; every scenario's link statistics
    and trip outcomes compared bit for bit with its own run."""
    import numpy as np
    import torch
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import ensemble as E
    steps = 3600
    log("%s generating %d scenarios" % (log_prefix, n))
    t = time.perf_counter()
    scens = ensemble_scenarios(n=n, steps=steps)
    log("%s generated in %.1f s, %d trips" % (log_prefix, time.perf_counter() - t,
                                              sum(s["demand"]["depart_step"].size for s in scens)))
    ens = E.Ensemble(scens)
    E.step_graph(ens, 60, args.chunk)
    tune = E.autotune(ens, steps_per_trial=60)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step_graph(ens, steps - 60, args.chunk)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    cb = ens.counters()
    est, etr = ens.edge_stats(), ens.trips()
    log("%s batched: %.3f s, %d vehicle-updates" % (log_prefix, t_batch, cb["vehicle_updates"]))
    loops = {}
    same = True
    for mode in ("plain", "graphs"):
        t_loop, upd_loop = 0.0, 0
        for q, sc in enumerate(scens):
            one = P.Sim(sc)
            if mode == "graphs":
                E.step_graph(one, 60, args.chunk)
            else:
                one.step(60)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "graphs":
                E.step_graph(one, steps - 60, args.chunk)
            else:
                one.step(steps - 60)
            torch.cuda.synchronize()
            t_loop += time.perf_counter() - t0
            upd_loop += one.counters()["vehicle_updates"]
            a, b = ens.scenario_edge_stats(q, est), one.edge_stats()
            same &= all(np.array_equal(a[k], b[k]) for k in b)
            vid = E.vehicle_ids(sc["demand"]["depart_step"])
            ta, tb = ens.scenario_trips(q, etr), one.trips()
            same &= all(np.array_equal(ta[k], tb[k][vid]) for k in tb)
            one.close()
        loops[mode] = (t_loop, upd_loop)
        log("%s per-scenario loop (%s launches): %.3f s" % (log_prefix, mode, t_loop))
    ens.close()
    return {"workload": "%d grid scenarios, side 20-120, 1e4-3e5 trips each, per-scenario IDM, 3,600 steps" % n,
            "launch": tune, "batched_s": t_batch, "plain_loop_s": loops["plain"][0],
            "graph_loop_s": loops["graphs"][0],
            "speedup_over_plain_loop": loops["plain"][0] / t_batch,
            "speedup_over_graph_loop": loops["graphs"][0] / t_batch,
            "batched_vehicle_updates_per_s": cb["vehicle_updates"] / t_batch,
            "plain_loop_vehicle_updates_per_s": loops["plain"][1] / loops["plain"][0],
            "graph_loop_vehicle_updates_per_s": loops["graphs"][1] / loops["graphs"][0],
            "bitwise_identical_per_scenario": bool(same)}


def bench_ensemble(args):
    r = ensemble_speedup(args, n=args.scenarios)
    out = {"metric": "ensemble speed-up over the per-scenario GPU loop (graph-captured launches)",
           "value": r["speedup_over_graph_loop"], "unit": "x", "n_gpus": 1, "steps": 3540, "warmup": 60,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": r["workload"], "launch": r["launch"]}, "detail": r}
    print(json.dumps(out), flush=True)


def adjoint_speedup(seed=1812, log_prefix="[adjoint]"):
    """Gradient of the link travel-time MSE w.r.t. 16 IDM parameters (4 link
    classes, (v0_scale, T, a, b)) on the differentiation workload, three ways:
      * adjoint: one taped forward (checkpoint every 60 steps) + sim_grad;
      * the per-parameter loop at equal accuracy: central differences
        (h = 1e-8, in double) of the frozen-event replay, 32 replays of the
        recorded window plus the forward that records it;
      * the plain per-scenario loop: central differences over 32 plain GPU
        runs (the events move with the parameters).
    Accuracy of each against the FP64 CPU adjoint of the FP32 oracle's tape
    (the oracle's forward is bit-identical to the GPU's), linearized at the
    recorded states and along the FP64-replayed states."""
    import numpy as np
    import torch
    import oracle
    import paper_1807_01148_amd as P
    import scenarios as S
    scen = S.diff_scenario(seed=seed)
    steps = scen["steps"]
    dt = float(np.float32(scen["params"]["dt"]))

    def run(idm, every=0):
        sc = dict(scen)
        sc["params"] = dict(scen["params"])
        sc["params"]["idm"] = np.asarray(idm, np.float32)
        sim = P.Sim(sc)
        if every:
            sim.tape_begin(every)
        sim.step(steps)
        return sim

    hid = run(scen["hidden_idm"])
    tgt, _ = hid.mean_travel_times()
    hid.close()
    theta = scen["params"]["idm"].astype(np.float32)

    def loss_terms(sim):
        tb, cnt = sim.mean_travel_times()
        m = cnt > 0
        return tb, cnt, m, float(((tb - tgt)[m] ** 2).mean())

    # warm-up: every timed path once (first launches; the checkpoints, adjoint
    # buffers and replay buffers taken from the allocator), so that the timed
    # runs measure the work and not first-time allocations
    w = run(theta, every=60)
    wb, _, wm, _ = loss_terms(w)
    w.grad(torch.where(wm, 2.0 * (wb - tgt) / int(wm.sum()), torch.zeros_like(wb)))
    w.close()
    w = run(theta, every=steps)
    w.replay(theta.astype(np.float64), fp64=True)
    w.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = run(theta, every=60)
    tb, cnt, m, L = loss_terms(sim)
    dL = torch.where(m, 2.0 * (tb - tgt) / int(m.sum()), torch.zeros_like(tb))
    g_adj = sim.grad(dL).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    sim.close()
    log("%s adjoint gradient in %.3f s" % (log_prefix, t_adj))

    tgt_np = tgt.double().cpu().numpy()
    # central differences of the frozen-event replay (double, h = 1e-8: far
    # enough below the steps at which a held branch stops making sense on this
    # workload; at 1e-6 some do): the window recorded as one segment, then 32
    # replays
    hr = 1e-8
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = run(theta, every=steps)
    es = rs.edge_stats()
    c0 = np.maximum(es["count"], 1)
    mk = es["count"] > 0
    th0 = theta.astype(np.float64)
    g_rep = np.zeros(theta.shape, np.float64)
    for c in range(theta.shape[0]):
        for j in range(4):
            lv = []
            for sgn in (1.0, -1.0):
                th = th0.copy()
                th[c, j] += sgn * hr
                # the replay's own mean link times: recorded whole steps plus replayed fractions
                tbp = dt * (es["tt_steps"] + rs.replay(th, fp64=True)) / c0
                lv.append(float(((tbp - tgt_np)[mk] ** 2).mean()))
            g_rep[c, j] = (lv[0] - lv[1]) / (2 * hr)
    torch.cuda.synchronize()
    t_rep = time.perf_counter() - t0
    rs.close()
    log("%s frozen-event replay differences in %.3f s" % (log_prefix, t_rep))
    h = 1e-3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_free = np.zeros(theta.shape, np.float64)
    for c in range(theta.shape[0]):
        for j in range(4):
            a, b = theta.astype(np.float64).copy(), theta.astype(np.float64).copy()
            a[c, j] += h
            b[c, j] -= h
            sa, sb = run(a), run(b)
            g_free[c, j] = (loss_terms(sa)[3] - loss_terms(sb)[3]) / (2 * h)
            sa.close()
            sb.close()
    torch.cuda.synchronize()
    t_free = time.perf_counter() - t0
    log("%s plain-run central differences in %.3f s; FP64 CPU references" % (log_prefix, t_free))
    o = oracle.Oracle(scen, "f32", tape=True)
    o.step(steps)
    mask = o.edge_stats()["count"] > 0
    th64 = theta.astype(np.float64)
    _, g_c, _, _, _ = oracle.replay(o.tape(), scen, th64, tgt_np, mask, at_tape_states=True)
    _, g_r, _, _, _ = oracle.replay(o.tape(), scen, th64, tgt_np, mask, at_tape_states=False)
    del o

    def err(g, ref):
        return float(np.abs(g - ref).max() / np.abs(ref).max())

    acc = {k: {"vs_fp64_at_recorded_states": err(v, g_c), "vs_fp64_replayed_states": err(v, g_r)}
           for k, v in (("adjoint", g_adj), ("replay_fd", g_rep), ("plain_runs_fd", g_free))}
    return {"workload": "50x50 grid, 100,000 trips, 1,800 steps, 4 link classes x (v0_scale, T, a, b)",
            "parameters": int(theta.size), "replay_fd_step": hr, "plain_fd_step": h, "checkpoint_every": 60,
            "loss": L, "adjoint_s": t_adj, "replay_fd_s": t_rep, "plain_runs_fd_s": t_free, "accuracy": acc}


def bench_adjoint(args):
    """The adjoint against the per-parameter loops (see adjoint_speedup)."""
    r = adjoint_speedup()
    out = {"metric": "adjoint gradient speed-up over the per-parameter GPU loop at equal accuracy",
           "value": r["replay_fd_s"] / r["adjoint_s"], "unit": "x", "n_gpus": 1, "steps": 1800,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": r["workload"], "checkpoint_every": 60},
           "speedup_over_plain_runs_fd": r["plain_runs_fd_s"] / r["adjoint_s"], "detail": r}
    print(json.dumps(out), flush=True)


# algorithmic bytes per relaxed link of the route search: its weight (8 B),
# its head node (4 B) and the 8-byte label it lowers
B_PER_RELAX = 20.0


def bench_reroute(args):
    """Iterative decaying re-routing (Sec. 6.3.1) on the workload: four
    iterations of (plan routes on the GPU, hand them to the simulation on
    the device, simulate the whole horizon, measured link times become the
    weights), re-planning all, all, half and a quarter of the trips; the
    hand-off through the host (routes read out, a new simulation loaded) is
    timed once beside it.  Reports the route search rate (relaxed links per
    second) of the full plan, per-iteration times and the mean trip time;
    the CPU baseline is the oracle's Dijkstra on a sample of origins."""
    import numpy as np
    import torch
    import oracle.routing as OR
    import paper_1807_01148_amd as P
    import scenarios as S
    from paper_1807_01148_amd.route import Router, with_routes
    log("[reroute] generating workload", args.workload)
    scen, desc = workload(args.workload)
    d = scen["demand"]
    n = int(d["depart_step"].size)
    masks = S.reroute_masks(1813, n)
    rt = Router(scen["net"])
    rt.set_trips(d["src_nodes"], d["trip_src"], d["trip_dst"])
    sim = P.Sim(scen)  # loaded once; every iteration replaces its routes on the device
    its = []
    host_handoff = None
    for k in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        total = rt.plan(None if k == 0 else masks[k])
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        relax, nsrc = rt.last_work()
        if k == 0:
            # for comparison, once: the routes read out and a new simulation loaded with them
            t0 = time.perf_counter()
            ptr, edges = rt.routes()
            t_read = time.perf_counter() - t0
            t0 = time.perf_counter()
            other = P.Sim(with_routes(scen, ptr, edges))
            torch.cuda.synchronize()
            host_handoff = {"read_routes_s": t_read, "load_s": time.perf_counter() - t0}
            other.close()
            del ptr, edges, other
        t0 = time.perf_counter()
        sim.reload_routes(*rt.route_views())
        torch.cuda.synchronize()
        t_load = time.perf_counter() - t0
        t0 = time.perf_counter()
        sim.step(scen["steps"])
        torch.cuda.synchronize()
        t_sim = time.perf_counter() - t0
        st = sim.edge_stats_device()
        rt.weights_from_stats(st["count"], st["tt_us"])
        tr = sim.trips()
        done = tr["arrive_step"] >= 0
        c = sim.counters()
        its.append({"replanned": int(n if k == 0 else masks[k].sum()), "origins": nsrc, "plan_s": t_plan,
                    "relaxations": relax, "route_edges": total, "load_s": t_load, "sim_s": t_sim,
                    "arrived": int(done.sum()),
                    "mean_trip_s": float((tr["arrive_step"][done] - tr["depart_actual"][done]).mean() *
                                         scen["params"]["dt"]) if done.any() else None,
                    "vehicle_updates": c["vehicle_updates"]})
        log("[reroute] iteration %d: %s" % (k, its[-1]))
    sim.close()
    # trees/s: shortest-path trees (one per origin zone) of the full plan per second
    rate = its[0]["origins"] / its[0]["plan_s"]
    # CPU baseline: the oracle's Dijkstra from a sample of origins, scaled
    w0 = OR.initial_weights(scen["net"])
    sample = d["src_nodes"][:: max(1, d["src_nodes"].size // 3)][:3]
    t0 = time.perf_counter()
    for s0 in sample:
        OR.sssp(scen["net"], w0, int(s0))
    t_cpu = (time.perf_counter() - t0) / len(sample)
    ne = int(scen["net"]["col_idx"].size)
    out = {"metric": "re-routing (Sec. 6.3.1): shortest-path trees/s of a full plan, 4 decaying iterations",
           "value": rate, "unit": "trees/s", "n_gpus": 1, "higher_is_better": True, "dtype": "int64",
           "data": "synthetic", "config": {"workload": desc, "iterations": 4, "replan_shares": [1, 1, 0.5, 0.25]},
           "full_plan_s": its[0]["plan_s"], "work_ratio": its[0]["relaxations"] / (its[0]["origins"] * ne),
           "relaxations_per_s": its[0]["relaxations"] / its[0]["plan_s"],
           "roofline": {"bound": "hbm", "achieved": rate * ne * B_PER_RELAX / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": rate * ne * B_PER_RELAX / 1e9 / HBM_PEAK_GBS, "traffic": None},
           "cpu_baseline": {"value": 1.0 / t_cpu, "unit": "trees/s", "cores": 1, "kind": "oracle",
                            "sample": "binary-heap Dijkstra (int64) from %d origins of the workload, each "
                                      "relaxing every link once" % len(sample), "host": host_cpu()},
           "iterations": its, "handoff": "device (sim_reload_routes; load_s of each iteration)",
           "host_handoff_once": host_handoff}
    print(json.dumps(out), flush=True)


def copy_ceiling(nbytes=1 << 29, reps=5):
    """Device-to-device copy bandwidth on this GPU (read + write bytes per
    second, GB/s), the practical ceiling for a streaming kernel."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def copy_calibration(args):
    """A plain device-to-device copy of 1 GiB, five times: the reference
    dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters (each copy
    reads and writes exactly 1 GiB)."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": 4 * n, "dispatches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1200)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--workload", default="metro", choices=["metro", "grid50", "grid10"])
    ap.add_argument("--start-step", type=int, default=-1,
                    help="step at which the warm-up and then the timed window start (default: the workload's "
                         "load peak)")
    ap.add_argument("--state-file", default="",
                    help="state image at the window start: loaded if it exists (instead of the approach), else "
                         "written after the approach")
    ap.add_argument("--no-kernel-timing", dest="kernel_timing", action="store_false",
                    help="skip the per-kernel replay of the timed window")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-training-patterns", dest="training_patterns", action="store_false",
                    help="skip the adjoint and ensemble speed-ups that follow the plain-step measurement")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--chunk", type=int, default=60, help="steps per captured HIP graph")
    ap.add_argument("--launch", default="",
                    help="launch shape GRID,SMALL_GRID,DECIDE_BLOCK,DECIDE_PER_THREAD instead of the tuned one")
    ap.add_argument("--tune-at", type=int, default=0,
                    help="simulate to this step, autotune the launch shape there, store it in the cache, exit")
    ap.add_argument("--mode", default="plain", choices=["plain", "ensemble", "adjoint", "reroute", "copycal"],
                    help="plain: the metric; ensemble / adjoint: speed-up of the batched and adjoint forms "
                         "over the plain per-scenario GPU loop")
    ap.add_argument("--scenarios", type=int, default=64)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import ensemble as E
    if args.mode == "ensemble":
        return bench_ensemble(args)
    if args.mode == "adjoint":
        return bench_adjoint(args)
    if args.mode == "reroute":
        return bench_reroute(args)
    if args.mode == "copycal":
        return copy_calibration(args)

    log("[bench] generating workload", args.workload)
    t = time.perf_counter()
    scen, desc = workload(args.workload)
    log("[bench] generated in %.1f s" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    t = time.perf_counter()
    sim = P.Sim(scen, device=0, stream=stream)
    log("[bench] loaded in %.1f s" % (time.perf_counter() - t))
    cache = os.path.join(ROOT, "paper_1807_01148_amd", "autotune_cache.json")
    if args.tune_at > 0:
        E.step_graph(sim, args.tune_at, args.chunk)
        torch.cuda.synchronize()
        res = E.autotune(sim, steps_per_trial=60)
        res.update({"workload": args.workload, "step": args.tune_at, "device": E.device_key(0)})
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
        db["%s|%s" % (res["device"], args.workload)] = {"grid": res["grid"], "grid_small": res["grid_small"],
                                                         "decide_block": res["decide_block"],
                                                         "decide_per_thread": res["decide_per_thread"],
                                                         "ms_per_step": res["ms_per_step"], "step": args.tune_at}
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        print(json.dumps(res), flush=True)
        return
    shape = "default"
    if args.launch:
        g, gs, db, dr = (int(v) for v in args.launch.split(","))
        E.apply_shape(sim, {"grid": g, "grid_small": gs, "decide_block": db, "decide_per_thread": dr})
        shape = "given"
    else:
        try:
            with open(cache) as f:
                hit = json.load(f).get("%s|%s" % (E.device_key(0), args.workload))
            if hit:
                E.apply_shape(sim, hit)
                shape = "autotuned"
        except (OSError, ValueError):
            pass
    launch = E.get_launch(sim) + E.get_decide_shape(sim)
    log("[bench] launch shape %s: grid %d, small grid %d, decide blocks of %d x %d entries"
        % (shape, launch[0], launch[1], launch[2], launch[3]))

    # the timed window sits at the load the workload is quoted on: the run is
    # advanced there untimed (graph replays), or its state there is loaded
    start = PEAK_STEP[args.workload] if args.start_step < 0 else args.start_step
    approach = None
    meta = {"workload": args.workload, "step": start}
    if args.state_file and os.path.exists(args.state_file) and os.path.exists(args.state_file + ".json"):
        with open(args.state_file + ".json") as f:
            got = json.load(f)
        if got != meta:
            raise SystemExit("state file %s holds %s, not %s" % (args.state_file, got, meta))
        import numpy as np
        sim.load_state(torch.from_numpy(np.fromfile(args.state_file, dtype=np.uint8)).to(dev))
        log("[bench] state at step %d loaded from %s" % (start, args.state_file))
    else:
        evp0, evp1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        evp0.record(stream)
        E.step_graph(sim, start, args.chunk)
        evp1.record(stream)
        torch.cuda.synchronize()
        # the untimed approach, reported beside the window: all steps from the
        # start of the run (ramp-up included; graph captures happen on the host)
        ca = sim.counters()
        approach = {"steps": ca["step"], "vehicle_updates": ca["vehicle_updates"],
                    "seconds": evp0.elapsed_time(evp1) / 1000.0}
        approach["value"] = approach["vehicle_updates"] / approach["seconds"] if approach["seconds"] > 0 else None
    img = sim.save_state()  # the window's start: warm-up, timed window and per-kernel replay all begin here
    if args.state_file and approach is not None:
        img.cpu().numpy().tofile(args.state_file)
        with open(args.state_file + ".json", "w") as f:
            json.dump(meta, f)
        log("[bench] state at step %d saved to %s" % (start, args.state_file))
    if args.warmup > 0:
        E.step_graph(sim, args.warmup, args.chunk)
        sim.load_state(img)
    # the window replays graphs of `wchunk` steps (a shorter window is one
    # graph): capture them here, untimed (two chunks, for both step parities),
    # then start again from the window
    wchunk = max(1, min(args.chunk, args.steps))
    if wchunk >= 2:
        E.step_graph(sim, 2 * wchunk, wchunk)
        sim.load_state(img)
    torch.cuda.synchronize()
    c0 = sim.counters()
    log("[bench] at step %d: en_route %d waiting %d" % (c0["step"], c0["en_route"], c0["waiting"]))
    host_state = None if args.no_cpu_baseline else gpu_state_for_oracle(sim)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    chunk = 1800
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        E.step_graph(sim, n, wchunk)
        done += n
        if done < args.steps:
            log("[bench] enqueued %d / %d steps" % (done, args.steps))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    c1 = sim.counters()
    upd = c1["vehicle_updates"] - c0["vehicle_updates"]
    claims = c1["claims"] - c0["claims"]
    lc_claims = c1["claims_lane_change"] - c0["claims_lane_change"]
    claims_cross = claims - (c1["claims_departure"] - c0["claims_departure"]) - lc_claims
    secs = ev_ms / 1000.0
    value = upd / secs if secs > 0 else 0.0
    log("[bench] %d steps in %.4f s (wall %.4f s), %d vehicle-updates, final en_route %d arrived %d"
        % (args.steps, secs, wall, upd, c1["en_route"], c1["arrived"]))

    # the same window again from its saved start, every step's kernels
    # launched with their own start and stop events (outside the graphs); the
    # replay must reach the same counters
    samples, avg, replay_same = 0, {}, None
    if args.steps > 0 and args.kernel_timing:
        sim.load_state(img)
        sim.set_timing(1)
        E.step_graph(sim, args.steps, args.chunk)
        kms, samples = sim.read_timing()
        sim.set_timing(0)
        replay_same = sim.counters() == c1
        avg = {k: v / samples for k, v in kms.items()} if samples else {}
        log("[bench] per-kernel replay: %d sampled steps, identical counters %s" % (samples, replay_same))
    del img

    roofline = None
    traffic = measured_traffic(args.workload, c0["step"], launch) if samples else None
    if samples:
        dom = max(avg, key=avg.get)
        per_launch_units = upd / args.steps
        # k_decide advances the vehicles and issues every claim of the step
        # (crossings, lane changes, departures)
        per_launch_claims = claims / args.steps
        alg_bytes = B_PER_VEH * per_launch_units + B_PER_EVENT * per_launch_claims
        achieved = alg_bytes / (avg[dom] * 1e-3) / 1e9
        tb = sum(traffic[dom]) if traffic and dom in traffic else None
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                    "avg_launch_us": avg[dom] * 1e3, "alg_bytes_per_launch": alg_bytes,
                    "sampled_steps": samples}
        if tb:
            # the measured HBM bytes over the same launch time, and their ratio to the algorithmic bytes
            roofline["traffic_gbs"] = tb / (avg[dom] * 1e-3) / 1e9
            roofline["traffic_frac"] = roofline["traffic_gbs"] / HBM_PEAK_GBS
            roofline["amplification"] = tb / alg_bytes
        roofline["copy_ceiling_gbs"] = copy_ceiling()
    step_traffic = None
    if traffic and samples and all(k in traffic for k in STEP_KERNELS):
        # every kernel's measured bytes per launch, over the step: bytes per
        # vehicle-update and their ratio to the method's algorithmic bytes
        tot = sum(sum(traffic[k]) for k in STEP_KERNELS)
        per_upd = tot / (upd / args.steps)
        alg_step = (B_PER_VEH * upd + B_PER_EVENT * claims) / args.steps
        step_traffic = {"bytes_per_step": tot, "bytes_per_vehicle_update": per_upd,
                        "alg_bytes_per_step": alg_step, "amplification": tot / alg_step,
                        "per_kernel_bytes": {k: sum(traffic[k]) for k in STEP_KERNELS},
                        "per_kernel_gbs": {k: sum(traffic[k]) / (avg[k] * 1e-3) / 1e9 for k in STEP_KERNELS
                                           if avg.get(k)}}
    step_achieved = (B_PER_VEH * upd + B_PER_EVENT * claims) / secs / 1e9 if secs > 0 else 0.0
    out = {
        "metric": METRIC, "value": value, "unit": "vehicle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ev_ms / args.steps if args.steps else 0.0,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "start_step": start, "simulated_steps": [c0["step"], c1["step"]],
                   "en_route_start": c0["en_route"], "waiting_start": c0["waiting"],
                   "vehicle_updates": upd, "claims": claims, "claims_crossing": claims_cross,
                   "claims_lane_change": lc_claims,
                   "lc_evaluated": c1["lc_evaluated"] - c0["lc_evaluated"], "en_route_end": c1["en_route"],
                   "arrived_end": c1["arrived"], "parallelism": "single GPU"},
        "roofline": roofline,
        "step_roofline": {"bound": "hbm", "achieved": step_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": step_achieved / HBM_PEAK_GBS},
        "step_traffic": step_traffic,
        "kernel_avg_us": {k: v * 1e3 for k, v in avg.items()} or None,
        "kernel_replay_identical": replay_same,
        "run_to_window": approach,
        "launch": {"grid": launch[0], "grid_small": launch[1], "decide_block": launch[2],
                   "decide_per_thread": launch[3], "shape": shape, "graph_chunk": wchunk},
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    out["cpu_baseline"] = None
    if host_state is not None:
        log("[bench] timing the CPU oracle baseline on the same state")
        out["cpu_baseline"] = cpu_baseline(scen, host_state, args.cpu_seconds)
    del scen, host_state
    # the metric's second half: the adjoint and the batched ensemble against
    # the plain per-scenario GPU loops, each with its accuracy
    if args.training_patterns:
        r = adjoint_speedup()
        acc = r["accuracy"]
        out["adjoint"] = {
            "speedup_at_equal_accuracy": r["replay_fd_s"] / r["adjoint_s"],
            "equal_accuracy_loop": "the recording forward + 32 frozen-event replays (double), central "
                                   "differences h = 1e-8",
            "speedup_over_plain_runs_fd": r["plain_runs_fd_s"] / r["adjoint_s"],
            "adjoint_s": r["adjoint_s"], "replay_fd_s": r["replay_fd_s"], "plain_runs_fd_s": r["plain_runs_fd_s"],
            "accuracy": acc, "workload": r["workload"]}
        e = ensemble_speedup(args, n=args.scenarios)
        out["ensemble"] = {"speedup_over_graph_loop": e["speedup_over_graph_loop"],
                           "speedup_over_plain_loop": e["speedup_over_plain_loop"],
                           "bitwise_identical_per_scenario": e["bitwise_identical_per_scenario"],
                           "batched_s": e["batched_s"], "graph_loop_s": e["graph_loop_s"],
                           "plain_loop_s": e["plain_loop_s"], "workload": e["workload"], "launch": e["launch"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
