#!/usr/bin/env python
"""Benchmark of the traffic microsimulation step on one MI355X.

A "step" is one synchronous simulation step (dt = 0.5 s) of the whole hot
path: leader search, IDM, lane changes, claims, crossings/arrivals/insertions
and the re-sort of the vehicle arrays.  The default workload is the
metro-scale configuration: random planar road graph with 1M nodes and 2.5M
directed links, 4M gravity-model trips with departures over a 3-hour two-peak
mixture, 21,600 steps.  ``--warmup W`` steps run untimed first (they advance
the simulation), then exactly ``--steps K`` steps are timed with the inputs
already resident in HBM.

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
# algorithmic bytes (per unit): x and v read and written once
# per vehicle-update, plus one 64-byte record per event (claim)
B_PER_VEH = 16.0
B_PER_EVENT = 64.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def cpu_baseline(seconds_budget=20.0):
    """The FP32 oracle, single-threaded, on a bounded sample of the metro
    workload: the metro network with a synthetic ~1M-vehicle snapshot
    (mid-simulation density), stepped until ~seconds_budget of CPU work."""
    import oracle
    import scenarios as S
    net = S.metro()
    net.pop("xy", None)
    scen = S.placed_snapshot(net, 1_000_000, seed=11)
    o = oracle.Oracle(scen, "f32")
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_budget or steps >= 200:
            break
    upd = o.counters()["vehicle_updates"]
    return {"value": upd / el, "unit": "vehicle-updates/s", "cores": 1, "kind": "oracle",
            "sample": "FP32 C oracle, 1 thread, metro network (1M nodes / 2.5M links) with a synthetic "
                      "snapshot of %d placed vehicles, %d steps, %.1f s" % (scen["demand"]["init_x"].size, steps, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=21540)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--workload", default="metro", choices=["metro", "grid50", "grid10"])
    ap.add_argument("--timing-every", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--chunk", type=int, default=60, help="steps per captured HIP graph")
    ap.add_argument("--tune-at", type=int, default=0,
                    help="simulate to this step, autotune the launch shape there, store it in the cache, exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_01148_amd as P
    from paper_1807_01148_amd import ensemble as E

    log("[bench] generating workload", args.workload)
    t = time.perf_counter()
    scen, desc = workload(args.workload)
    log("[bench] generated in %.1f s" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    t = time.perf_counter()
    sim = P.Sim(scen, device=0, stream=stream)
    del scen["demand"]
    log("[bench] loaded in %.1f s" % (time.perf_counter() - t))
    cache = os.path.join(ROOT, "paper_1807_01148_amd", "autotune_cache.json")
    if args.tune_at > 0:
        E.step_graph(sim, args.tune_at, args.chunk)
        torch.cuda.synchronize()
        res = E.autotune(sim, steps_per_trial=60)
        res.update({"workload": args.workload, "step": args.tune_at, "device": torch.cuda.get_device_name(0)})
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
        db["%s|%s" % (res["device"], args.workload)] = {"grid": res["grid"], "grid_small": res["grid_small"],
                                                         "ms_per_step": res["ms_per_step"], "step": args.tune_at}
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        print(json.dumps(res), flush=True)
        return
    shape = "default"
    try:
        with open(cache) as f:
            hit = json.load(f).get("%s|%s" % (torch.cuda.get_device_name(0), args.workload))
        if hit:
            E.set_launch(sim, hit["grid"], hit["grid_small"])
            shape = "autotuned"
    except (OSError, ValueError):
        pass
    launch = E.get_launch(sim)
    log("[bench] launch shape %s: grid %d, small grid %d" % (shape, launch[0], launch[1]))

    E.step_graph(sim, args.warmup, args.chunk)
    torch.cuda.synchronize()
    c0 = sim.counters()
    log("[bench] warmup done: step %d en_route %d" % (c0["step"], c0["en_route"]))
    sim.set_timing(args.timing_every)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    chunk = 1800
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        E.step_graph(sim, n, args.chunk)
        done += n
        if done < args.steps:
            log("[bench] enqueued %d / %d steps" % (done, args.steps))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    c1 = sim.counters()
    kms, samples = sim.read_timing()
    sim.set_timing(0)
    upd = c1["vehicle_updates"] - c0["vehicle_updates"]
    claims = c1["claims"] - c0["claims"]
    secs = ev_ms / 1000.0
    value = upd / secs
    log("[bench] %d steps in %.3f s (wall %.3f s), %d vehicle-updates, final en_route %d arrived %d"
        % (args.steps, secs, wall, upd, c1["en_route"], c1["arrived"]))

    avg = {k: (v / samples if samples else 0.0) for k, v in kms.items()}
    dom = max(avg, key=avg.get)
    per_launch_units = upd / args.steps
    per_launch_claims = claims / args.steps
    alg_bytes = B_PER_VEH * per_launch_units + B_PER_EVENT * per_launch_claims
    achieved = alg_bytes / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    step_achieved = (B_PER_VEH * upd + B_PER_EVENT * claims) / secs / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_us": avg[dom] * 1e3, "alg_bytes_per_launch": alg_bytes,
                "sampled_steps": samples}
    out = {
        "metric": METRIC, "value": value, "unit": "vehicle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ev_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "simulated_steps": [c0["step"], c1["step"]],
                   "vehicle_updates": upd, "claims": claims, "en_route_end": c1["en_route"],
                   "arrived_end": c1["arrived"], "parallelism": "single GPU"},
        "roofline": roofline,
        "step_roofline": {"bound": "hbm", "achieved": step_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": step_achieved / HBM_PEAK_GBS},
        "kernel_avg_us": {k: v * 1e3 for k, v in avg.items()},
        "launch": {"grid": launch[0], "grid_small": launch[1], "shape": shape, "graph_chunk": args.chunk},
    }
    sim.close()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
