"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code; no GPU involved) runs in a child process without a report:
the FP32 and FP64 step on the 10x10 grid with lane changes, lost claims and
arrivals, on a controlled grid (stop signs and signals), with trucks, and
with its tape; the FP64 adjoint of that tape; the route oracle's plans.  A
sanitizer finding ends the child with a non-zero status and its report."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

CHILD = r'''
import numpy as np
import oracle
import scenarios as S
from oracle import routing as R

scen = S.small_grid(n_trips=2000, steps=1200)
for prec in ("f32", "f64"):
    o = oracle.Oracle(scen, prec, tape=(prec == "f32"))
    o.step(1200)
    c = o.counters()
    assert c["claims_lost"] > 0 and c["arrived"] > 0, c
    if prec == "f32":
        tape = o.tape()
        mask = o.edge_stats()["count"] > 0
        th = scen["params"]["idm"].astype(np.float64)
        tgt = np.zeros(mask.size)
        oracle.replay(tape, scen, th, tgt, mask, at_tape_states=False)
    del o
ctl = S.small_grid(n_trips=2000, steps=1200)
ctl["net"]["node_control"] = S.random_control(ctl["net"], 7, 0.4, 0.4)
ctl["params"]["signal_green"] = 6
ctl["params"]["vehicle_types"] = np.array([(5.0, np.inf, np.inf), (12.0, 0.8, 12.0)], np.float32)
ctl["demand"]["trip_type"] = (np.random.default_rng(3).random(2000) < 0.3).astype(np.uint8)
o = oracle.Oracle(ctl, "f32")
o.step(1200)
assert o.counters()["arrived"] > 0
del o
d = scen["demand"]
net = scen["net"]
w = R.initial_weights(net)
R.plan(net, w, d["src_nodes"], d["trip_src"], d["trip_dst"])
print("sanitized oracle ran clean")
'''


def test_oracle_runs_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    asan = subprocess.check_output([gcc, "-print-file-name=libasan.so"]).decode().strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan")
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC"]
    libs = {}
    for key, src, defs in (("F32", "oracle.c", []), ("F64", "oracle.c", ["-DORACLE_F64"]),
                           ("ADJ", "adjoint.c", []), ("ROUTE", "routing.c", [])):
        out = str(tmp_path / ("lib_%s.so" % key.lower()))
        subprocess.check_call([gcc] + san + defs + ["-o", out, os.path.join(ORACLE, src), "-lm"])
        libs["ORACLE_LIB_" + key] = out
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", PYTHONPATH=ROOT, **libs)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "sanitized oracle ran clean" in r.stdout
