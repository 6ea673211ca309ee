"""Host logic of the benchmark that needs no GPU: the measured HBM traffic is
reported only for the kernel sources it was measured on, and the multi-GPU
request is refused with a message."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_summary(path, sha, fetch="1000", write="24", workload="metro", start=18300):
    with open(path, "w") as f:
        f.write("# summary\n\ntext: not a field\n\n")
        f.write("- kernel_sources_sha256: %s\n- workload: %s\n- window_start_step: %d\n- launch: 1024,256,256,2\n"
                % (sha, workload, start))
        for i, k in enumerate(bench.STEP_KERNELS):
            f.write("- %s_fetch_bytes_per_launch: %s\n- %s_write_bytes_per_launch: %s\n" % (k, fetch, k, i))
        f.write("- k_decide_write_bytes_per_launch: %s\n" % write)


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the sources the summary is checked against, copied so the test can edit them
    for rel in bench.KERNEL_SOURCES:
        os.makedirs(os.path.dirname(tmp_path / rel), exist_ok=True)
        with open(os.path.join(ROOT, rel), "rb") as src, open(tmp_path / rel, "wb") as dst:
            dst.write(src.read())
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", "summary.md")
    sha = bench.kernel_sources_sha()
    assert len(sha) == 64

    write_summary(tmp_path / "summary.md", sha)
    tr = bench.measured_traffic()
    assert sorted(tr) == sorted(bench.STEP_KERNELS)
    assert tr["k_decide"] == (1000.0, 24.0) and tr["k_lanes"] == (1000.0, float(bench.STEP_KERNELS.index("k_lanes")))
    assert bench.measured_traffic("metro", 18300) == tr
    assert bench.measured_traffic("metro", 18300, (1024, 256, 256, 2)) == tr
    # counters taken with another launch shape do not describe this one
    assert bench.measured_traffic("metro", 18300, (2048, 512, 256, 1)) is None
    # counters of another window or workload do not describe this one
    assert bench.measured_traffic("metro", 7205) is None
    assert bench.measured_traffic("grid50", 18300) is None

    # a changed kernel source: the counters no longer describe it
    with open(tmp_path / bench.KERNEL_SOURCES[-1], "ab") as f:
        f.write(b"\n// edited\n")
    assert bench.kernel_sources_sha() != sha
    assert bench.measured_traffic() is None

    # no summary, or a malformed one
    write_summary(tmp_path / "summary.md", bench.kernel_sources_sha(), fetch="n/a")
    assert bench.measured_traffic() is None
    os.remove(tmp_path / "summary.md")
    assert bench.measured_traffic() is None


def test_committed_summary_parses():
    with open(os.path.join(ROOT, bench.TRAFFIC_SUMMARY)) as f:
        kv = dict(line.strip()[2:].split(": ", 1) for line in f if line.startswith("- ") and ": " in line)
    assert len(kv["kernel_sources_sha256"]) == 64
    for k in bench.STEP_KERNELS:
        assert float(kv[k + "_fetch_bytes_per_launch"]) > 0 and float(kv[k + "_write_bytes_per_launch"]) > 0
    assert kv["workload"] in ("metro", "grid50", "grid10") and int(kv["window_start_step"]) >= 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
