"""The benchmark's command-line contract, on the CPU: one GPU only (any other
--gpus exits with a message and status 2 before touching a device), the
workloads it offers, and the stored counter records it reads for the
roofline's traffic entry."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in ("2", "8"):
        r = run("--gpus", n)
        assert r.returncode == 2, r.stderr
        assert "one GPU" in r.stderr
        assert r.stdout.strip() == ""


def test_every_workload_is_offered():
    r = run("--help")
    assert r.returncode == 0
    for w in ("plain", "batched", "mixed", "serve", "levels", "small", "host", "mfma"):
        assert w in r.stdout


def test_stored_traffic_records_have_what_the_bench_reads():
    with open(os.path.join(ROOT, "profiles", "schur_f64_n8192_b512_traffic.json")) as f:
        t = json.load(f)
    assert len(t["kernel_sha256_16"]) == 16
    # HBM bytes per trailing-update launch: at least the algorithmic bytes
    assert t["bytes_per_launch"] >= t["algorithmic_bytes_per_launch"] > 0
    with open(os.path.join(ROOT, "profiles", "batched_swept_step_traffic.json")) as f:
        b = json.load(f)
    assert len(b["sources_sha256_16"]) == 16
    assert b["bytes_per_launch"] >= b["algorithmic_bytes_per_step"] > 0
    assert b["bytes_per_batch"] == b["bytes_per_launch"] * b["steps_per_batch"] or \
        abs(b["bytes_per_batch"] - b["bytes_per_launch"] * b["steps_per_batch"]) <= b["steps_per_batch"]
