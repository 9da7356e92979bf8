"""Benchmark driver checks that need no GPU: the one-GPU rule and the
validity rules of the committed counter file."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_counter_traffic_only_for_its_workload_and_sources():
    d = json.load(open(bench.TRAFFIC_FILE))
    assert d["workload"].startswith("C3:")
    assert bench.traffic_for("fp32", workload="C2") is None
    if d["kernel_source_sha256_16"] == bench.lattice_source_hash():
        t = bench.traffic_for("fp32")
        alg = 2 * 19 * 4 * 256 ** 3
        # measured HBM bytes of the FP32 stream-collide pass: near the
        # algorithmic bytes, never below them
        assert alg <= t <= 1.2 * alg
    else:
        assert bench.traffic_for("fp32") is None
