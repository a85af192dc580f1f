"""Host-side checks of the benchmark script (no GPU): it refuses more than one GPU, and the
counter-calibrated HBM traffic it reports is read back only for kernels whose sources match
the recorded digest."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_entries_match_their_sources():
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    cal = t["calibration"]
    assert abs(cal["read_factor"] - 2.0) < 0.01 and abs(cal["write_factor"] - 1.0) < 0.01
    for name, e in t["kernels"].items():
        got = bench.measured_traffic(name)
        if e.get("mixed_configurations"):
            assert got is None
        elif e["source_sha256"] == bench.source_digest(e["sources"]):
            assert got == int(e["read_bytes"] + e["write_bytes"])
            if e.get("algorithmic_bytes"):
                # HBM bytes within a few per cent of the algorithmic bytes: no wasted re-reads
                assert 0.99 <= got / e["algorithmic_bytes"] <= 1.05, name
        else:
            assert got is None
    assert bench.measured_traffic("no_such_kernel") is None
