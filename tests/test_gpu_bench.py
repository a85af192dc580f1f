"""The benchmark's output contract on a GPU: one JSON line with the metric, the whole-step
throughput, the roofline object of the dominant kernel (bound, achieved, peak, unit, frac,
traffic), the probes, the 8-bit mode leg and the streaming service leg, from a short run of the
default workload."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_roofline():
    print("CASE bench short run", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1", "--fp32-steps", "0",
                        "--flags-steps", "0", "--beam-steps", "0", "--gains-steps", "0", "--no-cpu-baseline",
                        "--mfma-probe-iters", "256", "--copy-calibration-mib", "256", "--int8-steps", "2",
                        "--service-seconds", "3"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "roofline_other", "hbm_copy_gbs", "mfma_probe"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["value"] > 0
    assert d["unit"] == "TeraMAC/s" and d["config"]["stations"] == 76 and d["config"]["subbands"] == 64
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] in ("hbm", "mfma", "alu") and 0 < roof["frac"] < 1
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert d["mfma_probe"]["fp16_tflops"] > 0 and d["hbm_copy_gbs"] > 0
    i8 = d["int8_mode"]
    assert i8["value"] > 0 and i8["block_latency_ms"]["n"] >= 60
    for r in (i8["roofline_x"], i8["roofline_f"]):
        assert 0 < r["frac"] < 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    sv = d["service"]
    assert sv["blocks_completed"] + sv["dropped"] == sv["blocks_submitted"]
    assert len(sv["per_observation"]) == 3 and all(sv["admitted_at_open"])
    if sv["blocks_completed"]:
        assert 0 < sv["p50_ms"] <= sv["p99_ms"] <= sv["max_ms"]
