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


def _counter_csv(path, counter, rows):
    """A rocprofv3 counter_collection.csv with the columns the traffic writer reads."""
    import csv
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, value) in enumerate(rows):
            w.writerow([i, name, counter, value])


def test_write_traffic_calibrates_and_flags_mixed_launches(tmp_path, monkeypatch):
    """The counter summary: FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged per kernel) scaled
    by what the plain copy of 1 GiB reads; algorithmic bytes taken from the bench line; a kernel
    whose dispatches differ in size is marked mixed and reports no traffic."""
    f_dir, w_dir = str(tmp_path / "F"), str(tmp_path / "W")
    copy = "cobalt::(anonymous namespace)::device_copy_kernel(uint4*, uint4 const*, long)"
    fst = "void cobalt::(anonymous namespace)::fstage_kernel<2, 1, 64>(cobalt::FArgs)"
    beam = "void cobalt::(anonymous namespace)::beam_kernel<6, 1>(cobalt::BeamArgs)"
    _counter_csv(f_dir, "FETCH_SIZE", [(copy, 524288.0), (fst, 1000.0), (fst, 1000.0), (beam, 100.0), (beam, 300.0)])
    _counter_csv(w_dir, "WRITE_SIZE", [(copy, 1048576.0), (fst, 3000.0), (fst, 3000.0), (beam, 10.0), (beam, 10.0)])
    line = {"roofline": {"kernel": "fstage_kernel<2, 1, 64>", "algorithmic_bytes": 6000 * 1024},
            "beamformer": {"roofline": {"kernel": "beam_kernel<6, 1>", "algorithmic_bytes": 1}}}
    bj = tmp_path / "bench.json"
    bj.write_text("bench: a log line\n" + json.dumps(line) + "\n")
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    t = bench.write_traffic(f_dir, w_dir, str(bj))
    cal = t["calibration"]
    assert cal["read_factor"] == 2.0 and cal["write_factor"] == 1.0
    e = t["kernels"]["fstage_kernel<2, 1, 64>"]
    assert e["read_bytes"] == 2 * 1000 * 1024 and e["write_bytes"] == 3000 * 1024
    assert e["algorithmic_bytes"] == 6000 * 1024
    assert e["source_sha256"] == bench.source_digest(e["sources"])
    assert t["kernels"]["beam_kernel<6, 1>"].get("mixed_configurations")
    assert "device_copy_kernel" not in t["kernels"]
    assert json.loads(out.read_text()) == t
    assert bench.measured_traffic("fstage_kernel<2, 1, 64>") == 5000 * 1024
    assert bench.measured_traffic("beam_kernel<6, 1>") is None


def test_oracle_baselines_of_the_beamformer_transform_and_gains_legs():
    """The CPU baselines that sit beside the beamformer, output-resolution and gains legs run
    the oracle on a bounded sample and report a positive rate in the leg's unit."""
    from paper_1801_04834_amd import synth
    bw = synth.Workload(name="beam_small", S=4, SB=2, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, C=256,
                        N=256 * 32, sigma=64.0, seed=5, fp16_prescale_log2=-1)
    beam, xf = bench.beam_cpu_baselines(bw, 5, 16, n_sub=1, n_tb=3)
    assert beam["kind"] == xf["kind"] == "oracle"
    assert beam["unit"] == "TeraMAC/s" and xf["unit"] == "GB/s"
    assert beam["value"] > 0 and xf["value"] > 0 and beam["cores"] >= 1
    assert "1 of 2 subbands" in beam["sample"] and "3 of 5 beams" in xf["sample"]
    gw = synth.Workload(name="gains_small", S=3, SB=2, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, N=64 * 8,
                        fp16_prescale_log2=-1)
    g = bench.gains_cpu_baseline(gw)
    assert g["kind"] == "oracle" and g["unit"] == "GB/s" and g["value"] > 0
    assert f"({gw.SB * gw.C * 6 * 4} entries)" in g["sample"]
