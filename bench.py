"""Benchmark of the FX correlator hot path on one MI355X.

A step is one ~1 s block of the 16-bit one-GPU share (76 stations x 2 polarisations, 64
subbands, complex int16 samples, 16-tap PPF -> 64 channels, 3072 channel samples, FP16-split
MFMA X stage) through the whole chain: F stage (unpack, FIR, FFT, fine delay, bandpass,
transpose, FP16 hi/lo split) then X stage.  Inputs are synthetic and already resident in HBM
when timing starts.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--fp32-steps F]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "correlator TeraMACs/s and real-time factor at 76 stations; p99 block latency"
HBM_PEAK_GBS = 8000.0
FP16_MFMA_PEAK_TFLOPS = 2516.6       # dense fp16 MFMA, 256 CU x 2.4 GHz x 4096 flop/clk
INT8_MFMA_PEAK_TOPS = 5033.2
FP32_VALU_PEAK_TFLOPS = 157.3        # published vector FP32 (dual-issue/packed)
# FP32 vector FMA without packed math (these kernels are built with packed FP32 disabled):
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VALU_NOPACK_TFLOPS = 78.6
# F-stage arithmetic per complex sample: FIR 16 taps x 2 FMA (64 flop), 64-point FFT
# (5 N log2 N / N = 30 flop), phase rotation 6 + bandpass 2 flop
F_FLOP_PER_SAMPLE = 102


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_1801_04834_amd", "csrc")


def source_digest(files):
    """sha256 over the kernel's source files (csrc/), as recorded beside the counters."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch (read + write) of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy kernel's readings), or None when
    there is none or the kernel's sources changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            entry = json.load(fh)["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    if entry.get("source_sha256") != source_digest(entry["sources"]) or "read_bytes" not in entry:
        return None
    return int(entry["read_bytes"] + entry["write_bytes"])


KERNEL_SOURCES = (("fstage_kernel", "fstage.hip"), ("xstage_", "xstage.hip"), ("beam_transform_kernel", "beamxf.hip"),
                  ("beam_kernel", "beam.hip"))


def write_traffic(fetch_dir, write_dir, bench_json, copy_mib=1024):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs of one command (FETCH_SIZE,
    then WRITE_SIZE; per-dispatch values in KiB, averaged per kernel) and the bench JSON line of
    the same sources (for each kernel's algorithmic bytes).  The plain copy kernel of the same
    runs (copy_mib MiB read and written) calibrates both counters."""
    import csv
    import glob
    import re

    def per_kernel(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") != counter:
                        continue
                    m = re.search(r"(\w+_kernel(?:<[^()]*>)?)\(", row["Kernel_Name"])
                    if m:
                        vals.setdefault(m.group(1), []).append(float(row["Counter_Value"]))
        return vals

    fetch_d, write_d = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    fetch = {k: sum(v) / len(v) for k, v in fetch_d.items()}
    write = {k: sum(v) / len(v) for k, v in write_d.items()}
    # a kernel launched in more than one configuration (the beamformer with and without voltage
    # output) has dispatches of different sizes: no single per-launch figure applies
    mixed = {k for d in (fetch_d, write_d) for k, v in d.items() if max(v) > 1.1 * min(v) + 64}
    with open(bench_json) as fh:
        line = json.loads(fh.read().strip().splitlines()[-1])
    algo = {}

    def collect(o):
        if isinstance(o, dict):
            if "kernel" in o and o.get("algorithmic_bytes"):
                algo[o["kernel"]] = int(o["algorithmic_bytes"])
            for v in o.values():
                collect(v)
    collect(line)
    nbytes = copy_mib * 2**20
    cal_f, cal_w = fetch["device_copy_kernel"], write["device_copy_kernel"]
    rf, wf = nbytes / (cal_f * 1024), nbytes / (cal_w * 1024)
    out = {"calibration": {"kernel": "device_copy_kernel", "bytes_read": nbytes, "bytes_written": nbytes,
                           "FETCH_SIZE_kb": round(cal_f, 1), "WRITE_SIZE_kb": round(cal_w, 1),
                           "read_factor": round(rf, 4), "write_factor": round(wf, 4)},
           "kernels": {}}
    for name in sorted(set(fetch) & set(write)):
        src = next((f for prefix, f in KERNEL_SOURCES if name.startswith(prefix)), None)
        if src is None:
            continue
        files = [src, "cobalt_internal.h"]
        if name in mixed:
            out["kernels"][name] = {"sources": files, "source_sha256": source_digest(files),
                                    "mixed_configurations": True}
            continue
        out["kernels"][name] = {
            "sources": files, "source_sha256": source_digest(files),
            "FETCH_SIZE_kb": round(fetch[name], 1), "WRITE_SIZE_kb": round(write[name], 1),
            "read_bytes": int(round(fetch[name] * 1024 * rf)), "write_bytes": int(round(write[name] * 1024 * wf)),
            "algorithmic_bytes": algo.get(name)}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    return out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="int16_share", choices=["int16_share", "int8_full", "plain_fx"])
    ap.add_argument("--fp32-steps", type=int, default=2, help="steps of the plain FP32 form (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-subbands", type=int, default=6, help="subbands in the oracle sample")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="time only the serial F-then-X schedule (value = serial rate); for profiling runs")
    ap.add_argument("--flags-steps", type=int, default=3,
                    help="steps of the coarse-delay + lost-sample-flag path (0: skip)")
    ap.add_argument("--beam-steps", type=int, default=3,
                    help="steps of the beamformer workload (48 stations, 61 subbands, 256 channels, 127 beams; 0: skip)")
    ap.add_argument("--gains-steps", type=int, default=3,
                    help="steps of the differentiable gain-applied correlator (48 stations, 16 subbands; 0: skip)")
    ap.add_argument("--service", action="store_true",
                    help="only the streaming service leg: three concurrent observations (24/48/76 stations, "
                         "32/64/128 subbands, ci16/ci16/ci8), Poisson block arrivals, HBM-budget admission")
    ap.add_argument("--service-seconds", type=float, default=15.0,
                    help="length of the streaming service leg of the default run (0: skip)")
    ap.add_argument("--service-budget-gib", type=float, default=48.0)
    ap.add_argument("--int8-steps", type=int, default=20,
                    help="steps of the 8-bit mode leg (76 stations, 128 subbands, int8 X stage; 0: skip)")
    ap.add_argument("--mfma-probe-iters", type=int, default=16384,
                    help="rounds of the dense MFMA probe (FP16 and int8, 512 workgroups), run first: the MFMA rate "
                         "this GPU sustains under that load, reported as mfma_probe (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=1024,
                    help="plain device copy of this many MiB, run three times first: the HBM rate a streaming "
                         "kernel reaches (reported as hbm_copy_gbs) and the reference for counter calibration (0: skip)")
    ap.add_argument("--write-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "BENCH_JSON"),
                    help="no benchmark: write profiles/traffic.json from the rocprofv3 FETCH_SIZE and WRITE_SIZE "
                         "runs of one command and the bench JSON line of the same sources")
    return ap.parse_args()


def make_input(w, torch, device):
    """Synthetic block on the device, generated on the host one subband group at a time."""
    x = torch.empty((w.S, 2, w.SB, w.N, 2), dtype={1: torch.int8, 2: torch.int16, 3: torch.float32}[w.sample_type],
                    device=device)
    step = 8
    for sb0 in range(0, w.SB, step):
        sbs = list(range(sb0, min(w.SB, sb0 + step)))
        part = w.block(0, subbands=sbs)
        x[:, :, sb0:sb0 + len(sbs)].copy_(torch.from_numpy(part))
    return x


def time_steps(torch, plan, x, delays, steps, warmup):
    """F then X per step on the current stream, HIP events around each kernel."""
    chan = plan.empty_chan()
    vis = plan.empty_vis()
    for _ in range(warmup):
        plan.channelize(x, delays, out=chan)
        plan.correlate_channelized(chan, out=vis)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        plan.channelize(x, delays, out=chan)
        ev[k][1].record()
        plan.correlate_channelized(chan, out=vis)
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    f_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    x_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])
    return wall, f_ms, x_ms, vis


def time_pipelined(torch, plan, x, delays, steps, warmup):
    """Streaming schedule: the F stage of block k+1 (stream sF) overlaps the X stage of
    block k (stream sX); two channelised buffers, reuse ordered by events.  Every step is
    still one full F + X over one block; returns host wall time per step."""
    sF, sX = torch.cuda.Stream(), torch.cuda.Stream()
    chans = [plan.empty_chan(), plan.empty_chan()]
    vis = plan.empty_vis()
    f_done = [torch.cuda.Event() for _ in range(2)]
    x_done = [torch.cuda.Event() for _ in range(2)]

    def run(n):
        for k in range(n):
            b = k % 2
            if k >= 2:
                sF.wait_event(x_done[b])              # buffer b was read by X(k-2)
            plan.channelize(x, delays, out=chans[b], stream=sF)
            f_done[b].record(sF)
            sX.wait_event(f_done[b])
            plan.correlate_channelized(chans[b], out=vis, stream=sX)
            x_done[b].record(sX)

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_flagged(torch, binding, synth, plan, w, x, delays, steps):
    """The same block through cobalt_correlate_ex: rows with a guard of 2048 samples (32
    rows), per-station coarse offsets across the guard, lost packets of 16 samples with
    probability 0.2 % per station and subband, and weights.  Returns per-step times (ms) of
    the flagged call and of the plain call, each F + flags + X on one stream."""
    G = 2048
    xg = torch.empty((w.S, 2, w.SB, w.N + G, 2), dtype=x.dtype, device=x.device)
    xg[:, :, :, :w.N].copy_(x)
    xg[:, :, :, w.N:].copy_(x[:, :, :, :G])
    offs = np.random.default_rng([w.seed, 0xC0]).integers(0, G + 1, w.S).astype(np.int32)
    fl = synth.lost_sample_flags(w.seed, w.S, w.SB, w.N + G, p_packet=0.002, p_sample=0.0)
    fd = torch.from_numpy(synth.pack_flags(fl).view(np.int32)).to(x.device)
    wts = torch.empty(plan.weights_shape(), dtype=torch.int32, device=x.device)
    vis = plan.empty_vis()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    plan.correlate_ex(xg, delays, coarse=offs, flags=fd, weights=wts, out=vis)
    plan.correlate(x, delays, out=vis)
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record()
        plan.correlate_ex(xg, delays, coarse=offs, flags=fd, weights=wts, out=vis)
        ev[k][1].record()
        plan.correlate(x, delays, out=vis)     # the next plain call still runs the flag kernel
        ev[k][2].record()                      # for the carried rows; measured as the plain path
    torch.cuda.synchronize()
    flagged = np.array([e[0].elapsed_time(e[1]) for e in ev])
    plain = np.array([e[1].elapsed_time(e[2]) for e in ev])
    lost = float(fl.mean())
    del xg, fd, vis
    return flagged, plain, lost, float(wts.float().mean().item()) / w.n_c


def time_beamformer(torch, binding, synth, steps, device):
    """The beamformer workload: 48 stations x 2 pol, 61 subbands of 16-bit samples (a quarter of
    the paper's 244-subband beamformer requirement), 256 channels, 127 coherent beams with
    Stokes I summed over 16 channel samples, plus the incoherent Stokes I beam.  Returns
    per-step F-stage and beamformer times (ms) and the workload's sizes."""
    w = synth.Workload(name="beam_share", S=48, SB=61, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, C=256,
                       sigma=64.0, seed=1807, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05,
                       fp16_prescale_log2=-1)
    NB, n_int = 127, 16
    x = make_input(w, torch, device)
    plan = binding.plan_for(w)
    dtau = torch.from_numpy(np.random.default_rng(1808).uniform(-2e-6, 2e-6, (NB, w.S))).to(device)
    cs, _, isz = plan.beam_shapes(NB, 1, n_int)
    coh = torch.empty(cs, dtype=torch.float32, device=device)
    inc = torch.empty(isz, dtype=torch.float32, device=device)
    chan = plan.empty_chan()
    delays = w.delays(0)
    plan.channelize(x, delays, out=chan)
    plan.beamform_channelized(chan, dtau, 1, n_int, coherent=coh, incoherent=inc)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        plan.channelize(x, delays, out=chan)
        ev[k][1].record()
        plan.beamform_channelized(chan, dtau, 1, n_int, coherent=coh, incoherent=inc)
        ev[k][2].record()
    torch.cuda.synchronize()
    f_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    b_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])
    cs_numel = coh.numel()
    # output resolution: the same beams as complex voltages (rows padded to 128 beams, whole
    # 128-byte lines per 16 beams), transformed to 16 channels per subband, Stokes I summed over
    # 16 output samples; then the same transform writing the transformed voltages
    del coh
    NBS = (NB + 15) // 16 * 16
    _, vs, _ = plan.beam_shapes(NB, 1, 1, voltage_stride=NBS)
    volt = torch.empty(vs, dtype=torch.float32, device=device)
    tvs, tsz = plan.transform_shapes(NB, 16, 1, 16, voltage_stride=NBS)
    ts = torch.empty(tsz, dtype=torch.float32, device=device)
    tv = torch.empty(tvs, dtype=torch.float32, device=device)
    plan.beamform_channelized(chan, dtau, 1, 1, voltages=volt)
    plan.beam_transform(volt, 16, 1, 16, out_stokes=ts, n_beams=NB)
    plan.beam_transform(volt, 16, 1, 16, out_voltages=tv, n_beams=NB)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        plan.beamform_channelized(chan, dtau, 1, 1, voltages=volt)
        ev[k][1].record()
        plan.beam_transform(volt, 16, 1, 16, out_stokes=ts, n_beams=NB)
        ev[k][2].record()
        plan.beam_transform(volt, 16, 1, 16, out_voltages=tv, n_beams=NB)
        ev[k][3].record()
    torch.cuda.synchronize()
    beam_voltage_bytes = volt.numel() * 4 * NB // NBS        # the beams, not the padding
    xf = {"beam_bytes": w.SB * w.C * 2 * w.S * w.n_c * 8 + (cs_numel + inc.numel()) * 4,
          "voltages_ms": float(np.mean([e[0].elapsed_time(e[1]) for e in ev])),
          "transform_ms": float(np.mean([e[1].elapsed_time(e[2]) for e in ev])),
          "transform_voltages_ms": float(np.mean([e[2].elapsed_time(e[3]) for e in ev])),
          "voltage_bytes": beam_voltage_bytes, "stokes_bytes": ts.numel() * 4, "stride": NBS}
    plan.close()
    del x, chan, inc, volt, ts, tv
    return w, NB, n_int, f_ms, b_ms, xf


def time_gains(torch, binding, synth, steps, device):
    """Differentiable gain-applied correlator on 48 stations x 2 pol, 16 subbands x 64 channels:
    one correlated block, then per step the gain forward (V' = g_a conj(g_b) V0) and the
    hand-written adjoint (dL/dg for an upstream gradient of V's shape)."""
    w = synth.Workload(name="gains_48", S=48, SB=16, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, sigma=64.0,
                       seed=1809, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1)
    plan = binding.plan_for(w)
    x = make_input(w, torch, device)
    vis0 = torch.view_as_complex(plan.correlate(x, w.delays(0)))
    rng = np.random.default_rng(1810)
    g = rng.uniform(0.5, 1.5, plan.gains_shape) * np.exp(1j * rng.uniform(-np.pi, np.pi, plan.gains_shape))
    gains = torch.from_numpy(g.astype(np.complex64)).to(device)
    grad = torch.randn(vis0.shape, dtype=torch.complex64, device=device)
    out = torch.empty_like(vis0)
    gg = torch.empty_like(gains)
    plan.apply_gains(vis0, gains, out=out)
    plan.apply_gains_adjoint(vis0, gains, grad, out=gg)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        plan.apply_gains(vis0, gains, out=out)
        ev[k][1].record()
        plan.apply_gains_adjoint(vis0, gains, grad, out=gg)
        ev[k][2].record()
    torch.cuda.synchronize()
    fwd = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    adj = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    n_ent = vis0.numel()
    plan.close()
    del x
    return w, n_ent, fwd, adj


def intensity_roof(ops, nbytes, ms, peak_t):
    """Where a contraction sits on the roofline: its arithmetic intensity (ops per algorithmic
    HBM byte) against the ridge (MFMA peak / 8 TB/s); below the ridge HBM bounds it, and the
    attainable MFMA fraction is intensity / ridge.  hbm_frac = the kernel's algorithmic bytes
    per second against 8 TB/s."""
    intensity = ops / nbytes
    ridge = peak_t * 1e12 / (HBM_PEAK_GBS * 1e9)
    return {"intensity_op_per_byte": round(intensity, 1), "ridge_op_per_byte": round(ridge, 1),
            "bound_by_intensity": "hbm" if intensity < ridge else "mfma",
            "attainable_frac": round(min(1.0, intensity / ridge), 4),
            "hbm_frac": round(nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}


def int8_leg(args, torch, binding, synth, dev, probe):
    """The 8-bit mode workload: 76 stations x 2 pol, 128 subbands of ci8 samples, int8 X stage
    (int8 MFMA, int32 sums), F then X per step as in the main leg, the streaming schedule, and
    the block latency over 60 blocks.  Rooflines: X against the dense int8 MFMA peak; F against
    the non-packed FP32 vector rate (4 B per sample: bound by arithmetic), with its GB/s."""
    w = synth.workload("int8_full")
    log(f"bench: 8-bit leg {w.S} stations x {w.SB} subbands; generating input")
    x = make_input(w, torch, dev)
    delays = w.delays(0)
    plan = binding.plan_for(w)
    cmacs = plan.info["useful_cmacs"]
    block_s = w.N / synth.SAMPLE_RATE_HZ
    wall, f_ms, x_ms, vis = time_steps(torch, plan, x, delays, args.steps, args.warmup)
    del vis
    step_ms = wall * 1e3
    if not args.no_pipeline:
        step_ms = time_pipelined(torch, plan, x, delays, args.steps, args.warmup) * 1e3
    lat = block_latency(torch, plan, x, delays, max(args.steps, 60))
    vis_bytes = plan.info["vis_bytes"]
    plan.close()
    del x
    torch.cuda.empty_cache()
    samples = w.M * w.SB * w.N
    f_s, x_s = float(np.mean(f_ms)) * 1e-3, float(np.mean(x_ms)) * 1e-3
    f_tf = samples * F_FLOP_PER_SAMPLE / f_s / 1e12
    x_tops = cmacs * 8 / x_s / 1e12
    f_kernel = f"fstage_kernel<{w.sample_type}, {w.x_mode}, {w.C}>"
    x_kernel = f"xstage_mfma_kernel<{w.x_mode}, {(w.M + 31) // 32}>"
    out = {
        "workload": f"int8_full: {w.S} stations x 2 pol, {w.SB} subbands, ci8 N(0, 16^2) clipped to +-127, "
                    f"16-tap PPF -> 64 ch, N={w.N}; int8 MFMA X stage with int32 sums",
        "value": round(cmacs / (step_ms * 1e-3) / 1e12, 4), "unit": "TeraMAC/s",
        "ms_per_step": round(step_ms, 4), "ms_per_step_serial": round(wall * 1e3, 4),
        "real_time_factor": round(block_s / (step_ms * 1e-3), 2),
        "block_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                             "p99": round(float(np.percentile(lat, 99)), 3), "n": int(lat.size),
                             "deadline_ms": round(block_s * 1e3, 3)},
        "x_stage_tmacs": round(cmacs / x_s / 1e12, 3),
        "roofline_x": {"bound": "mfma", "achieved": round(x_tops, 1), "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s",
                       "frac": round(x_tops / INT8_MFMA_PEAK_TOPS, 4), "traffic": measured_traffic(x_kernel),
                       "kernel": x_kernel, "ms": round(x_s * 1e3, 4),
                       "operand_gbs": round(w.SB * w.C * w.M * w.n_c * 2 / x_s / 1e9, 1),
                       "algorithmic_bytes": w.SB * w.C * w.M * w.n_c * 2 + vis_bytes,
                       **intensity_roof(cmacs * 8, w.SB * w.C * w.M * w.n_c * 2 + vis_bytes, x_s * 1e3,
                                        INT8_MFMA_PEAK_TOPS)},
        "roofline_f": {"bound": "alu", "achieved": round(f_tf, 1), "peak": FP32_VALU_NOPACK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(f_tf / FP32_VALU_NOPACK_TFLOPS, 4), "traffic": measured_traffic(f_kernel),
                       "kernel": f_kernel, "ms": round(f_s * 1e3, 4),
                       "hbm_gbs": round(samples * 4 / f_s / 1e9, 1), "algorithmic_bytes": samples * 4},
    }
    if probe is not None:
        out["roofline_x"]["of_mfma_probe"] = round(x_tops / probe["int8_tops"], 4)
    log(f"bench: 8-bit leg F {f_s * 1e3:.3f} ms, X {x_s * 1e3:.3f} ms, step {step_ms:.3f} ms "
        f"({out['value']} TeraMAC/s), latency p99 {out['block_latency_ms']['p99']} ms")
    return out


def block_latency(torch, plan, x, delays, n):
    """Submit one block, wait for it; host-side enqueue-to-completion time (ms)."""
    vis = plan.empty_vis()
    out = []
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.correlate(x, delays, out=vis)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) * 1e3)
    return np.array(out)


def oracle_threads():
    """Threads the oracle's BLAS uses on this host."""
    try:
        import threadpoolctl
        return int(max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or 1)
    except Exception:
        return len(os.sched_getaffinity(0))


def cpu_baseline(w, n_sub):
    """The FP64 oracle on n_sub subbands of the same workload, on this host's cores."""
    import oracle
    from paper_1801_04834_amd import synth
    threads = oracle_threads()
    sbs = list(range(n_sub))
    x = synth.to_complex(w.block(0, subbands=sbs))
    hist = np.zeros((w.S, 2, n_sub, 960), np.complex128)
    mode = {synth.X_FP32: "fp32", synth.X_FP16_SPLIT: "fp16_split", synth.X_INT8: "int8"}[w.x_mode]
    t0 = time.perf_counter()
    oracle.fx_block(x, hist, w.fir(), w.bandpass(), w.subband_freqs()[:n_sub], synth.SAMPLE_RATE_HZ,
                    w.delays(0), 64, 16, mode=mode, gain=w.gain(), return_channelised=False)
    dt = time.perf_counter() - t0
    cmacs = w.n_baselines * 4 * n_sub * w.C * w.n_c
    return {"value": cmacs / dt / 1e12, "unit": "TeraMAC/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_sub} of {w.SB} subbands of the same block (all {w.S} stations, N={w.N}); "
                      f"{dt:.2f} s per sample, real-time factor {w.N / 195312.5 * n_sub / w.SB / dt:.4f} "
                      f"for the whole block",
            "seconds": dt}


def beam_cpu_baselines(bw, NB, n_int, n_sub=1, n_tb=16):
    """The FP64 beamformer oracle on n_sub subbands of the beamformer workload (F stage at 256
    channels, coherent beams, Stokes I over n_int samples, incoherent I), then its
    output-resolution transform (256 -> 16 channels, Stokes I over 16 output samples) on n_tb of
    those beams.  Returns the two baselines."""
    from oracle import beam as ob
    from paper_1801_04834_amd import synth
    threads = oracle_threads()
    sbs = list(range(n_sub))
    x = synth.to_complex(bw.block(0, subbands=sbs))
    hist = np.zeros((bw.S, 2, n_sub, (bw.T - 1) * bw.C), np.complex128)
    dtau = np.random.default_rng(1808).uniform(-2e-6, 2e-6, (NB, bw.S))
    t0 = time.perf_counter()
    r = ob.beamform_block(x, hist, bw.fir(), bw.bandpass(), bw.subband_freqs()[:n_sub], synth.SAMPLE_RATE_HZ,
                          bw.delays(0), dtau, bw.C, bw.T, which="I", n_int=n_int)
    dt_b = time.perf_counter() - t0
    cmacs = n_sub * bw.C * NB * bw.S * 2 * bw.n_c
    B = np.moveaxis(r["beams"][0][:, :n_tb], 0, -2)          # [beam, P, C, N_c]
    t0 = time.perf_counter()
    ob.transformed_stokes(B, 16, "I", 16)
    dt_t = time.perf_counter() - t0
    vbytes = B.size * 8                                     # complex64 voltages consumed
    beam = {"value": cmacs / dt_b / 1e12, "unit": "TeraMAC/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_sub} of {bw.SB} subbands (all {bw.S} stations, {NB} beams, N={bw.N}), F stage at "
                      f"{bw.C} channels included; {dt_b:.2f} s", "seconds": dt_b}
    xf = {"value": vbytes / dt_t / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
          "sample": f"{n_tb} of {NB} beams of 1 subband ({vbytes / 1e6:.0f} MB of voltages); {dt_t:.2f} s",
          "seconds": dt_t}
    return beam, xf


def gains_cpu_baseline(gw):
    """The FP64 gains oracle (forward and adjoint) on the whole gains workload: random
    visibilities, gains and upstream gradient of the same shapes.  GB/s of visibility entries
    (16 B per complex entry) through the forward and the adjoint together."""
    from oracle import gains as og
    rng = np.random.default_rng(1811)
    B = gw.S * (gw.S + 1) // 2
    shp = (gw.SB, gw.C, B, 4)
    V0 = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    G = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    g = np.exp(1j * rng.uniform(-np.pi, np.pi, (gw.SB, gw.C, gw.M)))
    t0 = time.perf_counter()
    og.apply_gains(V0, g, gw.S)
    og.apply_gains_adjoint(V0, g, G, gw.S)
    dt = time.perf_counter() - t0
    return {"value": 2 * V0.size * 16 / dt / 1e9, "unit": "GB/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": f"the whole workload ({V0.size} entries), forward and adjoint; {dt:.2f} s", "seconds": dt}


def service_workloads(synth):
    """The three concurrent observations of the streaming-service workload."""
    kw = dict(delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05)
    return [synth.Workload(name="O1", S=24, SB=32, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, seed=1805,
                           fp16_prescale_log2=-1, **kw),
            synth.Workload(name="O2", S=48, SB=64, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, seed=1806,
                           fp16_prescale_log2=-1, **kw),
            synth.Workload(name="O3", S=76, SB=128, sample_type=synth.CI8, x_mode=synth.X_INT8, sigma=16.0, seed=1807,
                           **kw)]


def service_leg(args, torch, binding, synth):
    """Streaming service: three concurrent observations (24 st x 32 SB ci16, 48 st x 64 SB ci16,
    76 st x 128 SB ci8), each producing one ~1 s block per Poisson arrival (mean inter-arrival =
    the block duration) for ``service_seconds``; blocks are submitted from pinned host memory
    and their visibilities copied back (latency includes both copies).  Returns latency
    percentiles (all blocks and per observation) against the block deadline, drops, late
    blocks and the sustained real-time factor (seconds of data correlated per wall second)."""
    import threading
    block_s = synth.BLOCK_SAMPLES / synth.SAMPLE_RATE_HZ
    ws = service_workloads(synth)
    t0 = time.perf_counter()
    host = []
    for w in ws:
        blk = torch.empty((w.S, 2, w.SB, w.N, 2), dtype={1: torch.int8, 2: torch.int16}[w.sample_type], pin_memory=True)
        for sb0 in range(0, w.SB, 16):
            sbs = list(range(sb0, min(w.SB, sb0 + 16)))
            blk[:, :, sb0:sb0 + len(sbs)].copy_(torch.from_numpy(w.block(0, subbands=sbs)))
        host.append(blk)
    log(f"bench: service inputs generated ({time.perf_counter() - t0:.1f} s)")
    budget = int(args.service_budget_gib * 2**30)
    svc = binding.Service(budget, n_slots=3, queue_depth=4, deadline_s=block_s)
    oids = [svc.open(**binding.plan_kwargs(w)) for w in ws]
    admitted = [svc.state(o) == binding.OBS_ADMITTED for o in oids]
    outs = [[svc.vis_buffer(o) for _ in range(4)] for o in oids]
    for i, w in enumerate(ws):                       # warm-up: one block per observation
        svc.wait(svc.submit(oids[i], host[i], w.delays(0), outs[i][0]))
    warm = svc.stats()
    rng = np.random.default_rng(1805)
    arrivals = []
    for i in range(len(ws)):
        t, k = rng.exponential(block_s), 0
        while t < args.service_seconds:
            arrivals.append((t, i, k))
            t += rng.exponential(block_s)
            k += 1
    arrivals.sort()
    queues = [[] for _ in ws]
    lats = [[] for _ in ws]
    cv = threading.Condition()
    state = {"stop": False}

    def waiter(i):
        while True:
            with cv:
                while not queues[i] and not state["stop"]:
                    cv.wait()
                if not queues[i]:
                    return
                tk = queues[i].pop(0)
            lats[i].append(svc.wait(tk))

    ths = [threading.Thread(target=waiter, args=(i,)) for i in range(len(ws))]
    for th in ths:
        th.start()
    start = time.perf_counter()
    submitted = [0] * len(ws)
    dropped = [0] * len(ws)
    for t, i, k in arrivals:
        dt = start + t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tk = svc.submit(oids[i], host[i], ws[i].delays(k), outs[i][k % 4])
        submitted[i] += 1
        if tk is None:
            dropped[i] += 1
            continue
        with cv:
            queues[i].append(tk)
            cv.notify_all()
    with cv:
        state["stop"] = True
        cv.notify_all()
    for th in ths:
        th.join()
    wall = time.perf_counter() - start
    st = svc.stats()
    svc.destroy()
    del host
    completed = st["completed"] - warm["completed"]
    allv = np.array([v for l in lats for v in l]) * 1e3
    pct = lambda a, q: round(float(np.percentile(a, q)), 3) if len(a) else None  # noqa: E731
    per_obs = []
    for i, w in enumerate(ws):
        a = np.array(lats[i]) * 1e3
        per_obs.append({"observation": f"{w.name}: {w.S} stations x 2 pol, {w.SB} subbands, "
                                       f"{'ci8 int8 X' if w.sample_type == synth.CI8 else 'ci16 FP16-split X'}",
                        "blocks": int(a.size), "dropped": dropped[i], "p50_ms": pct(a, 50), "p99_ms": pct(a, 99),
                        "max_ms": round(float(a.max()), 3) if a.size else None})
    out = {
        "workload": "three concurrent observations: 24 st x 32 SB ci16, 48 st x 64 SB ci16, 76 st x 128 SB ci8; "
                    "Poisson block arrivals, mean inter-arrival = block duration",
        "seconds": args.service_seconds, "slots": 3, "budget_gib": args.service_budget_gib,
        "admitted_at_open": admitted, "blocks_submitted": int(sum(submitted)), "blocks_completed": int(completed),
        "dropped": int(st["dropped"]), "late": int(st["late"] - warm["late"]),
        "p50_ms": pct(allv, 50), "p99_ms": pct(allv, 99), "max_ms": round(float(allv.max()), 3) if allv.size else None,
        "deadline_ms": round(block_s * 1e3, 3),
        "sustained_real_time_factor": round(completed * block_s / wall, 3),
        "offered_real_time_factor": round(sum(submitted) * block_s / args.service_seconds, 3),
        "per_observation": per_obs,
        "hbm_admitted_gib": round(st["hbm_used_bytes"] / 2**30, 2),
        "note": "latency = submit -> visibilities in host memory (host->device and device->host copies included); "
                "sustained real-time factor = seconds of station data correlated per wall-clock second, summed "
                "over the observations (3 when all keep up)",
    }
    log(f"bench: service {completed} blocks in {wall:.1f} s, p50 {out['p50_ms']} ms p99 {out['p99_ms']} ms, "
        f"dropped {out['dropped']}, late {out['late']}")
    return out


def main():
    args = parse()
    if args.write_traffic:
        t = write_traffic(*args.write_traffic, copy_mib=args.copy_calibration_mib)
        for name, e in t["kernels"].items():
            if e.get("mixed_configurations"):
                log(f"{name}: launched in several configurations, no per-launch figure")
                continue
            alg = e["algorithmic_bytes"]
            tot = e["read_bytes"] + e["write_bytes"]
            log(f"{name}: read {e['read_bytes'] / 1e9:.3f} GB, written {e['write_bytes'] / 1e9:.3f} GB"
                + (f", {tot / alg:.3f} x algorithmic" if alg else ""))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (the FX chain would shard over "
              "subbands with no exchange between GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1801_04834_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.service:
        svc = service_leg(args, torch, binding, synth)
        print(json.dumps({"metric": METRIC, "mode": "service", "value": svc["p99_ms"], "unit": "ms p99 block latency",
                          "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "service": svc}), flush=True)
        return
    w = synth.workload(args.workload)
    log(f"bench: workload {w.name} S={w.S} SB={w.SB} N={w.N} mode={w.x_mode}; generating input")
    t0 = time.perf_counter()
    x = make_input(w, torch, dev)
    delays = w.delays(0)
    torch.cuda.synchronize()
    log(f"bench: input {x.numel() * x.element_size() / 1e9:.2f} GB resident ({time.perf_counter() - t0:.1f} s)")

    copy_gbs = fanout_gbs = None
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * 2**20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        # the first copy is queued ahead of the start event, so the timed copies run back to back
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        binding.device_copy(dst, src)
        e0.record()
        for _ in range(3):
            binding.device_copy(dst, src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        copy_gbs = 2 * n / (ms * 1e-3) / 1e9
        log(f"bench: plain copy {n} B read + {n} B written in {ms:.3f} ms ({copy_gbs:.1f} GB/s)")
        # the same with two destinations: 1 byte read per 2 written, the 16-bit F stage's mix
        dst2 = torch.empty_like(src)
        binding.device_fanout(dst, dst2, src)
        e0.record()
        for _ in range(3):
            binding.device_fanout(dst, dst2, src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        fanout_gbs = 3 * n / (ms * 1e-3) / 1e9
        log(f"bench: fan-out copy {n} B read + {2 * n} B written in {ms:.3f} ms ({fanout_gbs:.1f} GB/s)")
        del src, dst, dst2

    probe = None
    if args.mfma_probe_iters > 0:
        sink = torch.empty(512 * 256, dtype=torch.float32, device=dev)
        probe = {"workgroups": 512, "iterations": args.mfma_probe_iters}
        for mode, name, k in ((synth.X_FP16_SPLIT, "fp16_tflops", 16), (synth.X_INT8, "int8_tops", 32)):
            binding.mfma_probe(mode, 64, sink)                     # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ops = binding.mfma_probe(mode, args.mfma_probe_iters, sink)
            e1.record()
            torch.cuda.synchronize()
            if not bool(torch.all(sink == float(args.mfma_probe_iters * k))):
                raise RuntimeError("MFMA probe returned wrong sums")
            probe[name] = round(ops / (e0.elapsed_time(e1) * 1e-3) / 1e12, 1)
        log(f"bench: MFMA probe {probe['fp16_tflops']} TFLOP/s FP16, {probe['int8_tops']} TOP/s int8 (dense, sustained)")
        del sink

    plan = binding.plan_for(w)
    info = plan.info
    cmacs = info["useful_cmacs"]
    block_s = w.N / synth.SAMPLE_RATE_HZ
    wall, f_ms, x_ms, vis = time_steps(torch, plan, x, delays, args.steps, args.warmup)
    log(f"bench: {args.steps} steps, wall {wall * 1e3:.3f} ms/step, F {np.mean(f_ms):.3f} ms, X {np.mean(x_ms):.3f} ms")
    serial_ms = wall * 1e3
    del vis
    if args.no_pipeline:
        step_ms = serial_ms
    else:
        wall_p = time_pipelined(torch, plan, x, delays, args.steps, args.warmup)
        log(f"bench: pipelined (F of block k+1 overlapping X of block k) {wall_p * 1e3:.3f} ms/step")
        step_ms = wall_p * 1e3
    lat = block_latency(torch, plan, x, delays, max(args.steps, 60))
    log(f"bench: block latency p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms")

    # algorithmic work per launch
    samples = w.M * w.SB * w.N
    sample_b = {synth.CI8: 2, synth.CI16: 4, synth.CF32: 8}[w.sample_type]
    chan_b = {synth.X_FP32: 8, synth.X_FP16_SPLIT: 8, synth.X_INT8: 2}[w.x_mode]
    f_bytes = samples * (sample_b + chan_b)
    f_ms_avg = float(np.mean(f_ms))
    x_ms_avg = float(np.mean(x_ms))
    f_gbs = f_bytes / (f_ms_avg * 1e-3) / 1e9
    x_tmacs = cmacs / (x_ms_avg * 1e-3) / 1e12
    if w.x_mode == synth.X_FP16_SPLIT:
        x_mfma_tflops = cmacs * 8 * 3 / (x_ms_avg * 1e-3) / 1e12
        x_peak, x_unit = FP16_MFMA_PEAK_TFLOPS, "TFLOP/s"
    elif w.x_mode == synth.X_INT8:
        x_mfma_tflops = cmacs * 8 / (x_ms_avg * 1e-3) / 1e12
        x_peak, x_unit = INT8_MFMA_PEAK_TOPS, "TOP/s"
    else:
        x_mfma_tflops = cmacs * 8 / (x_ms_avg * 1e-3) / 1e12
        x_peak, x_unit = FP32_VALU_PEAK_TFLOPS, "TFLOP/s"
    x_bytes = w.SB * w.C * w.M * w.n_c * chan_b
    f_kernel = f"fstage_kernel<{w.sample_type}, {w.x_mode}, {w.C}>"
    x_kernel = f"xstage_mfma_kernel<{w.x_mode}, {(w.M + 31) // 32}>" if w.x_mode != synth.X_FP32 else "xstage_fp32_kernel"
    if w.x_mode == synth.X_INT8:
        # 4 B per sample against ~100 flop: the 8-bit F stage is bound by vector arithmetic
        f_tf = samples * F_FLOP_PER_SAMPLE / (f_ms_avg * 1e-3) / 1e12
        f_roof = {"bound": "alu", "achieved": round(f_tf, 1), "peak": FP32_VALU_NOPACK_TFLOPS, "unit": "TFLOP/s",
                  "frac": round(f_tf / FP32_VALU_NOPACK_TFLOPS, 4), "traffic": measured_traffic(f_kernel),
                  "kernel": f_kernel, "ms": round(f_ms_avg, 4), "algorithmic_bytes": f_bytes,
                  "hbm_gbs": round(f_gbs, 1)}
    else:
        f_roof = {"bound": "hbm", "achieved": round(f_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(f_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(f_kernel), "kernel": f_kernel,
                  "ms": round(f_ms_avg, 4), "algorithmic_bytes": f_bytes,
                  "of_plain_copy": None if copy_gbs is None else round(f_gbs / copy_gbs, 4)}
        if fanout_gbs is not None and chan_b == 2 * sample_b:
            f_roof["of_same_mix_copy"] = round(f_gbs / fanout_gbs, 4)    # 1 read : 2 written
    x_roof = {"bound": "mfma" if w.x_mode != synth.X_FP32 else "alu", "achieved": round(x_mfma_tflops, 1),
              "peak": x_peak, "unit": x_unit, "frac": round(x_mfma_tflops / x_peak, 4),
              "traffic": measured_traffic(x_kernel), "kernel": x_kernel, "ms": round(x_ms_avg, 4),
              "operand_gbs": round(x_bytes / (x_ms_avg * 1e-3) / 1e9, 1),
              "algorithmic_bytes": x_bytes + info["vis_bytes"]}
    if probe is not None and w.x_mode != synth.X_FP32:
        ref = probe["fp16_tflops"] if w.x_mode == synth.X_FP16_SPLIT else probe["int8_tops"]
        x_roof["of_mfma_probe"] = round(x_mfma_tflops / ref, 4)
    if w.x_mode != synth.X_FP32:
        x_roof.update(intensity_roof(x_mfma_tflops * 1e12 * x_ms_avg * 1e-3, x_bytes + info["vis_bytes"], x_ms_avg, x_peak))
    dominant = f_roof if f_ms_avg >= x_ms_avg else x_roof
    other = x_roof if dominant is f_roof else f_roof

    fp32 = None
    if args.fp32_steps > 0 and w.x_mode != synth.X_FP32:
        plan32 = binding.plan_for(w, x_mode=synth.X_FP32)
        wall32, f32, x32, v32 = time_steps(torch, plan32, x, delays, args.fp32_steps, 1)
        fp32 = {"ms_per_step": round(wall32 * 1e3, 3), "x_ms": round(float(np.mean(x32)), 3),
                "f_ms": round(float(np.mean(f32)), 3),
                "x_tmacs": round(cmacs / (float(np.mean(x32)) * 1e-3) / 1e12, 3),
                "real_time_factor": round(block_s / wall32, 2)}
        log(f"bench: plain FP32 form {wall32 * 1e3:.3f} ms/step (X {np.mean(x32):.3f} ms)")
        del v32
        plan32.close()

    flagged = None
    if args.flags_steps > 0:
        fl_ms, pl_ms, lost, wfrac = time_flagged(torch, binding, synth, plan, w, x, delays, args.flags_steps)
        flagged = {"ms_per_step": round(float(np.mean(fl_ms)), 3), "plain_ms_per_step": round(float(np.mean(pl_ms)), 3),
                   "lost_sample_fraction": round(lost, 5), "mean_weight_fraction": round(wfrac, 4),
                   "guard_samples": 2048}
        log(f"bench: coarse delay + flags {np.mean(fl_ms):.3f} ms/step vs plain {np.mean(pl_ms):.3f} ms "
            f"(lost {lost:.4%}, mean weight {wfrac:.4f} of N_c)")

    beam = None
    if args.beam_steps > 0:
        bw, NB, n_int, bf_ms, bb_ms, xf = time_beamformer(torch, binding, synth, args.beam_steps, dev)
        cmac_b = bw.SB * bw.C * NB * bw.S * 2 * bw.n_c          # useful complex MACs per block
        b_ms = float(np.mean(bb_ms))
        mfma_tf = cmac_b * 8 * 3 * (128 / NB) / (b_ms * 1e-3) / 1e12     # executed: 3 products, beams padded to 128
        beam = {"workload": f"{bw.S} stations x 2 pol, {bw.SB} subbands ci16, 256 channels, {NB} beams, "
                            f"Stokes I summed over {n_int} samples + incoherent I",
                "f_stage_ms": round(float(np.mean(bf_ms)), 3), "beamformer_ms": round(b_ms, 3),
                "ms_per_step": round(float(np.mean(bf_ms)) + b_ms, 3),
                "beam_tcmacs": round(cmac_b / (b_ms * 1e-3) / 1e12, 3),
                "real_time_factor": round(bw.N / synth.SAMPLE_RATE_HZ / ((float(np.mean(bf_ms)) + b_ms) * 1e-3), 2),
                "roofline": {"bound": "mfma", "achieved": round(mfma_tf, 1), "peak": FP16_MFMA_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(mfma_tf / FP16_MFMA_PEAK_TFLOPS, 4),
                             "traffic": measured_traffic(f"beam_kernel<{(bw.S + 7) // 8}, 1, false>"),
                             "kernel": f"beam_kernel<{(bw.S + 7) // 8}, 1, false>", "algorithmic_bytes": xf["beam_bytes"]}}
        if probe is not None:
            beam["roofline"]["of_mfma_probe"] = round(mfma_tf / probe["fp16_tflops"], 4)
        t_gbs = (xf["voltage_bytes"] + xf["stokes_bytes"]) / (xf["transform_ms"] * 1e-3) / 1e9
        tv_gbs = 2 * xf["voltage_bytes"] / (xf["transform_voltages_ms"] * 1e-3) / 1e9
        beam["output_resolution"] = {
            "workload": "the same beams as complex voltages (rows of 127 beams padded to "
                        f"{xf['stride']}), transformed from 256 to 16 channels per subband, Stokes I summed over "
                        "16 output samples; and the same transform writing the transformed voltages",
            "voltages_ms": round(xf["voltages_ms"], 3), "transform_ms": round(xf["transform_ms"], 3),
            "transform_voltages_ms": round(xf["transform_voltages_ms"], 3),
            "transform_voltages_gbs": round(tv_gbs, 1),
            "roofline": {"bound": "hbm", "achieved": round(t_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(t_gbs / HBM_PEAK_GBS, 4), "kernel": "beam_transform_kernel<16, 1>",
                         "traffic": measured_traffic("beam_transform_kernel<16, 1>"),
                         "algorithmic_bytes": xf["voltage_bytes"] + xf["stokes_bytes"]}}
        log(f"bench: beam voltages {xf['voltages_ms']:.3f} ms, transform to 16 channels {xf['transform_ms']:.3f} ms "
            f"({t_gbs:.0f} GB/s), writing voltages {xf['transform_voltages_ms']:.3f} ms ({tv_gbs:.0f} GB/s)")
        log(f"bench: beamformer F {np.mean(bf_ms):.3f} ms + beams {b_ms:.3f} ms "
            f"({beam['beam_tcmacs']} TeraMAC/s useful, {mfma_tf:.0f} TFLOP/s executed)")

    gains = None
    if args.gains_steps > 0:
        gw, n_ent, fwd, adj = time_gains(torch, binding, synth, args.gains_steps, dev)
        gains = {"workload": f"{gw.S} stations x 2 pol, {gw.SB} subbands x 64 channels, complex gains per input and channel",
                 "forward_ms": round(fwd, 4), "adjoint_ms": round(adj, 4), "entries": n_ent,
                 "forward_gbs": round(n_ent * 16 / (fwd * 1e-3) / 1e9, 1),
                 "adjoint_gbs": round(n_ent * 16 / (adj * 1e-3) / 1e9, 1)}
        log(f"bench: gains forward {fwd:.3f} ms, adjoint {adj:.3f} ms ({n_ent} visibility entries)")

    if beam is not None and not args.no_cpu_baseline:
        log("bench: beamformer and output-resolution oracles for their CPU baselines")
        beam["cpu_baseline"], beam["output_resolution"]["cpu_baseline"] = beam_cpu_baselines(bw, NB, n_int)
        log(f"bench: beamformer oracle {beam['cpu_baseline']['seconds']:.2f} s, transform oracle "
            f"{beam['output_resolution']['cpu_baseline']['seconds']:.2f} s")

    if gains is not None and not args.no_cpu_baseline:
        gains["cpu_baseline"] = gains_cpu_baseline(gw)
        log(f"bench: gains oracle {gains['cpu_baseline']['seconds']:.2f} s")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"bench: oracle on {args.cpu_subbands} subband(s) for the CPU baseline")
        cpu = cpu_baseline(w, args.cpu_subbands)
        log(f"bench: oracle {cpu['seconds']:.2f} s -> {cpu['value']:.5f} TeraMAC/s")

    plan.close()
    del x
    torch.cuda.empty_cache()
    int8 = None
    if args.int8_steps > 0:
        a8 = argparse.Namespace(**vars(args))
        a8.steps = args.int8_steps
        int8 = int8_leg(a8, torch, binding, synth, dev, probe)
    service = None
    if args.service_seconds > 0:
        service = service_leg(args, torch, binding, synth)

    value = cmacs / (step_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TeraMAC/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {synth.X_FP16_SPLIT: "fp16x3-split/fp32-acc", synth.X_INT8: "int8/int32-acc",
                  synth.X_FP32: "fp32"}[w.x_mode],
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.S} stations x 2 pol, {w.SB} subbands, "
                               f"{'ci16' if w.sample_type == synth.CI16 else 'ci8' if w.sample_type == synth.CI8 else 'cf32'}, "
                               f"16-tap PPF -> 64 ch, N={w.N} ({w.n_c} channel samples, {block_s:.8f} s)",
                   "stations": w.S, "subbands": w.SB, "channels": w.C, "samples_per_block": w.N,
                   "x_mode": w.x_mode},
        "schedule": ("serial: F then X on one stream" if args.no_pipeline else
                     "pipelined: F stage of block k+1 overlaps X stage of block k on a second stream"),
        "ms_per_step_serial": round(serial_ms, 4),
        "real_time_factor": round(block_s / (step_ms * 1e-3), 2),
        "block_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                             "p99": round(float(np.percentile(lat, 99)), 3), "n": int(lat.size),
                             "deadline_ms": round(block_s * 1e3, 3)},
        "x_stage_tmacs": round(x_tmacs, 3),
        "hbm_copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
        "hbm_fanout_copy_gbs": None if fanout_gbs is None else round(fanout_gbs, 1),
        "mfma_probe": probe,
        "f_stage_gbs": round(f_gbs, 1),
        "roofline": dominant,
        "roofline_other": other,
        "traffic_source": "stored, not measured in this run: HBM bytes per launch from rocprofv3 FETCH_SIZE and "
                          "WRITE_SIZE passes (scaled by a plain copy's readings) over the same kernel sources, "
                          "profiles/traffic.json; null where a kernel's sources changed since",
        "plain_fp32_form": fp32,
        "coarse_delay_and_flags": flagged,
        "beamformer": beam,
        "differentiable_gains": gains,
        "int8_mode": int8,
        "service": service,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
