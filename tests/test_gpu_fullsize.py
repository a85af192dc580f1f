"""GPU parity at the full benchmark sizes, in the launch configuration the benchmark times
(F stage then X stage on one plan over the whole block), checked on sampled subbands that the
FP64 oracle computes on its own.

* 16-bit share: 76 stations x 2 pol, 64 subbands, ci16, 196 608 samples, FP16-split X stage;
  the visibilities of the first, a middle and the last subband against the oracle's, coherence
  error <= 1e-5.
* 8-bit mode: 76 stations x 2 pol, 128 subbands, ci8, int8 X stage; on the same three subbands
  the requantised channelised data follow the +-1-at-a-rounding-boundary rule against the
  oracle and the visibilities equal the exact integer correlation of the GPU's own int8 stream.
* plain FP32 form of the 16-bit share (FP32 channelised data, FP32 VALU X stage): coherence
  error <= 1e-6 on the same three subbands.
* the benchmark's flagged 16-bit share (rows with a 2048-sample guard, per-station coarse
  offsets across it, 16-sample packets lost with probability 0.2 %) through the full chain with
  weights: weights exact and coherence error <= 1e-5 on the same three subbands.
* the benchmark's beamformer workload (48 stations x 2 pol, 61 subbands, 256 channels, 127
  coherent beams, Stokes I over 16 channel samples, incoherent Stokes I), F stage then the
  beamformer as the benchmark runs them: coherent and incoherent Stokes of three sampled
  subbands within |dS| <= 2e-5 I + 1e-6 mean(I) of the oracle's.

Subbands are independent (each has its own streams, history and output), so the sampled ones
stand for the rest; the whole block runs on the GPU as in the benchmark.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import synth
from tests.layout import unblock
from tests.metrics import coherence_error, near_rounding_boundary, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS_FP16 = 1e-5
EPS_FP32 = 1e-6
MODE = {synth.X_FP32: "fp32", synth.X_FP16_SPLIT: "fp16_split", synth.X_INT8: "int8"}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _input(w):
    """The whole block on the device, generated on the host a few subbands at a time."""
    dt = {synth.CI8: torch.int8, synth.CI16: torch.int16, synth.CF32: torch.float32}[w.sample_type]
    x = torch.empty((w.S, 2, w.SB, w.N, 2), dtype=dt, device="cuda")
    for sb0 in range(0, w.SB, 8):
        sbs = list(range(sb0, min(w.SB, sb0 + 8)))
        x[:, :, sb0:sb0 + len(sbs)].copy_(torch.from_numpy(w.block(0, subbands=sbs)))
    return x


def _oracle(w, sbs):
    hist = np.zeros((w.S, 2, len(sbs), 15 * w.C), np.complex128)
    return oracle.fx_block(synth.to_complex(w.block(0, subbands=sbs)), hist, w.fir(), w.bandpass(),
                           w.subband_freqs()[sbs], synth.SAMPLE_RATE_HZ, w.delays(0), w.C, 16, mode=MODE[w.x_mode],
                           gain=w.gain())


@pytest.mark.parametrize("name,mode", [("int16_share", None), ("int8_full", None), ("int16_share", synth.X_FP32)])
def test_full_size_block_on_sampled_subbands(name, mode):
    from paper_1801_04834_amd import binding
    w = synth.workload(name) if mode is None else synth.workload(name, x_mode=mode)
    sbs = [0, w.SB // 2 + 3, w.SB - 1]
    _say(f"CASE fullsize {name} S={w.S} SB={w.SB} N={w.N} mode={w.x_mode} subbands={sbs} seed={w.seed}")
    x = _input(w)
    with binding.plan_for(w) as plan:
        chan = plan.empty_chan()
        vis = plan.empty_vis()
        plan.channelize(x, w.delays(0), out=chan)
        plan.correlate_channelized(chan, out=vis)
        torch.cuda.synchronize()
        del x
        Vg = vis[sbs].cpu().numpy()
        cg = chan[sbs].cpu().numpy() if w.x_mode == synth.X_INT8 else None
    o = _oracle(w, sbs)
    if w.x_mode == synth.X_INT8:
        Qg = unblock(cg)[..., :w.n_c, :]
        d = Qg.astype(np.int64) - o["Q"].astype(np.int64)
        bad = d != 0
        g = np.float64(np.float32(w.gain()))
        pre = np.stack([(g * o["Zf"].real).astype(np.float32), (g * o["Zf"].imag).astype(np.float32)], -1)
        _say(f"  int8 mismatches {int(bad.sum())} of {d.size}")
        assert np.all(np.abs(d) <= 1) and np.all(near_rounding_boundary(pre, 1e-3)[bad])
        np.testing.assert_array_equal(Vg.astype(np.int64), oracle.correlate_int(np.ascontiguousarray(Qg), w.S))
    else:
        eps = coherence_error(vis_complex(Vg), o["V"], w.S)
        _say(f"  eps {eps:.3e}")
        assert eps <= (EPS_FP32 if w.x_mode == synth.X_FP32 else EPS_FP16)


def test_full_size_coarse_delay_and_flags_on_sampled_subbands():
    from paper_1801_04834_amd import binding
    from oracle import flags as oflags
    from tests.test_gpu_flags import _eps
    w = synth.workload("int16_share")
    G = 2048
    sbs = [0, w.SB // 2 + 3, w.SB - 1]
    _say(f"CASE fullsize flagged int16_share S={w.S} SB={w.SB} N={w.N} G={G} subbands={sbs} seed={w.seed}")
    x = _input(w)
    xg = torch.empty((w.S, 2, w.SB, w.N + G, 2), dtype=x.dtype, device="cuda")
    xg[:, :, :, :w.N].copy_(x)
    xg[:, :, :, w.N:].copy_(x[:, :, :, :G])             # the guard repeats the block's first samples
    del x
    offs = np.random.default_rng([w.seed, 0xC0]).integers(0, G + 1, w.S).astype(np.int32)
    fl = synth.lost_sample_flags(w.seed, w.S, w.SB, w.N + G, p_packet=0.002, p_sample=0.0)
    fd = torch.from_numpy(synth.pack_flags(fl).view(np.int32)).to("cuda")
    with binding.plan_for(w) as plan:
        wts = torch.full(plan.weights_shape(), -1, dtype=torch.int32, device="cuda")
        vis = plan.correlate_ex(xg, w.delays(0), coarse=offs, flags=fd, weights=wts)
        torch.cuda.synchronize()
        Vg = vis[sbs].cpu().numpy()
        Wg = wts[sbs].cpu().numpy()
    del xg, fd, vis
    blk = w.block(0, subbands=sbs)
    rows = np.concatenate([blk, blk[:, :, :, :G]], axis=3)
    hist = np.zeros((w.S, 2, len(sbs), 15 * w.C), np.complex128)
    hrow = np.zeros((w.S, len(sbs), 15), bool)
    o = oflags.fx_block_flagged(synth.to_complex(rows), w.N, offs, fl[:, sbs], hist, hrow, w.fir(), w.bandpass(),
                                w.subband_freqs()[sbs], synth.SAMPLE_RATE_HZ, w.delays(0), w.C, 16,
                                mode=MODE[w.x_mode], gain=w.gain())
    _say(f"  lost {float(fl.mean()):.4%} of the samples, weights min {Wg.min()} of {w.n_c}")
    np.testing.assert_array_equal(Wg, o["W"])
    rms = np.sqrt(np.mean(np.abs(o["Z"]) ** 2))
    eps = _eps(vis_complex(Vg), o["V"], w.S, o["W"], rms)
    _say(f"  eps {eps:.3e}")
    assert eps <= EPS_FP16


def test_full_size_beamformer_on_sampled_subbands():
    from paper_1801_04834_amd import binding
    from oracle import beam as obeam
    w = synth.Workload(name="beam_share", S=48, SB=61, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, C=256,
                       sigma=64.0, seed=1807, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05,
                       fp16_prescale_log2=-1)
    NB, n_int = 127, 16
    sbs = [0, w.SB // 2, w.SB - 1]
    _say(f"CASE fullsize beamformer S={w.S} SB={w.SB} C={w.C} NB={NB} n_int={n_int} subbands={sbs} seed={w.seed}")
    dtau = np.random.default_rng(1808).uniform(-2e-6, 2e-6, (NB, w.S))
    x = _input(w)
    with binding.plan_for(w) as plan:
        cs, _, isz = plan.beam_shapes(NB, 1, n_int)
        coh = torch.full(cs, np.nan, dtype=torch.float32, device="cuda")
        inc = torch.full(isz, np.nan, dtype=torch.float32, device="cuda")
        chan = plan.channelize(x, w.delays(0))
        plan.beamform_channelized(chan, torch.from_numpy(dtau).cuda(), 1, n_int, coherent=coh, incoherent=inc)
        torch.cuda.synchronize()
        del x, chan
        cg = coh[sbs].cpu().numpy().transpose(0, 1, 4, 3, 2)      # -> [SB, C, NB, 1, n_out]
        ig = inc[sbs].cpu().numpy().transpose(0, 1, 3, 2)         # -> [SB, C, 1, n_out]
    hist = np.zeros((w.S, 2, len(sbs), 15 * w.C), np.complex128)
    o = obeam.beamform_block(synth.to_complex(w.block(0, subbands=sbs)), hist, w.fir(), w.bandpass(),
                             w.subband_freqs()[sbs], synth.SAMPLE_RATE_HZ, w.delays(0), dtau, w.C, 16, which="I",
                             n_int=n_int)
    for name, got, want in (("coherent", cg, o["coherent"]), ("incoherent", ig, o["incoherent"])):
        err = np.abs(got.astype(np.float64) - want)
        worst = float(np.max(err / (np.abs(want) + np.mean(np.abs(want)))))
        _say(f"  {name}: worst {worst:.3e}")
        assert np.all(err <= 2e-5 * np.abs(want) + 1e-6 * np.mean(np.abs(want))), f"{name} off, worst {worst:.3e}"


def test_full_size_output_resolution_on_sampled_rows():
    """The output-resolution transform at the benchmark's size and launch configuration (61
    subbands x 768 channel samples, 127 beams in rows padded to 128, 256 -> 16 channels, Stokes I
    over 16 output samples, and the transformed voltages): sampled (subband, channel sample)
    rows against the oracle's transform of the same voltages, row by row (FP32 transform error
    only: voltages <= 2e-6 of the rms, Stokes |dS| <= 4e-5 I + 1e-6 mean(I))."""
    from paper_1801_04834_amd import binding
    from oracle import beam as obeam
    w = synth.Workload(name="beam_share", S=48, SB=61, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, C=256,
                       sigma=64.0, seed=1807, fp16_prescale_log2=-1)
    NB, NBS, c_out, n_int = 127, 128, 16, 16
    rng = np.random.default_rng(4101)
    rows = [(int(rng.integers(w.SB)), int(rng.integers(w.n_c))) for _ in range(6)] + [(0, 0), (w.SB - 1, w.n_c - 1)]
    _say(f"CASE fullsize transform SB={w.SB} n_c={w.n_c} NB={NB} stride={NBS} c_out={c_out} n_int={n_int} rows={rows}")
    with binding.plan_for(w) as plan:
        _, vs, _ = plan.beam_shapes(NB, 1, 1, voltage_stride=NBS)
        g = torch.Generator(device="cuda").manual_seed(4102)
        volt = torch.randn(vs, generator=g, dtype=torch.float32, device="cuda")
        ov, osk = plan.transform_shapes(NB, c_out, 1, n_int, voltage_stride=NBS)
        tv = torch.full(ov, np.nan, dtype=torch.float32, device="cuda")
        ts = torch.full(osk, np.nan, dtype=torch.float32, device="cuda")
        plan.beam_transform(volt, c_out, 1, n_int, out_voltages=tv, out_stokes=ts, n_beams=NB)
        torch.cuda.synchronize()
        per = w.C // c_out                           # output samples per channel sample
        for sb, j in rows:
            v = volt[sb, :, j, :, :NB].cpu().numpy().astype(np.float64)           # [C, P, NB, 2]
            B = np.transpose(v[..., 0] + 1j * v[..., 1], (2, 1, 0))[..., None]    # [NB, P, C, 1]
            ref = obeam.resolution_transform(B, c_out)                            # [NB, P, per, c_out]
            got = tv[sb, j * per:(j + 1) * per, :, :, :NB].cpu().numpy().astype(np.float64)
            got = np.transpose(got[..., 0] + 1j * got[..., 1], (3, 2, 0, 1))      # [NB, P, per, c_out]
            rms = np.sqrt(np.mean(np.abs(ref) ** 2))
            e = float(np.max(np.abs(got - ref))) / rms
            st = obeam.transformed_stokes(B, c_out, "I", n_int)                   # [NB, per/n_int, c_out, 1]
            sg = ts[sb, j * per // n_int:(j + 1) * per // n_int].cpu().numpy().astype(np.float64)
            sg = np.transpose(sg, (3, 0, 1, 2))                                   # [NB, per/n_int, c_out, 1]
            err = np.abs(sg - st)
            worst = float(np.max(err / (np.abs(st) + np.mean(np.abs(st)))))
            _say(f"  row (sb {sb}, j {j}): voltages {e:.2e} rms, Stokes worst {worst:.2e}")
            assert e <= 2e-6
            assert np.all(err <= 4e-5 * np.abs(st) + 1e-6 * np.mean(np.abs(st)))
        assert bool(torch.isfinite(ts).all())
