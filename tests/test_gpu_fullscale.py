"""GPU parity on full-scale input in FP16-split mode: the largest channel samples valid 8/16-bit
input can produce stay finite and within tolerance.

The plan takes the largest prescale the library admits for the setting
(``cobalt_fp16_prescale_max``).  Four stations (``synth.full_scale_streams``): windows matched
to the signs of the taps at +-A (1 + i), with a delay that turns the DC channel's phase onto the
real axis so that one component reaches the bound; a full-scale tone over noise; full-scale
random signs; noise with a tone of A/16 (strong interference).  Every station carries a noise
floor, so every channel's autocorrelation is far from zero and the coherence error measures the
arithmetic rather than a division by an empty channel.  Two consecutive full-length blocks
(196 608 samples, history carried).
Checks: channelised hi/lo planes finite and equal to the oracle's Z within the channelised
tolerance, visibilities finite with coherence error <= 1e-5.  Float samples beyond the bound
saturate at +-65504 instead of becoming infinite.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import synth
from tests.layout import unblock_planes
from tests.metrics import coherence_error, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS_FP16 = 1e-5
FP16_MAX = 65504.0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _kw(st, C, n_c, k=None):
    from paper_1801_04834_amd import binding
    w = synth.Workload(name="fullscale", S=4, SB=1, sample_type=st, x_mode=synth.X_FP16_SPLIT, N=C * n_c, C=C,
                       ripple=0.05, f_sb0=150e6)
    kw = binding.plan_kwargs(w)
    kw["fp16_prescale_log2"] = binding.fp16_prescale_max(**kw) if k is None else k
    return w, kw


def _delays(f_sb):
    d = np.zeros((4, 2))
    d[0, :] = -1.0 / (8.0 * f_sb)              # DC-channel phase of (1 + i) -> real axis
    d[1, :] = 1.3e-6
    d[2, :] = (-0.7e-6, -0.69e-6)
    d[3, :] = 2.1e-6
    return d


@pytest.mark.parametrize("st,C", [(synth.CI16, 64), (synth.CI8, 64), (synth.CI16, 256)])
def test_full_scale_block_stays_finite_and_matches_oracle(st, C):
    from paper_1801_04834_amd import binding
    n_c = synth.BLOCK_SAMPLES // C
    w, kw = _kw(st, C, n_c)
    k = kw["fp16_prescale_log2"]
    d = _delays(150e6)
    _say(f"CASE fullscale st={st} C={C} n_c={n_c} k={k} blocks=2")
    hist = np.zeros((4, 2, 1, 15 * C), np.complex128)
    with binding.Plan(**kw) as plan:
        for blk in range(2):
            x = synth.full_scale_streams(w.fir(), C, 16, w.N, seed=21, sample_type=st, block=blk)
            xd = torch.from_numpy(x).cuda()
            ref = oracle.fx_block(synth.to_complex(x), hist, w.fir(), w.bandpass(), w.subband_freqs(),
                                  synth.SAMPLE_RATE_HZ, d, C, 16, mode="fp16_split")
            hist = ref["history"]
            chan = plan.channelize(xd, d)
            vis = plan.correlate_channelized(chan)
            torch.cuda.synchronize()
            hi, lo = unblock_planes(chan.cpu().numpy())
            assert np.all(np.isfinite(hi.astype(np.float32))) and np.all(np.isfinite(lo.astype(np.float32)))
            v = (hi.astype(np.float64) + lo.astype(np.float64)) * 2.0 ** (-k)
            Zg = (v[..., 0] + 1j * v[..., 1])[..., :n_c]
            Z = ref["Z"]
            peak = float(np.max(np.maximum(np.abs(Z.real), np.abs(Z.imag)))) * 2.0 ** k
            rms = np.sqrt(np.mean(np.abs(Z) ** 2))
            err = np.abs(Zg - Z)
            worst = float(np.max(err / (rms + np.abs(Z))))
            V = vis_complex(vis.cpu().numpy())
            eps = coherence_error(V, ref["V"], 4)
            _say(f"  block {blk}: largest stored component {peak:.1f} (limit {FP16_MAX:.0f}), "
                 f"channelised worst {worst:.3e}, eps {eps:.3e}")
            assert peak <= FP16_MAX
            assert np.all(err <= 5e-6 * rms + 2e-6 * np.abs(Z)), f"channelised worst {worst:.3e}"
            assert np.all(np.isfinite(V))
            assert eps <= EPS_FP16


def test_float_samples_beyond_the_bound_saturate():
    """CF32 input 4x full scale at k = 0: components above 65504 are stored as +-65504 with a
    zero lo part, the rest as usual; nothing is infinite."""
    from paper_1801_04834_amd import binding
    C, n_c = 64, 64
    w = synth.Workload(name="fullscale_f32", S=4, SB=1, sample_type=synth.CF32, x_mode=synth.X_FP16_SPLIT,
                       N=C * n_c, ripple=0.05, f_sb0=150e6, fp16_prescale_log2=0)
    x = synth.full_scale_streams(w.fir(), C, 16, w.N, seed=22, sample_type=synth.CI16).astype(np.float32) * 4
    d = _delays(150e6)
    _say(f"CASE fullscale cf32 saturation n_c={n_c} k=0")
    ref = oracle.fx_block(synth.to_complex(x), np.zeros((4, 2, 1, 15 * C), np.complex128), w.fir(), w.bandpass(),
                          w.subband_freqs(), synth.SAMPLE_RATE_HZ, d, C, 16, mode="fp16_split")
    with binding.plan_for(w) as plan:
        chan = plan.channelize(torch.from_numpy(x).cuda(), d)
        vis = plan.correlate_channelized(chan)
        torch.cuda.synchronize()
        hi, lo = unblock_planes(chan.cpu().numpy())
        V = vis_complex(vis.cpu().numpy())
    hi = hi[..., :n_c, :].astype(np.float64)
    lo = lo[..., :n_c, :].astype(np.float64)
    Z = ref["Z"]
    Zc = np.stack([Z.real, Z.imag], axis=-1)
    over = np.abs(Zc) > FP16_MAX * (1 + 1e-5)
    under = np.abs(Zc) < FP16_MAX * (1 - 1e-5)
    _say(f"  components above 65504: {int(over.sum())} of {over.size}")
    assert over.sum() > 0
    assert np.all(np.isfinite(hi)) and np.all(np.isfinite(lo)) and np.all(np.isfinite(V))
    assert np.all(hi[over] == np.sign(Zc[over]) * FP16_MAX) and np.all(lo[over] == 0.0)
    rms = np.sqrt(np.mean(np.abs(Z) ** 2))
    assert np.all(np.abs((hi + lo)[under] - Zc[under]) <= 5e-6 * rms + 2e-6 * np.abs(Zc[under]))
