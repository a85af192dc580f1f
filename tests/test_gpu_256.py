"""GPU parity at 256 channels per subband (the beamformer front end and the correlator's
finest resolution), through the C ABI, against the FP64 oracle.

Same tolerances as the 64-channel tests: channelised data 5e-6 rms + 2e-6 |Z| (float
modes), int8 +-1 only at rounding boundaries, coherence error <= 1e-5 for FP16-split / FP32
visibilities and bit-exact int8 X stage on the GPU's own int8 stream.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import synth
from tests.layout import unblock, unblock_planes
from tests.metrics import coherence_error, near_rounding_boundary, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C = 256
MODE = {synth.X_FP32: "fp32", synth.X_FP16_SPLIT: "fp16_split", synth.X_INT8: "int8"}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _work(S, SB, n_c, st, mode, seed):
    return synth.Workload(name="c256", S=S, SB=SB, sample_type=st, x_mode=mode, N=C * n_c, C=C,
                          sigma=16.0 if st == synth.CI8 else 64.0, seed=seed, delay_spread_s=5e-6,
                          delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1 if mode == synth.X_FP16_SPLIT else 0)


def _oracle_run(w, blocks):
    hist = np.zeros((w.S, 2, w.SB, 15 * C), np.complex128)
    outs = []
    for k, x in enumerate(blocks):
        o = oracle.fx_block(synth.to_complex(x), hist, w.fir(), w.bandpass(), w.subband_freqs(), synth.SAMPLE_RATE_HZ,
                            w.delays(k), C, 16, mode=MODE[w.x_mode], gain=w.gain())
        hist = o["history"]
        outs.append(o)
    return outs


@pytest.mark.parametrize("st", [synth.CI16, synth.CI8, synth.CF32])
@pytest.mark.parametrize("mode", [synth.X_FP16_SPLIT, synth.X_FP32, synth.X_INT8])
@pytest.mark.parametrize("n_c", [40, 300])
def test_256_channels_match_oracle(st, mode, n_c):
    from paper_1801_04834_amd import binding
    w = _work(3, 2, n_c, st, mode, 2500 + n_c + 10 * st + mode)
    _say(f"CASE c256 st={st} mode={mode} S={w.S} SB={w.SB} n_c={n_c} seed={w.seed}")
    blocks = [w.block(k) for k in range(2)]
    outs = _oracle_run(w, blocks)
    with binding.plan_for(w) as plan, binding.plan_for(w) as plan2:
        assert plan.chan_shape[1] == C
        for k in range(2):
            x = torch.from_numpy(blocks[k]).cuda()
            chan = plan.channelize(x, w.delays(k))
            vis = plan.correlate_channelized(chan)
            vis2 = plan2.correlate(x, w.delays(k))
            torch.cuda.synchronize()
            assert torch.equal(vis, vis2)
            c = chan.cpu().numpy()
            o = outs[k]
            if mode == synth.X_INT8:
                r = unblock(c)
                assert np.all(r[..., n_c:, :] == 0)
                Qg = r[..., :n_c, :]
                d = Qg.astype(np.int64) - o["Q"].astype(np.int64)
                bad = d != 0
                g = np.float64(np.float32(w.gain()))
                pre = np.stack([(g * o["Zf"].real).astype(np.float32), (g * o["Zf"].imag).astype(np.float32)], -1)
                _say(f"  block {k}: int8 mismatches {int(bad.sum())} of {d.size}")
                assert np.all(np.abs(d) <= 1) and np.all(near_rounding_boundary(pre, 1e-3)[bad])
                np.testing.assert_array_equal(vis.cpu().numpy().astype(np.int64),
                                              oracle.correlate_int(np.ascontiguousarray(Qg), w.S))
                continue
            if mode == synth.X_FP16_SPLIT:
                hi, lo = unblock_planes(c)
                v = (hi.astype(np.float64) + lo.astype(np.float64)) * 2.0 ** (-w.fp16_prescale_log2)
            else:
                v = unblock(c).astype(np.float64)
            Zg = (v[..., 0] + 1j * v[..., 1])[..., :n_c]
            rms = np.sqrt(np.mean(np.abs(o["Z"]) ** 2))
            err = np.abs(Zg - o["Z"])
            worst = float(np.max(err / (rms + np.abs(o["Z"]))))
            eps = coherence_error(vis_complex(vis.cpu().numpy()), o["V"], w.S)
            _say(f"  block {k}: chan worst {worst:.3e}  eps {eps:.3e}")
            assert np.all(err <= 5e-6 * rms + 2e-6 * np.abs(o["Z"]))
            assert eps <= 1e-5


def test_256_channel_tone_lands_in_its_channel():
    """A bin-centred tone at channel 201 of 256: the auto power of that channel dominates
    and equals N_c A^2 (sum h)^2 b^2 within FP32 error (zero delays, history warmed)."""
    from paper_1801_04834_amd import binding
    n_c, A, c0 = 64, 300.0, 201
    w = synth.Workload(name="tone256", S=2, SB=1, sample_type=synth.CF32, x_mode=synth.X_FP32, N=C * n_c, C=C,
                       sigma=0.0, seed=1, tone_amplitude=A, tone_channel=c0)
    _say(f"CASE c256 tone c0={c0}")
    with binding.plan_for(w) as plan:
        x0, x1 = torch.from_numpy(w.block(0)).cuda(), torch.from_numpy(w.block(1)).cuda()
        plan.correlate(x0, w.delays(0))
        V = vis_complex(plan.correlate(x1, w.delays(1)).cpu().numpy())[0]     # [C, B, 4]
        torch.cuda.synchronize()
    h = w.fir().astype(np.float64)
    want = n_c * A ** 2 * h.sum() ** 2
    auto = V[:, 0, 0].real
    assert int(np.argmax(auto)) == c0
    assert abs(auto[c0] - want) <= 1e-4 * want


def test_256_channel_flags_drop_whole_fir_windows():
    """One lost sample of station 0 at 256 channels: exactly the T = 16 channel samples whose
    window (16 rows of 256 samples) holds it are zero, station 0's baselines keep N_c - 16
    valid channel samples and the others all N_c (closed form; the flag path against the
    oracle at 256 channels is in the flag tests)."""
    from paper_1801_04834_amd import binding
    w = _work(2, 1, 40, synth.CI16, synth.X_FP16_SPLIT, 2590)
    _say("CASE c256 one lost sample")
    G, g0, lost = 3, 1, 10 * C + 77                   # sample 77 of row 10 of station 0's window
    with binding.plan_for(w) as plan:
        x = torch.from_numpy(synth.guarded_rows(w, 0, G)).cuda()
        fl = np.zeros((w.S, w.SB, w.N + G), bool)
        fl[0, 0, g0 + lost] = True
        fd = torch.from_numpy(synth.pack_flags(fl).view(np.int32)).cuda()
        wts = torch.zeros(plan.weights_shape(), dtype=torch.int32, device="cuda")
        chan = plan.channelize_ex(x, w.delays(0), coarse=np.array([g0, 0], np.int32), flags=fd, weights=wts)
        torch.cuda.synchronize()
        hi, lo = unblock_planes(chan.cpu().numpy())
        z0 = (hi[0, :, 0:2, :40] != 0).any(axis=(0, 1, 3))       # station 0, any channel / pol
        assert not z0[10:26].any() and z0[:10].all() and z0[26:].all()
        assert (hi[0, :, 2:4, :40] != 0).any(axis=(0, 1, 3)).all()
        np.testing.assert_array_equal(wts.cpu().numpy()[0], [40 - 16, 40 - 16, 40])
