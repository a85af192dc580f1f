"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every case prints its name, sizes and seed before touching the GPU.  Inputs come from
``paper_1801_04834_amd.synth``; expected values come from ``oracle`` only.

Tolerances:
* FP16-split mode: coherence error eps <= 1e-5 (the required 16-bit-mode bound).
* FP32 mode: eps <= 1e-6.  The X stage sums products over 128 channel samples into partial
  sums that are folded into running totals, which leaves a relative error of about
  u (128 / sqrt(N_c) + sqrt(N_c / 128)) / 6 (u = 2^-24): ~8e-8 rms at N_c = 3072, a few
  times that at the maximum over all entries (a single running sum would leave ~9e-7 rms).
* INT8 mode: the X stage is bit-exact on the same int8 stream; the requantised F output
  equals the oracle's except where the oracle's pre-rounding value lies within 1e-3 of a
  rounding boundary, where it may differ by exactly 1.
* Channelised data: |Z_gpu - Z| <= 5e-6 * rms(Z) + 2e-6 |Z| per element (FP32 / FP16 hi+lo).
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import synth
from tests.layout import block, block_planes, unblock, unblock_planes
from tests.metrics import coherence_error, frobenius_rel, near_rounding_boundary, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS_FP16 = 1e-5
EPS_FP32 = 1e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _binding():
    from paper_1801_04834_amd import binding
    return binding


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _small(name="small", S=3, SB=2, n_c=100, st=synth.CI16, mode=synth.X_FP32, seed=7, sigma=None, **kw):
    sig = sigma if sigma is not None else (16.0 if st == synth.CI8 else 64.0)
    return synth.Workload(name=name, S=S, SB=SB, sample_type=st, x_mode=mode, N=64 * n_c, sigma=sig, seed=seed,
                          delay_spread_s=kw.pop("spread", 5e-6), delay_drift_s=kw.pop("drift", 25e-9),
                          ripple=kw.pop("ripple", 0.05), fp16_prescale_log2=-1 if mode == synth.X_FP16_SPLIT else 0,
                          **kw)


def _oracle_run(w, blocks):
    """Oracle over consecutive blocks (history carried); returns per-block outputs."""
    hist = np.zeros((w.S, 2, w.SB, 15 * 64), np.complex128)
    outs = []
    mode = {synth.X_FP32: "fp32", synth.X_FP16_SPLIT: "fp16_split", synth.X_INT8: "int8"}[w.x_mode]
    for b, x in enumerate(blocks):
        o = oracle.fx_block(synth.to_complex(x), hist, w.fir(), w.bandpass(), w.subband_freqs(),
                            synth.SAMPLE_RATE_HZ, w.delays(b), 64, 16, mode=mode, gain=w.gain())
        hist = o["history"]
        outs.append(o)
    return outs


def _chan_rows(plan, chan):
    """Channelised tensor -> row-major numpy [SB, C, M, pitch, 2] (FP16: (hi, lo))."""
    c = chan.cpu().numpy()
    if plan.x_mode == synth.X_FP16_SPLIT:
        return unblock_planes(c)
    return unblock(c)


def _chan_complex(plan, chan):
    r = _chan_rows(plan, chan)
    if plan.x_mode == synth.X_FP16_SPLIT:
        k = plan.kw.get("fp16_prescale_log2", 0)
        v = (r[0].astype(np.float64) + r[1].astype(np.float64)) * 2.0 ** (-k)
    else:
        v = r.astype(np.float64)
    return (v[..., 0] + 1j * v[..., 1])[..., :plan.n_c]


def _check_chan_float(Zg, Z, label):
    rms = np.sqrt(np.mean(np.abs(Z) ** 2))
    err = np.abs(Zg - Z)
    bound = 5e-6 * rms + 2e-6 * np.abs(Z)
    worst = float(np.max(err / (rms + np.abs(Z))))
    _say(f"  {label}: max |dZ|/(rms+|Z|) = {worst:.3e}")
    assert np.all(err <= bound), f"{label}: channelised mismatch, worst {worst:.3e}"


def _check_int8_chan(Qg, out, gain, label, delta=1e-3):
    """Requantised F output vs oracle: equal except +-1 near a rounding boundary."""
    Q = out["Q"].astype(np.int64)
    Zf = out["Zf"]
    g = np.float64(np.float32(gain))
    pre = np.stack([(g * Zf.real).astype(np.float32), (g * Zf.imag).astype(np.float32)], axis=-1)
    diff = Qg.astype(np.int64) - Q
    bad = diff != 0
    amb = near_rounding_boundary(pre, delta)
    n_bad = int(bad.sum())
    _say(f"  {label}: int8 mismatches {n_bad} of {Q.size} (ambiguous {int(amb.sum())})")
    assert np.all(np.abs(diff) <= 1)
    assert np.all(amb[bad]), f"{label}: mismatch away from a rounding boundary"
    return bad


# ---------------------------------------------------------------- F stage ---------------

@pytest.mark.parametrize("st", [synth.CI16, synth.CI8, synth.CF32])
@pytest.mark.parametrize("mode", [synth.X_FP32, synth.X_FP16_SPLIT, synth.X_INT8])
@pytest.mark.parametrize("n_c", [100, 600])
def test_channelize_matches_oracle_two_blocks(st, mode, n_c):
    w = _small(S=3, SB=2, n_c=n_c, st=st, mode=mode, seed=11 + n_c)
    if st == synth.CI8 and mode != synth.X_INT8:
        w.sigma = 16.0
    _say(f"CASE channelize st={st} mode={mode} S={w.S} SB={w.SB} n_c={n_c} seed={w.seed}")
    blocks = [w.block(b) for b in range(2)]
    outs = _oracle_run(w, blocks)
    b = _binding()
    with b.plan_for(w) as plan:
        for k in range(2):
            chan = plan.channelize(_to_dev(blocks[k]), w.delays(k))
            torch.cuda.synchronize()
            rows = _chan_rows(plan, chan)
            if plan.x_mode == synth.X_INT8:
                assert np.all(rows[..., plan.n_c:, :] == 0)
                _check_int8_chan(rows[..., :plan.n_c, :], outs[k], w.gain(), f"block {k}")
            else:
                for r in (rows if plan.x_mode == synth.X_FP16_SPLIT else (rows,)):
                    assert np.all(r[..., plan.n_c:, :] == 0)
                _check_chan_float(_chan_complex(plan, chan), outs[k]["Z"], f"block {k}")


# ---------------------------------------------------------------- X stage only ----------

@pytest.mark.parametrize("S,n_c", [(1, 64), (3, 100), (8, 3072), (16, 96), (24, 70), (44, 130), (60, 96), (76, 128),
                                   (80, 160)])
def test_x_int8_bit_exact(S, n_c):
    _say(f"CASE x_int8 S={S} n_c={n_c}")
    b = _binding()
    w = _small(S=S, SB=1, n_c=n_c, st=synth.CI8, mode=synth.X_INT8)
    with b.plan_for(w) as plan:
        q = synth.int8_channelised(seed=S * 1000 + n_c, n_chan=64, M=2 * S, n_c=n_c, pitch=plan.pitch)
        chan = _to_dev(block(q).reshape(plan.chan_shape))
        V = plan.correlate_channelized(chan)
        torch.cuda.synchronize()
        ref = oracle.correlate_int(q[:, :, :n_c, :], S)              # [64, B, 4, 2]
        got = V.cpu().numpy().reshape(ref.shape).astype(np.int64)
        assert np.array_equal(got, ref)


def test_x_int8_overflow_bound_extremes():
    """All samples +-127 at the largest integration the int32 sums admit."""
    S, n_c = 4, 66560
    _say(f"CASE x_int8_extreme S={S} n_c={n_c}")
    b = _binding()
    w = _small(S=S, SB=1, n_c=n_c, st=synth.CI8, mode=synth.X_INT8)
    with b.plan_for(w) as plan:
        q = synth.int8_channelised(seed=3, n_chan=64, M=2 * S, n_c=n_c, pitch=plan.pitch, extreme=True)
        V = plan.correlate_channelized(_to_dev(block(q).reshape(plan.chan_shape)))
        torch.cuda.synchronize()
        ref = oracle.correlate_int(q[:, :, :n_c, :], S)
        got = V.cpu().numpy().reshape(ref.shape).astype(np.int64)
        assert np.array_equal(got, ref)
        assert got[:, 0, 0, 0].max() == n_c * 2 * 127 ** 2


@pytest.mark.parametrize("S,n_c", [(1, 32), (3, 100), (8, 1000), (24, 70), (40, 96), (60, 130), (76, 256), (80, 64)])
def test_x_fp16_split_matches_oracle(S, n_c):
    _say(f"CASE x_fp16 S={S} n_c={n_c}")
    b = _binding()
    k = -1  # the plan's prescale (the largest safe one for 16-bit input with these taps)
    w = _small(S=S, SB=1, n_c=n_c, st=synth.CI16, mode=synth.X_FP16_SPLIT)
    with b.plan_for(w) as plan:
        Z = synth.float_channelised(seed=S + n_c, n_chan=64, M=2 * S, n_c=n_c, sigma=7.7)
        # the hi/lo planes of 2^k Z (input construction; the oracle sees hi + lo exactly)
        zs = np.stack([Z.real, Z.imag], -1) * 2.0 ** k
        hi = zs.astype(np.float16)
        lo = (zs - hi.astype(np.float64)).astype(np.float16)
        hip_ = np.zeros((64, 2 * S, plan.pitch, 2), np.float16)
        lop_ = np.zeros((64, 2 * S, plan.pitch, 2), np.float16)
        hip_[:, :, :n_c] = hi
        lop_[:, :, :n_c] = lo
        planes = block_planes(hip_, lop_)
        exact = (hi.astype(np.float64) + lo.astype(np.float64)) * 2.0 ** (-k)
        Zx = exact[..., 0] + 1j * exact[..., 1]
        V = plan.correlate_channelized(_to_dev(planes.reshape(plan.chan_shape)))
        torch.cuda.synchronize()
        ref = oracle.correlate(Zx, S)
        got = vis_complex(V.cpu().numpy()).reshape(ref.shape)
        eps = coherence_error(got, ref, S)
        _say(f"  eps={eps:.3e} frob={frobenius_rel(got, ref):.3e}")
        assert eps <= EPS_FP16


@pytest.mark.parametrize("S,n_c", [(1, 16), (3, 100), (8, 3072), (20, 77), (76, 64), (128, 48)])
def test_x_fp32_matches_oracle(S, n_c):
    _say(f"CASE x_fp32 S={S} n_c={n_c}")
    b = _binding()
    w = _small(S=S, SB=1, n_c=n_c, st=synth.CI16, mode=synth.X_FP32)
    with b.plan_for(w) as plan:
        Z = synth.float_channelised(seed=S * 7 + n_c, n_chan=64, M=2 * S, n_c=n_c)
        buf = np.zeros((64, 2 * S, plan.pitch, 2), np.float32)
        buf[:, :, :n_c, 0] = Z.real
        buf[:, :, :n_c, 1] = Z.imag
        V = plan.correlate_channelized(_to_dev(block(buf).reshape(plan.chan_shape)))
        torch.cuda.synchronize()
        ref = oracle.correlate(Z, S)
        got = vis_complex(V.cpu().numpy()).reshape(ref.shape)
        eps = coherence_error(got, ref, S)
        _say(f"  eps={eps:.3e}")
        assert eps <= EPS_FP32


def test_x_ignores_columns_beyond_n_c():
    """Positions in [N_c, pitch) of a caller buffer do not enter the sums."""
    S, n_c = 5, 70
    b = _binding()
    rng = np.random.default_rng(0)
    for mode in (synth.X_FP32, synth.X_FP16_SPLIT, synth.X_INT8):
        _say(f"CASE x_pad mode={mode}")
        st = synth.CI8 if mode == synth.X_INT8 else synth.CI16
        w = _small(S=S, SB=1, n_c=n_c, st=st, mode=mode)
        with b.plan_for(w) as plan:
            dt = {synth.X_FP32: np.float32, synth.X_FP16_SPLIT: np.float16, synth.X_INT8: np.int8}[mode]
            rows = [np.rint(rng.uniform(-3, 3, (64, 2 * S, plan.pitch, 2))).astype(dt) for _ in range(2)]
            bufs = []
            for fill in (0, 5):
                rr = [r.copy() for r in rows]
                for r in rr:
                    r[..., n_c:, :] = fill
                arr = block_planes(*rr) if mode == synth.X_FP16_SPLIT else block(rr[0])
                bufs.append(_to_dev(arr.reshape(plan.chan_shape)))
            v1 = plan.correlate_channelized(bufs[0])
            v2 = plan.correlate_channelized(bufs[1])
            torch.cuda.synchronize()
            assert torch.equal(v1, v2)


# ---------------------------------------------------------------- full chain ------------

@pytest.mark.parametrize("mode", [synth.X_FP32, synth.X_FP16_SPLIT])
@pytest.mark.parametrize("st", [synth.CI16, synth.CF32])
def test_correlate_full_chain_float_modes(mode, st):
    w = _small(S=4, SB=2, n_c=300, st=st, mode=mode, seed=23)
    _say(f"CASE full_chain st={st} mode={mode} S={w.S} SB={w.SB} n_c={w.n_c}")
    blocks = [w.block(k) for k in range(2)]
    outs = _oracle_run(w, blocks)
    b = _binding()
    with b.plan_for(w) as plan:
        for k in range(2):
            V = plan.correlate(_to_dev(blocks[k]), w.delays(k))
            torch.cuda.synchronize()
            got = vis_complex(V.cpu().numpy())
            eps = coherence_error(got, outs[k]["V"], w.S)
            _say(f"  block {k}: eps={eps:.3e} frob={frobenius_rel(got, outs[k]['V']):.3e}")
            assert eps <= (EPS_FP16 if mode == synth.X_FP16_SPLIT else EPS_FP32)


def test_correlate_full_chain_int8():
    w = _small(S=4, SB=2, n_c=300, st=synth.CI8, mode=synth.X_INT8, seed=29)
    _say(f"CASE full_chain int8 S={w.S} SB={w.SB} n_c={w.n_c}")
    blocks = [w.block(k) for k in range(2)]
    outs = _oracle_run(w, blocks)
    b = _binding()
    with b.plan_for(w) as plan:
        for k in range(2):
            V = plan.correlate(_to_dev(blocks[k]), w.delays(k))
            torch.cuda.synchronize()
            got = V.cpu().numpy().astype(np.int64)                 # [SB, C, B, 4, 2]
            ref = outs[k]["V"]
            # which inputs hold elements the oracle itself marks as rounding-ambiguous
            g = np.float64(np.float32(w.gain()))
            Zf = outs[k]["Zf"]                                     # [SB, C, M, N_c]
            pre = np.stack([(g * Zf.real).astype(np.float32), (g * Zf.imag).astype(np.float32)], -1)
            amb_count = near_rounding_boundary(pre, 1e-3).any(-1).sum(-1)    # [SB, C, M]
            exact = 0
            for s1 in range(w.S):
                for s2 in range(s1 + 1):
                    bl = s1 * (s1 + 1) // 2 + s2
                    for p1 in range(2):
                        for p2 in range(2):
                            a, bb = 2 * s1 + p1, 2 * s2 + p2
                            n_amb = amb_count[:, :, a] + (amb_count[:, :, bb] if bb != a else 0)
                            d = np.abs(got[:, :, bl, 2 * p1 + p2] - ref[:, :, bl, 2 * p1 + p2]).max(-1)
                            # one flipped component moves a product sum by at most 2*127+1
                            assert np.all(d <= 2 * (2 * 127 + 1) * n_amb)
                            assert np.all(d[n_amb == 0] == 0)
                            exact += int((n_amb == 0).sum())
            _say(f"  block {k}: entries with no ambiguous input: {exact} (bit-exact)")


def test_correlate_equals_channelize_then_x():
    """cobalt_correlate is the F stage followed by the X stage (bit-identical)."""
    for mode in (synth.X_FP32, synth.X_FP16_SPLIT, synth.X_INT8):
        st = synth.CI8 if mode == synth.X_INT8 else synth.CI16
        w = _small(S=6, SB=2, n_c=256, st=st, mode=mode, seed=31)
        _say(f"CASE composition mode={mode}")
        b = _binding()
        x = _to_dev(w.block(0))
        with b.plan_for(w) as p1, b.plan_for(w) as p2:
            v1 = p1.correlate(x, w.delays(0))
            v2 = p2.correlate_channelized(p2.channelize(x, w.delays(0)))
            torch.cuda.synchronize()
            assert torch.equal(v1, v2)


def test_tone_lands_in_channel_with_fir_gain():
    """cf32 tone, continuous over the history: |Z(c0)| = A * sum(h) with zero delays and a
    flat bandpass; the autocorrelation there is N_c A^2 (sum h)^2 (closed form)."""
    A, c0, n_c = 256.0, 37, 200
    w = synth.Workload(name="tone", S=2, SB=1, sample_type=synth.CF32, x_mode=synth.X_FP32, N=64 * n_c,
                       sigma=0.0, tone_amplitude=A, tone_channel=c0, f_sb0=150e6)
    _say(f"CASE tone c0={c0} n_c={n_c}")
    b = _binding()
    h = w.fir().astype(np.float64)
    H0 = h.sum()
    with b.plan_for(w) as plan:
        plan.channelize(_to_dev(w.block(0)), w.delays(0))            # warm-up block (zero history)
        chan = plan.channelize(_to_dev(w.block(1)), w.delays(1))
        torch.cuda.synchronize()
        Z = _chan_complex(plan, chan)[0]                               # [C, M, n_c]
        mag = np.abs(Z[c0])
        np.testing.assert_allclose(mag, A * H0, rtol=2e-6)
        others = np.delete(np.abs(Z), c0, axis=0)
        assert others.max() < 1e-3 * A
        V = plan.correlate(_to_dev(w.block(2)), w.delays(2))
        torch.cuda.synchronize()
        auto = V.cpu().numpy()[0, c0, 0, 0, 0]
        assert abs(auto - n_c * A ** 2 * H0 ** 2) <= 2e-6 * n_c * A ** 2 * H0 ** 2


def test_plain_fx_configuration_matches_oracle():
    """The plain FX workload (8 stations, 1 subband, ci16 + tone at channel 37, full
    196608-sample block, FP32 X stage), two consecutive blocks."""
    w = synth.workload("plain_fx")
    _say(f"CASE plain_fx S={w.S} N={w.N}")
    blocks = [w.block(k) for k in range(2)]
    outs = _oracle_run(w, blocks)
    b = _binding()
    with b.plan_for(w) as plan:
        for k in range(2):
            V = plan.correlate(_to_dev(blocks[k]), w.delays(k))
            torch.cuda.synchronize()
            got = vis_complex(V.cpu().numpy())
            eps = coherence_error(got, outs[k]["V"], w.S)
            _say(f"  block {k}: eps={eps:.3e}")
            assert eps <= EPS_FP32
            # tone channel: autos carry the tone power, phase 0 across stations
            auto = got[0, w.tone_channel, 0, 0].real
            assert auto > 10 * np.median(got[0, :, 0, 0].real)


# ---------------------------------------------------------------- edge cases ------------

def test_empty_block_gives_zero_visibilities_and_keeps_history():
    b = _binding()
    for mode in (synth.X_FP32, synth.X_FP16_SPLIT, synth.X_INT8):
        st = synth.CI8 if mode == synth.X_INT8 else synth.CI16
        w = _small(S=2, SB=1, n_c=0, st=st, mode=mode)
        _say(f"CASE empty mode={mode}")
        with b.plan_for(w) as plan:
            x = torch.zeros(plan.input_shape, dtype=plan.input_dtype, device="cuda")
            out = torch.full(plan.vis_shape, 7, dtype=plan.vis_dtype, device="cuda")
            plan.correlate(x, w.delays(0), out=out)
            torch.cuda.synchronize()
            assert torch.count_nonzero(out).item() == 0


def test_reset_history_restarts_the_stream():
    w = _small(S=2, SB=1, n_c=128, st=synth.CI16, mode=synth.X_FP32, seed=41)
    _say("CASE reset_history")
    b = _binding()
    x0, x1 = _to_dev(w.block(0)), _to_dev(w.block(1))
    with b.plan_for(w) as plan:
        first = plan.correlate(x1, w.delays(0)).clone()
        plan.correlate(x0, w.delays(0))
        carried = plan.correlate(x1, w.delays(0)).clone()
        plan.reset_history()
        again = plan.correlate(x1, w.delays(0))
        torch.cuda.synchronize()
        assert torch.equal(first, again)
        assert not torch.equal(first, carried)


def test_short_block_history_spans_two_blocks():
    """N_c < T-1: the history carried out of a block reaches back into the previous one."""
    w = _small(S=2, SB=1, n_c=6, st=synth.CI16, mode=synth.X_FP32, seed=43)
    _say("CASE short blocks n_c=6")
    blocks = [w.block(k) for k in range(4)]
    outs = _oracle_run(w, blocks)
    b = _binding()
    with b.plan_for(w) as plan:
        for k in range(4):
            chan = plan.channelize(_to_dev(blocks[k]), w.delays(k))
            torch.cuda.synchronize()
            _check_chan_float(_chan_complex(plan, chan), outs[k]["Z"], f"block {k}")


def test_hermitian_and_auto_invariants_on_gpu():
    b = _binding()
    for mode in (synth.X_FP32, synth.X_FP16_SPLIT, synth.X_INT8):
        st = synth.CI8 if mode == synth.X_INT8 else synth.CI16
        w = _small(S=5, SB=1, n_c=200, st=st, mode=mode, seed=47)
        _say(f"CASE invariants mode={mode}")
        with b.plan_for(w) as plan:
            V = plan.correlate(_to_dev(w.block(0)), w.delays(0))
            torch.cuda.synchronize()
            v = V.cpu().numpy()
            for s in range(w.S):
                bl = s * (s + 1) // 2 + s
                assert np.all(v[:, :, bl, 0, 1] == 0) and np.all(v[:, :, bl, 3, 1] == 0)
                assert np.all(v[:, :, bl, 0, 0] >= 0) and np.all(v[:, :, bl, 3, 0] >= 0)
                xy, yx = v[:, :, bl, 1], v[:, :, bl, 2]
                if mode == synth.X_INT8:
                    assert np.array_equal(xy[..., 0], yx[..., 0]) and np.array_equal(xy[..., 1], -yx[..., 1])
                else:
                    scale = np.sqrt(v[:, :, bl, 0, 0] * v[:, :, bl, 3, 0]) + 1e-30
                    assert np.all(np.abs(xy[..., 0] - yx[..., 0]) <= 1e-6 * scale)
                    assert np.all(np.abs(xy[..., 1] + yx[..., 1]) <= 1e-6 * scale)


def test_calls_on_two_streams_are_ordered():
    """A plan used on two streams in turn gives the same results as on one stream."""
    w = _small(S=3, SB=1, n_c=256, st=synth.CI16, mode=synth.X_FP16_SPLIT, seed=53)
    _say("CASE two streams")
    b = _binding()
    xs = [_to_dev(w.block(k)) for k in range(4)]
    with b.plan_for(w) as p1, b.plan_for(w) as p2:
        ref = [p1.correlate(xs[k], w.delays(k)).clone() for k in range(4)]
        torch.cuda.synchronize()
        s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()
        got = []
        for k in range(4):
            st = s_a if k % 2 == 0 else s_b
            out = torch.empty(p2.vis_shape, dtype=p2.vis_dtype, device="cuda")
            p2.correlate(xs[k], w.delays(k), out=out, stream=st)
            got.append(out)
        torch.cuda.synchronize()
        for k in range(4):
            assert torch.equal(ref[k], got[k])


def test_pipelined_f_and_x_on_two_streams_match_serial():
    """F of block k+1 on one stream overlapping X of block k on another (two channelised
    buffers, events) gives the same visibilities as the serial chain."""
    w = _small(S=6, SB=2, n_c=512, st=synth.CI16, mode=synth.X_FP16_SPLIT, seed=59)
    _say("CASE pipelined two streams")
    b = _binding()
    xs = [_to_dev(w.block(k)) for k in range(5)]
    with b.plan_for(w) as p1, b.plan_for(w) as p2:
        ref = [p1.correlate(xs[k], w.delays(k)).clone() for k in range(5)]
        torch.cuda.synchronize()
        sF, sX = torch.cuda.Stream(), torch.cuda.Stream()
        chans = [p2.empty_chan(), p2.empty_chan()]
        outs = [p2.empty_vis() for _ in range(5)]
        f_done = [torch.cuda.Event() for _ in range(2)]
        x_done = [torch.cuda.Event() for _ in range(2)]
        for k in range(5):
            bb = k % 2
            if k >= 2:
                sF.wait_event(x_done[bb])
            p2.channelize(xs[k], w.delays(k), out=chans[bb], stream=sF)
            f_done[bb].record(sF)
            sX.wait_event(f_done[bb])
            p2.correlate_channelized(chans[bb], out=outs[k], stream=sX)
            x_done[bb].record(sX)
        torch.cuda.synchronize()
        for k in range(5):
            assert torch.equal(ref[k], outs[k])
