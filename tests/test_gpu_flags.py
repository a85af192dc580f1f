"""GPU parity of coarse delay windows, lost-sample flags and visibility weights against the
FP64 oracle (``oracle.flags``), through the C ABI.

Blocks run in sequence on one plan so that the FIR history and the carried row flags are
exercised; offsets change between blocks; one block passes no flags (the carried flags must
still apply).  Tolerances as in the plain parity tests: FP16-split / FP32 coherence error
<= 1e-5, channelised data 5e-6 rms + 2e-6 |Z|, int8 bit-exact X stage and the +-1 rule at
rounding boundaries for the requantised F output.  Flagged channel samples must be exactly
zero and the weights exact.
"""

import sys

import numpy as np
import pytest

from oracle import flags as of
from paper_1801_04834_amd import synth
from tests.layout import unblock, unblock_planes
from tests.metrics import near_rounding_boundary, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 1e-5
MODE = {synth.X_FP32: "fp32", synth.X_FP16_SPLIT: "fp16_split", synth.X_INT8: "int8"}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _work(S, SB, n_c, st, mode, seed, C=64):
    return synth.Workload(name="flags", S=S, SB=SB, sample_type=st, x_mode=mode, N=C * n_c, C=C,
                          sigma=16.0 if st == synth.CI8 else 64.0, seed=seed, delay_spread_s=1.5e-6,
                          delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1 if mode == synth.X_FP16_SPLIT else 0)


def _sequence(w, G, n_blocks, seed, flag_blocks):
    rng = np.random.default_rng([seed, 0xC0A5E])
    rows = [synth.guarded_rows(w, k, G) for k in range(n_blocks)]
    offs = [rng.integers(0, G + 1, w.S).astype(np.int32) for _ in range(n_blocks)]
    offs[0][0], offs[0][-1] = 0, G                     # both ends of the guard
    # loss rates scaled by 64/C: a channel sample's FIR window spans 16 C input samples, so the
    # same rates would flag most of a 256-channel block and leave sums of a handful of products
    # (whose coherence error is not averaged down)
    sc = 64 / w.C
    flags = [synth.lost_sample_flags(seed + k, w.S, w.SB, w.N + G, p_packet=0.004 * sc, p_sample=0.0004 * sc,
                                     clean_stations=(1,)) if k in flag_blocks else None
             for k in range(n_blocks)]
    return rows, offs, flags


def _oracle(w, rows, offs, flags):
    hist = np.zeros((w.S, 2, w.SB, 15 * w.C), np.complex128)
    hr = np.zeros((w.S, w.SB, 15), bool)
    outs = []
    for k in range(len(rows)):
        o = of.fx_block_flagged(synth.to_complex(rows[k]), w.N, offs[k], flags[k], hist, hr, w.fir(), w.bandpass(),
                                w.subband_freqs(), synth.SAMPLE_RATE_HZ, w.delays(k), w.C, 16, mode=MODE[w.x_mode],
                                gain=w.gain())
        hist, hr = o["history"], o["hist_row_flags"]
        outs.append(o)
    return outs


def _chan(plan, chan):
    c = chan.cpu().numpy()
    return unblock_planes(c) if plan.x_mode == synth.X_FP16_SPLIT else unblock(c)


def _check_block(plan, w, chan, wts, vis, o, label):
    n_c = plan.n_c
    W = wts.cpu().numpy()
    np.testing.assert_array_equal(W, o["W"], err_msg=f"{label}: weights")
    r = _chan(plan, chan)
    fl = np.repeat(o["chan_flags"].transpose(1, 0, 2), 2, axis=1)          # [SB, M, N_c]
    fl = np.broadcast_to(fl[:, None], (w.SB, w.C) + fl.shape[1:])
    n_fl = int(o["chan_flags"].sum())
    _say(f"  {label}: {n_fl} flagged channel samples (per station/subband), weights min {W.min()} of {n_c}")
    if plan.x_mode == synth.X_FP16_SPLIT:
        for part in r:
            assert np.all(part[..., :n_c, :][fl] == 0), f"{label}: flagged samples not zero"
        k = plan.kw.get("fp16_prescale_log2", 0)
        v = (r[0].astype(np.float64) + r[1].astype(np.float64)) * 2.0 ** (-k)
        Zg = (v[..., 0] + 1j * v[..., 1])[..., :n_c]
    else:
        assert np.all(r[..., :n_c, :][fl] == 0), f"{label}: flagged samples not zero"
        Zg = (r[..., 0].astype(np.float64) + 1j * r[..., 1])[..., :n_c]
    if plan.x_mode == synth.X_INT8:
        Qg = r[..., :n_c, :]
        d = Qg.astype(np.int64) - o["Q"].astype(np.int64)
        bad = d != 0
        g = np.float64(np.float32(w.gain()))
        pre = np.stack([(g * o["Zf"].real).astype(np.float32), (g * o["Zf"].imag).astype(np.float32)], axis=-1)
        _say(f"  {label}: int8 mismatches {int(bad.sum())} of {d.size}")
        assert np.all(np.abs(d) <= 1), f"{label}: int8 channelised off by more than 1"
        assert np.all(near_rounding_boundary(pre, 1e-3)[bad]), f"{label}: int8 mismatch away from a rounding boundary"
        # X stage bit-exact on the GPU's own int8 stream
        from oracle import fx as ofx
        Vx = ofx.correlate_int(np.ascontiguousarray(Qg).astype(np.int8), w.S)
        np.testing.assert_array_equal(vis.cpu().numpy().astype(np.int64), Vx, err_msg=f"{label}: int8 X stage")
        return
    rms = np.sqrt(np.mean(np.abs(o["Z"]) ** 2))
    err = np.abs(Zg - o["Z"])
    assert np.all(err <= 5e-6 * rms + 2e-6 * np.abs(o["Z"])), f"{label}: channelised mismatch"
    eps = _eps(vis_complex(vis.cpu().numpy()), o["V"], w.S, o["W"], rms)
    _say(f"  {label}: eps = {eps:.3e}")
    assert eps <= EPS


def _eps(Vg, Vo, S, W, rms, n_min=16):
    """Coherence error over entries whose stations keep valid samples; where a station lost
    every channel sample its entries must be exactly zero.  An entry of a baseline with fewer
    than n_min valid channel samples is a sum of a few products, whose error the sum does not
    average down (a station's few remaining samples may all be small against the channelised
    data's rms, to which the F stage's error is relative), so there the error is taken
    relative to the scale of such a sum, rms^2 times the sample count, instead."""
    autos = np.stack([Vo[..., s * (s + 1) // 2 + s, 0].real for s in range(S)] +
                     [Vo[..., s * (s + 1) // 2 + s, 3].real for s in range(S)], axis=-1)   # [SB, C, 2S]
    worst = 0.0
    for s1 in range(S):
        for s2 in range(s1 + 1):
            bl = s1 * (s1 + 1) // 2 + s2
            for q in range(4):
                p1, p2 = q // 2, q % 2
                den = np.sqrt(autos[..., p1 * S + s1] * autos[..., p2 * S + s2])
                few = (W[:, bl] < n_min)[:, None]                     # [SB, 1] over channels
                den = np.where(few & (den > 0), np.maximum(den, rms ** 2 * W[:, bl][:, None]), den)
                diff = np.abs(Vg[..., bl, q] - Vo[..., bl, q])
                zero = den == 0
                assert np.all(Vg[..., bl, q][zero] == 0)
                if (~zero).any():
                    worst = max(worst, float(np.max(diff[~zero] / den[~zero])))
    return worst


@pytest.mark.parametrize("st,mode,C", [(synth.CI16, synth.X_FP16_SPLIT, 64), (synth.CI16, synth.X_FP32, 64),
                                       (synth.CI8, synth.X_INT8, 64), (synth.CF32, synth.X_FP32, 64),
                                       (synth.CI16, synth.X_FP16_SPLIT, 256), (synth.CI8, synth.X_INT8, 256)])
@pytest.mark.parametrize("n_c", [300, 8])
def test_coarse_and_flagged_blocks_match_oracle(st, mode, C, n_c):
    from paper_1801_04834_amd import binding
    S, SB, G, nb = 5, 2, 37, 4
    if C == 256:
        n_c = n_c // 4 + 3                             # 78 and 5 channel samples of 256 inputs
    seed = 2100 + 10 * st + mode + n_c + C
    w = _work(S, SB, n_c, st, mode, seed, C)
    _say(f"CASE flags st={st} mode={mode} C={C} S={S} SB={SB} n_c={n_c} G={G} seed={seed}")
    rows, offs, flags = _sequence(w, G, nb, seed, flag_blocks=(0, 1, 3))     # block 2 passes no flags
    outs = _oracle(w, rows, offs, flags)
    with binding.plan_for(w) as plan, binding.plan_for(w) as plan2:
        for k in range(nb):
            x = _dev(rows[k])
            fd = _dev(synth.pack_flags(flags[k]).view(np.int32)) if flags[k] is not None else None
            wts = torch.full(plan.weights_shape(), -1, dtype=torch.int32, device="cuda")
            chan = plan.channelize_ex(x, w.delays(k), coarse=offs[k], flags=fd, weights=wts)
            vis = plan.correlate_channelized(chan)
            # the full chain on a second plan gives the same visibilities bit for bit
            wts2 = torch.full(plan.weights_shape(), -1, dtype=torch.int32, device="cuda")
            vis2 = plan2.correlate_ex(x, w.delays(k), coarse=offs[k], flags=fd, weights=wts2)
            torch.cuda.synchronize()
            _check_block(plan, w, chan, wts, vis, outs[k], f"block {k}")
            assert torch.equal(vis, vis2) and torch.equal(wts, wts2)


def test_reset_clears_carried_flags_and_plain_calls_honour_them():
    from paper_1801_04834_amd import binding
    S, SB, n_c = 3, 1, 40
    w = _work(S, SB, n_c, synth.CI16, synth.X_FP32, 2201)
    _say(f"CASE flags reset S={S} n_c={n_c}")
    fl = np.zeros((S, SB, w.N), bool)
    fl[0, 0, w.N - 3] = True                            # lost sample in the last row of block 0
    with binding.plan_for(w) as plan:
        x0, x1 = _dev(w.block(0)), _dev(w.block(1))
        plan.correlate_ex(x0, w.delays(0), flags=_dev(synth.pack_flags(fl).view(np.int32)))
        # the plain call on the next block still zeroes the 15 channel samples that read it
        chan = plan.channelize(x1, w.delays(1))
        wts = torch.zeros(plan.weights_shape(), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        r = _chan(plan, chan)
        assert np.all(r[:, :, 0:2, :15] == 0) and np.all(r[:, :, 0:2, 15:n_c].any(axis=-1).any(axis=1))
        plan.reset_history()
        plan.correlate_ex(x1, w.delays(1), weights=wts)
        torch.cuda.synchronize()
        assert (wts.cpu().numpy() == n_c).all()
        chan = plan.channelize(x1, w.delays(1))
        torch.cuda.synchronize()
        assert _chan(plan, chan)[:, :, 0:2, :15].any()


def test_zero_guard_equals_plain_correlate():
    from paper_1801_04834_amd import binding
    w = _work(4, 2, 64, synth.CI16, synth.X_FP16_SPLIT, 2202)
    _say("CASE flags zero-guard")
    with binding.plan_for(w) as a, binding.plan_for(w) as b:
        x = _dev(w.block(0))
        wts = torch.zeros(a.weights_shape(), dtype=torch.int32, device="cuda")
        va = a.correlate(x, w.delays(0))
        vb = b.correlate_ex(x, w.delays(0), coarse=np.zeros(w.S, np.int32), weights=wts)
        torch.cuda.synchronize()
        assert torch.equal(va, vb)
        assert (wts.cpu().numpy() == 64).all()


def test_invalid_extras_are_rejected():
    from paper_1801_04834_amd import binding
    w = _work(2, 1, 32, synth.CI16, synth.X_FP32, 2203)
    _say("CASE flags invalid")
    with binding.plan_for(w) as plan:
        G = 5
        x = _dev(synth.guarded_rows(w, 0, G))
        for off in ([0, G + 1], [-1, 0]):
            with pytest.raises(binding.CobaltError) as ei:
                plan.correlate_ex(x, w.delays(0), coarse=np.array(off, np.int32))
            assert ei.value.code == binding.EINVAL
        short = _dev(synth.guarded_rows(w, 0, 0)[..., :w.N - 64, :])
        with pytest.raises((binding.CobaltError, ValueError)):
            plan.correlate_ex(short, w.delays(0))
        # a failed call leaves the plan usable
        v = plan.correlate_ex(x, w.delays(0), coarse=np.array([0, G], np.int32))
        torch.cuda.synchronize()
        assert torch.isfinite(v).all()


def test_host_arrays_may_be_reused_as_soon_as_a_call_returns():
    """Delays and coarse offsets are host arrays that the library copies before a call returns
    (the kernels run later): overwriting them right after each call, while earlier work still
    occupies the GPU, changes nothing."""
    from paper_1801_04834_amd import binding
    S, SB, n_c, G = 3, 1, 64, 17
    w = _work(S, SB, n_c, synth.CI16, synth.X_FP16_SPLIT, 2204)
    _say(f"CASE flags host arrays reused S={S} n_c={n_c} G={G}")
    rows, offs, _ = _sequence(w, G, 3, 2204, flag_blocks=())
    xs = [_dev(r) for r in rows]
    with binding.plan_for(w) as p1, binding.plan_for(w) as p2:
        ref = [p1.correlate_ex(xs[k], w.delays(k).copy(), coarse=offs[k].copy()).clone() for k in range(3)]
        torch.cuda.synchronize()
        a = torch.ones(2**28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            binding.device_copy(b, a)                   # ~2 ms of work queued ahead
        got = []
        for k in range(3):
            d = np.ascontiguousarray(w.delays(k), np.float64)
            o = np.ascontiguousarray(offs[k], np.int32)
            got.append(p2.correlate_ex(xs[k], d, coarse=o))
            d[:] = 3e-6                                 # the caller reuses its arrays at once
            o[:] = G - o
        torch.cuda.synchronize()
        for k in range(3):
            assert torch.equal(ref[k], got[k])
