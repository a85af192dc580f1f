"""Pins of the coarse-delay and lost-sample-flag reference (``oracle.flags``), no GPU.

* flags: the channel samples flagged are exactly those whose FIR output changes when the
  lost input samples change (measured through the reference filter bank with random,
  nowhere-zero taps), including lost samples in the carried history;
* closed form: one lost sample flags T consecutive channel samples;
* weights: the flagged X stage equals sums over the intersection of the valid sample sets,
  computed with Python sets, and the weights are the sizes of those sets;
* history: two consecutive blocks equal one block twice as long (samples and flags);
* coarse delay: a noise stream delayed by a whole number of samples at one station is
  aligned exactly by the window offset; a sky tone delayed by a whole plus a fractional
  number of samples is aligned by the offset plus the residual fine delay.
"""

import numpy as np
import pytest

import oracle
from oracle import flags as of
from paper_1801_04834_amd import synth


def _rand_complex(rng, shape, scale=1.0):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale


def _setup(seed, S=3, P=2, SB=2, C=8, T=4, n_c=12, G=5):
    rng = np.random.default_rng(seed)
    N = n_c * C
    rows = _rand_complex(rng, (S, P, SB, N + G), 10.0)
    hist = _rand_complex(rng, (S, P, SB, (T - 1) * C), 10.0)
    h = rng.uniform(0.2, 1.0, T * C) * rng.choice([-1.0, 1.0], T * C)      # no zero tap
    offsets = rng.integers(0, G + 1, S)
    return rng, N, rows, hist, h, offsets


def _run(rows, N, offsets, flags, hist, hist_rows, h, C, T, delays=None, mode="fp32", gain=None,
         f_sb=(150e6, 150.1953125e6)):
    S, _, SB, _ = rows.shape
    d = np.zeros((S, 2)) if delays is None else delays
    return of.fx_block_flagged(rows, N, offsets, flags, hist, hist_rows, h, None, list(f_sb[:SB]),
                               synth.SAMPLE_RATE_HZ, d, C, T, mode=mode, gain=gain)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_flagged_channel_samples_are_exactly_those_reading_lost_samples(seed):
    S, P, SB, C, T, n_c, G = 3, 2, 2, 8, 4, 12, 5
    rng, N, rows, hist, h, offsets = _setup(seed, S, P, SB, C, T, n_c, G)
    flags = rng.random((S, SB, N + G)) < 0.01
    hist_rows = rng.random((S, SB, T - 1)) < 0.2
    # a lost sample's value is arbitrary: replace every lost sample (and one sample of each
    # flagged history row) by a different random value and see which outputs move
    rows2 = rows.copy()
    hist2 = hist.copy()
    for s in range(S):
        for sb in range(SB):
            lost = np.nonzero(flags[s, sb])[0]
            rows2[s, :, sb, lost] += _rand_complex(rng, (len(lost), P), 50.0)
            for r in np.nonzero(hist_rows[s, sb])[0]:
                k = r * C + int(rng.integers(C))
                hist2[s, :, sb, k] += _rand_complex(rng, P, 50.0)
    f_sb = [150e6] * SB
    Z1 = oracle.fx_block(of.coarse_window(rows, offsets, N), hist, h, None, f_sb, synth.SAMPLE_RATE_HZ,
                         np.zeros((S, 2)), C, T)["Z"]
    Z2 = oracle.fx_block(of.coarse_window(rows2, offsets, N), hist2, h, None, f_sb, synth.SAMPLE_RATE_HZ,
                         np.zeros((S, 2)), C, T)["Z"]
    moved = np.abs(Z1 - Z2).max(axis=1) > 1e-9                 # [SB, M, N_c]
    moved = moved.reshape(SB, S, P, n_c).any(axis=2).transpose(1, 0, 2)   # [S, SB, N_c]
    chan, _ = of.channel_flags(of.window_flags(flags, offsets, N), hist_rows, C, T)
    assert chan.any() and not chan.all()
    np.testing.assert_array_equal(chan, moved)


@pytest.mark.parametrize("k", [0, 7, 8, 37, 95])
def test_one_lost_sample_flags_T_channel_samples(k):
    C, T, n_c = 8, 4, 12
    fl = np.zeros((1, 1, n_c * C), bool)
    fl[0, 0, k] = True
    chan, new_rows = of.channel_flags(fl, np.zeros((1, 1, T - 1), bool), C, T)
    want = np.zeros(n_c, bool)
    want[k // C: min(k // C + T, n_c)] = True
    np.testing.assert_array_equal(chan[0, 0], want)
    np.testing.assert_array_equal(new_rows[0, 0], np.arange(n_c - T + 1, n_c) == k // C)


@pytest.mark.parametrize("mode", ["fp32", "int8"])
def test_weights_and_visibilities_are_sums_over_common_valid_samples(mode):
    S, P, SB, C, T, n_c, G = 4, 2, 2, 8, 4, 16, 3
    rng, N, rows, hist, h, offsets = _setup(7, S, P, SB, C, T, n_c, G)
    flags = rng.random((S, SB, N + G)) < 0.006
    hist_rows = rng.random((S, SB, T - 1)) < 0.3
    gain = 0.5 if mode == "int8" else None
    out = _run(rows, N, offsets, flags, hist, hist_rows, h, C, T, mode=mode, gain=gain)
    plain = oracle.fx_block(of.coarse_window(rows, offsets, N), hist, h, None, [150e6, 150.1953125e6],
                            synth.SAMPLE_RATE_HZ, np.zeros((S, 2)), C, T, mode=mode, gain=gain)
    chan = out["chan_flags"]
    for sb in range(SB):
        valid = [set(np.nonzero(~chan[s, sb])[0].tolist()) for s in range(S)]
        for s1 in range(S):
            for s2 in range(s1 + 1):
                both = sorted(valid[s1] & valid[s2])
                bl = oracle.baseline_index(s1, s2)
                assert out["W"][sb, bl] == len(both)
                for p1 in range(P):
                    for p2 in range(P):
                        q = 2 * p1 + p2
                        if mode == "int8":
                            a = plain["Q"][sb, :, s1 * P + p1][:, both].astype(np.int64)
                            b = plain["Q"][sb, :, s2 * P + p2][:, both].astype(np.int64)
                            re = np.sum(a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1], axis=-1)
                            im = np.sum(a[..., 1] * b[..., 0] - a[..., 0] * b[..., 1], axis=-1)
                            np.testing.assert_array_equal(out["V"][sb, :, bl, q, 0], re)
                            np.testing.assert_array_equal(out["V"][sb, :, bl, q, 1], im)
                        else:
                            za = plain["Z"][sb, :, s1 * P + p1][:, both]
                            zb = plain["Z"][sb, :, s2 * P + p2][:, both]
                            want = np.sum(za * np.conj(zb), axis=-1)
                            np.testing.assert_allclose(out["V"][sb, :, bl, q], want, rtol=0,
                                                       atol=1e-10 * max(1.0, np.abs(want).max()))
    assert (out["W"] < n_c).any() and (out["W"] > 0).all()


def test_two_blocks_equal_one_long_block():
    S, P, SB, C, T, n_c, G = 3, 2, 1, 8, 4, 10, 4
    rng = np.random.default_rng(11)
    N = n_c * C
    stream = _rand_complex(rng, (S, P, SB, 2 * N + G), 10.0)
    sflags = rng.random((S, SB, 2 * N + G)) < 0.01
    hist = _rand_complex(rng, (S, P, SB, (T - 1) * C), 10.0)
    hist_rows = rng.random((S, SB, T - 1)) < 0.3
    h = rng.standard_normal(T * C)
    offsets = rng.integers(0, G + 1, S)
    tau = rng.uniform(-2e-6, 2e-6, S)
    d = np.stack([tau, tau], 1)
    f_sb = (150e6,)
    b1 = _run(stream[..., :N + G], N, offsets, sflags[..., :N + G], hist, hist_rows, h, C, T, d, f_sb=f_sb)
    b2 = _run(stream[..., N:2 * N + G], N, offsets, sflags[..., N:2 * N + G], b1["history"], b1["hist_row_flags"],
              h, C, T, d, f_sb=f_sb)
    long = _run(stream, 2 * N, offsets, sflags, hist, hist_rows, h, C, T, d, f_sb=f_sb)
    np.testing.assert_array_equal(np.concatenate([b1["chan_flags"], b2["chan_flags"]], -1), long["chan_flags"])
    np.testing.assert_array_equal(b1["W"] + b2["W"], long["W"])
    np.testing.assert_allclose(np.concatenate([b1["Z"], b2["Z"]], -1), long["Z"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(b1["V"] + b2["V"], long["V"], rtol=0, atol=1e-8 * np.abs(long["V"]).max())
    np.testing.assert_array_equal(b2["hist_row_flags"], long["hist_row_flags"])


def test_integer_sample_delay_is_removed_exactly_by_the_window_offset():
    """Station 1 receives station 0's broadband signal n samples later; reading station 1's
    rows n samples further on gives identical channelised data, so every cross product
    equals the auto product."""
    S, P, C, T, n_c, n = 2, 2, 64, 16, 8, 3
    rng = np.random.default_rng(5)
    N = n_c * C
    G = 4
    u = _rand_complex(rng, (P, (T - 1) * C + N + G + 8), 20.0)     # sky signal per pol
    base = (T - 1) * C + 4                                          # row 0 = sample `base` of u
    rows = np.empty((S, P, 1, N + G), np.complex128)
    rows[0, :, 0] = u[:, base:base + N + G]
    rows[1, :, 0] = u[:, base - n:base - n + N + G]                 # x1[k] = u[k - n]
    offsets = np.array([0, n])
    hist = np.empty((S, P, 1, (T - 1) * C), np.complex128)
    hist[0, :, 0] = u[:, base - (T - 1) * C:base]
    hist[1, :, 0] = hist[0, :, 0]                                   # history of the aligned stream
    out = _run(rows, N, offsets, None, hist, np.zeros((S, 1, T - 1), bool), synth.fir_windowed_sinc(C, T), C, T,
               f_sb=(150e6,))
    np.testing.assert_array_equal(out["Z"][0, :, 2:4], out["Z"][0, :, 0:2])
    V = out["V"][0]
    for q in range(4):
        np.testing.assert_allclose(V[:, oracle.baseline_index(1, 0), q], V[:, oracle.baseline_index(0, 0), q],
                                   rtol=1e-12, atol=1e-9)
    assert (out["W"] == n_c).all()


def test_coarse_plus_residual_delay_aligns_a_delayed_sky_tone():
    """A sky tone at the centre frequency F of channel c0 reaches station s tau_s later,
    tau_s = n_s / f_s + r_s.  Baseband samples: A exp(2 pi i (F - f_SB)(k / f_s - tau_s))
    exp(-2 pi i f_SB tau_s).  With window offsets n_s and residual fine delays r_s every cross
    product in c0 equals the auto (f_SB a whole multiple of f_s, as for the LOFAR subbands)."""
    S, P, C, T, n_c, A, c0 = 4, 2, 64, 16, 16, 50.0, 27
    f_s = synth.SAMPLE_RATE_HZ
    f_sb = 768 * f_s                                                 # 150 MHz
    F = f_sb + (c0 - C / 2) * f_s / C
    nsh = np.array([0, 3, 1, 5])
    res = np.array([0.0, 1.1e-6, -2.3e-6, 0.4e-6])
    taus = nsh / f_s + res
    G = 6
    N = n_c * C
    k = np.arange(-(T - 1) * C, N + G)
    rows = np.empty((S, P, 1, N + G), np.complex128)
    hist = np.empty((S, P, 1, (T - 1) * C), np.complex128)
    for s in range(S):
        # rows hold samples k = 0 .. N+G-1; the window of station s starts at k = n_s and its
        # history is the (T-1)C samples before that
        sig = A * np.exp(2j * np.pi * (F - f_sb) * (k / f_s - taus[s])) * np.exp(-2j * np.pi * f_sb * taus[s])
        kk = k + nsh[s]
        full = A * np.exp(2j * np.pi * (F - f_sb) * (kk / f_s - taus[s])) * np.exp(-2j * np.pi * f_sb * taus[s])
        rows[s, :, 0] = sig[(T - 1) * C:]
        hist[s, :, 0] = full[:(T - 1) * C]
    out = _run(rows, N, nsh, None, hist, np.zeros((S, 1, T - 1), bool), synth.fir_windowed_sinc(C, T), C, T,
               delays=np.stack([res, res], 1), f_sb=(f_sb,))
    V = out["V"][0, c0]
    auto = V[oracle.baseline_index(0, 0), 0].real
    assert auto > 0
    for s1 in range(S):
        for s2 in range(s1 + 1):
            for q in range(4):
                assert abs(V[oracle.baseline_index(s1, s2), q] - auto) < 1e-9 * auto
    # the offsets alone (no residual) leave the stations misaligned
    out0 = _run(rows, N, nsh, None, hist, np.zeros((S, 1, T - 1), bool), synth.fir_windowed_sinc(C, T), C, T,
                f_sb=(f_sb,))
    assert abs(out0["V"][0, c0][oracle.baseline_index(2, 0), 0] - auto) > 1e-2 * auto


def test_no_flags_and_zero_offsets_reduce_to_the_plain_chain():
    S, P, SB, C, T, n_c, G = 2, 2, 2, 8, 4, 6, 0
    rng, N, rows, hist, h, _ = _setup(9, S, P, SB, C, T, n_c, G)
    out = _run(rows, N, np.zeros(S, int), None, hist, np.zeros((S, SB, T - 1), bool), h, C, T)
    plain = oracle.fx_block(rows, hist, h, None, [150e6, 150.1953125e6], synth.SAMPLE_RATE_HZ, np.zeros((S, 2)), C, T)
    np.testing.assert_array_equal(out["V"], plain["V"])
    assert (out["W"] == n_c).all()
