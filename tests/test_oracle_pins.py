"""Pins of the FP64 reference (``oracle``) to facts outside itself.

Each test checks the reference against something the mathematics or the paper fixes:
closed forms (tone response via the FIR's DTFT, geometric series for a drifting delay,
impulse response), reductions to independent routines (plain FIR by ``numpy.convolve``),
brute-force loops on tiny inputs, exact rational arithmetic, invariants (Hermitian,
real non-negative autos, exact power-of-two linearity) and noise statistics (the paper
validated its output by signal and noise properties, "Verification and validation").
No GPU is needed.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1801_04834_amd import synth


def _rand_complex(rng, shape, scale=1.0):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale


def _dtft(h, nu):
    """H(nu) = sum_m h[m] exp(-2 pi i nu m), written out (independent of the reference)."""
    m = np.arange(len(h), dtype=np.float64)
    return np.sum(np.asarray(h, np.float64) * np.exp(-2j * np.pi * nu * m))


# ---------------------------------------------------------------- brute force (tiny) ---

@pytest.mark.parametrize("C,T", [(4, 1), (4, 2), (8, 3), (2, 4), (1, 5)])
def test_ppf_matches_loops(C, T):
    rng = np.random.default_rng(11 + C * 10 + T)
    n_c = 5
    tl = _rand_complex(rng, (T - 1) * C + n_c * C)
    h = rng.standard_normal(T * C)
    ref = np.array(brute.ppf_loop(list(tl), list(h), C, T))
    got = oracle.polyphase_filterbank(tl, h, C, T)
    assert got.shape == (n_c, C)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("mode", ["fp32", "int8"])
def test_full_chain_matches_loops(mode):
    rng = np.random.default_rng(5)
    S, P, SB, C, T, n_c = 2, 2, 2, 4, 3, 6
    N = n_c * C
    x = np.rint(_rand_complex(rng, (S, P, SB, N), 20.0).real) + 1j * np.rint(_rand_complex(rng, (S, P, SB, N), 20.0).real)
    hist = np.rint(_rand_complex(rng, (S, P, SB, (T - 1) * C), 20.0).real) + 0j
    h = rng.standard_normal(T * C).astype(np.float32)
    b = (1 + 0.1 * rng.standard_normal(C)).astype(np.float32)
    f_sb = np.array([120e6, 121.3e6])
    f_s = 195312.5
    delays = np.stack([rng.uniform(-5e-6, 5e-6, S), rng.uniform(-5e-6, 5e-6, S)], 1)
    gain = float(np.float32(0.35))
    out = oracle.fx_block(x, hist, h, b, f_sb, f_s, delays, C, T, mode=mode, gain=gain)
    tl = oracle.stream_timeline(hist, x)
    for sb in range(SB):
        Z = []
        for s in range(S):
            for p in range(P):
                X = brute.ppf_loop(list(tl[s, p, sb]), [float(v) for v in h], C, T)
                Zs = brute.delay_rotate_loop(X, float(f_sb[sb]), C, f_s, delays[s, 0], delays[s, 1],
                                             [float(v) for v in b])
                Z.append(Zs)
        for c in range(C):
            rows = [[Z[a][j][c] for j in range(n_c)] for a in range(S * P)]
            if mode == "fp32":
                ref = np.array(brute.correlate_loop(rows, S, P))
                np.testing.assert_allclose(out["V"][sb, c], ref, rtol=0, atol=1e-9 * np.abs(ref).max())
                np.testing.assert_allclose(out["Z"][sb, c], np.array(rows), rtol=0,
                                           atol=1e-10 * np.abs(np.array(rows)).max())
            else:
                # the integer decision in single precision, written out term by term
                q = [[(int(np.clip(np.rint(np.float32(gain * v.real)), -127, 127)),
                       int(np.clip(np.rint(np.float32(gain * v.imag)), -127, 127))) for v in r] for r in rows]
                ref = np.array(brute.correlate_int_loop(q, S, P), np.int64)
                assert np.array_equal(out["V"][sb, c], ref)
                assert np.array_equal(out["Q"][sb, c], np.array(q, np.int8))


def test_correlate_matches_loops():
    rng = np.random.default_rng(3)
    S, P, n_c = 3, 2, 7
    Z = _rand_complex(rng, (S * P, n_c))
    ref = np.array(brute.correlate_loop([list(r) for r in Z], S, P))
    np.testing.assert_allclose(oracle.correlate(Z, S, P), ref, rtol=0, atol=1e-12)


def test_correlate_int_exact_against_python_ints():
    rng = np.random.default_rng(4)
    S, P, n_c = 3, 2, 40
    Q = rng.integers(-127, 128, size=(S * P, n_c, 2)).astype(np.int8)
    Q[0, :5] = 127
    Q[1, :5] = -127
    ref = brute.correlate_int_loop([[tuple(int(v) for v in Q[a, j]) for j in range(n_c)] for a in range(S * P)], S, P)
    assert np.array_equal(oracle.correlate_int(Q, S, P), np.array(ref, np.int64))


def test_correlate_int_at_overflow_bound():
    """All samples +-127 at the largest integration the int32 bound admits
    (N_c * 2 * 127^2 < 2^31): autos equal N_c * 2 * 127^2 exactly."""
    n_c = 66560
    assert n_c * 2 * 127 ** 2 < 2 ** 31 <= (n_c + 32 * 400) * 2 * 127 ** 2
    rng = np.random.default_rng(9)
    Q = rng.choice(np.array([-127, 127], np.int8), size=(4, n_c, 2))
    V = oracle.correlate_int(Q, 2, 2)
    for s in range(2):
        for p in range(2):
            assert V[oracle.baseline_index(s, s), 3 * p, 0] == n_c * 2 * 127 ** 2
            assert V[oracle.baseline_index(s, s), 3 * p, 1] == 0


# ---------------------------------------------------------------- reductions ------------

def test_single_channel_is_plain_fir():
    """C = 1: the filter bank is one FIR filter (compared with numpy.convolve)."""
    rng = np.random.default_rng(1)
    T, n = 16, 200
    h = rng.standard_normal(T)
    tl = _rand_complex(rng, T - 1 + n)
    got = oracle.polyphase_filterbank(tl, h, 1, T)[:, 0]
    ref = np.convolve(tl, h[::-1], mode="valid")
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("C", [4, 8, 64])
def test_impulse_response_closed_form(C):
    """One tap, h = 1, a unit impulse at phase p0 of row j0:
    X_j0[c] = exp(-2 pi i p0 (c - C/2) / C), every other row zero."""
    for p0 in (0, 1, C - 1, C // 3):
        n_c = 3
        tl = np.zeros(n_c * C, np.complex128)
        tl[1 * C + p0] = 1.0
        X = oracle.polyphase_filterbank(tl, np.ones(C), C, 1)
        c = np.arange(C)
        want = np.exp(-2j * np.pi * p0 * (c - C // 2) / C)
        np.testing.assert_allclose(X[1], want, rtol=0, atol=1e-13)
        assert np.all(X[0] == 0) and np.all(X[2] == 0)


def test_dft_unnormalised_parseval():
    """T = 1, h = 1: sum_c |X_j[c]|^2 = C * sum_p |x_j[p]|^2 (forward DFT, no 1/C)."""
    rng = np.random.default_rng(2)
    C = 64
    tl = _rand_complex(rng, 10 * C)
    X = oracle.polyphase_filterbank(tl, np.ones(C), C, 1)
    lhs = np.sum(np.abs(X) ** 2, axis=1)
    rhs = C * np.sum(np.abs(tl.reshape(10, C)) ** 2, axis=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)


# ---------------------------------------------------------------- tone closed forms -----

@pytest.mark.parametrize("f0", [5 / 64, -27 / 64, 0.123456, -0.4321, 0.0])
def test_tone_closed_form_steady_state(f0):
    """Continuous complex tone x[n] = A exp(2 pi i f0 n) (history included):
    X_j[k] = A exp(2 pi i f0 (j-T+1) C) H(k/C - f0) with H the FIR's DTFT."""
    C, T, n_c, A = 64, 16, 8, 3.0
    h = synth.fir_windowed_sinc(C, T).astype(np.float64)
    n = np.arange(-(T - 1) * C, n_c * C)
    tl = A * np.exp(2j * np.pi * f0 * n)
    X = oracle.polyphase_filterbank(tl, h, C, T)
    for j in (0, 3, n_c - 1):
        for c in range(C):
            k = (c - C // 2) % C
            want = A * np.exp(2j * np.pi * f0 * (j - T + 1) * C) * _dtft(h, k / C - f0)
            assert abs(X[j, c] - want) < 1e-11


def test_bin_centred_tone_lands_in_its_channel_with_fir_gain():
    """A tone at baseband (c0 - C/2)/C cycles/sample appears in channel c0 (ascending
    frequency order) with |X| = A * sum(h); all other channels are far below it."""
    C, T, n_c, A = 64, 16, 4, 256.0
    h = synth.fir_windowed_sinc(C, T).astype(np.float64)
    for c0 in (0, 5, 31, 32, 37, 63):
        f0 = (c0 - C // 2) / C
        n = np.arange(-(T - 1) * C, n_c * C)
        X = oracle.polyphase_filterbank(A * np.exp(2j * np.pi * f0 * n), h, C, T)
        mag = np.abs(X)
        assert np.all(np.argmax(mag, axis=1) == c0)
        np.testing.assert_allclose(mag[:, c0], A * h.sum(), rtol=1e-12)
        others = np.delete(mag, c0, axis=1)
        assert others.max() < 1e-3 * A


def test_tone_warm_up_rows_after_reset():
    """Zero history (first block after a reset): rows j < T-1 see only the part of the
    FIR that overlaps the block, X_j[k] = A e^{..} sum_{m >= (T-1-j)C} h[m] e^{-2 pi i m nu}."""
    C, T, n_c, A, f0 = 8, 4, 6, 2.0, 0.19
    rng = np.random.default_rng(8)
    h = rng.standard_normal(T * C)
    n = np.arange(n_c * C)
    block = A * np.exp(2j * np.pi * f0 * n)
    tl = oracle.stream_timeline(np.zeros((T - 1) * C), block)
    X = oracle.polyphase_filterbank(tl, h, C, T)
    m = np.arange(T * C)
    for j in range(n_c):
        for c in range(C):
            nu = ((c - C // 2) % C) / C - f0
            mask = m >= max(0, (T - 1 - j) * C)
            want = A * np.exp(2j * np.pi * f0 * (j - T + 1) * C) * np.sum(h[mask] * np.exp(-2j * np.pi * nu * m[mask]))
            assert abs(X[j, c] - want) < 1e-11


def _tone_block(S, P, C, T, n_c, A, f0, phases=None):
    n = np.arange(-(T - 1) * C, n_c * C)
    x = np.empty((S, P, 1, len(n)), np.complex128)
    for s in range(S):
        for p in range(P):
            ph = 0.0 if phases is None else phases[s]
            x[s, p, 0] = A * np.exp(2j * np.pi * (f0 * n + ph))
    return x[..., (T - 1) * C:], x[..., :(T - 1) * C]


def test_autocorrelation_closed_form():
    """Steady-state tone in channel c0: V_aa(c0) = N_c A^2 (sum h)^2 b_c0^2, imaginary 0."""
    S, P, C, T, n_c, A, c0 = 2, 2, 64, 16, 32, 100.0, 37
    h = synth.fir_windowed_sinc(C, T)
    b = synth.bandpass_ripple(C, 0.2)
    x, hist = _tone_block(S, P, C, T, n_c, A, (c0 - C // 2) / C)
    out = oracle.fx_block(x, hist, h, b, [150e6], synth.SAMPLE_RATE_HZ, np.zeros((S, 2)), C, T)
    V = out["V"][0, c0]
    want = n_c * A ** 2 * float(np.sum(h.astype(np.float64))) ** 2 * float(b[c0]) ** 2
    for s in range(S):
        bl = oracle.baseline_index(s, s)
        for q in (0, 3):
            assert abs(V[bl, q].real - want) < 1e-9 * want
            assert V[bl, q].imag == 0.0


def test_delay_sign_and_frequency_align_a_delayed_sky_tone():
    """A sky tone at the centre frequency F of channel c0, arriving tau_s later at station
    s, has baseband samples A exp(2 pi i f0 n) exp(-2 pi i F tau_s).  Compensating with
    tau_s must align all stations: every cross V(c0) equals the auto (real, positive)."""
    S, P, C, T, n_c, A, c0 = 4, 2, 64, 16, 16, 50.0, 21
    f_s, f_sb = synth.SAMPLE_RATE_HZ, 140e6
    F = f_sb + (c0 - C / 2) * f_s / C
    taus = np.array([0.0, 1.3e-6, -4.1e-6, 2.7e-7])
    x, hist = _tone_block(S, P, C, T, n_c, A, (c0 - C // 2) / C, phases=-F * taus)
    delays = np.stack([taus, taus], 1)
    out = oracle.fx_block(x, hist, synth.fir_windowed_sinc(C, T), None, [f_sb], f_s, delays, C, T)
    V = out["V"][0, c0]
    auto = V[oracle.baseline_index(0, 0), 0].real
    assert auto > 0
    for s1 in range(S):
        for s2 in range(s1 + 1):
            for q in range(4):
                v = V[oracle.baseline_index(s1, s2), q]
                assert abs(v - auto) < 1e-9 * auto
    # with the opposite sign (or without compensation) the phases stay spread
    out0 = oracle.fx_block(x, hist, synth.fir_windowed_sinc(C, T), None, [f_sb], f_s, np.zeros((S, 2)), C, T)
    assert abs(out0["V"][0, c0][oracle.baseline_index(1, 0), 0] - auto) > 1e-2 * auto


def test_constant_delay_rotates_each_baseline():
    """Constant delays on noise: V_ab(tau) = exp(2 pi i f_c (tau_a - tau_b)) V_ab(0)."""
    rng = np.random.default_rng(21)
    S, P, SB, C, T, n_c = 3, 2, 1, 64, 16, 8
    x = _rand_complex(rng, (S, P, SB, n_c * C), 30.0)
    hist = _rand_complex(rng, (S, P, SB, (T - 1) * C), 30.0)
    h = synth.fir_windowed_sinc(C, T)
    f_sb, f_s = 180e6, synth.SAMPLE_RATE_HZ
    taus = rng.uniform(-5e-6, 5e-6, S)
    V0 = oracle.fx_block(x, hist, h, None, [f_sb], f_s, np.zeros((S, 2)), C, T)["V"][0]
    V1 = oracle.fx_block(x, hist, h, None, [f_sb], f_s, np.stack([taus, taus], 1), C, T)["V"][0]
    fc = f_sb + (np.arange(C) - C / 2) * f_s / C
    for s1 in range(S):
        for s2 in range(s1 + 1):
            rot = np.exp(2j * np.pi * fc * (taus[s1] - taus[s2]))
            bl = oracle.baseline_index(s1, s2)
            for q in range(4):
                np.testing.assert_allclose(V1[:, bl, q], rot * V0[:, bl, q], rtol=0,
                                           atol=1e-8 * np.abs(V0[:, bl, q]).max())


def test_linear_delay_drift_geometric_series():
    """Tone in channel c0, station 1 with tau(j) = tau0 + D j / N_c, station 0 undelayed:
    V_10(c0) = A^2 H0^2 e^{2 pi i F tau0} sum_j e^{i alpha j}, alpha = 2 pi F D / N_c,
    whose sum is e^{i alpha (N_c-1)/2} sin(N_c alpha / 2) / sin(alpha / 2)."""
    S, P, C, T, n_c, A, c0 = 2, 2, 64, 16, 64, 10.0, 40
    f_s, f_sb = synth.SAMPLE_RATE_HZ, 160e6
    F = f_sb + (c0 - C / 2) * f_s / C
    tau0, D = 1.0e-6, 3.1e-9
    x, hist = _tone_block(S, P, C, T, n_c, A, (c0 - C // 2) / C)
    delays = np.array([[0.0, 0.0], [tau0, tau0 + D]])
    h = synth.fir_windowed_sinc(C, T)
    V = oracle.fx_block(x, hist, h, None, [f_sb], f_s, delays, C, T)["V"][0, c0]
    H0 = float(np.sum(h.astype(np.float64)))
    alpha = 2 * np.pi * F * D / n_c
    series = np.exp(1j * alpha * (n_c - 1) / 2) * np.sin(n_c * alpha / 2) / np.sin(alpha / 2)
    want = A ** 2 * H0 ** 2 * np.exp(2j * np.pi * F * tau0) * series
    got = V[oracle.baseline_index(1, 0), 0]
    assert abs(got - want) < 1e-8 * abs(want)
    assert abs(series) < 0.95 * n_c      # the drift really decorrelates


# ---------------------------------------------------------------- range reduction -------

def test_range_reduction_against_exact_rationals():
    rng = np.random.default_rng(31)
    n_c = 3072
    for _ in range(40):
        f_c = float(rng.uniform(10e6, 250e6))
        t0 = float(rng.uniform(-5e-6, 5e-6))
        t1 = t0 + float(rng.uniform(-3e-8, 3e-8))
        js = rng.integers(0, n_c, 8)
        cyc = oracle.delay_cycles(np.array([f_c]), t0, t1, n_c)[js, 0]
        r = oracle.reduce_cycles(cyc)
        for j, rv in zip(js, r):
            exact = Fraction(f_c) * (Fraction(t0) + (Fraction(t1) - Fraction(t0)) * int(j) / n_c)
            frac = exact - round(exact)
            assert abs(float(frac) - rv) < 1e-12 or abs(abs(float(frac)) - 0.5) < 1e-12
            assert -0.5 <= rv <= 0.5


# ---------------------------------------------------------------- invariants ------------

def _noise_run(seed, S=3, C=64, T=16, n_c=16, scale=1.0, mode="fp32"):
    rng = np.random.default_rng(seed)
    x = np.rint(_rand_complex(rng, (S, 2, 2, n_c * C), 40.0).real) + 1j * np.rint(_rand_complex(rng, (S, 2, 2, n_c * C), 40.0).real)
    hist = np.zeros((S, 2, 2, (T - 1) * C), np.complex128)
    delays = np.stack([rng.uniform(-5e-6, 5e-6, S)] * 2, 1)
    return oracle.fx_block(scale * x, scale * hist, synth.fir_windowed_sinc(C, T), synth.bandpass_ripple(C),
                           [110e6, 111e6], synth.SAMPLE_RATE_HZ, delays, C, T, mode=mode, gain=0.7)


def test_invariants_hermitian_autos_linearity():
    out = _noise_run(41)
    V, S = out["V"], 3
    # exact in the mathematics; float64 summation order leaves ~1e-16 relative residue
    for s in range(S):
        bl = oracle.baseline_index(s, s)
        for q in (0, 3):
            assert np.all(np.abs(V[..., bl, q].imag) <= 1e-13 * V[..., bl, q].real)
            assert np.all(V[..., bl, q].real > 0)
        scale = np.sqrt(V[..., bl, 0].real * V[..., bl, 3].real)
        assert np.all(np.abs(V[..., bl, 2] - np.conj(V[..., bl, 1])) <= 1e-13 * scale)
    out4 = _noise_run(41, scale=4.0)
    assert np.array_equal(out4["V"], 16.0 * V)


def test_int8_mode_invariants():
    out = _noise_run(42, mode="int8")
    V = out["V"]
    for s in range(3):
        bl = oracle.baseline_index(s, s)
        assert np.all(V[..., bl, 0, 1] == 0) and np.all(V[..., bl, 0, 0] >= 0)
        assert np.array_equal(V[..., bl, 2, 0], V[..., bl, 1, 0])
        assert np.array_equal(V[..., bl, 2, 1], -V[..., bl, 1, 1])
    assert np.abs(out["Q"]).max() <= 127


def test_requantise_rounding_and_clipping():
    Z = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 127.4, 127.5, 200.0, -126.5, -1000.0, 0.49999997])
    q = oracle.requantise_int8(Z + 0j, 1.0)[..., 0]
    assert list(q) == [0, 2, 2, 0, -2, 127, 127, 127, -126, -127, 0]
    q = oracle.requantise_int8(1j * Z, 1.0)[..., 1]
    assert list(q) == [0, 2, 2, 0, -2, 127, 127, 127, -126, -127, 0]


def test_history_carry_equals_one_long_block():
    """Two consecutive blocks with carried history equal one block of twice the length."""
    rng = np.random.default_rng(51)
    S, C, T, n_c = 2, 16, 4, 10
    x = _rand_complex(rng, (S, 2, 1, 2 * n_c * C), 9.0)
    h = rng.standard_normal(T * C).astype(np.float32)
    args = (h, None, [100e6], synth.SAMPLE_RATE_HZ, np.zeros((S, 2)), C, T)
    z0 = np.zeros((S, 2, 1, (T - 1) * C), np.complex128)
    a = oracle.fx_block(x[..., :n_c * C], z0, *args)
    b = oracle.fx_block(x[..., n_c * C:], a["history"], *args)
    both = oracle.fx_block(x, z0, *args)
    np.testing.assert_allclose(both["Z"][..., :n_c], a["Z"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(both["Z"][..., n_c:], b["Z"], rtol=0, atol=1e-12)


# ---------------------------------------------------------------- statistics ------------

def test_white_noise_power_and_decorrelation():
    """White complex Gaussian input (std sigma per component, rounded to integers):
    E[V_aa(c)] = N_c * 2 (sigma^2 + 1/12) * sum(h^2) * b_c^2, and independent stations
    give cross terms consistent with zero."""
    S, C, T, n_c, sigma = 4, 64, 16, 256, 32.0
    rng = np.random.default_rng(61)
    x = np.rint(rng.standard_normal((S, 2, 1, n_c * C)) * sigma) + 1j * np.rint(rng.standard_normal((S, 2, 1, n_c * C)) * sigma)
    hist = np.rint(rng.standard_normal((S, 2, 1, (T - 1) * C)) * sigma) + 1j * np.rint(rng.standard_normal((S, 2, 1, (T - 1) * C)) * sigma)
    h = synth.fir_windowed_sinc(C, T)
    b = synth.bandpass_ripple(C, 0.1)
    V = oracle.fx_block(x, hist, h, b, [130e6], synth.SAMPLE_RATE_HZ, np.zeros((S, 2)), C, T)["V"][0]
    h2 = float(np.sum(h.astype(np.float64) ** 2))
    mu = n_c * 2 * (sigma ** 2 + 1 / 12) * h2 * b.astype(np.float64) ** 2        # per channel
    autos = np.array([V[:, oracle.baseline_index(s, s), q].real for s in range(S) for q in (0, 3)])  # [8, C]
    ratio = autos / mu[None, :]
    # 8 inputs x 64 channels x 256 samples: the mean is within 1 % (many std errors)
    assert abs(ratio.mean() - 1) < 0.01
    assert np.all(np.abs(ratio - 1) < 0.6)
    cross = np.array([V[:, oracle.baseline_index(1, 0), q] for q in range(4)])
    # |V_ab| / sqrt(V_aa V_bb) ~ 1/sqrt(N_c_eff); with N_c = 256 allow 5 std
    coh = np.abs(cross) / np.sqrt(autos[0] * autos[2])[None, :]
    assert coh.mean() < 5 / math.sqrt(n_c)
