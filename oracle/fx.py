"""FP64 reference of the correlator's FX chain, written from the paper's description.

Test infrastructure only (see the package docstring).  Everything here is plain numpy in
float64 / complex128 / int64.  Library primitives used as single steps: ``numpy.fft.fft``
(the DFT of one row), ``numpy.matmul`` (the sum over time of the X stage).  There is no
blocking, fusion or reordering beyond what the definitions below state.

Citations name the paper's sections: "Processing steps" (sec. 3.2), "Hardware requirements
and design priorities" (sec. 6.1), "Dealing with jitter and hardware failure" (sec. 7.2),
"Workload distribution" (sec. 7.3, Table "Dimensions to map"), "Signal processing with GPU
kernels" (sec. 7.5), "Verification and validation" (sec. 8).

Notation
--------
S stations (antenna fields), P = 2 polarisations, M = S*P inputs, SB subbands, C channels,
T FIR taps, N samples per subband per input per block, N_c = N / C channel samples,
f_s the subband sample rate, h[T*C] the prototype FIR, b[C] the bandpass correction.

Readings where the paper is silent:
* FIR tap alignment: output j uses timeline rows j .. j+T-1 (the newest row last), i.e.
  ``y_j[p] = sum_t h[t*C + p] * x[(j - T + 1 + t)*C + p]`` over the block's own sample
  index, with the T-1 rows before the block taken from the carried history.
* DFT: forward, ``exp(-2 pi i p k / C)``, unnormalised; channel ``c = (k + C/2) mod C``
  (ascending sky frequency, DC at c = C/2).
* Channel sky frequency ``f_c = f_SB + (c - C/2) * f_s / C``.
* Fine delay: ``tau(j) = tau0 + (tau1 - tau0) * j / N_c`` (block start / end values,
  linear in between), phase in cycles ``f_c * tau(j)`` in float64, reduced to
  ``r = cyc - rint(cyc)``; the sample is multiplied by ``exp(+2 pi i r) * b_c``.
* Integration is a plain sum over the block (no division by N_c).
* Baselines ``s1 >= s2`` including autos, ``V = sum Z_{s1,p1} conj(Z_{s2,p2})``, pol pair
  ``q = 2*p1 + p2`` (XX, XY, YX, YY), baseline index ``s1*(s1+1)/2 + s2``.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "stream_timeline",
    "polyphase_filterbank",
    "channel_sky_freqs",
    "delay_cycles",
    "reduce_cycles",
    "fine_delay_bandpass",
    "requantise_int8",
    "correlate",
    "correlate_int",
    "visibilities_from_full",
    "baseline_index",
    "fx_block",
]


def stream_timeline(history: np.ndarray, block: np.ndarray) -> np.ndarray:
    """History samples followed by the block's samples, along the last axis.

    The FIR history of one block is carried into the next ("Signal processing with GPU
    kernels", sec. 7.5).  ``history`` holds the (T-1)*C samples that precede the block.
    """
    return np.concatenate([np.asarray(history, np.complex128), np.asarray(block, np.complex128)], axis=-1)


def polyphase_filterbank(timeline: np.ndarray, h: np.ndarray, C: int, T: int) -> np.ndarray:
    """Polyphase filter bank: C FIR filters of T taps feeding a C-point DFT.

    "Hardware requirements and design priorities" (sec. 6.1) describes the PPF as many FIR
    filters feeding an FFT; sec. 7.5 runs it as FIR then FFT kernels.

    ``timeline``: complex [..., (T-1)*C + N] (history then block).
    Returns X: complex128 [..., N_c, C], channel axis in ascending sky frequency.
    """
    timeline = np.asarray(timeline, np.complex128)
    h = np.asarray(h, np.float64)
    assert h.shape == (T * C,)
    n_rows = timeline.shape[-1] // C
    assert timeline.shape[-1] == n_rows * C and n_rows >= T - 1
    n_c = n_rows - (T - 1)
    rows = timeline.reshape(timeline.shape[:-1] + (n_rows, C))      # rows[..., r, p]
    taps = h.reshape(T, C)                                           # taps[t, p] = h[t*C + p]
    # FIR per phase p:  y[j, p] = sum_t taps[t, p] * rows[j + t, p]
    y = np.zeros(timeline.shape[:-1] + (n_c, C), np.complex128)
    for t in range(T):
        y += taps[t] * rows[..., t:t + n_c, :]
    # Forward unnormalised DFT over the phase axis, then ascending-frequency channel order.
    X = np.fft.fft(y, axis=-1)
    return np.roll(X, C // 2, axis=-1)          # channel c holds DFT bin (c - C/2) mod C


def channel_sky_freqs(f_sb: float, C: int, f_s: float) -> np.ndarray:
    """Sky centre frequency of each channel of one subband: f_SB + (c - C/2) * f_s / C."""
    c = np.arange(C, dtype=np.float64)
    return f_sb + (c - C / 2) * (f_s / C)


def delay_cycles(f_c: np.ndarray, tau0: float, tau1: float, n_c: int) -> np.ndarray:
    """Delay phase in cycles, ``f_c * tau(j)``, for every channel sample j of the block.

    Sec. 7.5: channel-dependent phase angles come from the residual delays at the start
    and end of the block, computed in double precision and interpolated linearly.
    Returns float64 [N_c, C].
    """
    j = np.arange(n_c, dtype=np.float64)
    tau = tau0 + (tau1 - tau0) * j / n_c if n_c > 0 else j
    return tau[:, None] * np.asarray(f_c, np.float64)[None, :]


def reduce_cycles(cyc: np.ndarray) -> np.ndarray:
    """Range reduction of a phase in cycles to [-1/2, 1/2]: ``cyc - rint(cyc)`` (float64)."""
    cyc = np.asarray(cyc, np.float64)
    return cyc - np.rint(cyc)


def fine_delay_bandpass(X: np.ndarray, cyc: np.ndarray, bandpass: np.ndarray) -> np.ndarray:
    """Fine delay compensation and bandpass correction of one input's channelised data.

    Sec. 7.5: rotate back the phase of each sample by a complex multiplication and apply
    the bandpass correction.  ``X``: [..., N_c, C]; ``cyc``: [N_c, C] cycles;
    ``bandpass``: real [C].  Returns ``X * exp(2 pi i r) * b_c`` with r the reduced cycles.
    """
    r = reduce_cycles(cyc)
    rot = np.exp(2j * np.pi * r) * np.asarray(bandpass, np.float64)[None, :]
    return np.asarray(X, np.complex128) * rot


def requantise_int8(Z: np.ndarray, gain: float) -> np.ndarray:
    """8-bit requantisation of channelised samples (reading; the paper gives no rule).

    The integer decision is taken in single precision, the arithmetic the paper's pipeline
    uses for samples ("Processing steps", sec. 3.2): ``v = float32(gain * Z)`` per
    component, rounded half to even, clipped to [-127, 127].  Returns int8 [..., 2] (re, im).
    """
    g = np.float64(np.float32(gain))
    Z = np.asarray(Z, np.complex128)
    out = np.empty(Z.shape + (2,), np.int8)
    for comp, part in ((0, Z.real), (1, Z.imag)):
        v = (g * part).astype(np.float32)
        out[..., comp] = np.clip(np.rint(v), -127, 127).astype(np.int8)
    return out


def baseline_index(s1: int, s2: int) -> int:
    """Index of baseline (s1, s2), s1 >= s2, in the lower-triangle order."""
    assert s1 >= s2 >= 0
    return s1 * (s1 + 1) // 2 + s2


def visibilities_from_full(Vfull: np.ndarray, S: int, P: int = 2) -> np.ndarray:
    """Pick the stored entries out of full M x M correlation matrices.

    ``Vfull[..., a, b]`` with input index ``a = s*P + p``.  Returns [..., B, P*P] with
    B = S(S+1)/2, baselines s1 >= s2 (autos included) and pol pair ``q = P*p1 + p2``.
    """
    B = S * (S + 1) // 2
    out = np.empty(Vfull.shape[:-2] + (B, P * P), Vfull.dtype)
    for s1 in range(S):
        for s2 in range(s1 + 1):
            bl = baseline_index(s1, s2)
            for p1 in range(P):
                for p2 in range(P):
                    out[..., bl, P * p1 + p2] = Vfull[..., s1 * P + p1, s2 * P + p2]
    return out


def correlate(Z: np.ndarray, S: int, P: int = 2) -> np.ndarray:
    """X stage: ``V[a, b] = sum_j Z[a, j] * conj(Z[b, j])`` per channel, float modes.

    Sec. 7.5: the last kernel correlates all pairs of antenna fields and integrates over
    the ~1 s block.  ``Z``: complex [..., M, N_c] (one channel per leading index).
    Returns complex128 [..., B, P*P].
    """
    Z = np.asarray(Z, np.complex128)
    Vfull = np.matmul(Z, np.conj(np.swapaxes(Z, -1, -2)))
    return visibilities_from_full(Vfull, S, P)


def correlate_int(Q: np.ndarray, S: int, P: int = 2) -> np.ndarray:
    """X stage on 8-bit samples with exact integer sums.

    ``Q``: int8 [..., M, N_c, 2] (re, im).  Every product and partial sum is an integer of
    magnitude below 2**53, so the float64 matmul below is exact in any summation order.
    Returns int64 [..., B, P*P, 2] (re, im).
    """
    qr = np.asarray(Q[..., 0], np.float64)
    qi = np.asarray(Q[..., 1], np.float64)
    assert np.abs(qr).max(initial=0) <= 128 and np.abs(qi).max(initial=0) <= 128
    n_c = Q.shape[-2]
    assert n_c * 2 * 128 * 128 < 2 ** 53
    T_ = lambda a: np.swapaxes(a, -1, -2)  # noqa: E731
    re = np.matmul(qr, T_(qr)) + np.matmul(qi, T_(qi))          # sum ar*br + ai*bi
    im = np.matmul(qi, T_(qr)) - np.matmul(qr, T_(qi))          # sum ai*br - ar*bi
    Vfull = np.stack([re, im], axis=-1).astype(np.int64)
    out = np.empty(Vfull.shape[:-3] + (S * (S + 1) // 2, P * P, 2), np.int64)
    for s1 in range(S):
        for s2 in range(s1 + 1):
            bl = baseline_index(s1, s2)
            for p1 in range(P):
                for p2 in range(P):
                    out[..., bl, P * p1 + p2, :] = Vfull[..., s1 * P + p1, s2 * P + p2, :]
    return out


def fx_block(x, history, h, bandpass, subband_freqs, sample_rate, delays, C, T,
             mode="fp32", gain=None, fp16_prescale_log2=0, return_channelised=True):
    """One block of the full FX chain for all subbands.

    Parameters
    ----------
    x : complex [S, P, SB, N]  block samples (exact integers for 8/16-bit input).
    history : complex [S, P, SB, (T-1)*C]  samples preceding the block (zeros after a reset).
    h : float [T*C] FIR prototype (float32 values, promoted to float64 here).
    bandpass : float [C] or None (ones).
    subband_freqs : float64 [SB] subband sky centre frequencies, Hz.
    sample_rate : subband sample rate f_s, Hz.
    delays : float64 [S, 2]  residual delay (s) at block start and block end.
    mode : "fp32" | "fp16_split" | "int8".  Float modes keep Z in float64 (no emulation of
        device rounding); "int8" requantises Z with ``requantise_int8`` before the X stage.
    fp16_prescale_log2 : accepted for interface symmetry; the float64 result does not
        depend on the power-of-two prescale.

    Returns dict with ``V`` ([SB, C, B, 4] complex128, or int64 [SB, C, B, 4, 2] in int8
    mode), ``Z`` ([SB, C, M, N_c] complex128, float modes) or ``Q`` (int8 [SB, C, M, N_c, 2]),
    ``Zf`` (the float64 channelised data before requantisation, int8 mode) and
    ``history`` (the carried samples for the next block).
    """
    x = np.asarray(x, np.complex128)
    S, P, SB, N = x.shape
    assert N % C == 0
    n_c = N // C
    M = S * P
    bandpass = np.ones(C) if bandpass is None else np.asarray(bandpass, np.float64)
    bandpass = bandpass.astype(np.float32).astype(np.float64)
    delays = np.asarray(delays, np.float64).reshape(S, 2)
    tl = stream_timeline(history, x)                           # [S, P, SB, (T-1)C + N]
    new_hist = tl[..., tl.shape[-1] - (T - 1) * C:].copy()
    Zall = np.empty((SB, C, M, n_c), np.complex128)
    for sb in range(SB):
        f_c = channel_sky_freqs(float(subband_freqs[sb]), C, sample_rate)
        X = polyphase_filterbank(tl[:, :, sb, :], h, C, T)      # [S, P, N_c, C]
        for s in range(S):
            cyc = delay_cycles(f_c, delays[s, 0], delays[s, 1], n_c)
            Zs = fine_delay_bandpass(X[s], cyc, bandpass)       # [P, N_c, C]
            for p in range(P):
                Zall[sb, :, s * P + p, :] = Zs[p].T
    out = {"history": new_hist}
    if mode == "int8":
        Q = requantise_int8(Zall, gain)
        out["V"] = correlate_int(Q, S, P)
        if return_channelised:
            out["Q"] = Q
            out["Zf"] = Zall
    else:
        out["V"] = correlate(Zall, S, P)
        if return_channelised:
            out["Z"] = Zall
    return out
