"""FP64 reference of the beamformer pipeline, written from the paper's description.

Test infrastructure only (see the package docstring).

Paper ("Signal processing with GPU kernels", sec. 7.5; "System requirements", sec. 5): the
beamformer shares the first kernels with the correlator -- polyphase filter bank, fine delay
compensation and bandpass correction -- but channelises to 256 channels per subband.
Coherent beams then shift each station's data by a per-beam phase (beams pointed away from
the centre direction, computed like the delay compensation: angle in double precision,
rotation in single precision) and sum over stations; the output is either the complex
voltages of both polarisations or the Stokes parameters I or IQUV.  Incoherent beams compute
Stokes parameters per station first and then sum over stations.  Time resolution can be
traded for frequency resolution within a subband.

Readings where the paper is silent:
* channelisation, fine delay and bandpass exactly as ``fx.fx_block`` with C = 256;
* beam weights ``w[b][s] = exp(+2 pi i f_c dtau[b][s])`` with ``dtau`` the extra arrival
  delay of beam b's direction at station s relative to the centre (same sign convention as
  the fine delay), constant over the block, phase reduced to ``cyc - rint(cyc)`` in FP64;
* ``beam[b][p][t] = sum_s w[b][s] Z[s*P + p][t]`` for both polarisations p;
* Stokes from the two polarisations X (p = 0), Y (p = 1): ``I = |X|^2 + |Y|^2``,
  ``Q = |X|^2 - |Y|^2``, ``U = 2 Re(X conj Y)``, ``V = 2 Im(X conj Y)``;
* time integration: plain sums over ``n_int`` consecutive channel samples (N_c a multiple
  of n_int);
* output resolution (the paper transforms the 256 beamformed channels "to the requested
  output resolution, often 1 or 16 channels per subband", and time resolution is traded for
  frequency resolution within a subband): ``resolution_transform`` takes each channel
  sample's C values back to C time samples with an inverse DFT (scaled 1/C, channel c
  carrying frequency index c - C/2), joins the rows into one time series at the subband
  sample rate, cuts it into consecutive groups of C_out samples and gives each group an
  unnormalised forward C_out-point DFT (output channel c' carrying index c' - C_out/2).
  C_out = 1 is the time series itself; C_out = C reproduces the input.  Stokes of the
  transformed voltages are summed over n_int consecutive output samples.
"""

from __future__ import annotations

import numpy as np

from . import fx

__all__ = ["beam_cycles", "beam_weights", "coherent_beams", "stokes", "integrate", "incoherent_stokes",
           "beamform_block", "resolution_transform", "transformed_stokes"]


def beam_cycles(f_c: np.ndarray, dtau: np.ndarray) -> np.ndarray:
    """Phase of beam b at station s in channel c, in cycles: f_c * dtau[b][s] (FP64).
    Returns [C, NB, S]."""
    return np.asarray(f_c, np.float64)[:, None, None] * np.asarray(dtau, np.float64)[None, :, :]


def beam_weights(f_c: np.ndarray, dtau: np.ndarray) -> np.ndarray:
    """exp(+2 pi i r) with r the phase reduced to [-1/2, 1/2] cycles: [C, NB, S] complex."""
    return np.exp(2j * np.pi * fx.reduce_cycles(beam_cycles(f_c, dtau)))


def coherent_beams(Z: np.ndarray, W: np.ndarray, S: int, P: int = 2) -> np.ndarray:
    """Z [C, M, N_c] channelised (row s*P + p); W [C, NB, S].  Returns [C, NB, P, N_c]:
    the weighted sum over stations for each polarisation."""
    Z = np.asarray(Z, np.complex128)
    C, M, n_c = Z.shape
    Zp = Z.reshape(C, S, P, n_c)
    return np.einsum("cbs,cspt->cbpt", np.asarray(W, np.complex128), Zp)


def stokes(X: np.ndarray, Y: np.ndarray, which: str = "IQUV") -> np.ndarray:
    """Stokes parameters of two polarisation voltages, stacked on a new axis -2 (``which``
    = "I" or "IQUV")."""
    xx = np.abs(X) ** 2
    yy = np.abs(Y) ** 2
    xy = X * np.conj(Y)
    parts = {"I": xx + yy, "Q": xx - yy, "U": 2 * xy.real, "V": 2 * xy.imag}
    return np.stack([parts[k] for k in which], axis=-2)


def integrate(v: np.ndarray, n_int: int) -> np.ndarray:
    """Plain sums over n_int consecutive samples of the last axis."""
    v = np.asarray(v)
    n = v.shape[-1]
    assert n % n_int == 0, (n, n_int)
    return v.reshape(v.shape[:-1] + (n // n_int, n_int)).sum(axis=-1)


def incoherent_stokes(Z: np.ndarray, S: int, P: int = 2, which: str = "IQUV") -> np.ndarray:
    """Stokes per station from its two polarisations, summed over stations: Z [C, M, N_c]
    -> [C, len(which), N_c]."""
    Z = np.asarray(Z, np.complex128)
    C, M, n_c = Z.shape
    Zp = Z.reshape(C, S, P, n_c)
    return stokes(Zp[:, :, 0], Zp[:, :, 1], which).sum(axis=1)


def beamform_block(x, history, h, bandpass, subband_freqs, sample_rate, delays, beam_dtau, C, T,
                   which="IQUV", n_int=1, return_channelised=False):
    """One block of the beamformer pipeline for all subbands.

    x complex [S, P, SB, N]; history [S, P, SB, (T-1)*C]; h [T*C]; delays [S, 2] (centre
    pointing, fine delay); beam_dtau [NB, S] seconds.  Returns a dict with ``beams``
    ([SB, C, NB, P, N_c] complex voltages), ``coherent`` ([SB, C, NB, len(which), N_c/n_int]),
    ``incoherent`` ([SB, C, len(which), N_c/n_int]), ``history`` and optionally ``Z``."""
    x = np.asarray(x, np.complex128)
    S, P, SB, N = x.shape
    res = fx.fx_block(x, history, h, bandpass, subband_freqs, sample_rate, delays, C, T, mode="fp32")
    Z = res["Z"]                                           # [SB, C, M, N_c]
    NB = np.asarray(beam_dtau).shape[0]
    n_c = N // C
    beams = np.empty((SB, C, NB, P, n_c), np.complex128)
    coh = np.empty((SB, C, NB, len(which), n_c // n_int))
    inc = np.empty((SB, C, len(which), n_c // n_int))
    for sb in range(SB):
        f_c = fx.channel_sky_freqs(float(subband_freqs[sb]), C, sample_rate)
        W = beam_weights(f_c, beam_dtau)
        B = coherent_beams(Z[sb], W, S, P)
        beams[sb] = B
        coh[sb] = integrate(stokes(B[:, :, 0], B[:, :, 1], which), n_int)
        inc[sb] = integrate(incoherent_stokes(Z[sb], S, P, which), n_int)
    out = {"beams": beams, "coherent": coh, "incoherent": inc, "history": res["history"]}
    if return_channelised:
        out["Z"] = Z
    return out


def resolution_transform(B, C_out: int) -> np.ndarray:
    """Beamformed voltages at C channels -> C_out channels (the reading in the module
    docstring).  ``B`` complex [..., C, n_c] (channel axis -2, channel sample axis -1).
    Returns complex [..., n_c * C / C_out, C_out]: output sample g, output channel c'.

        u[j C + n] = (1/C) sum_c B[c, j] exp(+2 pi i n (c - C/2) / C),      n < C
        O[g, c']   = sum_m u[g C_out + m] exp(-2 pi i m (c' - C_out/2) / C_out),  m < C_out
    """
    B = np.asarray(B, np.complex128)
    *lead, C, n_c = B.shape
    assert C % C_out == 0, (C, C_out)
    n = np.arange(C)
    E = np.exp(2j * np.pi * np.outer(n, np.arange(C) - C // 2) / C) / C      # [n, c]
    u = np.einsum("nc,...cj->...jn", E, B).reshape(*lead, n_c * C)           # time t = j C + n
    m = np.arange(C_out)
    F = np.exp(-2j * np.pi * np.outer(m, np.arange(C_out) - C_out // 2) / C_out)   # [m, c']
    return u.reshape(*lead, n_c * C // C_out, C_out) @ F


def transformed_stokes(beams, C_out: int, which: str = "IQUV", n_int: int = 1) -> np.ndarray:
    """Stokes of the transformed voltages of both polarisations, summed over n_int output
    samples.  ``beams`` [..., P = 2, C, n_c] -> [..., n_c C / C_out / n_int, C_out, len(which)]."""
    O = resolution_transform(beams, C_out)                 # [..., 2, G, C_out]
    st = stokes(O[..., 0, :, :], O[..., 1, :, :], which)   # [..., G, len(which), C_out]
    st = np.moveaxis(st, -3, -1)                           # [..., len(which), C_out, G]
    st = integrate(st, n_int)                              # [..., len(which), C_out, G / n_int]
    return np.moveaxis(st, -1, -3).swapaxes(-1, -2)        # [..., G / n_int, C_out, len(which)]
