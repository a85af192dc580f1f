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
* output resolution stays at 256 channels (the optional transform to 1 or 16 channels per
  subband is not part of this reference).
"""

from __future__ import annotations

import numpy as np

from . import fx

__all__ = ["beam_cycles", "beam_weights", "coherent_beams", "stokes", "integrate", "incoherent_stokes",
           "beamform_block"]


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
