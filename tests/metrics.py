"""Comparison helpers shared by the GPU parity tests (no FX arithmetic here)."""

import numpy as np


def vis_complex(v):
    """[..., 4, 2] float (re, im) -> complex128 [..., 4]."""
    v = np.asarray(v)
    return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)


def coherence_error(V, Vref, S):
    """max |V - Vref| / sqrt(Vref[a,a] Vref[b,b]) over all stored entries.

    ``V``, ``Vref``: complex [..., B, 4] with baseline b(s1, s2) = s1(s1+1)/2 + s2 and pol
    pair q = 2 p1 + p2.  The error is in correlation-coefficient units: per-element relative
    error is meaningless for cross terms whose expectation is zero.
    """
    V = np.asarray(V)
    Vref = np.asarray(Vref)
    autos = np.empty(Vref.shape[:-2] + (S, 2))
    for s in range(S):
        bl = s * (s + 1) // 2 + s
        autos[..., s, 0] = Vref[..., bl, 0].real
        autos[..., s, 1] = Vref[..., bl, 3].real
    err = 0.0
    for s1 in range(S):
        for s2 in range(s1 + 1):
            bl = s1 * (s1 + 1) // 2 + s2
            for p1 in range(2):
                for p2 in range(2):
                    q = 2 * p1 + p2
                    den = np.sqrt(np.maximum(autos[..., s1, p1] * autos[..., s2, p2], 1e-300))
                    err = max(err, float(np.max(np.abs(V[..., bl, q] - Vref[..., bl, q]) / den)))
    return err


def frobenius_rel(V, Vref):
    return float(np.linalg.norm(np.asarray(V) - np.asarray(Vref)) / np.linalg.norm(np.asarray(Vref)))


def near_rounding_boundary(v, delta):
    """True where float ``v`` lies within ``delta`` of a half-integer (an int8 rounding
    boundary) or of the clip boundary +-127.5."""
    v = np.asarray(v, np.float64)
    frac = np.abs(v - np.floor(v) - 0.5)
    return (frac < delta) | (np.abs(np.abs(v) - 127.5) < delta)
