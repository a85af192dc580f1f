"""FP64 reference of the gain-applied correlator and its adjoint (test infrastructure).

Per-input complex gains g (one per station, polarisation, subband and channel, constant over
the block) multiply the channelised samples before the X stage: Z'_a = g_a Z_a.  Because the
gains do not depend on the channel sample j, the gain-applied visibilities are the ungained
ones scaled per entry:

    V'_ab = sum_j g_a Z_a conj(g_b Z_b) = g_a conj(g_b) V0_ab.

For a real loss L(V') the gradient in PyTorch's convention (dL/dRe g + i dL/dIm g) follows
from the Wirtinger derivatives of V'_ab (which depends on g_a and on conj(g_b)):

    grad_k = sum_{entries with b = k} conj(G_ab) g_a V0_ab
           + sum_{entries with a = k} G_ab g_b conj(V0_ab),

with G = dL/dRe V' + i dL/dIm V' the upstream gradient.  An auto (a = b = k) takes both terms.
Layouts follow the library: gains [..., M] with input a = s*P + p; visibilities [..., B, 4]
with baseline s1(s1+1)/2 + s2 (s1 >= s2) and pol pair q = 2 p1 + p2.
"""

from __future__ import annotations

import numpy as np

from .fx import baseline_index


def _entries(S, P=2):
    """(bl, q, a, b) for every stored entry."""
    out = []
    for s1 in range(S):
        for s2 in range(s1 + 1):
            bl = baseline_index(s1, s2)
            for p1 in range(P):
                for p2 in range(P):
                    out.append((bl, P * p1 + p2, s1 * P + p1, s2 * P + p2))
    return out


def apply_gains(V0, g, S, P=2):
    """V'[..., bl, q] = g[..., a] conj(g[..., b]) V0[..., bl, q]."""
    V0 = np.asarray(V0, np.complex128)
    g = np.asarray(g, np.complex128)
    out = np.empty_like(V0)
    for bl, q, a, b in _entries(S, P):
        out[..., bl, q] = g[..., a] * np.conj(g[..., b]) * V0[..., bl, q]
    return out


def apply_gains_adjoint(V0, g, G, S, P=2):
    """Gradient with respect to g of a real loss whose gradient with respect to V' is G."""
    V0 = np.asarray(V0, np.complex128)
    g = np.asarray(g, np.complex128)
    G = np.asarray(G, np.complex128)
    grad = np.zeros_like(g)
    for bl, q, a, b in _entries(S, P):
        grad[..., b] += np.conj(G[..., bl, q]) * g[..., a] * V0[..., bl, q]
        grad[..., a] += G[..., bl, q] * g[..., b] * np.conj(V0[..., bl, q])
    return grad


def model_loss(V0, g, Mdl, S, P=2):
    """L = sum over stored entries |V' - M|^2 and its upstream gradient G = 2 (V' - M)."""
    E = apply_gains(V0, g, S, P) - np.asarray(Mdl, np.complex128)
    return float(np.sum(np.abs(E) ** 2)), 2.0 * E
