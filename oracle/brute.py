"""The FX chain's defining sums as plain Python loops (tiny inputs only).

Test infrastructure, like the rest of ``oracle``.  Each function evaluates one definition
term by term with Python complex numbers and ``cmath``: no numpy FFT, no matmul, no
vectorisation.  The vectorised reference in ``oracle.fx`` is checked against these on
inputs small enough for loops (a few stations, C <= 8, a few dozen samples).
"""

from __future__ import annotations

import cmath
import math


def ppf_loop(timeline, h, C, T):
    """Polyphase filter bank of one input by direct summation.

    ``timeline``: list of complex, history ((T-1)*C samples) followed by the block.
    Returns ``X[j][c]`` for j < N_c, channel c, with
    ``X[j][c] = sum_p exp(-2 pi i p k / C) * sum_t h[t*C+p] * x[(j+t)*C + p]`` where
    ``k = (c - C/2) mod C`` and x indexes the timeline.
    """
    n_rows = len(timeline) // C
    n_c = n_rows - (T - 1)
    out = []
    for j in range(n_c):
        y = []
        for p in range(C):
            acc = 0j
            for t in range(T):
                acc += h[t * C + p] * timeline[(j + t) * C + p]
            y.append(acc)
        row = []
        for c in range(C):
            k = (c - C // 2) % C
            s = 0j
            for p in range(C):
                s += y[p] * cmath.exp(-2j * math.pi * p * k / C)
            row.append(s)
        out.append(row)
    return out


def delay_rotate_loop(X, f_sb, C, f_s, tau0, tau1, bandpass):
    """Fine delay + bandpass, one term at a time: ``X * exp(2 pi i f_c tau(j)) * b_c``.

    Uses the unreduced phase ``2 pi f_c tau(j)`` (the reduction to [-1/2, 1/2] cycles is an
    exact identity of the exponential; only its rounding differs).
    """
    n_c = len(X)
    out = []
    for j in range(n_c):
        tau = tau0 + (tau1 - tau0) * j / n_c
        row = []
        for c in range(C):
            f_c = f_sb + (c - C / 2) * f_s / C
            row.append(X[j][c] * cmath.exp(2j * math.pi * f_c * tau) * bandpass[c])
        out.append(row)
    return out


def correlate_loop(Z, S, P=2):
    """X stage by direct summation for one channel.

    ``Z[a][j]`` complex, a = s*P + p.  Returns ``V[bl][q]`` with bl = s1(s1+1)/2 + s2,
    q = P*p1 + p2, ``V = sum_j Z[s1*P+p1][j] * conj(Z[s2*P+p2][j])``.
    """
    n_c = len(Z[0])
    V = []
    for s1 in range(S):
        for s2 in range(s1 + 1):
            entry = []
            for p1 in range(P):
                for p2 in range(P):
                    a, b = s1 * P + p1, s2 * P + p2
                    acc = 0j
                    for j in range(n_c):
                        acc += Z[a][j] * Z[b][j].conjugate()
                    entry.append(acc)
            V.append(entry)
    return V


def correlate_int_loop(Q, S, P=2):
    """X stage on integer samples with Python integers (exact).

    ``Q[a][j] = (re, im)`` ints.  Returns ``V[bl][q] = (re, im)`` ints.
    """
    n_c = len(Q[0])
    V = []
    for s1 in range(S):
        for s2 in range(s1 + 1):
            entry = []
            for p1 in range(P):
                for p2 in range(P):
                    a, b = s1 * P + p1, s2 * P + p2
                    re = im = 0
                    for j in range(n_c):
                        ar, ai = Q[a][j]
                        br, bi = Q[b][j]
                        re += ar * br + ai * bi
                        im += ai * br - ar * bi
                    entry.append((re, im))
            V.append(entry)
    return V
