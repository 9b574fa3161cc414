"""Uniform B-splines for the oracle (test infrastructure only).

The B-spline basis of degree d on a knot vector is defined by the Cox-de Boor
recurrence quoted in Section 4.2 (the recurrence used to derive eq. recIq).
On integer knots every basis function is a translate of the cardinal B-spline
M_d supported on [0, d+1]; a closed curve uses the periodic (cyclic) basis of
Section 3, B_i(t) = M_d(N t - i mod N) on N uniform elements of [0, 1).
"""
from __future__ import annotations

import numpy as np


def cardinal(p: int, x) -> np.ndarray:
    """M_p(x) via the Cox-de Boor recurrence on the integer knots 0..p+1.

    Degree 0: indicator of [k, k+1).  Degree r from degree r-1:
    B_{k,r}(x) = (x - k)/r * B_{k,r-1}(x) + (k + r + 1 - x)/r * B_{k+1,r-1}(x).
    """
    x = np.asarray(x, dtype=np.float64)
    B = [((x >= k) & (x < k + 1)).astype(np.float64) for k in range(p + 1)]
    for r in range(1, p + 1):
        B = [(x - k) / r * B[k] + (k + r + 1 - x) / r * B[k + 1] for k in range(p + 1 - r)]
    return B[0]


def cardinal_deriv(p: int, x) -> np.ndarray:
    """M_p'(x) = M_{p-1}(x) - M_{p-1}(x - 1) (derivative of the recurrence)."""
    if p == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return cardinal(p - 1, x) - cardinal(p - 1, np.asarray(x, dtype=np.float64) - 1.0)


def periodic(p: int, N: int, i: int, t) -> np.ndarray:
    """Cyclic basis function B_i of degree p on N uniform elements of [0, 1);
    supported on [i/N, (i+p+1)/N) mod 1."""
    t = np.asarray(t, dtype=np.float64)
    return cardinal(p, np.mod(N * t - i, N))


def piece_monomials(p: int) -> np.ndarray:
    """coef[c, a] with M_p(c + u) = sum_a coef[c, a] u^a for u in [0, 1],
    c = 0..p, from the truncated-power form
    M_p(x) = (1/p!) sum_k (-1)^k C(p+1, k) (x - k)_+^p."""
    from math import comb, factorial
    coef = np.zeros((p + 1, p + 1))
    for c in range(p + 1):
        for k in range(c + 1):
            for a in range(p + 1):
                coef[c, a] += (-1) ** k * comb(p + 1, k) * comb(p, a) * float(c - k) ** (p - a)
    return coef / factorial(p)


def general(knots, d: int, j: int, t) -> np.ndarray:
    """B_{j,d}(t) on an arbitrary non-decreasing knot vector by the Cox-de Boor
    recurrence (Section 4.2), with the convention that a term whose knot
    difference vanishes is dropped.  Degree-0 functions are right-open
    indicators, except that the last non-empty span also contains its right end."""
    T = np.asarray(knots, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    last = np.max(np.nonzero(T[1:] > T[:-1])[0])

    def rec(i, r):
        if r == 0:
            inside = (t >= T[i]) & (t < T[i + 1])
            if i == last:
                inside = inside | (t == T[i + 1])
            return inside.astype(np.float64)
        out = np.zeros_like(t)
        if T[i + r] > T[i]:
            out = out + (t - T[i]) / (T[i + r] - T[i]) * rec(i, r - 1)
        if T[i + r + 1] > T[i + 1]:
            out = out + (T[i + r + 1] - t) / (T[i + r + 1] - T[i + 1]) * rec(i + 1, r - 1)
        return out

    return rec(j, d)
