"""Reference matrices for the log part of coincident / adjacent element pairs
(test infrastructure only).

On a pair of elements of length h, the element-by-element rule (Section 5,
Remark) splits ln|f(s) - f(t)| = [ln|f(s) - f(t)| - ln|s - t|] + ln|s - t|.
The log part of the pair integral is integrated after interpolating each
smooth factor phi = B J at the Gs Gauss-Legendre points of its element:

  int_e1 int_e2 l_a(s) l_b(t) ln|s - t| dt ds = h^2 (ln h w_a w_b + Mhat_ab),

with l_a the Lagrange polynomials on [0, 1] and w_a = int l_a the Gauss weights.
Mhat is evaluated here in 60-digit arithmetic from two exact monomial moment
formulas (derived by splitting the unit square along its diagonal and
substituting v = u x, resp. u = 1 - x, in the triangles):

coincident  C_mn = int_0^1 int_0^1 u^m v^n ln|u - v| du dv
            = -(1/(m+1) + 1/(n+1)) / (m+n+2)^2 - (H_{m+1}/(m+1) + H_{n+1}/(n+1)) / (m+n+2)
adjacent    D_mn = int_0^1 int_0^1 u^m v^n ln(1 + v - u) du dv        (u left, v right)
            = sum_k C(m,k) (-1)^k E_kn,
            E_kn = int int x^k y^n ln(x + y) = -(1/(k+1) + 1/(n+1)) / (k+n+2)^2 + (L_k + L_n) / (k+n+2),
            L_q = int_0^1 z^q ln(1 + z) dz = (ln 2 - T_{q+1}) / (q+1),
            T_q = int_0^1 z^q / (1 + z) dz,  T_0 = ln 2,  T_q = 1/q - T_{q-1}.
"""
from __future__ import annotations

import functools
from math import comb

import mpmath as mp
import numpy as np

_DPS = 60


def _harmonic(n):
    return mp.fsum(mp.mpf(1) / k for k in range(1, n + 1))


def coincident_moment(m: int, n: int):
    s = m + n + 2
    return (-(mp.mpf(1) / (m + 1) + mp.mpf(1) / (n + 1)) / s ** 2
            - (_harmonic(m + 1) / (m + 1) + _harmonic(n + 1) / (n + 1)) / s)


def _T(q):
    t = mp.log(2)
    for k in range(1, q + 1):
        t = mp.mpf(1) / k - t
    return t


def _L(q):
    return (mp.log(2) - _T(q + 1)) / (q + 1)


def _E(k, n):
    s = k + n + 2
    return -(mp.mpf(1) / (k + 1) + mp.mpf(1) / (n + 1)) / s ** 2 + (_L(k) + _L(n)) / s


def adjacent_moment(m: int, n: int):
    return mp.fsum(comb(m, k) * (-1) ** k * _E(k, n) for k in range(m + 1))


def _gauss_nodes_mp(n):
    """Gauss-Legendre nodes / weights on [0, 1] in mp precision (Newton on P_n)."""
    x0, _ = np.polynomial.legendre.leggauss(n)
    xs, ws = [], []
    for x in x0:
        x = mp.mpf(float(x))
        for _ in range(100):
            pn = mp.legendre(n, x)
            dp = n * (x * pn - mp.legendre(n - 1, x)) / (x * x - 1)
            dx = pn / dp
            x -= dx
            if abs(dx) < mp.mpf(10) ** (-_DPS + 5):
                break
        dp = n * (x * mp.legendre(n, x) - mp.legendre(n - 1, x)) / (x * x - 1)
        w = 2 / ((1 - x * x) * dp * dp)
        xs.append((x + 1) / 2)
        ws.append(w / 2)
    return xs, ws


@functools.lru_cache(maxsize=None)
def reference_matrices(Gs: int = 16):
    """Return (u, w, Mco, Madj) as float64 arrays: Gauss nodes / weights on [0, 1]
    and the (Gs x Gs) coincident / adjacent matrices (row index: s-element on the
    left for the adjacent case)."""
    with mp.workdps(_DPS):
        u, w = _gauss_nodes_mp(Gs)
        V = mp.matrix(Gs, Gs)
        for a in range(Gs):
            for m in range(Gs):
                V[a, m] = u[a] ** m
        L = V ** -1            # l_b(u) = sum_m L[m, b] u^m
        C = mp.matrix(Gs, Gs)
        D = mp.matrix(Gs, Gs)
        for m in range(Gs):
            for n in range(Gs):
                C[m, n] = coincident_moment(m, n)
                D[m, n] = adjacent_moment(m, n)
        Mco = L.T * C * L
        Madj = L.T * D * L
        tof = lambda X: np.array([[float(X[i, j]) for j in range(Gs)] for i in range(Gs)])
        return (np.array([float(x) for x in u]), np.array([float(x) for x in w]), tof(Mco), tof(Madj))
