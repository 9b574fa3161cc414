"""O1: closed forms on the exact circle x(t) = r (cos 2 pi t, sin 2 pi t)
(test infrastructure only).

On the circle |f(s) - f(t)| = 2 r |sin(pi (s - t))| and J = 2 pi r, and
ln|2 sin(pi x)| = -sum_{k>=1} cos(2 pi k x)/k.  The cyclic B-spline B_i on N
uniform elements has Fourier coefficients
int B_i(s) e^{-2 pi i k s} ds = (1/N) e^{-2 pi i k (i + (p+1)/2)/N} sinc(k/N)^{p+1}.
Inserting both into eq. final_1 (with the factor -1/(2 pi) of eq. Gmatrix) gives

  A_ij = (2 pi r^2 / N^2) [ -ln r + sum_{k>=1} sinc(k/N)^{2p+2} cos(2 pi k (i-j)/N) / k ],

and, grouping k = c + N m, the exact finite sum with the Hurwitz zeta function

  A_ij = (2 pi r^2 / N^2) [ -ln r + pi^{-(2p+2)} N^{-1}
          sum_{c=1}^{N-1} sin(pi c/N)^{2p+2} cos(2 pi c (i-j)/N) zeta(2p+3, c/N) ].

The single-layer operator V = -(1/2 pi) int ln|x - y| . dgamma acts on the
circle as V[1] = -r ln r and V[cos k theta] = (r / 2k) cos k theta.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import zeta


def matrix(r: float, N: int, p: int) -> np.ndarray:
    """Exact Galerkin matrix A (N x N) on the circle of radius r."""
    c = np.arange(1, N)
    m = np.arange(N)
    terms = np.sin(math.pi * c / N) ** (2 * p + 2) * zeta(2 * p + 3, c / N)
    series = (np.cos(2.0 * math.pi * np.outer(m, c) / N) @ terms) / (math.pi ** (2 * p + 2) * N)
    row0 = 2.0 * math.pi * r * r / N ** 2 * (-math.log(r) + series)   # A_{0,m} = A_{i,i+m}
    idx = (np.arange(N)[None, :] - np.arange(N)[:, None]) % N
    return row0[idx]


def matrix_series(r: float, N: int, p: int, m: int, K: int = 400000) -> float:
    """A_{i,i+m} from the truncated Fourier series (slow cross-check)."""
    k = np.arange(1, K + 1, dtype=np.float64)
    return 2.0 * math.pi * r * r / N ** 2 * (
        -math.log(r) + np.sum(np.sinc(k / N) ** (2 * p + 2) * np.cos(2.0 * math.pi * k * m / N) / k))


def rhs_x2_minus_y2(r: float, N: int, p: int) -> np.ndarray:
    """beta_i = int B_i J g ds (eq. final_b1) for g = x1^2 - x2^2 = r^2 cos(4 pi t):
    beta_i = (2 pi r^3 / N) sinc(2/N)^{p+1} cos(4 pi (i + (p+1)/2) / N)."""
    i = np.arange(N)
    return 2.0 * math.pi * r ** 3 / N * np.sinc(2.0 / N) ** (p + 1) * np.cos(4.0 * math.pi * (i + (p + 1) / 2.0) / N)


def density_x2_minus_y2(r: float, t) -> np.ndarray:
    """Exact density phi of V phi = g for g = r^2 cos(2 theta): phi = 4 r cos(2 theta)."""
    return 4.0 * r * np.cos(4.0 * math.pi * np.asarray(t, dtype=np.float64))
