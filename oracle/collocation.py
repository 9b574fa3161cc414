"""O5: collocation BEM with the weighted quadrature rules (test infrastructure only).

Conclusions of the paper: the rules serve collocation BEM too, with the outer
collocation point fixed and the new rules used for the inner integral.  The
single-layer equation V phi = u_D is collocated at x_i, phi(f(t)) ~ sum_j
alpha_j B_j(t):

    A_ij = -1/(2 pi) int K(x_i, t) B_j(t) J(t) dt
         ~ -1/(2 pi) [ sum_n w_n^(j) K1(x_i, eta_n) J(eta_n)             (Alg. 1, weight B_j)
                       + sum_n w_n^(x_i) J(eta_n) B_j(eta_n) ]          (Alg. 2, source x_i)

with the periodic split K = K1 + K2 of the Galerkin oracle.  Reading of the
collocation points: the Greville abscissae of the cyclic basis,
x_i = (i + (p+1)/2) / N, which are nodes of eta (index 2 R i + R (p+1):
breakpoints for odd p, midpoints for even p), so the singular rule at x_i is one
of the rules the Galerkin assembly already uses.
"""
from __future__ import annotations

import math

import numpy as np

from . import bspline, curves, wq


def points(p: int, N: int, R: int) -> np.ndarray:
    """Node indices of the collocation points: 2 R i + R (p+1), i = 0..N-1 (mod 2RN)."""
    return (2 * R * np.arange(N) + R * (p + 1)) % (2 * R * N)


def matrix(curve, p: int, N: int, R: int) -> np.ndarray:
    """The N x N collocation matrix (not symmetric), dense."""
    eta = wq.nodes(N, R)
    x, y, _, _, J = curves.evaluate(curve, eta)
    rows = points(p, N, R)
    K1 = wq.K1_rows(x, y, J, eta, rows)                 # (N, 2M)
    Ws = wq.singular_weights(p, N, R, sources=rows)     # (N, 2M)
    A = np.zeros((N, N))
    Wd = wq.regular_weights(p, N, R)
    for j in range(N):
        nset, w = Wd[j]
        A[:, j] = K1[:, nset] @ (w * J[nset])
        Bj = bspline.periodic(p, N, j, eta)
        A[:, j] += Ws @ (J * Bj)
    return -A / (2.0 * math.pi)


def rhs(curve, p: int, N: int, R: int, g) -> np.ndarray:
    """u_D at the collocation points."""
    t = wq.nodes(N, R)[points(p, N, R)]
    x, y = curves.evaluate(curve, t)[:2]
    return g(x, y)
