"""O4: right-hand side of the direct formulation (test infrastructure only).

The direct boundary integral equation of the interior Dirichlet problem
(Section 2, eq. seconda_BIE, weak form eq. weakpb) has the same Galerkin
matrix as the indirect one and the right-hand side

    F_i = 1/2 b1_i - 1/(2 pi) b2_i,

b1 of eq. final_b1 and b2 of eq. final_b2 (Section 3.2):

    b2_i = int B_i(s) J(s) int Kbar(s, t) u_D(t) dt ds,
    Kbar(s, t) = d ln|x - y| / d n_y (x = f(s), y = f(t)) * J(t).

Its solution is the outward flux q = du/dn on the curve, q(f(t)) ~ sum_j alpha_j B_j(t).

Reading of the sign: the expression of Kbar written out in Section 3.2 belongs
to the normal (-f2', f1') / J, which points outward for a clockwise
parametrisation.  The curves here run counter-clockwise, so the outward normal
is (f2', -f1') / J and

    Kbar(s, t) = [(f1(t) - f1(s)) f2'(t) - (f2(t) - f2(s)) f1'(t)] / |f(s) - f(t)|^2,

the printed expression with the opposite sign; with it eq. seconda_BIE holds
for the outward flux (on the circle of radius r, Kbar = pi everywhere).

Quadrature (Section 5): the outer integral by the regular weighted rule of
Alg. 1 on the nodes eta (the weights of b1), the inner one by composite
Gauss-Legendre with G points per element.  G is even, so no Gauss point falls
on a node and Kbar is never evaluated at coincident points.
"""
from __future__ import annotations

import math

import numpy as np

from . import curves, wq


def kbar(curve, s, t) -> np.ndarray:
    """Kbar(s, t) for arrays s, t (broadcast), s != t, outward normal of a
    counter-clockwise curve."""
    xs, ys = curves.evaluate(curve, s)[:2]
    xt, yt, dxt, dyt, _ = curves.evaluate(curve, t)
    ax, ay = xt - xs, yt - ys
    return (ax * dyt - ay * dxt) / (ax * ax + ay * ay)


def gauss_points(N: int, G: int):
    """Composite G-point Gauss-Legendre on the N elements of [0, 1):
    parameters t[e G + g] = (e + u_g) / N and weights w_g / N."""
    u, w = np.polynomial.legendre.leggauss(G)
    u = 0.5 * (u + 1.0)
    w = 0.5 * w
    t = (np.arange(N)[:, None] + u[None, :]).ravel() / N
    wt = np.tile(w, N) / N
    return t, wt


def inner_sums(curve, N: int, R: int, G: int, g, rows=None) -> np.ndarray:
    """v_n = sum over the Gauss points of w Kbar(eta_n, xi) u_D(xi), for the
    nodes n in `rows` (all 2 R N nodes by default)."""
    if G % 2:
        raise ValueError("G must be even")
    eta = wq.nodes(N, R)
    rows = np.arange(eta.size) if rows is None else np.asarray(rows)
    t2, wt = gauss_points(N, G)
    x2, y2, dx2, dy2, _ = curves.evaluate(curve, t2)
    coef = wt * g(x2, y2)
    x1, y1 = curves.evaluate(curve, eta[rows])[:2]
    v = np.zeros(rows.size)
    for c0 in range(0, rows.size, 256):
        ax = x2[None, :] - x1[c0:c0 + 256, None]
        ay = y2[None, :] - y1[c0:c0 + 256, None]
        K = (ax * dy2[None, :] - ay * dx2[None, :]) / (ax * ax + ay * ay)
        v[c0:c0 + 256] = K @ coef
    return v


def b2(curve, p: int, N: int, R: int, G: int, g) -> np.ndarray:
    """eq. final_b2 by the rule of Section 5: b2_i = sum_n w_n^(i) J(eta_n) v_n."""
    eta = wq.nodes(N, R)
    J = curves.evaluate(curve, eta)[4]
    v = inner_sums(curve, N, R, G, g)
    out = np.zeros(N)
    for i, (nset, w) in wq.regular_weights(p, N, R).items():
        out[i] = np.sum(w * J[nset] * v[nset])
    return out


def rhs(curve, p: int, N: int, R: int, G: int, g) -> np.ndarray:
    """F = 1/2 b1 - 1/(2 pi) b2 (eq. seconda_BIE in the weak form eq. weakpb)."""
    return 0.5 * wq.rhs(curve, p, N, R, g) - b2(curve, p, N, R, G, g) / (2.0 * math.pi)


def outward_flux(curve, t, grad) -> np.ndarray:
    """du/dn at f(t) for a function u with gradient grad(x, y) -> (ux, uy)."""
    x, y, dx, dy, J = curves.evaluate(curve, t)
    ux, uy = grad(x, y)
    return (ux * dy - uy * dx) / J
