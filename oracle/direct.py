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

Reading of the rule's value: the quadrature sum itself, every term exact.  For
a Gauss point close to the node, f(t) - f(s) is nearly tangent to f'(t), and
in FP64 the numerator and the denominator of Kbar cancel to a relative error
of about eps / |t - s| (1e-10 for the closest points at N = 16384).  Those
terms (the Gauss points of the node's element and of its two neighbours) are
therefore evaluated from the exact rational parameters in exact arithmetic:
rational de Boor for B-spline geometry, 50-digit mpmath for polar curves.
Farther points carry at most a few eps, and FP64 keeps them.
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np

from . import curves, wq


def kbar(curve, s, t) -> np.ndarray:
    """Kbar(s, t) for arrays s, t (broadcast), s != t, outward normal of a
    counter-clockwise curve."""
    xs, ys = curves.evaluate(curve, s)[:2]
    xt, yt, dxt, dyt, _ = curves.evaluate(curve, t)
    ax, ay = xt - xs, yt - ys
    return (ax * dyt - ay * dxt) / (ax * ax + ay * ay)


def _exact_point(curve, t):
    """f(t) and f'(t) at an exact rational parameter t, as exact fractions
    (B-spline geometry: de Boor's algorithm on the span holding t, right-continuous)
    or as 50-digit mpmath numbers (polar curves)."""
    if curve.kind == "polar":
        th = 2 * mpmath.pi * mpmath.mpf(t.numerator) / t.denominator
        r, dr = mpmath.mpf(1), mpmath.mpf(0)
        for k, (a, ph) in enumerate(zip(curve.a, curve.phi), start=1):
            r += mpmath.mpf(a) * mpmath.cos(k * th + mpmath.mpf(ph))
            dr -= k * mpmath.mpf(a) * mpmath.sin(k * th + mpmath.mpf(ph))
        r, dr = mpmath.mpf(curve.r0) * r, mpmath.mpf(curve.r0) * dr
        c, sn = mpmath.cos(th), mpmath.sin(th)
        return r * c, r * sn, 2 * mpmath.pi * (dr * c - r * sn), 2 * mpmath.pi * (dr * sn + r * c)
    if curve.kind != "bspline":
        raise ValueError(f"exact evaluation: unsupported curve kind {curve.kind!r}")
    d = curve.degree
    Q = [(Fraction(float(q[0])), Fraction(float(q[1]))) for q in np.asarray(curve.ctrl, dtype=np.float64)]
    n = len(Q)
    if getattr(curve, "knots", None) is not None:
        tau = [Fraction(float(v)) for v in np.asarray(curve.knots, dtype=np.float64)[:-1]]
        knot = lambda k: tau[k % n] + (k // n)      # periodic extension, tau_{k+n} = tau_k + 1
    else:
        knot = lambda k: Fraction(k, n)
    l = math.floor(t) * n                           # the span l with knot(l) <= t < knot(l + 1)
    while knot(l + 1) <= t:
        l += 1
    P = [Q[(l - d + i) % n] for i in range(d + 1)]
    T = [knot(l - d + i) for i in range(2 * d + 2)]

    def deboor(ctrl, deg, T0):
        c = list(ctrl)
        for rr in range(1, deg + 1):
            for i in range(deg, rr - 1, -1):
                al = (t - T0[i]) / (T0[i + deg + 1 - rr] - T0[i])
                c[i] = ((1 - al) * c[i - 1][0] + al * c[i][0], (1 - al) * c[i - 1][1] + al * c[i][1])
        return c[deg]

    x, y = deboor(P, d, T)
    D = [(d * (P[i][0] - P[i - 1][0]) / (T[i + d] - T[i]), d * (P[i][1] - P[i - 1][1]) / (T[i + d] - T[i]))
         for i in range(1, d + 1)]
    dx, dy = deboor(D, d - 1, T[1:]) if d > 1 else D[0]
    return x, y, dx, dy


def kbar_exact(curve, s, t, cache=None) -> float:
    """Kbar(s, t) for exact rational parameters s != t (mod 1), evaluated exactly
    (B-spline geometry) or with 50 digits (polar curves), then rounded.  cache:
    an optional dict of exact points by parameter."""
    def point(u):
        if cache is None:
            return _exact_point(curve, u)
        if u not in cache:
            cache[u] = _exact_point(curve, u)
        return cache[u]
    with mpmath.workdps(50):
        x1, y1 = point(s)[:2]
        x2, y2, dx2, dy2 = point(t)
        ax, ay = x2 - x1, y2 - y1
        return float((ax * dy2 - ay * dx2) / (ax * ax + ay * ay))


def near_window(n: int, N: int, R: int):
    """The elements whose Gauss points are evaluated exactly for node n: its
    own element and the two neighbours (fewer for N < 3)."""
    e = n // (2 * R)
    return sorted({(e - 1) % N, e % N, (e + 1) % N})


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
    # the near terms, exactly: replace the FP64 value of each by the exact one
    u = 0.5 * (np.polynomial.legendre.leggauss(G)[0] + 1.0)
    cache = {}
    for i, n in enumerate(rows):
        s = Fraction(int(n), 2 * R * N)
        for e in near_window(int(n), N, R):
            for q in range(G):
                k = e * G + q
                t = (e + Fraction(float(u[q]))) / N
                ax = x2[k] - x1[i]
                ay = y2[k] - y1[i]
                Kd = (ax * dy2[k] - ay * dx2[k]) / (ax * ax + ay * ay)
                v[i] += coef[k] * (kbar_exact(curve, s, t, cache) - Kd)
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
