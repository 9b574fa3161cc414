"""Pins for O1 (circle closed forms) and O2 (element-by-element oracle), CPU."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import bspline, circle, curves, ebe, nearfield


def _relmax(A, B):
    return np.abs(A - B).max() / np.abs(B).max()


# ------------------------------------------------------------------ O1
@pytest.mark.parametrize("N,p,m", [(8, 2, 1), (64, 3, 5), (256, 4, 0)])
def test_circle_hurwitz_equals_series(N, p, m):
    A = circle.matrix(0.5, N, p)
    assert abs(A[0, m] - circle.matrix_series(0.5, N, p, m)) < 1e-15 * abs(A[0, 0])


def test_circle_entries_brute_force():
    """Two entries of A on the circle r = 0.5, N = 8, p = 2 by nested adaptive
    quadrature of eq. final_1 with K = ln|f(s) - f(t)| (no series involved)."""
    r, N, p = 0.5, 8, 2
    J = 2 * math.pi * r
    A = circle.matrix(r, N, p)

    def K(s, t):
        return math.log(2 * r * abs(math.sin(math.pi * (s - t))))

    def B(i, t):
        return float(bspline.periodic(p, N, i, t))

    def entry(i, j):
        def inner(s):
            pts = sorted({(j + m) / N for m in range(p + 2)} | {s})
            tot = 0.0
            for a, b in zip(pts[:-1], pts[1:]):
                if b > a:
                    tot += integrate.quad(lambda t: B(j, t) * K(s, t), a, b, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
            return tot
        tot = sum(integrate.quad(lambda s: B(i, s) * inner(s), (i + e) / N, (i + e + 1) / N,
                                 epsabs=1e-15, epsrel=1e-12, limit=200)[0] for e in range(p + 1))
        return -J * J * tot / (2 * math.pi)

    for (i, j) in [(0, 0), (0, 2)]:
        assert abs(entry(i, j) - A[i, j]) < 1e-11 * abs(A[0, 0])


@pytest.mark.parametrize("N,p", [(16, 2), (64, 3)])
def test_circle_row_sum_is_V_of_one(N, p):
    """sum_j B_j = 1 and V[1] = -r ln r, so (A 1)_i = -2 pi r^2 ln r / N."""
    for r in (0.5, 0.3):
        A = circle.matrix(r, N, p)
        assert np.abs(A.sum(axis=1) + 2 * math.pi * r * r * math.log(r) / N).max() < 1e-16 * N


def test_circle_rhs_closed_form_vs_quadrature():
    r, N, p = 0.5, 16, 3
    beta = circle.rhs_x2_minus_y2(r, N, p)
    for i in (0, 5):
        f = lambda t: float(bspline.periodic(p, N, i, t)) * 2 * math.pi * r * (r * r * math.cos(4 * math.pi * t))
        num = sum(integrate.quad(f, (i + e) / N, (i + e + 1) / N, epsabs=1e-16, epsrel=1e-14)[0] for e in range(p + 1))
        assert abs(num - beta[i]) < 1e-14


# ------------------------------------------------------------------ near-field reference matrices
@pytest.mark.parametrize("m,n", [(0, 0), (1, 0), (3, 2), (6, 5)])
def test_nearfield_moments_brute_force(m, n):
    with mp.workdps(25):
        def inner_c(v):
            return mp.quad(lambda u: u ** m * mp.log(abs(u - v)) if u != v else mp.mpf(0), [0, v, 1])
        c = mp.quad(lambda v: v ** n * inner_c(v), [0, 1])
        a = mp.quad(lambda v: v ** n * mp.quad(lambda u: u ** m * mp.log(1 + v - u), [0, 1]), [0, 1])
        assert abs(float(nearfield.coincident_moment(m, n)) - float(c)) < 1e-15
        assert abs(float(nearfield.adjacent_moment(m, n)) - float(a)) < 1e-15


def test_nearfield_matrices_reproduce_moments():
    u, w, Mco, Madj = nearfield.reference_matrices(16)
    assert abs(Mco.sum() + 1.5) < 1e-14                       # int int ln|u - v| = -3/2
    assert abs(Madj.sum() - (2 * math.log(2) - 1.5)) < 1e-14  # int int ln(1 + v - u)
    assert np.abs(Mco - Mco.T).max() < 1e-17
    for m, n in [(1, 2), (7, 3), (15, 15)]:
        assert abs((u ** m) @ Mco @ (u ** n) - float(nearfield.coincident_moment(m, n))) < 1e-14
        # the float64 products with u^15 themselves round at ~1e-14
        assert abs((u ** m) @ Madj @ (u ** n) - float(nearfield.adjacent_moment(m, n))) < 5e-14


# ------------------------------------------------------------------ O2
@pytest.mark.parametrize("N,p", [(64, 2), (32, 3), (24, 4)])
def test_ebe_converged_equals_circle_closed_form(N, p):
    A = ebe.matrix(synth.circle(0.5), p, N, 24)
    E = circle.matrix(0.5, N, p)
    assert _relmax(A, E) < 1e-13
    assert np.abs(A - A.T).max() < 1e-15 * np.abs(A).max()


def test_ebe_gauss_order_convergence():
    E = circle.matrix(0.5, 32, 2)
    errs = [_relmax(ebe.matrix(synth.circle(0.5), 2, 32, G), E) for G in (2, 3, 4, 6, 8)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[0] > 1e-5 and errs[3] < 1e-10


def test_ebe_star_entries_brute_force():
    """Coincident / adjacent / far entries on a star (J not constant), N = 8, p = 2,
    against nested adaptive quadrature of eq. final_1."""
    curve, N, p = synth.star(5), 8, 2
    A = ebe.EBEProblem(curve, p, N, 24)

    def geo(t):
        x, y, _, _, J = curves.evaluate(curve, np.array([t]))
        return x[0], y[0], J[0]

    def entry(i, j):
        def inner(s):
            xs, ys, _ = geo(s)
            pts = sorted({(j + m) / N for m in range(p + 2)} | {s, s + 1, s - 1})
            lo, hi = j / N, (j + p + 1) / N
            pts = [q for q in pts if lo <= q <= hi]
            tot = 0.0
            for a, b in zip(pts[:-1], pts[1:]):
                def f(t):
                    xt, yt, Jt = geo(t % 1.0)
                    return float(bspline.periodic(p, N, j, t % 1.0)) * Jt * math.log(math.hypot(xs - xt, ys - yt))
                tot += integrate.quad(f, a, b, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
            return tot
        tot = 0.0
        for e in range(p + 1):
            def g(s):
                return float(bspline.periodic(p, N, i, s % 1.0)) * geo(s % 1.0)[2] * inner(s % 1.0)
            tot += integrate.quad(g, (i + e) / N, (i + e + 1) / N, epsabs=1e-14, epsrel=1e-11, limit=100)[0]
        return -tot / (2 * math.pi)

    vals = A.entries([0, 0], [0, 1])
    for v, (i, j) in zip(vals, [(0, 0), (0, 1)]):
        assert abs(v - entry(i, j)) < 1e-9 * abs(vals[0])


def test_solution_converges_at_order_p_plus_1():
    """Circle, g = x1^2 - x2^2: the Galerkin density converges to 4 r cos(4 pi t)
    in relative L2 at the rate p+1 (Section 6, Table 2 caption)."""
    r, p = 0.5, 2
    errs = []
    for N in (8, 16, 32):
        alpha = np.linalg.solve(circle.matrix(r, N, p), circle.rhs_x2_minus_y2(r, N, p))
        t = (np.arange(4000) + 0.5) / 4000
        phi = sum(alpha[j] * bspline.periodic(p, N, j, t) for j in range(N))
        ex = circle.density_x2_minus_y2(r, t)
        errs.append(np.sqrt(np.mean((phi - ex) ** 2) / np.mean(ex ** 2)))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(2.6 < q < 3.6 for q in rates), rates


# ------------------------------------------------------------------ O2 right-hand side (eq. final_b1)
@pytest.mark.parametrize("N,p,G", [(64, 2, 8), (32, 3, 10), (20, 4, 12)])
def test_ebe_rhs_equals_circle_closed_form(N, p, G):
    """beta_i = int B_i J g ds for g = x1^2 - x2^2 on the circle has the closed
    form of O1; the G-point element rule reaches it to rounding for G >= 8.
    A swapped piece index (p - a for a), a dropped element length or a shifted
    element fails this (the closed form carries the phase (i + (p+1)/2)/N)."""
    r = 0.5
    beta = ebe.EBEProblem(synth.circle(r), p, N, G).rhs(synth.g_x2_minus_y2)
    ref = circle.rhs_x2_minus_y2(r, N, p)
    assert np.abs(beta - ref).max() < 1e-14 * np.abs(ref).max()


def test_ebe_rhs_star_adaptive_quadrature():
    """On a star (J not constant, g = exp(x1) cos(x2)) the element rule at G = 12
    equals beta_i by adaptive quadrature over the p+1 elements of supp B_i."""
    curve, p, N, G = synth.star(3), 3, 12, 12
    beta = ebe.EBEProblem(curve, p, N, G).rhs(synth.g_exp_cos)

    def integrand(i, s):
        x, y, _, _, J = curves.evaluate(curve, np.array([s % 1.0]))
        return float(bspline.periodic(p, N, i, s % 1.0)) * J[0] * float(synth.g_exp_cos(x[0], y[0]))

    for i in (0, 5, N - 1):
        ref = sum(integrate.quad(lambda s: integrand(i, s), (i + e) / N, (i + e + 1) / N,
                                 epsabs=1e-15, epsrel=1e-13, limit=200)[0] for e in range(p + 1))
        assert abs(beta[i] - ref) < 1e-13 * np.abs(beta).max(), (i, beta[i], ref)
