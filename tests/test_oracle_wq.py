"""Pins for O3, the weighted-quadrature oracle (CPU)."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import bspline, circle, open_arc, wq


def _quad_pieces(f, pts):
    return sum(integrate.quad(f, a, b, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
               for a, b in zip(pts[:-1], pts[1:]) if b > a)


@pytest.mark.parametrize("p,N,R", [(2, 8, 1), (3, 10, 2), (2, 8, 3)])
def test_alg1_exactness_and_mass(p, N, R):
    """eq. reg_exactness with mu computed by adaptive quadrature; sum w = int B_i = 1/N."""
    M = R * N
    eta = wq.nodes(N, R)
    W = wq.regular_weights(p, N, R)
    for i in (0, N - 1):
        nset, w = W[i]
        assert abs(w.sum() - 1.0 / N) < 4e-15 / N      # a few ulp of 1/N
        for k in wq.exactness_set(p, N, R, i):
            f = lambda t: float(bspline.periodic(p, M, k, t) * bspline.periodic(p, N, i, t))
            mu = _quad_pieces(f, np.arange(M + 1) / M)
            assert abs(np.dot(w, bspline.periodic(p, M, k, eta[nset])) - mu) < 1e-15
        assert nset.size == 2 * R * (p + 1) - 1


@pytest.mark.parametrize("p,R", [(2, 1), (3, 2)])
def test_alg1_polynomial_exactness(p, R):
    """Polynomials of degree <= p lie in the exactness space on a support that
    does not wrap: sum_n w_n eta_n^q = int t^q B_i(t) dt."""
    N, i = 12, 3
    nset, w = wq.regular_weights(p, N, R, rows=[i])[i]
    eta = wq.nodes(N, R)[nset]
    for q in range(p + 1):
        ex = _quad_pieces(lambda t: t ** q * float(bspline.periodic(p, N, i, t)), np.arange(N + 1) / N)
        assert abs(np.dot(w, eta ** q) - ex) < 1e-16


@pytest.mark.parametrize("p,M", [(2, 8), (3, 9)])
def test_moments_brute_force(p, M):
    """mu_k(s) = int Bbar_k(t) ln|sin(pi (t - s)) / pi| dt against mpmath quadrature,
    for s inside, next to, far from and across the wrap of supp Bbar_k."""
    with mp.workdps(25):
        for s in (0.0, 0.5 / M, 3.5 / M, 0.61, 1 - 0.5 / M):
            mu = wq.moments(p, M, s)
            for k in (0, 2, M - 1):
                knots = [mp.mpf(k + c) / M for c in range(p + 2)]
                pts = sorted(set(knots + [mp.mpf(s) + q for q in (-1, 0, 1) if knots[0] < s + q < knots[-1]]))

                def f(t):
                    x = t - s
                    if mp.sin(mp.pi * x) == 0:
                        return mp.mpf(0)
                    return float(bspline.cardinal(p, float(M * t - k))) * mp.log(abs(mp.sin(mp.pi * x)) / mp.pi)
                ex = mp.quad(f, pts)
                assert abs(mu[k] - float(ex)) < 2e-15 * max(1.0, abs(float(ex))), (s, k)


def test_singular_weights_two_routes_agree():
    p, N, R = 3, 12, 2
    Ws = wq.singular_weights(p, N, R)
    src = [0, 1, 7, 2 * R * N - 1]
    Wn = wq.singular_weights_normal(p, N, R, src)
    assert np.abs(Ws[src] - Wn).max() < 1e-14 * np.abs(Ws).max()
    B = wq.collocation(p, R * N, wq.nodes(N, R))
    for m in src:
        assert np.abs(B @ Ws[m] - wq.moments(p, R * N, wq.nodes(N, R)[m])).max() < 1e-15


def test_K1_constant_on_circle():
    r = 0.7
    eta = wq.nodes(16, 1)
    from oracle import curves
    x, y, _, _, J = curves.evaluate(synth.circle(r), eta)
    K1 = wq.K1_rows(x, y, J, eta, np.arange(eta.size))
    assert np.abs(K1 - math.log(2 * math.pi * r)).max() < 1e-13


def test_circle_assembly_brute_force_same_rule():
    """On the circle K1 = ln(2 pi r) and J is constant, so the inner sums of
    eqs. IK1e2 / IK1e2_bis are exact: A_full[i, j] must equal
    -(J^2 / 2 pi) sum_n1 w_n1^(i) [ln(2 pi r) / N + int B_j(t) K2(eta_n1, t) dt]
    with the inner integral by adaptive quadrature."""
    r, p, N, R = 0.5, 2, 8, 1
    J = 2 * math.pi * r
    A_full, tab = wq.full_matrix(synth.circle(r), p, N, R)
    eta = tab["eta"]
    W = wq.regular_weights(p, N, R)
    for (i, j) in [(0, 0), (0, 1), (2, 6), (7, 0)]:
        nset, w = W[i]
        tot = 0.0
        for n1, wn in zip(nset, w):
            s = eta[n1]
            pts = sorted({(j + m) / N for m in range(p + 2)} | {q for q in (s, s + 1, s - 1) if j / N < q < (j + p + 1) / N})
            inner = _quad_pieces(lambda t: float(bspline.periodic(p, N, j, t % 1.0)) * float(wq.K2(s, t)), pts)
            tot += wn * (math.log(2 * math.pi * r) / N + inner)
        assert abs(-J * J * tot / (2 * math.pi) - A_full[i, j]) < 1e-14 * abs(A_full[0, 0])


@pytest.mark.parametrize("p,R,lo,hi", [(2, 1, 1e-4, 5e-4), (2, 2, 1e-5, 5e-5), (2, 4, 5e-7, 3e-6), (3, 1, 5e-5, 2e-4)])
def test_circle_quadrature_error_band(p, R, lo, hi):
    """The weighted-quadrature matrix differs from the exact one only by the
    quadrature error of the outer rule, which shrinks with N_ref."""
    N = 64
    err = np.abs(wq.matrix(synth.circle(0.5), p, N, R) - circle.matrix(0.5, N, p)).max() / circle.matrix(0.5, N, p).max()
    assert lo < err < hi


def test_full_rows_match_dense():
    curve, p, N, R = synth.star(2), 3, 16, 2
    A_full, _ = wq.full_matrix(curve, p, N, R)
    rows = [0, 5, 15]
    assert np.abs(wq.full_rows(curve, p, N, R, rows) - A_full[rows]).max() < 1e-14 * np.abs(A_full).max()


def test_rhs_constant_on_circle():
    r, p, N, R = 0.5, 3, 16, 1
    beta = wq.rhs(synth.circle(r), p, N, R, lambda x, y: np.ones_like(x))
    assert np.abs(beta - 2 * math.pi * r / N).max() < 1e-15


def test_wq_solution_converges_at_order_p_plus_1():
    r, p = 0.5, 2
    errs = []
    for N in (8, 16, 32):
        A = wq.matrix(synth.circle(r), p, N, 1)
        al = np.linalg.solve(A, wq.rhs(synth.circle(r), p, N, 1, synth.g_x2_minus_y2))
        t = (np.arange(4000) + 0.5) / 4000
        phi = sum(al[j] * bspline.periodic(p, N, j, t) for j in range(N))
        ex = circle.density_x2_minus_y2(r, t)
        errs.append(np.sqrt(np.mean((phi - ex) ** 2) / np.mean(ex ** 2)))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(2.8 < q < 3.8 for q in rates), rates


# ------------------------------------------------------------------ open interval (Section 4.2)
def _int_monomial_log(q, s):
    with mp.workdps(40):
        s = mp.mpf(s)
        Phi = lambda j, z: mp.mpf(0) if z == 0 else z ** (j + 1) / (j + 1) * (mp.log(abs(z)) - mp.mpf(1) / (j + 1))
        return float(mp.fsum(mp.binomial(q, j) * s ** (q - j) * (Phi(j, 1 - s) - Phi(j, -1 - s)) for j in range(q + 1)))


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_open_singular_rule_exact_on_t_power_d(d):
    """Section 4.2, first test: the rule integrates t^d against ln|t - s| up to
    machine precision for d <= 5."""
    Nh = 10
    eta = open_arc.open_nodes(d, Nh)
    assert eta.size == 2 * d + 2 * Nh - 1
    Q = open_arc.singular_weights(d, Nh) @ eta ** d
    I = np.array([_int_monomial_log(d, s) for s in eta])
    assert np.abs(Q - I).max() < 1e-14 * np.abs(I).max()


def _table1():
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_err.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows[(int(parts[0]), parts[1])] = [float(x) for x in parts[2:]]
    return rows


@pytest.mark.parametrize("d,v", [(2, "t^3"), (2, "t^4"), (3, "t^4"), (2, "tsal"), (4, "tsal")])
def test_open_singular_rule_table1_bounds(d, v):
    """Table 1: the paper's knot / index conventions are not stated, so its ERR
    values serve as upper bounds, and ERR must fall monotonically in N_h."""
    ref = _table1()[(d, v)]
    errs = []
    for Nh in (10, 20, 40):
        eta = open_arc.open_nodes(d, Nh)
        Ws = open_arc.singular_weights(d, Nh)
        if v == "tsal":
            Q, I = Ws @ open_arc.tsal_integrand(eta), open_arc.tsal_exact(eta)
        else:
            q = int(v[2:])
            Q, I = Ws @ eta ** q, np.array([_int_monomial_log(q, s) for s in eta])
        errs.append(open_arc.err_ratio(Q, I))
    assert all(e <= r for e, r in zip(errs, ref[:3]))
    assert errs[0] > errs[1] > errs[2]


def test_tsal_closed_form():
    """eq. testdiff against mpmath quadrature."""
    with mp.workdps(20):
        for s in (0.0, 0.3, -0.77, 1.0):
            f = lambda t: mp.log(abs(t - s)) * mp.sqrt(1 - t * t) / (t * t + 25) if t != s else mp.mpf(0)
            num = mp.quad(f, sorted({-1, s, 1}))
            assert abs(float(num) - float(open_arc.tsal_exact(s))) < 1e-14
