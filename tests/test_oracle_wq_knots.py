"""Pins for the oracle's weighted quadrature on non-uniform periodic knots
(oracle/wq_knots.py; Section 3, Algorithms 1 and 2, eqs. IK1e2 / IK1e2_bis), CPU.

Each pin checks the general-knot rules against something other than their own
arithmetic: scipy's B-splines, adaptive quadrature of the exactness conditions,
the uniform oracle when the knots are uniform, the circle's constant K1 with
brute-force inner integrals, and the convergence of the Galerkin solution on a
graded mesh to the exact density."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

import synth
from oracle import bspline, circle, wq
from oracle import wq_knots as K


def graded(N, amp=0.3):
    """tau_k = u + amp sin(2 pi u) / (2 pi) at u = k / N: smooth, strictly increasing,
    element lengths between (1 - amp) / N and (1 + amp) / N."""
    u = np.arange(N + 1) / N
    tau = u + amp * np.sin(2 * math.pi * u) / (2 * math.pi)
    tau[0], tau[-1] = 0.0, 1.0
    return tau


def random_knots(N, seed, spread=0.6):
    rng = np.random.default_rng(seed)
    u = (np.arange(N + 1) + spread * (rng.uniform(0, 1, N + 1) - 0.5)) / N
    u[0], u[-1] = 0.0, 1.0
    return u


def _quad(f, a, b, points):
    pts = sorted({q for q in points if a < q < b})
    edges = [a] + pts + [b]
    return sum(integrate.quad(f, lo, hi, limit=200, epsabs=1e-16, epsrel=1e-14)[0] for lo, hi in zip(edges, edges[1:]))


@pytest.mark.parametrize("p,N,R", [(2, 10, 1), (3, 12, 2), (4, 11, 1)])
def test_uniform_knots_reduce_to_the_uniform_oracle(p, N, R):
    tau = np.arange(N + 1) / N
    # two evaluations of the same basis (cardinal vs general Cox-de Boor) through the local
    # minimum-norm systems: equal to the conditioning of those systems
    eta = wq.nodes(N, R)
    nset = wq.support_nodes(p, N, R, 0)
    Bloc = np.stack([bspline.periodic(p, R * N, k, eta[nset]) for k in wq.exactness_set(p, N, R, 0)])
    Wu = wq.regular_weight_matrix(p, N, R)
    tol = 20 * np.finfo(float).eps * np.linalg.cond(Bloc) * np.abs(Wu).max()
    assert np.abs(K.regular_weight_matrix(tau, p, R) - Wu).max() < tol
    Wsu = wq.singular_weights(p, N, R)
    assert np.abs(K.singular_weights(tau, p, R) - Wsu).max() < 1e-13 * np.abs(Wsu).max()
    A = wq.matrix(synth.star(4), p, N, R)
    assert np.abs(K.matrix(synth.star(4), tau, p, R) - A).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_basis_matches_scipy_and_pieces(p):
    tau = random_knots(9, 3)
    n = tau.size - 1
    text = np.concatenate([tau[n - p:n] - 1.0, tau, tau[1:p + 1] + 1.0])
    t = np.linspace(0, 1, 501, endpoint=False)
    tot = np.zeros_like(t)
    for i in range(n):
        c = np.zeros(n + p)
        c[(i + p) % n] = 1.0           # scipy's basis element i + p is B_i (index shift of the extension)
        if (i + p) % n + n < n + p:
            c[(i + p) % n + n] = 1.0
        ref = BSpline(text, c, p)(t)
        mine = K.basis(tau, p, i, t)
        assert np.abs(mine - ref).max() < 1e-13
        tot += mine
        for e in range(n):             # local pieces reproduce the function
            u = np.linspace(0.03, 0.97, 9)
            te = tau[e] + (tau[e + 1] - tau[e]) * u
            assert np.abs(np.polynomial.polynomial.polyval(u, K.piece_poly(tau, p, i, e)) - K.basis(tau, p, i, te)).max() < 1e-13
    assert np.abs(tot - 1.0).max() < 1e-14


@pytest.mark.parametrize("p,R,seed", [(2, 1, 0), (3, 2, 1), (4, 1, 2)])
def test_regular_rules_exact_by_adaptive_quadrature(p, R, seed):
    """Algorithm 1 on non-uniform knots: sum_n w_n^(i) Bbar_k(eta_n) equals
    int Bbar_k B_i for every refined k meeting supp B_i (eq. reg_exactness)."""
    tau = random_knots(10, seed)
    N = tau.size - 1
    tb = K.refine(tau, R)
    eta = K.nodes(tau, R)
    rules = K.regular_weights(tau, p, R, rows=[0, 3, N - 1])
    for i, (nset, w) in rules.items():
        a, b = K.ext(tau, i), K.ext(tau, i + p + 1)
        brk = [K.ext(tb, j) for j in range(R * i, R * (i + p + 1) + 1)]
        for k in K.exactness_set(p, N, R, i):
            ref = _quad(lambda t: K.basis(tb, p, int(k), np.array([t % 1.0]))[0] * K.basis(tau, p, i, np.array([t % 1.0]))[0],
                        a, b, brk)
            got = float(np.dot(w, K.basis(tb, p, int(k), eta[nset])))
            assert abs(got - ref) < 1e-15 + 1e-13 * abs(ref)
        # mass: the rule integrates B_i exactly (the refined functions sum to 1)
        assert abs(w.sum() - (b - a) / (p + 1)) < 1e-14


@pytest.mark.parametrize("p,R", [(2, 1), (3, 2)])
def test_singular_rules_exact_by_adaptive_quadrature(p, R):
    """Algorithm 2 on non-uniform knots: for sampled sources eta_m,
    sum_n w_n^(eta_m) Bbar_k(eta_n) equals int Bbar_k(t) ln|sin(pi (eta_m - t)) / pi| dt
    (eq. sing_exactness), the integral split at the singularity and the knots."""
    tau = random_knots(8, 7)
    tb = K.refine(tau, R)
    eta = K.nodes(tau, R)
    Ws = K.singular_weights(tau, p, R)
    M = tb.size - 1
    for m in [0, 3, 2 * M - 1]:
        s = eta[m]
        for k in range(M):
            a, b = K.ext(tb, k), K.ext(tb, k + p + 1)
            f = lambda t: K.basis(tb, p, k, np.array([t % 1.0]))[0] * math.log(abs(math.sin(math.pi * (s - t))) / math.pi)
            ref = _quad(f, a, b, [K.ext(tb, j) for j in range(k + 1, k + p + 1)] + [s, s + 1.0, s - 1.0])
            got = float(np.dot(Ws[m], K.basis(tb, p, k, eta)))
            assert abs(got - ref) < 1e-13, (m, k, got, ref)


def test_circle_entries_by_brute_force_inner_integrals():
    """On the circle K1 = ln(2 pi r) is constant (|f(s) - f(t)| = 2 r |sin(pi (s - t))|),
    so with the exactness of both rules (B_j lies in the refined space)
    A_ij = -(J^2 / 2 pi) sum_n1 w_n1^(i) [ln(2 pi r) int B_j + int B_j(t) K2(eta_n1, t) dt]:
    the inner integrals by adaptive quadrature, the outer rule the oracle's, for
    non-uniform knots and n_ref = 2."""
    r, p, R = 0.5, 2, 2
    tau = random_knots(7, 11)
    N = tau.size - 1
    A_full, tab = K.full_matrix(synth.circle(r), tau, p, R)
    eta = tab["eta"]
    J = 2 * math.pi * r
    rules = K.regular_weights(tau, p, R)
    for i, j in [(0, 0), (0, 1), (2, 5), (6, 3)]:
        nset, w = rules[i]
        a, b = K.ext(tau, j), K.ext(tau, j + p + 1)
        brk = [K.ext(tau, q) for q in range(j + 1, j + p + 1)]
        mass = (b - a) / (p + 1)
        tot = 0.0
        for n1, wn in zip(nset, w):
            s = eta[n1]
            inner = _quad(lambda t: K.basis(tau, p, j, np.array([t % 1.0]))[0] * float(wq.K2(s, t)), a, b,
                          brk + [s, s + 1.0, s - 1.0])
            tot += wn * (math.log(2 * math.pi * r) * mass + inner)
        assert abs(-J * J * tot / (2 * math.pi) - A_full[i, j]) < 1e-14 * abs(A_full[0, 0])


def test_solution_converges_on_graded_knots():
    """The Galerkin solution on the circle with graded non-uniform knots
    converges to the exact density at order p + 1 (p = 2)."""
    r, p = 0.5, 2
    errs = []
    t = (np.arange(4000) + 0.5) / 4000
    ex = circle.density_x2_minus_y2(r, t)
    for N in (8, 16, 32):
        tau = graded(N)
        A = K.matrix(synth.circle(r), tau, p, 1)
        al = np.linalg.solve(A, K.rhs(synth.circle(r), tau, p, 1, synth.g_x2_minus_y2))
        phi = sum(al[j] * K.basis(tau, p, j, t) for j in range(N))
        errs.append(np.sqrt(np.mean((phi - ex) ** 2) / np.mean(ex ** 2)))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(2.6 < q < 4.0 for q in rates), (errs, rates)
