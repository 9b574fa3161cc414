"""Pins for the open-arc oracle (oracle/wq_open.py; Section 2 eq. prima_BIE on
an open arc, Section 3 eq. lift, Section 4 node vector and Algorithms 1 and 2
with K2 = ln|s - t|, Section 5 eqs. IK1e2 / IK1e2_bis, Section 6 parabola
test), CPU.

Each pin checks the oracle against something other than its own arithmetic:
scipy's B-splines, adaptive quadrature (with QUADPACK's logarithmic weights) of
the exactness conditions and of the Dirichlet datum, the closed form of the
parabola, and the values the paper prints in Table 2 (tests/golden)."""
import math
from pathlib import Path

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

import synth
from oracle import wq_open as O

GOLDEN = Path(__file__).parent / "golden" / "table2_parabola.txt"


def random_breaks(n, seed, a=-1.0, b=1.0, spread=0.6):
    rng = np.random.default_rng([1703, 60000 + seed])
    u = (np.arange(n + 1) + spread * (rng.uniform(0, 1, n + 1) - 0.5)) / n
    u[0], u[-1] = 0.0, 1.0
    return a + (b - a) * u


def scipy_basis(T, p, k):
    c = np.zeros(T.size - p - 1)
    c[k] = 1.0
    return BSpline(T, c, p, extrapolate=False)


def log_quad(f, a, b, s):
    """int_a^b f(t) ln|t - s| dt: QUADPACK's algebraic-logarithmic weights where s is an end of a piece
    ([a, s] and [s, b] when s is inside), plain adaptive quadrature when s is outside [a, b]."""
    kw = dict(epsabs=1e-15, epsrel=1e-13, limit=200)
    if s < a or s > b:
        return integrate.quad(lambda t: f(t) * math.log(abs(t - s)), a, b, **kw)[0]
    out = 0.0
    if s > a:
        out += integrate.quad(f, a, s, weight="alg-logb", wvar=(0.0, 0.0), **kw)[0]
    if s < b:
        out += integrate.quad(f, s, b, weight="alg-loga", wvar=(0.0, 0.0), **kw)[0]
    return out


def test_parabola_geometry_closed_form():
    t = np.linspace(-1, 1, 41)
    x, y, dx, dy, J = O.arc_evaluate(synth.parabola(), t)
    assert np.abs(x - t).max() < 1e-15 and np.abs(y - (1 - t * t)).max() < 1e-15
    assert np.abs(dx - 1).max() < 1e-14 and np.abs(dy + 2 * t).max() < 1e-14
    assert np.abs(J - np.sqrt(1 + 4 * t * t)).max() < 1e-14


def test_open_arc_geometry_matches_scipy():
    cur = synth.open_arc_bspline(3)
    T = np.asarray(cur.knots)
    spl = BSpline(T, np.asarray(cur.ctrl), cur.degree)
    t = np.linspace(0, 1, 77)
    x, y, dx, dy, J = O.arc_evaluate(cur, t)
    ref = spl(t)
    dref = spl.derivative()(t)
    assert np.abs(x - ref[:, 0]).max() < 1e-14 and np.abs(y - ref[:, 1]).max() < 1e-14
    assert np.abs(dx - dref[:, 0]).max() < 1e-12 and np.abs(dy - dref[:, 1]).max() < 1e-12


@pytest.mark.parametrize("p,n,R", [(1, 4, 1), (2, 5, 1), (3, 3, 2), (2, 1, 2), (5, 7, 1), (4, 2, 3)])
def test_node_vector_of_section_4(p, n, R):
    br = random_breaks(n, p + 10 * n)
    xb = O.refine(br, R)
    M = R * n
    eta = O.nodes(br, p, R)
    assert eta.size == 2 * p + 2 * M - 1
    assert np.all(np.diff(eta) > 0) and eta[0] == br[0] and eta[-1] == br[-1]
    h0, h1 = xb[1] - xb[0], xb[-1] - xb[-2]
    assert np.allclose(eta[:p + 2], xb[0] + h0 * np.arange(p + 2) / (p + 1), rtol=0, atol=1e-15)
    assert np.allclose(eta[-(p + 2):], xb[-2] + h1 * np.arange(p + 2) / (p + 1), rtol=0, atol=1e-15)
    inner = eta[p + 1:eta.size - p - 1]              # x_1, mid, x_2, mid, ..., x_{M-1}
    assert np.allclose(inner[0::2], xb[1:M], rtol=0, atol=1e-15)
    assert np.allclose(inner[1::2], 0.5 * (xb[1:M - 1] + xb[2:M]), rtol=0, atol=1e-15)
    # Schoenberg-Whitney: the collocation matrix of the exactness space has full row rank
    B = O.collocation(O.knot_vector(xb, p), p, eta)
    assert np.linalg.matrix_rank(B) == M + p


@pytest.mark.parametrize("p", [1, 2, 3, 6])
def test_open_basis_matches_scipy(p):
    br = random_breaks(6, p)
    T = O.knot_vector(br, p)
    t = np.linspace(br[0], br[-1], 301)
    tot = np.zeros_like(t)
    for k in range(T.size - p - 1):
        mine = O.basis(T, p, k, t)
        ref = np.nan_to_num(scipy_basis(T, p, k)(t))
        assert np.abs(mine[:-1] - ref[:-1]).max() < 1e-14
        tot += mine
    assert np.abs(tot - 1.0).max() < 1e-14
    assert O.basis(T, p, 0, br[0]) == 1.0 and O.basis(T, p, T.size - p - 2, br[-1]) == 1.0


@pytest.mark.parametrize("p,n,R,seed", [(2, 6, 1, 0), (3, 5, 2, 1), (4, 7, 1, 2), (1, 4, 3, 3)])
def test_regular_rule_is_exact_on_the_exactness_space(p, n, R, seed):
    """eq. reg_exactness: int Bbar_k B_i for every refined function meeting supp B_i, by adaptive quadrature
    of scipy's B-splines; polynomials up to degree p are in the space."""
    br = random_breaks(n, seed)
    T = O.knot_vector(br, p)
    Tb = O.knot_vector(O.refine(br, R), p)
    eta = O.nodes(br, p, R)
    rules = O.regular_weights(br, p, R)
    for i, (nset, w) in rules.items():
        Bi = scipy_basis(T, p, i)
        assert np.all(np.nan_to_num(Bi(eta[nset])) > 0) or i in (0, len(rules) - 1)
        lo, hi = T[i], T[i + p + 1]
        pts = sorted({float(x) for x in Tb if lo < x < hi})
        for k in O.exactness_set(br, p, R, i):
            Bk = scipy_basis(Tb, p, int(k))
            ex = integrate.quad(lambda t: np.nan_to_num(Bk(t)) * np.nan_to_num(Bi(t)), lo, hi, points=pts or None,
                                epsabs=1e-16, epsrel=1e-13, limit=200)[0]
            assert abs(np.sum(w * O.basis(Tb, p, int(k), eta[nset])) - ex) < 1e-13
        for m in range(p + 1):
            ex = integrate.quad(lambda t: t ** m * np.nan_to_num(Bi(t)), lo, hi, points=pts or None,
                                epsabs=1e-16, epsrel=1e-13, limit=200)[0]
            assert abs(np.sum(w * eta[nset] ** m) - ex) < 1e-13


@pytest.mark.parametrize("p,n,R,seed", [(2, 5, 1, 4), (3, 4, 2, 5), (5, 6, 1, 6)])
def test_singular_rule_is_exact(p, n, R, seed):
    """eq. sing_exactness with K2 = ln|t - s| on the open interval: the moments of every refined B-spline and
    of the monomials, against QUADPACK's logarithmic-weight quadrature, at every node and between nodes."""
    br = random_breaks(n, seed)
    xb = O.refine(br, R)
    Tb = O.knot_vector(xb, p)
    eta = O.nodes(br, p, R)
    src = np.concatenate([eta, [br[0] + 0.37 * (br[1] - br[0]), 0.5 * (eta[3] + eta[4])]])
    Ws = O.singular_weights(br, p, R, sources=src)
    B = O.collocation(Tb, p, eta)
    for m, s in enumerate(src):
        mu = O.moments(xb, p, s)
        assert np.abs(B @ Ws[m] - mu).max() < 1e-13
        for k in (0, Tb.size - p - 2, (Tb.size - p - 1) // 2):
            Bk = scipy_basis(Tb, p, k)
            lo, hi = Tb[k], Tb[k + p + 1]
            ex = 0.0
            for a, b in zip(xb[:-1], xb[1:]):
                if a >= lo and b <= hi:
                    ex += log_quad(lambda t: float(np.nan_to_num(Bk(t))), a, b, s)
            assert abs(mu[k] - ex) < 1e-12, (m, k)
        for q in range(p + 1):
            ex = log_quad(lambda t: t ** q, br[0], br[-1], s)
            assert abs(np.sum(Ws[m] * eta ** q) - ex) < 1e-12


def test_uD_closed_form_matches_the_defining_integral():
    """u_D(f(s)) = -(1/2pi) int ln|f(s) - f(t)| phi(f(t)) J(t) dt with the arc's own geometry, by adaptive
    quadrature split at the log singularity."""
    for s in (-1.0, -0.93, -0.4, 0.0, 0.21, 0.77, 1.0):
        def f(t):
            dx, dy = s - t, (1 - s * s) - (1 - t * t)
            return 0.5 * math.log(dx * dx + dy * dy) * (1 + 4 * t * t)
        pts = [q for q in (s,) if -1 < q < 1]
        edges = [-1.0] + pts + [1.0]
        ex = sum(integrate.quad(f, a, b, epsabs=1e-15, epsrel=1e-13, limit=400)[0] for a, b in zip(edges, edges[1:]))
        assert abs(synth.parabola_uD(s) - (-ex / (2 * math.pi))) < 1e-12


def test_K1_limit_and_split():
    cur = synth.open_arc_bspline(1)
    br = np.linspace(0, 1, 9)
    eta = O.nodes(br, 3, 1)
    x, y, _, _, J = O.arc_evaluate(cur, eta)
    K1 = O.K1_open(x, y, J, eta)
    for n in (0, 7, eta.size - 1):
        t = eta[n] + (1e-5 if n < eta.size - 1 else -1e-5)
        xx, yy, _, _, _ = O.arc_evaluate(cur, np.array([t]))
        lim = 0.5 * math.log(((xx[0] - x[n]) ** 2 + (yy[0] - y[n]) ** 2) / (t - eta[n]) ** 2)
        assert abs(K1[n, n] - lim) < 1e-4
    m, n = 3, 11
    assert abs(K1[m, n] + math.log(abs(eta[m] - eta[n])) - 0.5 * math.log((x[m] - x[n]) ** 2 + (y[m] - y[n]) ** 2)) < 1e-14


def _golden():
    rows = []
    for line in GOLDEN.read_text().splitlines():
        if line.startswith("#") or not line.strip():
            continue
        v = line.split()
        rows.append((int(v[0]), int(v[1]), int(v[2])) + tuple(float(q) for q in v[3:]))
    return rows


def _solve_parabola(p, n):
    br = np.linspace(-1.0, 1.0, n + 1)
    cur = synth.parabola()
    A = O.matrix(cur, br, p, 1)
    b = O.rhs(cur, br, p, 1, synth.parabola_uD)
    al = np.linalg.solve(A, b)
    return A, al, O.errors(br, p, al)


@pytest.mark.parametrize("row", [r for r in _golden() if r[1] <= 320], ids=lambda r: f"d{r[0]}_n{r[1]}")
def test_parabola_reproduces_table2(row):
    """Table 2: the errors lie between the element-by-element column (exact Galerkin up to its quadrature)
    and the new-assembly column; from n_el = 80 on, E_R, E_M and the condition number agree with the
    new-assembly column to the printed digits (1.5%)."""
    d, n, dof, ebe_cond, ebe_ER, ebe_EM, new_cond, new_ER, new_EM = row
    A, al, (ER, EM) = _solve_parabola(d, n)
    assert A.shape == (dof, dof)
    assert 0.98 * min(ebe_ER, new_ER) <= ER <= 1.02 * new_ER, (ER, ebe_ER, new_ER)
    assert 0.9 * min(ebe_EM, new_EM) <= EM <= 1.05 * max(ebe_EM, new_EM), (EM, ebe_EM, new_EM)
    cond = np.linalg.cond(A)
    assert 0.95 * min(ebe_cond, new_cond) <= cond <= 1.05 * max(ebe_cond, new_cond), cond
    if n >= 80:
        for mine, ref in ((ER, new_ER), (EM, new_EM), (cond, new_cond)):
            assert abs(mine / ref - 1) < 0.015, (mine, ref)


@pytest.mark.parametrize("p,ns,lo,hi", [(2, (20, 40, 80), 2.9, 3.2), (3, (16, 32, 64), 3.9, 4.5)])
def test_parabola_converges_at_order_d_plus_1(p, ns, lo, hi):
    """Section 6: E_R of order d + 1 in h (Fig. Parabola_conv for d = 2)."""
    errs = [_solve_parabola(p, n)[2][0] for n in ns]
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(lo < r < hi for r in rates), (errs, rates)


def test_mirrored_rows_lose_the_row_exactness():
    """Each row of eq. IK1e2_bis integrates the whole spline space with the singular rule, so the rows applied
    to a smooth density are accurate although single entries near the clamped ends carry errors of about 1%;
    mirroring the upper rows (as a closed curve's uniform rules allow) breaks that near the ends."""
    br = np.linspace(-1.0, 1.0, 11)
    cur = synth.parabola()
    A_full = O.full_matrix(cur, br, 2, 1)[0]
    A_ref = O.full_matrix(cur, br, 2, 6)[0]
    assert np.abs(A_full - A_ref).max() > 5e-3 * np.abs(A_ref).max()
    b = O.rhs(cur, br, 2, 1, synth.parabola_uD)
    up = np.triu(A_full)
    ER_full = O.errors(br, 2, np.linalg.solve(A_full, b))[0]
    ER_mirror = O.errors(br, 2, np.linalg.solve(up + np.triu(up, 1).T, b))[0]
    assert ER_full < 2e-4 < 1e-2 < ER_mirror
