"""O7: IgA-SGBEM on an open arc with B-spline weighted quadrature (test
infrastructure only).

The exterior Dirichlet problem of Section 2 (eq. BVP_arco) in the indirect
form eq. prima_BIE, discretised as in Sections 3-5 and written with dense
linear algebra:

* parameter interval I = [a, b] with breakpoints a = x_0 < x_1 < ... < x_n = b;
  approximation space (Section 3, eq. lift): all N = n + p B-splines of degree
  p on the open knot vector with p + 1 copies of a and of b (simple inner
  knots), B_i supported on [T_i, T_{i+p+1}]; B_0(a) = B_{N-1}(b) = 1;
* exactness space: the same construction on the refined mesh, every element
  split into R equal parts (M = R n refined elements, N_E = M + p functions);
* nodes (Section 4): p + 2 equally spaced points in the first and in the last
  refined element, midpoints and breakpoints elsewhere, N_quad = 2p + 2M - 1;
* Algorithm 1 per test function on the nodes where B_i is non-zero (the open
  support, plus the end point where the clamped end function equals one),
  Algorithm 2 per source on all nodes, both minimum-norm by LAPACK least
  squares (the systems are underdetermined where an end element is involved);
* the kernel split of Section 3.1 as printed: K2(s, t) = ln|s - t|,
  K1 = ln|f(s) - f(t)| - K2 with the diagonal limit ln J (eq. F1_lim);
* modified moments (eq. mod_mom_gen) from the closed form of int z^j ln|z|
  (Section 4.2) in the local variable of each refined element, the local
  monomial coefficients of each piece from its values at p + 1 points;
* assembly by eqs. IK1e2 / IK1e2_bis, every entry (not mirrored), right-hand
  side F_i = int B_i J u_D (the indirect form) with the regular rule.

``errors`` gives E_R and E_M of the parabola test of Section 6 (Table 2) for a
computed density, against the exact phi(f(t)) = sqrt(1 + 4 t^2).
"""
from __future__ import annotations

import math

import numpy as np

from . import bspline
from .wq import log_piece


# ---------------------------------------------------------------- knots, nodes
def check_breaks(breaks) -> np.ndarray:
    x = np.asarray(breaks, dtype=np.float64)
    assert x.ndim == 1 and x.size >= 2 and np.all(np.diff(x) > 0)
    return x


def knot_vector(breaks, p: int) -> np.ndarray:
    """Open (clamped) extended knot vector of Section 3: p + 1 copies of each end."""
    x = check_breaks(breaks)
    return np.concatenate([np.full(p, x[0]), x, np.full(p, x[-1])])


def refine(breaks, R: int) -> np.ndarray:
    """Every element [x_e, x_{e+1}] split into R equal parts: x_e + (x_{e+1} - x_e) r / R."""
    x = check_breaks(breaks)
    inner = x[:-1, None] + (np.diff(x)[:, None] * np.arange(R)[None, :]) / R
    return np.append(inner.ravel(), x[-1])


def nodes(breaks, p: int, R: int) -> np.ndarray:
    """Section 4: p + 2 uniformly spaced points in the first and in the last
    refined element, every midpoint and breakpoint of the inner elements."""
    xb = refine(breaks, R)
    M = xb.size - 1
    assert M >= 2
    pts = set()
    first = xb[0] + (xb[1] - xb[0]) * np.arange(p + 2) / (p + 1)
    last = xb[M - 1] + (xb[M] - xb[M - 1]) * np.arange(p + 2) / (p + 1)
    first[-1], last[0], last[-1] = xb[1], xb[M - 1], xb[M]
    pts.update(first.tolist())
    pts.update(last.tolist())
    for e in range(1, M - 1):
        pts.add(float(xb[e]))
        pts.add(float(xb[e + 1]))
        pts.add(float(0.5 * (xb[e] + xb[e + 1])))
    eta = np.array(sorted(pts))
    assert eta.size == 2 * p + 2 * M - 1
    return eta


def basis(T, p: int, i: int, t) -> np.ndarray:
    return bspline.general(T, p, i, t)


def collocation(T, p: int, t) -> np.ndarray:
    n_fun = np.asarray(T).size - p - 1
    return np.stack([basis(T, p, k, t) for k in range(n_fun)])


# ---------------------------------------------------------------- Algorithm 1
def support_nodes(breaks, p: int, R: int, i: int, eta=None) -> np.ndarray:
    """N^(i): nodes where B_i is non-zero: inside (T_i, T_{i+p+1}), plus a for
    B_0 and b for B_{N-1}.  eta: ``nodes(breaks, p, R)`` if already formed."""
    T = knot_vector(breaks, p)
    eta = nodes(breaks, p, R) if eta is None else eta
    inside = (eta > T[i]) & (eta < T[i + p + 1])
    if i == 0:
        inside |= eta == T[0]
    if i == T.size - p - 2:
        inside |= eta == T[-1]
    return np.nonzero(inside)[0]


def exactness_set(breaks, p: int, R: int, i: int) -> np.ndarray:
    """J^(i): refined functions whose support meets supp B_i in an interval."""
    T = knot_vector(breaks, p)
    Tb = knot_vector(refine(breaks, R), p)
    lo, hi = T[i], T[i + p + 1]
    k = np.arange(Tb.size - p - 1)
    return k[(np.minimum(Tb[k + p + 1], hi) - np.maximum(Tb[k], lo)) > 0]


def regular_weights(breaks, p: int, R: int, rows=None) -> dict:
    """Algorithm 1: for each test function B_i the minimum-norm weights on N^(i)
    that integrate every Bbar_k, k in J^(i), against B_i exactly (eq.
    reg_exactness); int Bbar_k B_i by (p + 1)-point Gauss per refined element
    (exact for the degree-2p pieces)."""
    T = knot_vector(breaks, p)
    xb = refine(breaks, R)
    Tb = knot_vector(xb, p)
    eta = nodes(breaks, p, R)
    gu, gw = np.polynomial.legendre.leggauss(p + 1)
    gu, gw = (gu + 1.0) / 2.0, gw / 2.0
    out = {}
    N = T.size - p - 1
    for i in (range(N) if rows is None else rows):
        Jset = exactness_set(breaks, p, R, i)
        Nset = support_nodes(breaks, p, R, i, eta)
        el = np.nonzero((xb[:-1] >= T[i]) & (xb[1:] <= T[i + p + 1]))[0]
        h = xb[el + 1] - xb[el]
        tq = (xb[el][:, None] + h[:, None] * gu[None, :]).ravel()
        wq = (h[:, None] * gw[None, :]).ravel()
        Bi = basis(T, p, i, tq)
        mu = np.array([np.sum(wq * basis(Tb, p, int(k), tq) * Bi) for k in Jset])
        Bloc = np.stack([basis(Tb, p, int(k), eta[Nset]) for k in Jset])
        out[i] = (Nset, np.linalg.lstsq(Bloc, mu, rcond=None)[0])
    return out


def regular_weight_matrix(breaks, p: int, R: int) -> np.ndarray:
    N = check_breaks(breaks).size - 1 + p
    W = np.zeros((N, nodes(breaks, p, R).size))
    for i, (nset, w) in regular_weights(breaks, p, R).items():
        W[i, nset] = w
    return W


# ---------------------------------------------------------------- modified moments
def pieces(xb, p: int):
    """(k, e, coef): local monomial coefficients, in u = (t - xb_e) / h_e on
    [0, 1], of every non-zero piece of the refined Bbar_k, from its values at
    p + 1 Chebyshev points of the element."""
    Tb = knot_vector(xb, p)
    M = xb.size - 1
    u = (1.0 - np.cos(math.pi * (np.arange(p + 1) + 0.5) / (p + 1))) / 2.0
    V = np.vander(u, p + 1, increasing=True)
    ks, es, cs = [], [], []
    for e in range(M):
        a, h = xb[e], xb[e + 1] - xb[e]
        for k in range(e, e + p + 1):        # Bbar_k is non-zero on element e for k = e .. e + p
            vals = basis(Tb, p, k, a + h * u)
            ks.append(k)
            es.append(e)
            cs.append(np.linalg.solve(V, vals))
    return np.array(ks), np.array(es), np.array(cs)


def moments(xb, p: int, s: float, pcs=None) -> np.ndarray:
    """mu_k(s) = int_I Bbar_k(t) ln|t - s| dt (eq. mod_mom_gen), element by element:
    h_e [ln h_e int_0^1 P + int_0^1 P(u) ln|u - sigma_e| du], sigma_e = (s - xb_e) / h_e."""
    ks, es, cs = pieces(xb, p) if pcs is None else pcs
    h = np.diff(xb)[es]
    sigma = (s - xb[es]) / h
    vals = h * (np.log(h) * (cs @ (1.0 / np.arange(1, p + 2))) + log_piece(cs, sigma))
    return np.bincount(ks, weights=vals, minlength=xb.size - 1 + p)


# ---------------------------------------------------------------- Algorithm 2
def singular_weights(breaks, p: int, R: int, sources=None) -> np.ndarray:
    """Algorithm 2: for each source s the minimum-norm weights on all nodes that
    integrate every Bbar_k against ln|t - s| exactly (eq. sing_exactness).
    Returns Ws[m, n]; the sources default to the nodes."""
    xb = refine(breaks, R)
    eta = nodes(breaks, p, R)
    src = eta if sources is None else np.asarray(sources, dtype=np.float64)
    B = collocation(knot_vector(xb, p), p, eta)
    pcs = pieces(xb, p)
    Mu = np.stack([moments(xb, p, s, pcs) for s in src], axis=1)
    return np.linalg.lstsq(B, Mu, rcond=None)[0].T


# ---------------------------------------------------------------- geometry
def arc_evaluate(curve, t):
    """(x, y, dx, dy, J) of the open B-spline arc f(t) = sum_j Q_j B_j(t) on its
    clamped knot vector; f' = sum_j d (Q_j - Q_{j-1}) / (T_{j+d} - T_j) B_{j,d-1}
    on the same knots without the end copies (derivative of the recurrence)."""
    t = np.asarray(t, dtype=np.float64)
    T = np.asarray(curve.knots, dtype=np.float64)
    Q = np.asarray(curve.ctrl, dtype=np.float64)
    d = curve.degree
    n = Q.shape[0]
    assert T.size == n + d + 1
    x = sum(Q[j, 0] * basis(T, d, j, t) for j in range(n))
    y = sum(Q[j, 1] * basis(T, d, j, t) for j in range(n))
    Td = T[1:-1]
    dx = np.zeros_like(t)
    dy = np.zeros_like(t)
    for j in range(1, n):
        c = d / (T[j + d] - T[j])
        b = basis(Td, d - 1, j - 1, t)
        dx += c * (Q[j, 0] - Q[j - 1, 0]) * b
        dy += c * (Q[j, 1] - Q[j - 1, 1]) * b
    return x, y, dx, dy, np.sqrt(dx * dx + dy * dy)


def K1_open(x, y, J, eta) -> np.ndarray:
    """K1(s, t) = ln(|f(s) - f(t)|^2 / (s - t)^2) / 2 on the node grid, ln J on the diagonal."""
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    dt = eta[:, None] - eta[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        K = 0.5 * np.log((dx * dx + dy * dy) / (dt * dt))
    K[np.diag_indices_from(K)] = np.log(J)
    return K


# ---------------------------------------------------------------- assembly
def full_matrix(curve, breaks, p: int, R: int):
    """A_full = -(1/2pi) (W D_J) [K1 (W D_J)^T + Ws D_J Bmat^T], Bmat[j, n] = B_j(eta_n)
    (eqs. IK1e2, IK1e2_bis)."""
    eta = nodes(breaks, p, R)
    x, y, _, _, J = arc_evaluate(curve, eta)
    W = regular_weight_matrix(breaks, p, R)
    Ws = singular_weights(breaks, p, R)
    Bmat = collocation(knot_vector(breaks, p), p, eta)
    K1 = K1_open(x, y, J, eta)
    What = W * J[None, :]
    A_full = -(What @ (K1 @ What.T + Ws @ (J[:, None] * Bmat.T))) / (2.0 * math.pi)
    return A_full, dict(W=W, Ws=Ws, Bmat=Bmat, K1=K1, x=x, y=y, J=J, eta=eta)


def full_rows(curve, breaks, p: int, R: int, rows) -> np.ndarray:
    """Rows of A_full (eqs. IK1e2, IK1e2_bis) without the whole matrix: the
    singular weights only for the sources in the supports of those rows."""
    eta = nodes(breaks, p, R)
    x, y, _, _, J = arc_evaluate(curve, eta)
    W = regular_weight_matrix(breaks, p, R)
    Bmat = collocation(knot_vector(breaks, p), p, eta)
    What = W * J[None, :]
    src = np.unique(np.concatenate([np.nonzero(W[i])[0] for i in rows]))
    Ws = singular_weights(breaks, p, R, sources=eta[src])
    dx = x[src, None] - x[None, :]
    dy = y[src, None] - y[None, :]
    dt = eta[src, None] - eta[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        K1 = 0.5 * np.log((dx * dx + dy * dy) / (dt * dt))
    K1[np.arange(src.size), src] = np.log(J[src])
    inner = K1 @ What.T + Ws @ (J[:, None] * Bmat.T)          # (sources, N)
    return np.array([-(What[i, src] @ inner) / (2.0 * math.pi) for i in rows])


def matrix(curve, breaks, p: int, R: int) -> np.ndarray:
    """Every entry of eq. IK1e2_bis, not mirrored: each row integrates the whole
    spline space with the singular rule, which keeps the row applied to a
    smooth density accurate near the clamped ends although single entries
    there are not; mirroring the upper rows loses that."""
    return full_matrix(curve, breaks, p, R)[0]


def rhs(curve, breaks, p: int, R: int, uD) -> np.ndarray:
    """F_i = sum_n w_n^(i) J(eta_n) u_D(f(eta_n)) (indirect form, regular rule)."""
    eta = nodes(breaks, p, R)
    x, y, _, _, J = arc_evaluate(curve, eta)
    u = uD(x, y)
    N = check_breaks(breaks).size - 1 + p
    beta = np.zeros(N)
    for i, (nset, w) in regular_weights(breaks, p, R).items():
        beta[i] = np.sum(w * J[nset] * u[nset])
    return beta


# ---------------------------------------------------------------- errors of Section 6
def _phi(t):
    """Exact density of the parabola test at f(t): sqrt(1 + 4 t^2)."""
    t = np.asarray(t, dtype=np.float64)
    return np.sqrt(1.0 + 4.0 * t * t)


def density(breaks, p: int, alpha, t) -> np.ndarray:
    T = knot_vector(breaks, p)
    return sum(a * basis(T, p, j, t) for j, a in enumerate(alpha))


def errors(breaks, p: int, alpha):
    """(E_R, E_M) of Section 6: the relative L2(I) error of phi_h against phi
    (Gauss, 8 points per element) and the maximum error on 500 uniformly spaced
    points of I."""
    x = check_breaks(breaks)
    gu, gw = np.polynomial.legendre.leggauss(8)
    gu, gw = (gu + 1.0) / 2.0, gw / 2.0
    h = np.diff(x)
    tq = (x[:-1, None] + h[:, None] * gu[None, :]).ravel()
    wq = (h[:, None] * gw[None, :]).ravel()
    e = density(breaks, p, alpha, tq) - _phi(tq)
    ER = math.sqrt(np.sum(wq * e * e) / np.sum(wq * _phi(tq) ** 2))
    tu = np.linspace(x[0], x[-1], 500)
    EM = float(np.max(np.abs(density(breaks, p, alpha, tu) - _phi(tu))))
    return ER, EM
