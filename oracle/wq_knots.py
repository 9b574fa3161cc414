"""O6: B-spline weighted quadrature and row assembly on non-uniform periodic
knots (test infrastructure only).

The general form of Section 4 (Algorithms 1 and 2) and Section 5 (eqs. IK1e2,
IK1e2_bis) for a closed curve, written with dense linear algebra:

* approximation space (Section 3): periodic B-splines B_i of degree p on the
  knots tau_0 = 0 < tau_1 < ... < tau_N = 1 of one period, extended by
  tau_{k+N} = tau_k + 1; B_i is supported on [tau_i, tau_{i+p+1}) mod 1;
* exactness space: the same construction on the refined knots, every element
  [tau_e, tau_{e+1}] split into R equal parts (M = R N refined elements);
* nodes: every breakpoint and every midpoint of the refined mesh (the
  closed-curve reading of the node vector of Section 4), eta_{2k} = taubar_k,
  eta_{2k+1} = (taubar_k + taubar_{k+1}) / 2;
* Algorithm 1 per test function (the local systems are no longer shifts of
  one another), Algorithm 2 per source (no translation invariance: the full
  2M x 2M table of singular weights), both minimum-norm by LAPACK least
  squares;
* the periodic kernel split K2(s, t) = ln|sin(pi (s - t)) / pi| of the
  uniform oracle, K1 = K - K2 with the diagonal limit ln J (eq. F1_lim).

Modified moments (eq. mod_mom_gen) use the closed forms of Section 4.2 in the
local variable of each refined element, with the local monomial coefficients
of every piece obtained from the Cox-de Boor recurrence (Section 4.2) carried
out on polynomials of the local variable.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as npoly

from . import bspline, curves
from .wq import K1_rows, log_piece, symmetrize_upper


# ---------------------------------------------------------------- knots, nodes
def check_knots(tau) -> np.ndarray:
    tau = np.asarray(tau, dtype=np.float64)
    assert tau.ndim == 1 and tau.size >= 2 and tau[0] == 0.0 and tau[-1] == 1.0 and np.all(np.diff(tau) > 0)
    return tau


def refine(tau, R: int) -> np.ndarray:
    """Every element split into R equal parts: M + 1 breakpoints, M = R N."""
    tau = check_knots(tau)
    N = tau.size - 1
    tb = np.empty(R * N + 1)
    for e in range(N):
        tb[R * e:R * e + R] = tau[e] + (tau[e + 1] - tau[e]) * np.arange(R) / R
    tb[-1] = 1.0
    return tb


def nodes(tau, R: int) -> np.ndarray:
    tb = refine(tau, R)
    M = tb.size - 1
    eta = np.empty(2 * M)
    eta[0::2] = tb[:-1]
    eta[1::2] = 0.5 * (tb[:-1] + tb[1:])
    return eta


def ext(tau, k: int) -> float:
    """Extended periodic knot tau_k for any integer k."""
    n = tau.size - 1
    q, r = divmod(k, n)
    return float(tau[r] + q)


def basis(tau, p: int, i: int, t) -> np.ndarray:
    """Periodic B_i on the knots tau at t in [0, 1): the Cox-de Boor function
    on tau_i .. tau_{i+p+1} plus its part that wraps past t = 1."""
    t = np.asarray(t, dtype=np.float64)
    T = np.array([ext(tau, k) for k in range(i, i + p + 2)])

    def one(s):
        inside = (s >= T[0]) & (s < T[-1])
        out = np.zeros_like(s)
        if inside.any():
            out[inside] = bspline.general(T, p, 0, s[inside])
        return out

    return one(t) + one(t + 1.0)


def piece_poly(tau, p: int, k: int, e: int) -> np.ndarray:
    """Local monomial coefficients (low to high, in u = (t - tau_e) / h_e on
    [0, 1]) of the periodic B_k of degree p on element e (zero if e is not in
    its support): the Cox-de Boor recurrence on polynomials of u."""
    n = tau.size - 1
    a, b = ext(tau, e), ext(tau, e + 1)
    h = b - a
    # functions j = e - r .. e of degree r nonzero on span e, by degree
    polys = {e: np.array([1.0])}
    for r in range(1, p + 1):
        new = {}
        for j in range(e - r, e + 1):
            acc = np.zeros(1)
            if j in polys:                      # (t - tau_j) / (tau_{j+r} - tau_j) B_{j, r-1}
                lin = np.array([a - ext(tau, j), h]) / (ext(tau, j + r) - ext(tau, j))
                acc = npoly.polyadd(acc, npoly.polymul(lin, polys[j]))
            if j + 1 in polys:                  # (tau_{j+r+1} - t) / (tau_{j+r+1} - tau_{j+1}) B_{j+1, r-1}
                lin = np.array([ext(tau, j + r + 1) - a, -h]) / (ext(tau, j + r + 1) - ext(tau, j + 1))
                acc = npoly.polyadd(acc, npoly.polymul(lin, polys[j + 1]))
            new[j] = acc
        polys = new
    out = np.zeros(p + 1)
    for j, c in polys.items():
        if j % n == k % n:
            out[:c.size] += c
    return out


# ---------------------------------------------------------------- Algorithm 1
def support_nodes(p: int, N: int, R: int, i: int) -> np.ndarray:
    """Nodes inside the open support of B_i (the same indices as for uniform knots)."""
    return (2 * R * i + np.arange(1, 2 * R * (p + 1))) % (2 * R * N)


def exactness_set(p: int, N: int, R: int, i: int) -> np.ndarray:
    M = R * N
    elems = {(R * i + c) % M for c in range(R * (p + 1))}
    return np.array(sorted({(e - c) % M for e in elems for c in range(p + 1)}))


def regular_weights(tau, p: int, R: int, rows=None) -> dict:
    """Algorithm 1 for each test function B_i: the weights on the nodes inside
    supp B_i that integrate every refined Bbar_k meeting supp B_i against B_i
    exactly (eq. reg_exactness), minimum-norm.  The moments int Bbar_k B_i are
    integrals of piecewise polynomials of degree 2p on the refined mesh: Gauss
    with p + 1 points per refined element is exact."""
    tau = check_knots(tau)
    N = tau.size - 1
    tb = refine(tau, R)
    M = R * N
    eta = nodes(tau, R)
    gu, gw = np.polynomial.legendre.leggauss(p + 1)
    gu, gw = (gu + 1.0) / 2.0, gw / 2.0
    out = {}
    for i in (range(N) if rows is None else rows):
        Jset = exactness_set(p, N, R, i)
        Nset = support_nodes(p, N, R, i)
        elems = np.array(sorted({(R * i + c) % M for c in range(R * (p + 1))}))
        h = tb[elems + 1] - tb[elems]
        tq = (tb[elems][:, None] + h[:, None] * gu[None, :]).ravel()
        wq = (h[:, None] * gw[None, :]).ravel()
        Bi = basis(tau, p, i, tq)
        mu = np.array([np.sum(wq * basis(tb, p, int(k), tq) * Bi) for k in Jset])
        Bloc = np.stack([basis(tb, p, int(k), eta[Nset]) for k in Jset])
        out[i] = (Nset, np.linalg.lstsq(Bloc, mu, rcond=None)[0])
    return out


def regular_weight_matrix(tau, p: int, R: int) -> np.ndarray:
    N = np.asarray(tau).size - 1
    W = np.zeros((N, 2 * R * N))
    for i, (nset, w) in regular_weights(tau, p, R).items():
        W[i, nset] = w
    return W


# ---------------------------------------------------------------- modified moments
_GFAR = 16


def pieces(tb, p: int) -> np.ndarray:
    """C[e, c] = local coefficients of the piece of Bbar_{(e - c) mod M} on refined element e."""
    M = tb.size - 1
    return np.array([[piece_poly(tb, p, (e - c) % M, e) for c in range(p + 1)] for e in range(M)])


def moments(tb, p: int, s: float, C=None) -> np.ndarray:
    """mu_k(s) = int Bbar_k(t) K2(s, t) dt for every refined function k (eq.
    mod_mom_gen, periodic K2).  On refined element e = [a, a + h] with local
    coefficients P of the piece and s* the image of s nearest the element:
    ln|sin(pi x)/pi| = ln|x| + ln sinc(x), x = t - s*;
    ln|x| = ln h + ln|u - sigma|, sigma = (s* - a) / h, by ``log_piece``; the
    smooth ln sinc by 16-point Gauss.  C: ``pieces(tb, p)`` if already formed."""
    M = tb.size - 1
    if C is None:
        C = pieces(tb, p)
    gu, gw = np.polynomial.legendre.leggauss(_GFAR)
    gu, gw = (gu + 1.0) / 2.0, gw / 2.0
    a, h = tb[:-1], np.diff(tb)
    s_star = s + np.round((a + 0.5 * h) - s)
    sigma = (s_star - a) / h                                              # (M,)
    L = log_piece(C, sigma[:, None])                                      # (M, p+1)
    ip = C @ (1.0 / np.arange(1, p + 2))                                  # int_0^1 P
    lsinc = np.log(np.sinc(a[:, None] + h[:, None] * gu[None, :] - s_star[:, None]))   # (M, G)
    Pg = np.einsum("eca,ga->ecg", C, gu[:, None] ** np.arange(p + 1)[None, :])
    S = np.einsum("ecg,g,eg->ec", Pg, gw, lsinc)
    part = h[:, None] * (L + np.log(h)[:, None] * ip + S)                 # (M, p+1)
    mu = np.zeros(M)
    k = (np.arange(M)[:, None] - np.arange(p + 1)[None, :]) % M
    np.add.at(mu, k, part)
    return mu


# ---------------------------------------------------------------- Algorithm 2
def collocation(tb, p: int, t) -> np.ndarray:
    M = tb.size - 1
    return np.stack([basis(tb, p, k, t) for k in range(M)])


def singular_weights(tau, p: int, R: int) -> np.ndarray:
    """Algorithm 2 with sigma = eta: for every source eta_m the minimum-norm
    weights on all nodes that integrate every refined Bbar_k against
    K2(eta_m, .) exactly (eq. sing_exactness).  Returns Ws[m, n] (2M x 2M)."""
    tb = refine(tau, R)
    eta = nodes(tau, R)
    B = collocation(tb, p, eta)
    C = pieces(tb, p)
    Mu = np.stack([moments(tb, p, s, C) for s in eta], axis=1)
    return np.linalg.lstsq(B, Mu, rcond=None)[0].T


# ---------------------------------------------------------------- assembly
def full_matrix(curve, tau, p: int, R: int):
    """A_full = -(1/2pi) (W D_J) [K1 (W D_J)^T + Ws D_J Bmat^T], Bmat[j, n] = B_j(eta_n)
    (eqs. IK1e2, IK1e2_bis)."""
    tau = check_knots(tau)
    N = tau.size - 1
    eta = nodes(tau, R)
    x, y, _, _, J = curves.evaluate(curve, eta)
    W = regular_weight_matrix(tau, p, R)
    Ws = singular_weights(tau, p, R)
    Bmat = np.stack([basis(tau, p, j, eta) for j in range(N)])
    K1 = K1_rows(x, y, J, eta, np.arange(eta.size))
    What = W * J[None, :]
    A_full = -(What @ (K1 @ What.T + Ws @ (J[:, None] * Bmat.T))) / (2.0 * math.pi)
    return A_full, dict(W=W, Ws=Ws, Bmat=Bmat, K1=K1, x=x, y=y, J=J, eta=eta)


def matrix(curve, tau, p: int, R: int) -> np.ndarray:
    return symmetrize_upper(full_matrix(curve, tau, p, R)[0])


def rhs(curve, tau, p: int, R: int, g) -> np.ndarray:
    """b1_i = sum_n w_n^(i) J(eta_n) u_D(f(eta_n)) (Section 5)."""
    eta = nodes(tau, R)
    x, y, _, _, J = curves.evaluate(curve, eta)
    gv = g(x, y)
    N = np.asarray(tau).size - 1
    beta = np.zeros(N)
    for i, (nset, w) in regular_weights(tau, p, R).items():
        beta[i] = np.sum(w * J[nset] * gv[nset])
    return beta
