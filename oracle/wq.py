"""O3: B-spline weighted quadrature and row assembly (test infrastructure only).

Section 4 / Section 5 of the paper, for a closed curve with the cyclic basis
B_i (degree p, N uniform elements of [0, 1)) and the exactness space of the
refined cyclic B-splines Bbar_k (M = N_ref N elements), written with dense
linear algebra and no use of the problem's translation invariance.

Readings taken where the paper leaves the closed-curve case open:

* nodes (Section 4): every breakpoint and every midpoint of the refined mesh,
  eta_n = n / (2M), n = 0..2M-1 (the paper's d+2 points in the end elements
  only exist on an open arc);
* kernel split (Section 3.1) made periodic: K2(s,t) = ln|sin(pi (s-t)) / pi|,
  K1 = K - K2, K1(s,s) = ln J(s) (eq. F1_lim); the paper's ln|s-t| would leave
  K1 singular at the wrap corner s -> 0, t -> 1 where f(0) = f(1);
* "minimum Euclidean norm" solutions are computed by LAPACK's least squares
  (SVD), never by rescaling the collocation rows;
* the row of eq. IK1e2_bis is not exactly symmetric; the assembled matrix keeps
  rows i <= j and mirrors them.
"""
from __future__ import annotations

import math
from math import comb

import numpy as np

from . import bspline, curves


# ---------------------------------------------------------------- nodes, bases
def nodes(N: int, R: int) -> np.ndarray:
    M = R * N
    return np.arange(2 * M, dtype=np.float64) / (2 * M)


def support_nodes(p: int, N: int, R: int, i: int) -> np.ndarray:
    """N^(i): nodes inside the open support (i/N, (i+p+1)/N) of B_i (mod 1)."""
    M = R * N
    return (2 * R * i + np.arange(1, 2 * R * (p + 1))) % (2 * M)


def support_refined_elements(p: int, N: int, R: int, i: int) -> np.ndarray:
    M = R * N
    return np.array(sorted({(R * (i + c) + r) % M for c in range(p + 1) for r in range(R)}))


def exactness_set(p: int, N: int, R: int, i: int) -> np.ndarray:
    """J^(i): refined functions Bbar_k whose support meets supp B_i."""
    M = R * N
    return np.array(sorted({(e - c) % M for e in support_refined_elements(p, N, R, i) for c in range(p + 1)}))


def collocation(p: int, M: int, t) -> np.ndarray:
    """B[k, n] = Bbar_k(t_n) for the M refined cyclic functions."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([bspline.periodic(p, M, k, t) for k in range(M)])


# ---------------------------------------------------------------- Algorithm 1
def regular_weights(p: int, N: int, R: int, rows=None) -> dict:
    """Algorithm 1: for each test function B_i, the weights w^(i) on N^(i) that
    integrate every Bbar_k, k in J^(i), against B_i exactly (eq. reg_exactness),
    minimum-norm when the local system is underdetermined.
    Returns {i: (node indices, weights)}."""
    M = R * N
    eta = nodes(N, R)
    gu, gw = np.polynomial.legendre.leggauss(p + 1)       # exact for degree 2p per element
    gu = (gu + 1.0) / 2.0
    gw = gw / 2.0
    out = {}
    for i in (range(N) if rows is None else rows):
        Jset = exactness_set(p, N, R, i)
        Nset = support_nodes(p, N, R, i)
        elems = support_refined_elements(p, N, R, i)
        tq = ((elems[:, None] + gu[None, :]) / M).ravel()
        wq = np.tile(gw / M, elems.size)
        Bi = bspline.periodic(p, N, i, tq)
        mu = np.array([np.sum(wq * bspline.periodic(p, M, k, tq) * Bi) for k in Jset])
        Bloc = np.stack([bspline.periodic(p, M, k, eta[Nset]) for k in Jset])
        w = np.linalg.lstsq(Bloc, mu, rcond=None)[0]
        out[i] = (Nset, w)
    return out


def regular_weight_matrix(p: int, N: int, R: int) -> np.ndarray:
    M = R * N
    W = np.zeros((N, 2 * M))
    for i, (nset, w) in regular_weights(p, N, R).items():
        W[i, nset] = w
    return W


# ---------------------------------------------------------------- modified moments
def _Phi(j: int, z):
    """Antiderivative z^{j+1}/(j+1) (ln|z| - 1/(j+1)) of z^j ln|z| (Section 4.2), 0 at z = 0."""
    z = np.asarray(z, dtype=np.float64)
    az = np.abs(z)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = z ** (j + 1) / (j + 1) * (np.log(az) - 1.0 / (j + 1))
    return np.where(az == 0.0, 0.0, v)


_GFAR = 16


def log_piece(coef, sigma) -> np.ndarray:
    """int_0^1 P(u) ln|u - sigma| du for P(u) = sum_a coef[..., a] u^a.

    |sigma - 1/2| <= 3/2: the closed form of Section 4.2 in the local variable,
      u^a = sum_j C(a,j) sigma^{a-j} (u - sigma)^j, int z^j ln|z| = Phi_j;
    otherwise the integrand is smooth on [0, 1]: 16-point Gauss-Legendre."""
    coef = np.asarray(coef, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    deg = coef.shape[-1] - 1
    near = np.abs(sigma - 0.5) <= 1.5
    out = np.zeros(np.broadcast(coef[..., 0], sigma).shape)
    sig = np.broadcast_to(sigma, out.shape)
    cf = np.broadcast_to(coef, out.shape + (deg + 1,))
    # closed form
    s = np.where(near, sig, 0.0)
    base = [_Phi(j, 1.0 - s) - _Phi(j, -s) for j in range(deg + 1)]
    cl = np.zeros(out.shape)
    for a in range(deg + 1):
        ia = np.zeros(out.shape)
        for j in range(a + 1):
            ia += comb(a, j) * s ** (a - j) * base[j]
        cl += cf[..., a] * ia
    # Gauss far field
    gu, gw = np.polynomial.legendre.leggauss(_GFAR)
    gu = (gu + 1.0) / 2.0
    gw = gw / 2.0
    sf = np.where(near, 2.0, sig)[..., None]
    P = np.zeros(out.shape + (_GFAR,))
    for a in range(deg + 1):
        P += cf[..., a][..., None] * gu ** a
    far = np.sum(gw * P * np.log(np.abs(gu - sf)), axis=-1)
    return np.where(near, cl, far)


def moments(p: int, M: int, s: float) -> np.ndarray:
    """mu_k(s) = int Bbar_k(t) K2(s, t) dt for k = 0..M-1 (eq. mod_mom_gen with
    the periodic K2).  On a refined element e of supp Bbar_k, with s* the image of
    s nearest the element and x = t - s* (|x| < 1):
    ln|sin(pi x)/pi| = ln|x| + ln sinc(x); ln|x| = ln|u - sigma| - ln M with
    u = M t - e, sigma = M s* - e, handled by ``log_piece``; the smooth
    ln sinc(x) by 16-point Gauss."""
    coef = bspline.piece_monomials(p)                      # M_p(c + u)
    k = np.arange(M)[:, None]
    c = np.arange(p + 1)[None, :]
    e = (k + c) % M                                        # element of piece c of Bbar_k
    centre = (e + 0.5) / M
    s_star = s + np.round(centre - s)
    sigma = M * s_star - e
    L = log_piece(coef[None, :, :], sigma)                 # (M, p+1)
    gu, gw = np.polynomial.legendre.leggauss(_GFAR)
    gu = (gu + 1.0) / 2.0
    gw = gw / 2.0
    Pg = np.stack([np.polyval(coef[cc, ::-1], gu) for cc in range(p + 1)])   # (p+1, G)
    x = (gu[None, None, :] - sigma[..., None]) / M
    S = np.sum(gw * Pg[None, :, :] * np.log(np.sinc(x)), axis=-1)
    piece_int = coef @ (1.0 / np.arange(1, p + 2))        # int_0^1 M_p(c + u) du
    return np.sum((L - math.log(M) * piece_int[None, :] + S) / M, axis=1)


# ---------------------------------------------------------------- Algorithm 2
def singular_weights(p: int, N: int, R: int, sources=None) -> np.ndarray:
    """Algorithm 2 with sigma = eta: for each source eta_m the weights w^(eta_m)
    on all nodes, the minimum-norm solution of B w = mu(eta_m)
    (eq. sing_exactness).  Returns Ws[m, n] for m in ``sources`` (default all)."""
    M = R * N
    eta = nodes(N, R)
    src = np.arange(2 * M) if sources is None else np.asarray(sources)
    B = collocation(p, M, eta)
    Mu = np.stack([moments(p, M, eta[m]) for m in src], axis=1)
    return np.linalg.lstsq(B, Mu, rcond=None)[0].T


def singular_weights_normal(p: int, N: int, R: int, sources) -> np.ndarray:
    """The same minimum-norm weights as w = B^T (B B^T)^{-1} mu with a sparse
    direct factorisation of B B^T (for sampled rows at sizes where the dense
    least-squares solve does not fit)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    M = R * N
    eta = nodes(N, R)
    rows, cols, vals = [], [], []
    for k in range(M):
        n = (2 * k + np.arange(1, 2 * (p + 1))) % (2 * M)
        v = bspline.periodic(p, M, k, eta[n])
        rows += [k] * n.size
        cols += list(n)
        vals += list(v)
    B = sp.csr_matrix((vals, (rows, cols)), shape=(M, 2 * M))
    G = (B @ B.T).tocsc()
    lu = spl.splu(G)
    Mu = np.stack([moments(p, M, eta[m]) for m in sources], axis=1)
    return (B.T @ lu.solve(Mu)).T


# ---------------------------------------------------------------- kernel on nodes
def K2(s, t):
    return np.log(np.abs(np.sin(math.pi * (np.asarray(s) - np.asarray(t)))) / math.pi)


def K1_rows(x, y, J, eta, rows) -> np.ndarray:
    """K1(eta_n1, eta_n2) = ln|f(eta_n1) - f(eta_n2)| - K2 for n1 in rows; the
    diagonal takes the limit ln J (eq. F1_lim)."""
    rows = np.asarray(rows)
    dx = x[rows, None] - x[None, :]
    dy = y[rows, None] - y[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        K = 0.5 * np.log(dx * dx + dy * dy) - K2(eta[rows, None], eta[None, :])
    for r, n in enumerate(rows):
        K[r, n] = math.log(J[n])
    return K


# ---------------------------------------------------------------- assembly
def full_matrix(curve, p: int, N: int, R: int):
    """A_full[i, j] = -(1/2pi) (I_K1 + I_K2) by eqs. IK1e2 and IK1e2_bis:
    A_full = -(1/2pi) (W D_J) [K1 (W D_J)^T + Ws D_J Bmat^T],  Bmat[j, n] = B_j(eta_n).
    Returns (A_full, tables) with the intermediate rules."""
    M = R * N
    eta = nodes(N, R)
    x, y, _, _, J = curves.evaluate(curve, eta)
    W = regular_weight_matrix(p, N, R)
    Ws = singular_weights(p, N, R)
    Bmat = np.stack([bspline.periodic(p, N, j, eta) for j in range(N)])
    K1 = K1_rows(x, y, J, eta, np.arange(2 * M))
    What = W * J[None, :]
    A_full = -(What @ (K1 @ What.T + Ws @ (J[:, None] * Bmat.T))) / (2.0 * math.pi)
    return A_full, dict(W=W, Ws=Ws, Bmat=Bmat, K1=K1, x=x, y=y, J=J, eta=eta)


def symmetrize_upper(A_full: np.ndarray) -> np.ndarray:
    U = np.triu(A_full)
    return U + np.triu(A_full, 1).T


def matrix(curve, p: int, N: int, R: int) -> np.ndarray:
    return symmetrize_upper(full_matrix(curve, p, N, R)[0])


def full_rows(curve, p: int, N: int, R: int, rows) -> np.ndarray:
    """Rows of A_full for sampled rows at large N: only the node rows n1 in the
    supports of the requested rows are formed (sparse W, sparse Bmat)."""
    import scipy.sparse as sp
    M = R * N
    eta = nodes(N, R)
    x, y, _, _, J = curves.evaluate(curve, eta)
    rows = list(rows)
    need = sorted({int(n) for i in rows for n in support_nodes(p, N, R, i)})
    col = {n: c for c, n in enumerate(need)}
    # regular weights of every test function (all columns j need W[j])
    Wd = regular_weights(p, N, R)
    r_, c_, v_ = [], [], []
    rb, cb, vb = [], [], []
    for j in range(N):
        nset, w = Wd[j]
        r_ += [j] * nset.size
        c_ += list(nset)
        v_ += list(w * J[nset])
        bv = bspline.periodic(p, N, j, eta[nset])
        rb += [j] * nset.size
        cb += list(nset)
        vb += list(bv * J[nset])
    What = sp.csr_matrix((v_, (r_, c_)), shape=(N, 2 * M))
    BJ = sp.csr_matrix((vb, (rb, cb)), shape=(N, 2 * M))
    K1 = K1_rows(x, y, J, eta, need)                     # (len(need), 2M)
    Ws = singular_weights_normal(p, N, R, need)          # (len(need), 2M)
    C1 = (What @ K1.T).T + (BJ @ Ws.T).T                 # (len(need), N): [n1, j]
    out = np.zeros((len(rows), N))
    for r, i in enumerate(rows):
        nset, w = Wd[i]
        for n, wn in zip(nset, w):
            out[r] += wn * J[n] * C1[col[int(n)]]
    return -out / (2.0 * math.pi)


def rhs(curve, p: int, N: int, R: int, g) -> np.ndarray:
    """b1^(i) = sum_n w_n^(i) J(eta_n) u_D(eta_n) (Section 5)."""
    eta = nodes(N, R)
    x, y, _, _, J = curves.evaluate(curve, eta)
    gv = g(x, y)
    beta = np.zeros(N)
    for i, (nset, w) in regular_weights(p, N, R).items():
        beta[i] = np.sum(w * J[nset] * gv[nset])
    return beta
