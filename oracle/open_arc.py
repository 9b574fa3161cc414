"""Singular weighted quadrature on an open interval (test infrastructure only).

The paper's own test setting for the singular rule (Section 4.2, eq. ERR,
Table 1): I = [-1, 1] with an open (clamped) knot vector of N_h uniform
elements, degree d, exactness space = the same spline space (N_ref = 1), and
the node vector of Section 4: d+2 uniformly spaced points in the first and the
last element, breakpoints and midpoints elsewhere (N_quad = 2d + 2 N_h - 1).
It pins the modified-moment routine shared with the closed-curve oracle
against closed forms (t^d, eq. testdiff) and against the paper's Table 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import bspline
from .wq import log_piece


def open_knots(d: int, Nh: int) -> np.ndarray:
    inner = np.linspace(-1.0, 1.0, Nh + 1)
    return np.concatenate([np.full(d, -1.0), inner, np.full(d, 1.0)])


def open_nodes(d: int, Nh: int) -> np.ndarray:
    br = np.linspace(-1.0, 1.0, Nh + 1)
    h = 2.0 / Nh
    first = -1.0 + h * np.arange(d + 2) / (d + 1)
    last = 1.0 - h + h * np.arange(d + 2) / (d + 1)
    mids = (br[1:-2] + br[2:-1]) / 2.0          # inner elements 1..Nh-2
    inner_br = br[2:-2]
    return np.sort(np.concatenate([first, last, mids, inner_br]))


def _piece_coefs(knots, d, j, a, b):
    """Monomial coefficients in u in [0, 1] of B_{j,d} restricted to [a, b]."""
    u = (1.0 - np.cos(math.pi * (np.arange(d + 1) + 0.5) / (d + 1))) / 2.0
    vals = bspline.general(knots, d, j, a + (b - a) * u)
    return np.linalg.solve(np.vander(u, d + 1, increasing=True), vals)


def _pieces(d: int, Nh: int):
    """(j, e, coef) for every non-empty piece of every B_j on [-1, 1]."""
    T = open_knots(d, Nh)
    br = np.linspace(-1.0, 1.0, Nh + 1)
    js, es, cs = [], [], []
    for j in range(Nh + d):
        for e in range(Nh):
            a, b = br[e], br[e + 1]
            if b <= T[j] or a >= T[j + d + 1]:
                continue
            js.append(j)
            es.append(e)
            cs.append(_piece_coefs(T, d, j, a, b))
    return np.array(js), np.array(es), np.array(cs)


def moments(d: int, Nh: int, s: float, pieces=None) -> np.ndarray:
    """mu_j(s) = int_{-1}^{1} B_j(t) ln|t - s| dt (eq. mod_mom_gen), j = 0..Nh+d-1,
    element by element: h [ln h int P + int_0^1 P(u) ln|u - sigma| du]."""
    js, es, cs = _pieces(d, Nh) if pieces is None else pieces
    h = 2.0 / Nh
    sigma = (s - (-1.0 + h * es)) / h
    vals = h * (math.log(h) * (cs @ (1.0 / np.arange(1, d + 2))) + log_piece(cs, sigma))
    return np.bincount(js, weights=vals, minlength=Nh + d)


def singular_weights(d: int, Nh: int, sources=None) -> np.ndarray:
    """Algorithm 2 on the open interval: Ws[m, n], minimum-norm."""
    T = open_knots(d, Nh)
    eta = open_nodes(d, Nh)
    src = eta if sources is None else np.asarray(sources, dtype=np.float64)
    B = np.stack([bspline.general(T, d, j, eta) for j in range(Nh + d)])
    pcs = _pieces(d, Nh)
    Mu = np.stack([moments(d, Nh, s, pcs) for s in src], axis=1)
    return np.linalg.lstsq(B, Mu, rcond=None)[0].T


def tsal_exact(s):
    """eq. testdiff: int_{-1}^1 ln|t - s| sqrt(1 - t^2) / (t^2 + 25) dt."""
    s = np.asarray(s, dtype=np.float64)
    return math.pi * math.log(2.0) + math.pi * math.sqrt(26.0) / 5.0 * np.log(
        np.sqrt(25.0 + s * s) / (5.0 + math.sqrt(26.0)))


def tsal_integrand(t):
    t = np.asarray(t, dtype=np.float64)
    return np.sqrt(np.maximum(1.0 - t * t, 0.0)) / (t * t + 25.0)


def err_ratio(Q: np.ndarray, I: np.ndarray) -> float:
    """eq. ERR: sum (Q - I)^2 / sum Q^2 over the source nodes."""
    return float(np.sum((Q - I) ** 2) / np.sum(Q ** 2))
