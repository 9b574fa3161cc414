"""Curve geometry for the oracle (test infrastructure only): f(t), f'(t) and
the parametric speed J(t) = |f'(t)| (Section 3, eq. J), for t in [0, 1).

* polar kind: x(t) = r(theta) (cos theta, sin theta), theta = 2 pi t,
  r(theta) = r0 (1 + sum_k a_k cos(k theta + phi_k)), differentiated in closed form;
* B-spline kind: f(t) = sum_j Q_j B_j(t) over the cyclic basis (Section 3).
"""
from __future__ import annotations

import math

import numpy as np

from . import bspline


def evaluate(curve, t):
    """Return (x, y, dx, dy, J) at parameters t (any shape)."""
    t = np.asarray(t, dtype=np.float64)
    if curve.kind == "polar":
        th = 2.0 * math.pi * t
        r = np.ones_like(th)
        dr = np.zeros_like(th)
        for k, (a, ph) in enumerate(zip(curve.a, curve.phi), start=1):
            r = r + a * np.cos(k * th + ph)
            dr = dr - k * a * np.sin(k * th + ph)
        r = curve.r0 * r
        dr = curve.r0 * dr
        c, s = np.cos(th), np.sin(th)
        x, y = r * c, r * s
        dx = 2.0 * math.pi * (dr * c - r * s)
        dy = 2.0 * math.pi * (dr * s + r * c)
    elif curve.kind == "bspline":
        d = curve.degree
        Q = np.asarray(curve.ctrl, dtype=np.float64)
        n = Q.shape[0]
        x = np.zeros_like(t)
        y = np.zeros_like(t)
        dx = np.zeros_like(t)
        dy = np.zeros_like(t)
        for j in range(n):
            u = np.mod(n * t - j, n)
            b = bspline.cardinal(d, u)
            db = n * bspline.cardinal_deriv(d, u)
            x += Q[j, 0] * b
            y += Q[j, 1] * b
            dx += Q[j, 0] * db
            dy += Q[j, 1] * db
    else:
        raise ValueError(f"unknown curve kind {curve.kind!r}")
    J = np.sqrt(dx * dx + dy * dy)
    return x, y, dx, dy, J
