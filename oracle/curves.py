"""Curve geometry for the oracle (test infrastructure only): f(t), f'(t) and
the parametric speed J(t) = |f'(t)| (Section 3, eq. J), for t in [0, 1).

* polar kind: x(t) = r(theta) (cos theta, sin theta), theta = 2 pi t,
  r(theta) = r0 (1 + sum_k a_k cos(k theta + phi_k)), differentiated in closed form;
* B-spline kind: f(t) = sum_j Q_j B_j(t) over the cyclic basis (Section 3),
  on uniform knots or on the periodic extension of the breakpoints
  0 = tau_0 < ... < tau_n = 1 of one period.
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
    elif curve.kind == "bspline" and getattr(curve, "knots", None) is not None:
        x, y, dx, dy = _bspline_periodic_knots(curve.degree, np.asarray(curve.ctrl, dtype=np.float64),
                                               np.asarray(curve.knots, dtype=np.float64), t)
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


def _bspline_periodic_knots(d, Q, tau, t):
    """f and f' of the closed B-spline of degree d with control points Q[n] on
    the periodic knots tau_{k + n} = tau_k + 1 (Section 3).  B_j is the
    Cox-de Boor function on the knots tau_j .. tau_{j+d+1} of the extended
    vector; on [0, 1) it is G_j(t) + G_j(t + 1), the second term its part that
    wraps past t = 1.  f' = sum_j d (Q_j - Q_{j-1}) / (tau_{j+d} - tau_j) B_{j,d-1}
    (the derivative of the recurrence, Section 4.2)."""
    n = Q.shape[0]
    assert tau.shape == (n + 1,) and tau[0] == 0.0 and tau[-1] == 1.0 and np.all(np.diff(tau) > 0)
    ext = np.concatenate([tau[:-1] - 1.0, tau[:-1], tau[:-1] + 1.0, [2.0]])    # tau_k, k = -n .. 2n
    off = n

    def knot(k):
        return ext[k + off]

    def basis(j, r, s):
        T = np.array([knot(k) for k in range(j, j + r + 2)])
        inside = (s >= T[0]) & (s < T[-1])
        out = np.zeros_like(s)
        if inside.any():
            out[inside] = bspline.general(T, r, 0, s[inside])
        return out

    x = np.zeros_like(t)
    y = np.zeros_like(t)
    dx = np.zeros_like(t)
    dy = np.zeros_like(t)
    for j in range(n):
        b = basis(j, d, t) + basis(j, d, t + 1.0)
        x += Q[j, 0] * b
        y += Q[j, 1] * b
        # derivative control point D_j = d (Q_j - Q_{j-1}) / (tau_{j+d} - tau_j) on B_{j,d-1}
        Dj = d * (Q[j] - Q[j - 1]) / (knot(j + d) - knot(j))
        db = basis(j, d - 1, t) + basis(j, d - 1, t + 1.0)
        dx += Dj[0] * db
        dy += Dj[1] * db
    return x, y, dx, dy
