"""Seeded synthetic inputs for the IgA-SGBEM Galerkin assembly.

This module only *describes* problem instances: curve descriptions (control
points or polar Fourier coefficients), discretisation parameters and
Dirichlet data functions.  It holds none of the method's arithmetic (no
B-spline evaluation, no quadrature, no kernel), so that both the HIP path and
the CPU oracle can take their inputs from here without sharing any code.

Workloads (the paper's own test curves are an open parabola and an S-shape
whose control points only exist in a missing figure, Section 6, so these
synthetic closed curves stand in for them):

* ``circle``: x(t) = r (cos 2 pi t, sin 2 pi t), the closed-form check case.
* ``ellipse_bspline``: semi-axes (1, 0.5) as a closed uniform cubic B-spline
  of 32 control points interpolating the ellipse at the knots.  A closed
  curve is a periodic B-spline whose last d control points repeat the first
  ones (Section 3); here the periodic repetition is implicit.
* ``star``: r(theta) = 1 + sum_{k=1..6} a_k cos(k theta + phi_k) with
  a_k ~ U(0, 0.1/k), phi_k ~ U(0, 2 pi), drawn from numpy's PCG64 seeded
  with ``[1703, idx]``.

Open arcs (Section 2, exterior problem; Section 6, parabola test):

* ``parabola``: f(t) = (t, 1 - t^2), t in [-1, 1], the quadratic arc with
  control points (-1, 0), (0, 2), (1, 0) on the knots [-1, -1, -1, 1, 1, 1];
* ``parabola_phi``: the density sqrt(1 + 4 x1^2) of the test, and
  ``parabola_uD``: its single-layer potential u_D = V phi on the arc, the
  Dirichlet datum, in closed form (an exact integral, not a quadrature);
* ``open_arc_bspline``: seeded open cubic arcs (a wavy open curve) for
  the general open-arc paths.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Tuple

import numpy as np

__all__ = [
    "PolarCurve", "BSplineCurve", "OpenBSplineCurve", "circle", "parabola", "parabola_uD", "parabola_phi",
    "open_arc_bspline", "ellipse_bspline", "ellipse_bspline_nonuniform", "star",
    "g_x2_minus_y2", "g_exp_cos", "Problem", "config_circle", "config_ellipse",
    "config_stars", "config_batch", "config_serving",
]


@dataclass(frozen=True)
class PolarCurve:
    """r(theta) = r0 * (1 + sum_k a[k-1] cos(k theta + phi[k-1])), theta = 2 pi t,
    traversed counter-clockwise for t in [0, 1)."""
    r0: float
    a: np.ndarray = field(default_factory=lambda: np.zeros(0))
    phi: np.ndarray = field(default_factory=lambda: np.zeros(0))
    kind: str = "polar"


@dataclass(frozen=True)
class BSplineCurve:
    """Closed curve f(t) = sum_j ctrl[j] B_j(t) with periodic knots on n_ctrl
    elements of [0, 1); B_j is supported on [tau_j, tau_{j+degree+1}) mod 1.
    ``ctrl`` has shape (n_ctrl, 2); the first ``degree`` points are not repeated.
    ``knots``: None for uniform knots tau_k = k / n_ctrl, else the n_ctrl + 1
    breakpoints tau_0 = 0 < tau_1 < ... < tau_n = 1 of one period (extended
    periodically, tau_{k+n} = tau_k + 1)."""
    degree: int
    ctrl: np.ndarray
    kind: str = "bspline"
    knots: np.ndarray = None


@dataclass(frozen=True)
class OpenBSplineCurve:
    """Open arc f(t) = sum_j ctrl[j] B_j(t), t in [knots[0], knots[-1]], on the
    clamped knot vector ``knots`` (n_ctrl + degree + 1 values, the first and the
    last degree + 1 equal, the inner ones strictly increasing)."""
    degree: int
    ctrl: np.ndarray
    knots: np.ndarray
    kind: str = "bspline_open"


def circle(r: float = 0.5) -> PolarCurve:
    return PolarCurve(r0=float(r))


def ellipse_bspline(a: float = 1.0, b: float = 0.5, n_ctrl: int = 32) -> BSplineCurve:
    """Closed uniform cubic B-spline interpolating the ellipse (a cos th, b sin th)
    at its n_ctrl knots.  B_j peaks at the knot (j+2)/n; (cos th, sin th) are
    single Fourier modes, so the control polygon is the ellipse scaled by
    3 / (2 + cos(2 pi / n)) (the cubic's knot values are 1/6, 2/3, 1/6)."""
    th = 2.0 * math.pi * (np.arange(n_ctrl) + 2) / n_ctrl
    scale = 3.0 / (2.0 + math.cos(2.0 * math.pi / n_ctrl))
    ctrl = scale * np.stack([a * np.cos(th), b * np.sin(th)], axis=1)
    return BSplineCurve(degree=3, ctrl=np.ascontiguousarray(ctrl))


def ellipse_bspline_nonuniform(idx: int = 0, n_ctrl: int = 32, jitter: float = 0.35) -> BSplineCurve:
    """The control polygon of ``ellipse_bspline`` on non-uniform periodic knots
    tau_k = (k + jitter (u_k - 1/2)) / n_ctrl, u_k ~ U(0, 1) from PCG64 seeded
    with [1703, 30000 + idx], tau_0 = 0 and tau_n = 1 (element lengths between
    (1 - jitter) / n and (1 + jitter) / n).  The control polygon is convex, so
    the curve is a simple closed convex curve near the ellipse."""
    rng = np.random.default_rng([1703, 30000 + int(idx)])
    u = rng.uniform(0.0, 1.0, n_ctrl)
    u[0] = 0.5
    tau = (np.arange(n_ctrl + 1) + jitter * (np.append(u, 0.5) - 0.5)) / n_ctrl
    base = ellipse_bspline(n_ctrl=n_ctrl)
    return BSplineCurve(degree=3, ctrl=base.ctrl, knots=np.ascontiguousarray(tau))


def star(idx: int, n_modes: int = 6) -> PolarCurve:
    rng = np.random.default_rng([1703, int(idx)])
    k = np.arange(1, n_modes + 1)
    a = rng.uniform(0.0, 0.1 / k)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return PolarCurve(r0=1.0, a=a, phi=phi)


def parabola() -> OpenBSplineCurve:
    """The arc of the parabola test: x1 = t, x2 = 1 - t^2, t in [-1, 1]."""
    return OpenBSplineCurve(degree=2, ctrl=np.array([[-1.0, 0.0], [0.0, 2.0], [1.0, 0.0]]),
                            knots=np.array([-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]))


def open_arc_bspline(idx: int = 0, n_ctrl: int = 12) -> OpenBSplineCurve:
    """Open cubic arc over [0, 1]: control points (x_j, y_j) with x_j = j / (n - 1)
    and y_j = 0.3 sin(3 x_j + c) + 0.1 u_j, c ~ U(0, 2 pi), u_j ~ U(-1, 1) from
    PCG64 seeded with [1703, 50000 + idx]; clamped knots with uniform inner
    knots (a graph over x1: no self-intersection)."""
    rng = np.random.default_rng([1703, 50000 + int(idx)])
    c = rng.uniform(0.0, 2.0 * math.pi)
    x = np.arange(n_ctrl) / (n_ctrl - 1)
    y = 0.3 * np.sin(3.0 * x + c) + 0.1 * rng.uniform(-1.0, 1.0, n_ctrl)
    d = 3
    inner = np.arange(1, n_ctrl - d) / (n_ctrl - d)
    knots = np.concatenate([np.zeros(d + 1), inner, np.ones(d + 1)])
    return OpenBSplineCurve(degree=d, ctrl=np.ascontiguousarray(np.stack([x, y], axis=1)), knots=knots)


def parabola_phi(t):
    """The exact density of the parabola test at f(t): sqrt(1 + 4 t^2)."""
    t = np.asarray(t, dtype=np.float64)
    return np.sqrt(1.0 + 4.0 * t * t)


def _zlogz(k: int, z):
    """int_0^z w^k ln|w| dw = z^(k+1) (ln|z| / (k+1) - 1 / (k+1)^2), 0 at z = 0."""
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = z ** (k + 1) * (np.log(np.abs(z)) / (k + 1) - 1.0 / (k + 1) ** 2)
    return np.where(z == 0.0, 0.0, v)


def _ulog1p(k: int, u):
    """Antiderivatives of u^k ln(1 + u^2), k = 0, 1, 2."""
    u = np.asarray(u, dtype=np.float64)
    L = np.log1p(u * u)
    if k == 0:
        return u * L - 2.0 * u + 2.0 * np.arctan(u)
    if k == 1:
        return 0.5 * ((1.0 + u * u) * L - u * u)
    return u ** 3 / 3.0 * L - 2.0 * u ** 3 / 9.0 + 2.0 * u / 3.0 - 2.0 / 3.0 * np.arctan(u)


def parabola_uD(x1, x2=None):
    """Dirichlet datum of the parabola test, u_D(f(s)) = -(1/2pi) int_{-1}^{1}
    ln|f(s) - f(t)| phi(f(t)) J(t) dt at the arc point with x1 = s.  On this arc
    |f(s) - f(t)| = |s - t| sqrt(1 + (s + t)^2) and phi J = 1 + 4 t^2, so the
    integral is int ln|z| [(1 + 4 s^2) + 8 s z + 4 z^2] dz over z = t - s plus
    one half of int ln(1 + u^2) [(1 + 4 s^2) - 8 s u + 4 u^2] du over u = s + t,
    both elementary."""
    s = np.asarray(x1, dtype=np.float64)
    c1 = (1.0 + 4.0 * s * s, 8.0 * s, 4.0)
    I1 = sum(ck * (_zlogz(k, 1.0 - s) - _zlogz(k, -1.0 - s)) for k, ck in enumerate(c1))
    c2 = (1.0 + 4.0 * s * s, -8.0 * s, 4.0)
    I2 = sum(ck * (_ulog1p(k, s + 1.0) - _ulog1p(k, s - 1.0)) for k, ck in enumerate(c2))
    return -(I1 + 0.5 * I2) / (2.0 * math.pi)


# Dirichlet data: harmonic functions of the physical point (x1, x2).
def g_x2_minus_y2(x1, x2):
    return x1 * x1 - x2 * x2


def g_exp_cos(x1, x2):
    return np.exp(x1) * np.cos(x2)


@dataclass(frozen=True)
class Problem:
    name: str
    curve: object
    p: int
    N: int
    g: Callable
    g_name: str


def config_circle() -> Problem:
    """Circle r = 0.5, p = 2, N = 64, g = x1^2 - x2^2."""
    return Problem("circle_r0.5_p2_N64", circle(0.5), 2, 64, g_x2_minus_y2, "x1^2-x2^2")


def config_ellipse() -> Problem:
    """Ellipse (1, 0.5) as a 32-point closed cubic B-spline, p = 3, N = 1024."""
    return Problem("ellipse_bspline32_p3_N1024", ellipse_bspline(), 3, 1024, g_exp_cos, "exp(x1)cos(x2)")


def config_stars(n_per: int = 8) -> List[Problem]:
    """Stars for p in {2,3,4} x N in {4096, 16384}, n_per curves each."""
    out = []
    idx = 0
    for p in (2, 3, 4):
        for N in (4096, 16384):
            for _ in range(n_per):
                out.append(Problem(f"star{idx}_p{p}_N{N}", star(idx), p, N, g_exp_cos, "exp(x1)cos(x2)"))
                idx += 1
    return out


def config_batch(n: int = 256) -> List[Problem]:
    """n stars with N ~ U{128..2048}, p in {2,3}: seeds [1703, 10000 + idx]."""
    out = []
    for idx in range(n):
        rng = np.random.default_rng([1703, 10000 + idx])
        N = int(rng.integers(128, 2049))
        p = int(rng.choice([2, 3]))
        out.append(Problem(f"batch{idx}_p{p}_N{N}", star(10000 + idx), p, N, g_exp_cos, "exp(x1)cos(x2)"))
    return out


def config_serving(rate: float, n: int = 2000, n_min: int = 256, n_max: int = 8192
                   ) -> Tuple[np.ndarray, List[Problem]]:
    """Poisson arrivals at ``rate`` req/s: exponential inter-arrival times and
    log-uniform N in [n_min, n_max], p in {2,3,4}; seed [1703, 20000 + rate]."""
    rng = np.random.default_rng([1703, 20000 + int(round(rate))])
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps)
    probs = []
    for idx in range(n):
        N = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        p = int(rng.choice([2, 3, 4]))
        probs.append(Problem(f"req{idx}_p{p}_N{N}", star(30000 + idx), p, N, g_exp_cos, "exp(x1)cos(x2)"))
    return arrivals, probs
