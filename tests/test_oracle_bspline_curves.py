"""Pins for the oracle's B-splines and curve geometry (CPU)."""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import synth
from oracle import bspline, curves


@pytest.mark.parametrize("p", range(0, 7))
def test_cardinal_matches_scipy(p):
    x = np.linspace(-0.5, p + 1.5, 997)
    ref = np.nan_to_num(BSpline.basis_element(np.arange(p + 2), extrapolate=False)(x))
    assert np.abs(bspline.cardinal(p, x) - ref).max() < 1e-14


def test_cardinal_cubic_knot_values():
    assert np.allclose(bspline.cardinal(3, np.array([1.0, 2.0, 3.0])), [1 / 6, 2 / 3, 1 / 6], atol=1e-16)


@pytest.mark.parametrize("p,N", [(2, 7), (3, 16), (4, 10)])
def test_periodic_partition_of_unity(p, N):
    t = np.random.default_rng(0).uniform(0, 1, 500)
    s = sum(bspline.periodic(p, N, i, t) for i in range(N))
    assert np.abs(s - 1).max() < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_piece_monomials_and_derivative(p):
    coef = bspline.piece_monomials(p)
    u = np.linspace(0, 0.999, 50)
    for c in range(p + 1):
        assert np.abs(np.polyval(coef[c, ::-1], u) - bspline.cardinal(p, c + u)).max() < 1e-13
    x = (np.arange(p + 1)[:, None] + np.linspace(0.05, 0.95, 19)[None, :]).ravel()
    fd = (bspline.cardinal(p, x + 1e-6) - bspline.cardinal(p, x - 1e-6)) / 2e-6
    assert np.abs(fd - bspline.cardinal_deriv(p, x)).max() < 1e-6


@pytest.mark.parametrize("d,Nh", [(2, 5), (3, 8), (5, 6)])
def test_general_open_knots_match_scipy(d, Nh):
    T = np.concatenate([np.full(d, -1.0), np.linspace(-1, 1, Nh + 1), np.full(d, 1.0)])
    t = np.linspace(-1, 1, 301)
    tot = np.zeros_like(t)
    for j in range(Nh + d):
        ref = BSpline.basis_element(T[j:j + d + 2], extrapolate=False)(t)
        mine = bspline.general(T, d, j, t)
        ok = ~np.isnan(ref) & (t < 1.0)      # scipy's element is right-open at t = 1
        assert np.abs(mine[ok] - ref[ok]).max() < 1e-13
        tot += mine
    assert np.abs(tot - 1).max() < 1e-13


def test_circle_geometry():
    x, y, dx, dy, J = curves.evaluate(synth.circle(0.5), np.linspace(0, 1, 33))
    assert np.abs(np.hypot(x, y) - 0.5).max() < 1e-15
    assert np.abs(J - math.pi).max() < 1e-14


@pytest.mark.parametrize("curve", [synth.star(3), synth.ellipse_bspline()])
def test_derivative_matches_finite_difference(curve):
    t = np.random.default_rng(1).uniform(0, 1, 200)
    h = 1e-6
    xp, yp, *_ = curves.evaluate(curve, t + h)
    xm, ym, *_ = curves.evaluate(curve, t - h)
    _, _, dx, dy, J = curves.evaluate(curve, t)
    assert np.abs((xp - xm) / (2 * h) - dx).max() < 1e-6 * np.abs(dx).max()
    assert np.abs((yp - ym) / (2 * h) - dy).max() < 1e-6 * np.abs(dy).max()


def test_ellipse_bspline_interpolates_at_knots():
    c = synth.ellipse_bspline()
    t = np.arange(32) / 32
    x, y, *_ = curves.evaluate(c, t)
    th = 2 * math.pi * t
    assert np.abs(x - np.cos(th)).max() < 1e-14
    assert np.abs(y - 0.5 * np.sin(th)).max() < 1e-14
    tm = (np.arange(32) + 0.5) / 32
    x, y, *_ = curves.evaluate(c, tm)
    assert np.abs(np.hypot(x, 2 * y) - 1).max() < 5e-6


def _scipy_periodic(curve):
    """scipy's BSpline on the extended knot vector tau_{-d} .. tau_{n+d} with
    coefficients Q_{(i - d) mod n}: the closed curve on [0, 1)."""
    d, Q, tau = curve.degree, np.asarray(curve.ctrl), np.asarray(curve.knots)
    n = Q.shape[0]
    text = np.concatenate([tau[n - d:n] - 1.0, tau, tau[1:d + 1] + 1.0])
    return BSpline(text, np.array([Q[(i - d) % n] for i in range(n + d)]), d)


@pytest.mark.parametrize("curve", [
    synth.ellipse_bspline_nonuniform(0),
    synth.ellipse_bspline_nonuniform(5, n_ctrl=9, jitter=0.6),
    synth.BSplineCurve(degree=2, ctrl=np.random.default_rng(4).normal(size=(7, 2)),
                       knots=np.array([0.0, 0.05, 0.3, 0.35, 0.6, 0.8, 0.93, 1.0])),
    synth.BSplineCurve(degree=5, ctrl=np.random.default_rng(6).normal(size=(11, 2)),
                       knots=np.sort(np.concatenate([[0.0, 1.0], np.random.default_rng(7).uniform(0, 1, 10)]))),
])
def test_periodic_knots_match_scipy(curve):
    t = np.concatenate([np.linspace(0, 1, 777, endpoint=False), np.asarray(curve.knots[:-1])])
    S = _scipy_periodic(curve)
    ref, dref = S(t), S.derivative()(t)
    x, y, dx, dy, J = curves.evaluate(curve, t)
    sc = np.abs(ref).max()
    assert np.abs(x - ref[:, 0]).max() < 1e-14 * sc and np.abs(y - ref[:, 1]).max() < 1e-14 * sc
    dsc = np.abs(dref).max()
    assert np.abs(dx - dref[:, 0]).max() < 1e-13 * dsc and np.abs(dy - dref[:, 1]).max() < 1e-13 * dsc
    assert np.allclose(J, np.hypot(dref[:, 0], dref[:, 1]), rtol=1e-12, atol=0)


def test_uniform_knot_vector_reduces_to_the_uniform_curve():
    import dataclasses
    u = synth.ellipse_bspline()
    uk = dataclasses.replace(u, knots=np.arange(33) / 32)
    t = np.random.default_rng(2).uniform(0, 1, 400)
    for a, b in zip(curves.evaluate(u, t), curves.evaluate(uk, t)):
        assert np.abs(a - b).max() < 1e-13 * max(1.0, np.abs(a).max())


def test_nonuniform_ellipse_is_closed_and_convex():
    c = synth.ellipse_bspline_nonuniform(0)
    t = np.linspace(0, 1, 2001)
    x, y, dx, dy, J = curves.evaluate(c, np.mod(t, 1.0))
    assert J.min() > 0.1
    # turning direction never changes sign (convex, counter-clockwise)
    cross = dx[:-1] * dy[1:] - dy[:-1] * dx[1:]
    assert (cross > 0).all()
