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
