"""Pins of the direct-formulation oracle (O4: eq. final_b2, Section 5) against
facts that do not come from its own formula."""
import math

import numpy as np
import pytest

import synth
from oracle import bspline, curves, direct, wq


def test_kbar_is_pi_on_the_circle():
    """On a circle of radius r, (y - x) . n_y = r (1 - cos d) and |x - y|^2 =
    2 r^2 (1 - cos d), so the outward normal derivative of ln|x - y| is 1/(2r)
    and Kbar = J / (2r) = pi for every pair of distinct points."""
    rng = np.random.default_rng(5)
    s, t = rng.random(200), rng.random(200)
    keep = np.abs(((s - t + 0.5) % 1.0) - 0.5) > 0.01      # away from the cancellation of near pairs
    s, t = s[keep], t[keep]
    for r in (0.5, 1.7):
        assert np.abs(direct.kbar(synth.circle(r), s, t) - math.pi).max() < 1e-12


@pytest.mark.parametrize("curve", [synth.star(3), synth.ellipse_bspline()], ids=["star", "ellipse"])
def test_kbar_is_the_outward_normal_derivative(curve):
    """Central difference of ln|f(s) - y| along the outward normal at y = f(t),
    with the normal taken from a difference quotient of f (tangent rotated by
    -90 degrees) and the orientation from the shoelace area (counter-clockwise
    curves have positive area), times the parametric speed."""
    tt = np.linspace(0.0, 1.0, 4001)[:-1]
    x, y = curves.evaluate(curve, tt)[:2]
    area = 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)
    assert area > 0
    rng = np.random.default_rng(9)
    s, t = rng.random(50), rng.random(50)
    keep = np.abs(((s - t + 0.5) % 1.0) - 0.5) > 0.02
    s, t = s[keep], t[keep]
    d = 1e-6
    xs, ys = curves.evaluate(curve, s)[:2]
    xp, yp = curves.evaluate(curve, t + d)[:2]
    xm, ym = curves.evaluate(curve, t - d)[:2]
    tx, ty = (xp - xm) / (2 * d), (yp - ym) / (2 * d)
    J = np.hypot(tx, ty)
    nx, ny = ty / J, -tx / J
    xt, yt = curves.evaluate(curve, t)[:2]
    h = 1e-5
    lp = np.log(np.hypot(xs - (xt + h * nx), ys - (yt + h * ny)))
    lm = np.log(np.hypot(xs - (xt - h * nx), ys - (yt - h * ny)))
    fd = (lp - lm) / (2 * h) * J
    assert np.abs(direct.kbar(curve, s, t) - fd).max() < 1e-6 * max(1.0, np.abs(fd).max())


@pytest.mark.parametrize("curve,p,N", [(synth.star(4), 3, 40), (synth.ellipse_bspline(), 2, 64)], ids=["star", "ellipse"])
def test_constant_datum_gives_zero_direct_rhs(curve, p, N):
    """Gauss's lemma: for x on a smooth closed curve the double layer of the
    constant 1 is 1/2, i.e. (1/2pi) int Kbar(s, t) dt = 1/2, so u_D = 1 (whose
    flux is 0) gives F = b1/2 - b2/(2pi) = 0 node by node and entry by entry."""
    one = lambda x, y: np.ones_like(x)
    v = direct.inner_sums(curve, N, 1, 8, one)
    assert np.abs(v / (2 * math.pi) - 0.5).max() < 1e-11
    F = direct.rhs(curve, p, N, 1, 8, one)
    b1 = wq.rhs(curve, p, N, 1, one)
    assert np.abs(F).max() < 1e-11 * np.abs(b1).max()


def test_direct_solution_converges_to_the_exact_flux():
    """u = exp(x1) cos(x2) is harmonic; the direct Galerkin solution of
    A alpha = F approximates its outward flux q = grad u . n, and the error
    falls at least fourfold per mesh halving for p = 2 (order p + 1 = 3)."""
    curve, p, G = synth.star(6), 2, 8
    g = synth.g_exp_cos
    grad = lambda x, y: (np.exp(x) * np.cos(y), -np.exp(x) * np.sin(y))
    ts = np.linspace(0.0, 1.0, 997, endpoint=False)
    q = direct.outward_flux(curve, ts, grad)
    errs = []
    for N in (16, 32, 64):
        A = wq.matrix(curve, p, N, 1)
        alpha = np.linalg.solve(A, direct.rhs(curve, p, N, 1, G, g))
        qh = sum(alpha[j] * bspline.periodic(p, N, j, ts) for j in range(N))
        errs.append(np.abs(qh - q).max() / np.abs(q).max())
    assert errs[0] / errs[1] > 4 and errs[1] / errs[2] > 4, errs
    assert errs[2] < 1e-3, errs


def test_exact_kbar_is_pi_on_the_circle_at_any_separation():
    """The exact evaluation of the near terms keeps the circle's closed form
    Kbar = pi down to separations where the FP64 formula has lost every digit."""
    from fractions import Fraction
    c = synth.circle(0.5)
    s = Fraction(3, 7)
    for h in (Fraction(1, 10 ** 12), Fraction(1, 3 * 10 ** 7), Fraction(-1, 10 ** 5), Fraction(1, 40)):
        assert abs(direct.kbar_exact(c, s, s + h) - math.pi) < 1e-15
    # across the period
    assert abs(direct.kbar_exact(c, Fraction(0), Fraction(-1, 10 ** 9) + 1) - math.pi) < 1e-15


@pytest.mark.parametrize("curve", [synth.star(3), synth.ellipse_bspline(), synth.ellipse_bspline_nonuniform(2)],
                         ids=["star", "ellipse", "ellipse-nonuniform-knots"])
def test_exact_kbar_limit_is_half_the_curvature_term(curve):
    """As t -> s, f(t) - f(s) = f' h + f'' h^2 / 2 + O(h^3), so Kbar tends to
    (f' x f'') / (2 |f'|^2) (the curvature times J / 2), with an O(h) remainder:
    the exact evaluation at h = 1e-9 against f'' from scipy's B-spline
    derivative or a central difference of the FP64 first derivative."""
    from fractions import Fraction
    rng = np.random.default_rng(11)
    for s in rng.random(6):
        sf = Fraction(float(s))
        d = 1e-5
        x, y, dx, dy, _ = curves.evaluate(curve, np.array([s]))
        ddx = (curves.evaluate(curve, np.array([s + d]))[2] - curves.evaluate(curve, np.array([s - d]))[2]) / (2 * d)
        ddy = (curves.evaluate(curve, np.array([s + d]))[3] - curves.evaluate(curve, np.array([s - d]))[3]) / (2 * d)
        lim = float(((dx * ddy - dy * ddx) / (2 * (dx * dx + dy * dy)))[0])
        ke = direct.kbar_exact(curve, sf, sf + Fraction(1, 10 ** 9))
        assert abs(ke - lim) < 1e-6 * max(1.0, abs(lim)), (s, ke, lim)


def test_exact_kbar_meets_fp64_away_from_the_node():
    """Where FP64 does not cancel (separations of a few hundredths) the exact
    evaluation and the FP64 formula agree to rounding."""
    from fractions import Fraction
    for curve in (synth.star(5), synth.ellipse_bspline()):
        for s, h in ((Fraction(1, 3), Fraction(1, 40)), (Fraction(5, 9), Fraction(-3, 100)), (Fraction(0), Fraction(1, 25))):
            t = s + h
            kd = float(direct.kbar(curve, np.array(float(s)), np.array(float(t % 1))))
            assert abs(direct.kbar_exact(curve, s, t) - kd) < 1e-13 * abs(kd)


def test_near_window_holds_every_term_fp64_cannot_carry():
    """Tiny case, every term exact (brute force): the inner sums with only the
    window exact match it to rounding, i.e. the terms left in FP64 carry no
    visible cancellation error."""
    from fractions import Fraction
    curve, N, R, G = synth.star(7), 12, 1, 4
    g = synth.g_exp_cos
    v = direct.inner_sums(curve, N, R, G, g)
    t2, wt = direct.gauss_points(N, G)
    x2, y2 = curves.evaluate(curve, t2)[:2]
    coef = wt * g(x2, y2)
    u = 0.5 * (np.polynomial.legendre.leggauss(G)[0] + 1.0)
    for n in range(2 * R * N):
        s = Fraction(n, 2 * R * N)
        exact = sum(coef[e * G + q] * direct.kbar_exact(curve, s, (e + Fraction(float(u[q]))) / N)
                    for e in range(N) for q in range(G))
        assert abs(v[n] - exact) < 1e-14 * max(1.0, abs(exact)), (n, v[n], exact)
