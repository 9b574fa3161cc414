"""Pins of the collocation oracle (O5) against facts independent of its formula."""
import math

import numpy as np
import pytest

import synth
from oracle import bspline, circle, collocation


@pytest.mark.parametrize("p,N,R", [(2, 24, 1), (3, 17, 1), (4, 20, 2)])
def test_circle_rows_sum_to_the_single_layer_of_one(p, N, R):
    """On a circle of radius r: K1 = ln(2 pi r) is constant and the exactness of
    both rules covers constants, sum_j B_j = 1, and int ln|sin(pi t)/pi| dt =
    -ln(2 pi); so every row sums to V[1](x) = -r ln r exactly."""
    for r in (0.5, 1.3):
        A = collocation.matrix(synth.circle(r), p, N, R)
        assert np.abs(A.sum(axis=1) + r * math.log(r)).max() < 1e-12


def test_collocation_points_are_the_greville_abscissae():
    """x_i = (i + (p+1)/2)/N is where the cyclic B_i peaks (symmetric support)."""
    for p, N in [(2, 10), (3, 12)]:
        t = collocation.points(p, N, 1) / (2.0 * N)
        for i in range(N):
            s = np.linspace(i / N, (i + p + 1) / N, 2001) % 1.0
            v = bspline.periodic(p, N, i, s)
            assert abs(s[np.argmax(v)] - t[i]) < 1e-3


def test_collocation_solution_converges_to_the_exact_circle_density():
    """V phi = x1^2 - x2^2 on the circle r = 0.5 has phi = 4 r cos(2 theta);
    the collocation solution converges at order >= p (here p = 2: >= 4x per halving)."""
    r, p = 0.5, 2
    g = synth.g_x2_minus_y2
    ts = np.linspace(0.0, 1.0, 991, endpoint=False)
    exact = circle.density_x2_minus_y2(r, ts)
    errs = []
    for N in (16, 32, 64):
        A = collocation.matrix(synth.circle(r), p, N, 1)
        a = np.linalg.solve(A, collocation.rhs(synth.circle(r), p, N, 1, g))
        ph = sum(a[j] * bspline.periodic(p, N, j, ts) for j in range(N))
        errs.append(np.abs(ph - exact).max() / np.abs(exact).max())
    assert errs[0] / errs[1] > 4 and errs[1] / errs[2] > 4, errs


def test_star_rows_sum_to_the_single_layer_of_one_by_adaptive_quadrature():
    """Off the circle the matrix is not circulant: row sums must equal
    V[1](x_i) = -(1/2pi) int ln|f(x_i) - f(t)| J(t) dt, computed by adaptive
    quadrature split at the singular point, to the rules' quadrature error
    (order ~p+1: 4e-3, 1e-5, 4e-7 relative at N = 24, 48, 96); column sums differ
    by O(1e-3), so a transposed operand fails."""
    from scipy.integrate import quad
    from oracle import curves, wq
    curve, p, N = synth.star(8), 3, 96
    A = collocation.matrix(curve, p, N, 1)
    ts = wq.nodes(N, 1)[collocation.points(p, N, 1)]
    for i in (0, 7, 30):
        s = ts[i]
        xs, ys = curves.evaluate(curve, s)[:2]

        def f(t):
            x, y, _, _, J = curves.evaluate(curve, t)
            return -math.log(math.hypot(x - xs, y - ys)) * J / (2 * math.pi)
        v = quad(f, s, s + 1.0, limit=400, epsabs=1e-13)[0]   # periodic: one period starting at the singularity
        assert abs(A[i].sum() - v) < 1e-8
    assert np.abs(A.sum(axis=0) - A.sum(axis=1)).max() > 1e-3
