"""Collocation BEM with the weighted rules (O5) through the C ABI."""
import math

import numpy as np
import pytest

import synth
from oracle import bspline, circle, collocation, wq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1703_10016_amd.runtime import Context
    c = Context(0)
    yield c
    c.close()


def tol(p, N, R):
    """1e-12, or for p >= 5 the conditioning of the local Alg. 1 systems (as for
    the Galerkin matrix: both routes solve them, by different algorithms)."""
    if p <= 4:
        return 1e-12
    eta = wq.nodes(N, R)
    nset = wq.support_nodes(p, N, R, 0)
    Bloc = np.stack([bspline.periodic(p, R * N, k, eta[nset]) for k in wq.exactness_set(p, N, R, 0)])
    return 40 * np.finfo(float).eps * np.linalg.cond(Bloc)


CASES = [
    ("circle", synth.circle(0.5), 2, 64, 1),
    ("star_ragged", synth.star(31), 3, 100, 1),
    ("ellipse_R2", synth.ellipse_bspline(), 3, 70, 2),
    ("star_p5", synth.star(32), 5, 40, 1),
    ("star_p6_R2", synth.star(33), 6, 36, 2),
    ("star_minimal", synth.star(34), 1, 4, 1),
    ("star_p4_tiles", synth.star(35), 4, 200, 1),
]


@pytest.mark.parametrize("name,curve,p,N,R", CASES, ids=[c[0] for c in CASES])
def test_collocation_matrix_matches_oracle(ctx, name, curve, p, N, R):
    A = ctx.assemble_collocation(curve, p, N, n_ref=R).cpu().numpy()
    ref = collocation.matrix(curve, p, N, R)
    assert np.abs(A - ref).max() < tol(p, N, R) * np.abs(ref).max()


def test_collocation_full_size_ellipse(ctx):
    c = synth.config_ellipse()
    A = ctx.assemble_collocation(c.curve, c.p, c.N).cpu().numpy()
    ref = collocation.matrix(c.curve, c.p, c.N, 1)
    assert np.abs(A - ref).max() < 1e-12 * np.abs(ref).max()


def test_circle_row_sums_at_large_size(ctx):
    """Every row of the circle's collocation matrix sums to -r ln r (rule
    exactness), at N = 16384."""
    r, p, N = 0.7, 3, 16384
    A = ctx.assemble_collocation(synth.circle(r), p, N)
    s = A.sum(dim=1).cpu().numpy()
    assert np.abs(s + r * math.log(r)).max() < 1e-11


def test_collocation_rhs_and_solve_converge_to_the_exact_density(ctx):
    r, p = 0.5, 3
    g = synth.g_x2_minus_y2
    ts = np.linspace(0.0, 1.0, 991, endpoint=False)
    exact = circle.density_x2_minus_y2(r, ts)
    errs = []
    for N in (16, 32, 64):
        b = ctx.collocation_rhs(synth.circle(r), p, N, g)
        assert np.abs(b.cpu().numpy() - collocation.rhs(synth.circle(r), p, N, 1, g)).max() < 1e-14
        A = ctx.assemble_collocation(synth.circle(r), p, N)
        x, info = ctx.solve(A, b, tol=1e-13)
        assert info.pivoted == 1          # not symmetric: partial pivoting from the start
        a = x.cpu().numpy()
        ph = sum(a[j] * bspline.periodic(p, N, j, ts) for j in range(N))
        errs.append(np.abs(ph - exact).max() / np.abs(exact).max())
    assert errs[0] / errs[1] > 4 and errs[1] / errs[2] > 4, errs


def test_collocation_error_paths(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    curve = synth.star(36)
    r3 = ctx.rules(2, 24, 3)
    A = torch.empty((24, 24), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_assemble_collocation(ctx.ctx, curve, r3, A.data_ptr(), 24)
    assert e.value.status == S.SGBEM_E_UNSUPPORTED
    r1 = ctx.rules(2, 24, 1)
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_assemble_collocation(ctx.ctx, curve, r1, A.data_ptr(), 10)
    assert e.value.status == S.SGBEM_E_INVAL
