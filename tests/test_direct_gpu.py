"""Direct-formulation right-hand side (eq. final_b2 by the rule of Section 5,
F = b1/2 - b2/(2 pi)) through the C ABI, against the CPU oracle O4."""
import math

import numpy as np
import pytest

import synth
from oracle import bspline, direct, wq

pytestmark = pytest.mark.gpu


def tol(N, G):
    """1e-12 in max-norm relative error at every N and G: the Gauss points near a
    node, where Kbar's numerator and denominator cancel in FP64 (relative
    eps / |t - s|, 2e-10 at N = 16384), are evaluated without cancellation on
    the device (second-order differences of the curve) and exactly in the
    oracle."""
    return 1e-12


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1703_10016_amd.runtime import Context
    c = Context(0)
    yield c
    c.close()


CASES = [
    ("circle", synth.circle(0.5), 2, 64, 1, 4),
    ("star_p3_G6", synth.star(21), 3, 100, 1, 6),
    ("ellipse", synth.ellipse_bspline(), 3, 256, 1, 4),
    ("star_p4_R2_G2", synth.star(22), 4, 37, 2, 2),
    ("star_p2_G8_ragged", synth.star(23), 2, 520, 1, 8),
    ("star_minimal", synth.star(24), 1, 4, 1, 4),
    ("ellipse_nonuniform_knots_R2", synth.ellipse_bspline_nonuniform(3), 3, 96, 2, 4),
    ("ellipse_8_ctrl_minimal", synth.ellipse_bspline(n_ctrl=8), 1, 4, 1, 4),
]


@pytest.mark.parametrize("name,curve,p,N,R,G", CASES, ids=[c[0] for c in CASES])
def test_direct_rhs_matches_oracle(ctx, name, curve, p, N, R, G):
    g = synth.g_exp_cos
    F, b2 = ctx.rhs_direct(curve, p, N, g, n_gauss=G, n_ref=R, with_b2=True)
    F, b2 = F.cpu().numpy(), b2.cpu().numpy()
    ref_b2 = direct.b2(curve, p, N, R, G, g)
    ref_F = direct.rhs(curve, p, N, R, G, g)
    scale = np.abs(wq.rhs(curve, p, N, R, g)).max()
    assert np.abs(b2 - ref_b2).max() < tol(N, G) * np.abs(ref_b2).max()
    assert np.abs(F - ref_F).max() < tol(N, G) * scale


def test_direct_rhs_full_size_ellipse(ctx):
    c = synth.config_ellipse()
    F, b2 = ctx.rhs_direct(c.curve, c.p, c.N, c.g, n_gauss=4, with_b2=True)
    ref = direct.b2(c.curve, c.p, c.N, 1, 4, c.g)
    assert np.abs(b2.cpu().numpy() - ref).max() < tol(c.N, 4) * np.abs(ref).max()


@pytest.mark.parametrize("curve", [synth.star(25), synth.ellipse_bspline()], ids=["star", "ellipse"])
def test_direct_rhs_large_sampled_rows(ctx, curve):
    """N = 16384 (the large configuration, a polar and a B-spline curve): b2 rows
    from the oracle's inner sums at their support nodes only, where the
    closest Gauss points lie 3e-6 from the nodes."""
    p, N, G, g = 3, 16384, 4, synth.g_exp_cos
    _, b2 = ctx.rhs_direct(curve, p, N, g, n_gauss=G, with_b2=True)
    b2 = b2.cpu().numpy()
    rows = [0, 1, 8191, N - 1]
    Wd = wq.regular_weights(p, N, 1, rows=rows)
    J = direct.curves.evaluate(curve, wq.nodes(N, 1))[4]
    for i in rows:
        nset, w = Wd[i]
        v = direct.inner_sums(curve, N, 1, G, g, rows=nset)
        ref = np.sum(w * J[nset] * v)
        assert abs(b2[i] - ref) < tol(N, G) * np.abs(b2).max()


def test_constant_datum_gives_zero_at_full_size(ctx):
    """Gauss's lemma (the double layer of 1 is 1/2 on a smooth closed curve):
    u_D = 1 has zero flux, so F = 0 up to the quadrature error."""
    one = lambda x, y: np.ones_like(x)
    curve, p, N = synth.star(26), 3, 16384
    F = ctx.rhs_direct(curve, p, N, one, n_gauss=4).cpu().numpy()
    b1 = ctx.rhs(curve, p, N, one).cpu().numpy()
    assert np.abs(F).max() < 1e-10 * np.abs(b1).max()


def test_direct_solve_converges_to_the_exact_flux(ctx):
    """Assemble + direct right-hand side + mixed-precision solve on the device:
    the solution approximates the outward flux of u = exp(x1) cos(x2) and the
    error falls at least fourfold per mesh halving (p = 3)."""
    curve, p, g = synth.star(27), 3, synth.g_exp_cos
    grad = lambda x, y: (np.exp(x) * np.cos(y), -np.exp(x) * np.sin(y))
    ts = np.linspace(0.0, 1.0, 1999, endpoint=False)
    q = direct.outward_flux(curve, ts, grad)
    errs = []
    for N in (32, 64, 128):
        A = ctx.assemble(curve, p, N, "wq")
        F = ctx.rhs_direct(curve, p, N, g, n_gauss=8)
        x, info = ctx.solve(A, F, tol=1e-13)
        a = x.cpu().numpy()
        qh = sum(a[j] * bspline.periodic(p, N, j, ts) for j in range(N))
        errs.append(np.abs(qh - q).max() / np.abs(q).max())
    assert errs[0] / errs[1] > 4 and errs[1] / errs[2] > 4, errs
    assert errs[2] < 1e-4, errs


def test_direct_rhs_error_paths(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    curve, p, N = synth.star(28), 2, 32
    r = ctx.rules(p, N, 1)
    buf = torch.zeros(4 * N * 8, dtype=torch.float64, device="cuda")
    for G in (0, 3, 10):
        with pytest.raises(S.SgbemError) as e:
            S.sgbem_rhs_direct(ctx.ctx, curve, r, G, buf.data_ptr(), buf.data_ptr(), buf.data_ptr())
        assert e.value.status == S.SGBEM_E_INVAL
    with pytest.raises(S.SgbemError):
        S.sgbem_rhs_direct(ctx.ctx, curve, r, 4, 0, buf.data_ptr(), buf.data_ptr())
