"""Parity of the HIP path (through the C ABI) with the CPU oracle, on an MI355X.

Tolerances: FP64 matrices within 1e-12 of the oracle in max-norm relative
error (the oracle and the library compute the same rule by different
routes); for p >= 5 the bound grows with the conditioning of the paper's
local collocation systems (Alg. 1).  FP32 results are compared with stated
bounds.  Sizes span several 32 x 32 tiles with ragged tails and the minimal
N = 2(p+1)."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import bspline, circle, ebe, wq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1703_10016_amd.runtime import Context
    c = Context(0)
    yield c
    c.close()


def relmax(A, B):
    return float(np.abs(A - B).max() / np.abs(B).max())


def wq_tol(p, N, R):
    if p <= 4:
        return 1e-12
    eta = wq.nodes(N, R)
    nset = wq.support_nodes(p, N, R, 0)
    Bloc = np.stack([bspline.periodic(p, R * N, k, eta[nset]) for k in wq.exactness_set(p, N, R, 0)])
    return 40 * np.finfo(float).eps * np.linalg.cond(Bloc)


WQ_CASES = [
    ("circle", synth.circle(0.5), 2, 64, 1),
    ("star1", synth.star(1), 3, 40, 1),
    ("ellipse", synth.ellipse_bspline(), 3, 64, 2),
    ("star2", synth.star(2), 4, 37, 1),
    ("star3", synth.star(3), 2, 50, 3),
    ("star4", synth.star(4), 3, 33, 4),
    ("star5", synth.star(5), 1, 16, 1),
    ("star6", synth.star(6), 5, 20, 1),
    ("star7", synth.star(7), 6, 28, 2),
    ("star8_minimal", synth.star(8), 3, 8, 1),
    ("star9_p2R4", synth.star(9), 2, 70, 4),
]


@pytest.mark.parametrize("name,curve,p,N,R", WQ_CASES, ids=[c[0] for c in WQ_CASES])
def test_wq_fp64_matches_oracle(ctx, name, curve, p, N, R):
    A = ctx.assemble(curve, p, N, "wq", n_ref=R).cpu().numpy()
    ref = wq.matrix(curve, p, N, R)
    assert np.array_equal(A, A.T)
    assert relmax(A, ref) < wq_tol(p, N, R)


EBE_CASES = [
    ("circle_config", synth.circle(0.5), 2, 64, 6),
    ("star1", synth.star(1), 3, 40, 4),
    ("ellipse", synth.ellipse_bspline(), 3, 48, 3),
    ("star2_G1", synth.star(2), 2, 37, 1),
    ("star3_G8", synth.star(3), 4, 20, 8),
    ("star5_p6", synth.star(5), 6, 14, 2),
    ("star6_minimal", synth.star(6), 1, 4, 5),
    ("star7_G7", synth.star(7), 5, 66, 7),
]


@pytest.mark.parametrize("name,curve,p,N,G", EBE_CASES, ids=[c[0] for c in EBE_CASES])
def test_ebe_fp64_matches_oracle(ctx, name, curve, p, N, G):
    A = ctx.assemble(curve, p, N, "ebe", n_gauss=G).cpu().numpy()
    ref = ebe.matrix(curve, p, N, G)
    assert np.array_equal(A, A.T)
    assert relmax(A, ref) < 1e-12


def test_ebe_converged_equals_circle_closed_form(ctx):
    A = ctx.assemble(synth.circle(0.5), 3, 48, "ebe", n_gauss=8).cpu().numpy()
    assert relmax(A, circle.matrix(0.5, 48, 3)) < 1e-12


# ------------------------------------------------------------------ full size: ellipse, p = 3, N = 1024
@pytest.fixture(scope="module")
def ellipse_full(ctx):
    c = synth.config_ellipse()
    return c, ctx.assemble(c.curve, c.p, c.N, "wq").cpu().numpy(), ctx.assemble(c.curve, c.p, c.N, "ebe", n_gauss=6).cpu().numpy()


def test_full_size_wq_sampled_rows(ellipse_full):
    c, A, _ = ellipse_full
    rows = [0, 1, 517, 1023]
    ref = wq.full_rows(c.curve, c.p, c.N, 1, rows)
    assert np.array_equal(A, A.T)
    for r, i in enumerate(rows):
        assert np.abs(A[i, i:] - ref[r, i:]).max() < 1e-12 * np.abs(ref[r]).max()


def test_full_size_ebe_sampled_entries(ellipse_full):
    c, _, A = ellipse_full
    P = ebe.EBEProblem(c.curve, c.p, c.N, 6)
    rng = np.random.default_rng(0)
    ii = rng.integers(0, c.N, 1500)
    jj = rng.integers(0, c.N, 1500)
    band_i = np.repeat(np.arange(0, c.N, 97), 11)
    band_j = (band_i + np.tile(np.arange(-5, 6), band_i.size // 11)) % c.N
    ii = np.concatenate([ii, band_i])
    jj = np.concatenate([jj, band_j])
    ref = P.entries(ii, jj)
    assert np.abs(A[ii, jj] - ref).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("p,N,prec", [(2, 4096, "fp64"), (4, 4096, "fp64"), (3, 16384, "fp64"), (3, 16384, "fp32"),
                                      (2, 16384, "fp32"), (4, 16384, "fp32"), (3, 4096, "fp32")])
def test_large_wq_sampled_rows(ctx, p, N, prec):
    """Star curves at the sizes of the large configurations (the launch that
    switches to the large-matrix tile instance from N = 4096): sampled rows
    against the oracle's sparse row route, upper triangle and its mirror."""
    import torch
    curve = synth.star(11)
    rows = [0, 1, N // 2 + 1, N - 1]
    A = ctx.assemble(curve, p, N, "wq", precision=prec)
    got = A[rows].double().cpu().numpy()
    col = A[:, rows].double().cpu().numpy().T
    del A
    torch.cuda.empty_cache()
    ref = wq.full_rows(curve, p, N, 1, rows)
    tol = 1e-12 if prec == "fp64" else 2e-5
    # the row formula (eq. IK1e2_bis) is not symmetric: entries j >= i come from
    # row i, the others are mirrored from row j
    for r, i in enumerate(rows):
        assert np.abs(got[r, i:] - ref[r, i:]).max() < tol * np.abs(ref[r]).max()
    assert got[1, 0] == got[0, 1] and np.array_equal(got, col)


def test_full_size_wq_vs_ebe_quadrature_gap(ellipse_full):
    """Both forms approximate the same Galerkin matrix; their difference is the
    quadrature error of the weighted rules (near-diagonal, ~1e-4 relative)."""
    _, A, E = ellipse_full
    d = relmax(A, E)
    assert 1e-6 < d < 1e-3


# ------------------------------------------------------------------ FP32
@pytest.mark.parametrize("method", ["wq", "ebe"])
def test_fp32_error_bound(ctx, method):
    curve, p, N = synth.star(11), 3, 300
    A64 = ctx.assemble(curve, p, N, method, n_gauss=4).cpu().numpy()
    A32 = ctx.assemble(curve, p, N, method, n_gauss=4, precision="fp32").cpu().numpy().astype(np.float64)
    assert np.array_equal(A32, A32.T)
    err = relmax(A32, A64)
    assert err < 2e-6, err


def test_fp32_ebe_matches_oracle(ctx):
    """The FP32 plain form against the FP64 oracle of the same rule (not the
    GPU's own FP64 matrix): FP32 kernel values and sums, FP64 node differences."""
    curve, p, N, G = synth.star(11), 3, 300, 4
    A32 = ctx.assemble(curve, p, N, "ebe", n_gauss=G, precision="fp32").cpu().numpy().astype(np.float64)
    ref = ebe.matrix(curve, p, N, G)
    assert np.array_equal(A32, A32.T)
    assert relmax(A32, ref) < 2e-6


# ------------------------------------------------------------------ right-hand side
@pytest.mark.parametrize("method,R,G", [("wq", 1, 0), ("wq", 2, 0), ("ebe", 1, 5)])
def test_rhs_matches_oracle(ctx, method, R, G):
    curve, p, N, g = synth.star(12), 3, 45, synth.g_exp_cos
    beta = ctx.rhs(curve, p, N, g, method=method, n_ref=R, n_gauss=max(G, 1)).cpu().numpy()
    ref = wq.rhs(curve, p, N, R, g) if method == "wq" else ebe.EBEProblem(curve, p, N, G).rhs(g)
    assert np.abs(beta - ref).max() < 1e-13 * np.abs(ref).max()
    xy = ctx.rhs_points(curve, p, N, method=method, n_ref=R, n_gauss=max(G, 1)).cpu().numpy()
    from oracle import curves
    t = wq.nodes(N, R) if method == "wq" else ((np.arange(N)[:, None] + ebe.gauss01(G)[0][None, :]) / N).ravel()
    x, y, *_ = curves.evaluate(curve, t)
    assert np.abs(xy[:, 0] - x).max() < 1e-14 and np.abs(xy[:, 1] - y).max() < 1e-14


# ------------------------------------------------------------------ solve
SOLVE_SIZES = [(20, "fp64"), (65, "fp32"), (100, "fp64"), (256, "fp64"), (200, "fp32"), (1000, "fp64"),
               (2500, "fp64"), (4096, "fp64"), (4500, "fp32"), (9000, "fp64")]


def skew_perturbed(A, seed):
    """A + 1e-3 (A o S), S antisymmetric with entries in [-1, 1]: no longer
    symmetric (so the solve pivots), conditioned like A."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    R = torch.rand(A.shape, generator=g, dtype=torch.float64) * 2 - 1
    S = (torch.triu(R, 1) - torch.triu(R, 1).T).to(A.device, A.dtype)
    return A + 1e-3 * A * S


@pytest.mark.parametrize("sym", [True, False], ids=["symmetric", "nonsymmetric"])
@pytest.mark.parametrize("N,prec", SOLVE_SIZES)
def test_mixed_solve_matches_fp64_solve(ctx, N, prec, sym):
    """Symmetric Galerkin matrices take the factorisation without interchanges
    (star curves: indefinite, capacity > 1) unless it fails; a non-symmetric
    matrix is factored with partial pivoting (every panel shape of either kind
    runs across these sizes)."""
    curve, p = synth.star(13), 3
    A = ctx.assemble(curve, p, N, "wq", precision=prec)
    if not sym:
        A = skew_perturbed(A, N)
    beta = ctx.rhs(curve, p, N, synth.g_exp_cos)
    x, info = ctx.solve(A, beta, tol=1e-12, max_iter=30)
    Ah = A.cpu().numpy().astype(np.float64)
    ref = np.linalg.solve(Ah, beta.cpu().numpy())
    xh = x.cpu().numpy()
    err = np.linalg.norm(xh - ref) / np.linalg.norm(ref)
    assert err < 1e-10, (err, info.iters, info.rel_update, info.backward_err, info.pivoted)
    assert info.backward_err < 1e-14 and info.iters >= 1
    if not sym:
        assert info.pivoted == 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_positive_definite_solve_without_interchanges(ctx, prec):
    """The ellipse (capacity 0.75 < 1: positive definite Galerkin matrix, the
    paper's setting), assembled in either precision (exactly symmetric: the
    lower triangle mirrors the upper): factored without interchanges, same
    solution."""
    c = synth.config_ellipse()
    A = ctx.assemble(c.curve, c.p, c.N, "wq", precision=prec)
    beta = ctx.rhs(c.curve, c.p, c.N, c.g)
    x, info = ctx.solve(A, beta, tol=1e-12)
    assert info.pivoted == 0
    ref = np.linalg.solve(A.cpu().numpy().astype(np.float64), beta.cpu().numpy())
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [4200, 4301, 8200])
def test_positive_definite_large_keeps_factor_without_interchanges(ctx, N, prec):
    """Beyond N = 4096 the factorisation without interchanges runs in 256-column
    blocks of four 64-column quarters; N = 4200 and 8200 leave ragged last
    blocks (104 and 8 columns) and take the symmetric form (U = D L^T, updates
    of the lower blocks only, U filled in at the end), N = 4301 (not a multiple
    of 4) the general form.  On the ellipse (positive definite) that factor must
    be kept (no silent fallback to partial pivoting) and the refined solution
    must equal LAPACK's FP64 solve of the same stored matrix."""
    c = synth.config_ellipse()
    A = ctx.assemble(c.curve, c.p, N, "wq", precision=prec)
    beta = ctx.rhs(c.curve, c.p, N, c.g)
    x, info = ctx.solve(A, beta, tol=1e-12)
    assert info.pivoted == 0, (info.iters, info.rel_update, info.backward_err)
    ref = np.linalg.solve(A.cpu().numpy().astype(np.float64), beta.cpu().numpy())
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-10


@pytest.mark.parametrize("bad", [float("nan"), float("inf")], ids=["nan", "inf"])
def test_non_finite_matrix_is_never_reported_converged(ctx, bad):
    """A symmetric matrix with one non-finite pair of entries: the refinement's
    norms propagate NaN, so the solve ends with an error status (no convergence
    or a zero pivot), never with SGBEM_OK."""
    import torch
    from paper_1703_10016_amd import sgbem as S
    N = 96
    A = circle.matrix(0.5, N, 2)
    A[5, 7] = A[7, 5] = bad
    b = torch.from_numpy(circle.rhs_x2_minus_y2(0.5, N, 2)).cuda()
    x, info = ctx.solve(torch.from_numpy(A).cuda(), b, check=False)
    assert info.status in (S.SGBEM_E_NOCONV, S.SGBEM_E_SINGULAR), info.status


@pytest.mark.parametrize("N", [300, 4200], ids=["64-column blocks", "128-column blocks"])
def test_symmetric_zero_pivot_falls_back_to_pivoting(ctx, N):
    """A symmetric matrix with a zero diagonal (every first pivot is zero):
    the attempt without interchanges fails and partial pivoting solves it."""
    import torch
    rng = np.random.default_rng(5)
    B = rng.standard_normal((N // 2, N // 2)) + 4 * np.eye(N // 2)
    A = np.zeros((N, N))
    A[:N // 2, N // 2:] = B
    A[N // 2:, :N // 2] = B.T
    beta = rng.standard_normal(N)
    x, info = ctx.solve(torch.from_numpy(A).cuda(), torch.from_numpy(beta).cuda(), tol=1e-12)
    assert info.pivoted == 1
    ref = np.linalg.solve(A, beta)
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-10


def test_symmetric_tiny_pivot_stalls_and_falls_back(ctx):
    """A well-conditioned symmetric matrix whose first diagonal entry is tiny
    but not zero: without interchanges the FP32 factors carry a growth of
    ~1e12, the refinement stalls, and partial pivoting takes over."""
    import torch
    N = 200
    rng = np.random.default_rng(6)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    A = Q @ np.diag(np.linspace(1.0, 4.0, N)) @ Q.T
    A = 0.5 * (A + A.T)
    A[0, 0] = 1e-12
    beta = rng.standard_normal(N)
    x, info = ctx.solve(torch.from_numpy(A).cuda(), torch.from_numpy(beta).cuda(), tol=1e-12)
    assert info.pivoted == 1
    ref = np.linalg.solve(A, beta)
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-10


@pytest.mark.parametrize("N,sym", [(16384, True), (16500, True), (16500, False)])
def test_large_solve_backward_error(ctx, N, sym):
    """N = 16384 (the tallest panels without interchanges), N = 16500 (partial
    pivoting: panels taller than 16384 rows at the start, every register panel
    shape after): the FP64 residual of the refined solution, formed
    independently by a library matrix-vector product, is at rounding level."""
    import torch
    curve, p = synth.star(14), 3
    A = ctx.assemble(curve, p, N, "wq", precision="fp32")
    if not sym:
        A = skew_perturbed(A, N)
    beta = ctx.rhs(curve, p, N, synth.g_exp_cos)
    x, info = ctx.solve(A, beta, tol=1e-10, max_iter=30)
    if N > 16384:
        assert info.pivoted == 1
    A64 = A.double()
    r = beta - A64 @ x
    bwd = (r.abs().max() / (A64.abs().sum(dim=1).max() * x.abs().max() + beta.abs().max())).item()
    del A64
    assert bwd < 1e-14, (bwd, info.iters, info.backward_err)
    assert abs(bwd - info.backward_err) < 1e-15 + 0.1 * bwd


def test_solve_circle_exact_discrete_solution(ctx):
    r, p, N = 0.5, 2, 64
    import torch
    A = torch.from_numpy(circle.matrix(r, N, p)).cuda()
    beta = torch.from_numpy(circle.rhs_x2_minus_y2(r, N, p)).cuda()
    x, info = ctx.solve(A, beta)
    lam = np.fft.fft(circle.matrix(r, N, p)[0]).real[2]   # eigenvalue of the k = 2 mode
    assert np.abs(x.cpu().numpy() - circle.rhs_x2_minus_y2(r, N, p) / lam).max() < 1e-12 * np.abs(x.cpu().numpy()).max()


def test_solve_error_paths(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    N = 64
    Z = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    b = torch.ones(N, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SgbemError) as e:
        ctx.solve(Z, b)
    assert e.value.status == S.SGBEM_E_SINGULAR
    A = torch.from_numpy(circle.matrix(0.5, N, 2)).cuda()
    x, info = ctx.solve(A, b, max_iter=0, check=False)
    assert info.status == S.SGBEM_E_NOCONV


def test_assemble_error_paths(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    out = torch.empty((16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_assemble(ctx.ctx, synth.star(1), ctx.rules(2, 16, 1), S.SGBEM_EBE, 9, S.SGBEM_FP64, out.data_ptr(), 16)
    assert e.value.status == S.SGBEM_E_INVAL
    with pytest.raises(S.SgbemError):
        S.sgbem_assemble(ctx.ctx, synth.star(1), ctx.rules(2, 16, 1), S.SGBEM_WQ, 0, S.SGBEM_FP64, out.data_ptr(), 8)
    bad = synth.PolarCurve(r0=1.0, a=np.array([0.7, 0.6]), phi=np.zeros(2))
    with pytest.raises(S.SgbemError):
        S.sgbem_assemble(ctx.ctx, bad, ctx.rules(2, 16, 1), S.SGBEM_WQ, 0, S.SGBEM_FP64, out.data_ptr(), 16)
