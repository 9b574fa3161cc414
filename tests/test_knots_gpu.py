"""Fast-form assembly on non-uniform periodic knots (Section 3; Algorithms 1
and 2 in their general form, eqs. IK1e2 / IK1e2_bis) on an MI355X, through the
C ABI, against the oracle's dense route (oracle/wq_knots.py).

Tolerance: 1e-12 in max-norm relative error for p <= 4; for p >= 5 the bound
grows with the conditioning of the local collocation systems of Alg. 1, as in
the uniform parity tests."""
import math

import numpy as np
import pytest

import synth
from oracle import circle
from oracle import wq_knots as K

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


def knots(N, seed, spread=0.6):
    rng = np.random.default_rng([1703, 40000 + seed])
    u = (np.arange(N + 1) + spread * (rng.uniform(0, 1, N + 1) - 0.5)) / N
    u[0], u[-1] = 0.0, 1.0
    return u


def graded(N, amp=0.3):
    u = np.arange(N + 1) / N
    t = u + amp * np.sin(2 * math.pi * u) / (2 * math.pi)
    t[0], t[-1] = 0.0, 1.0
    return t


def tol(p, N, R, tau):
    if p <= 4:
        return 1e-12
    tb = K.refine(tau, R)
    eta = K.nodes(tau, R)
    worst = 1.0
    for i in range(N):
        nset = K.support_nodes(p, N, R, i)
        B = np.stack([K.basis(tb, p, int(k), eta[nset]) for k in K.exactness_set(p, N, R, i)])
        worst = max(worst, np.linalg.cond(B))
    return 40 * np.finfo(float).eps * worst


CASES = [
    ("star-p3", synth.star(21), 3, 96, 1, 0),
    ("ellipse-p2-R2", synth.ellipse_bspline(), 2, 50, 2, 1),
    ("knotted-curve-p4", synth.ellipse_bspline_nonuniform(2), 4, 40, 1, 2),
    ("star-p1", synth.star(22), 1, 24, 1, 3),
    ("star-p6", synth.star(23), 6, 30, 1, 4),
    ("star-p5-R2", synth.star(24), 5, 20, 2, 5),
    ("circle-minimal", synth.circle(0.5), 3, 8, 1, 6),
]


@pytest.mark.parametrize("name,curve,p,N,R,seed", CASES, ids=[c[0] for c in CASES])
def test_knots_fast_form_matches_oracle(ctx, name, curve, p, N, R, seed):
    tau = knots(N, seed)
    print(f"case {name}: p={p} N={N} n_ref={R}", flush=True)
    A = ctx.assemble(curve, p, N, "wq", n_ref=R, knots=tau).cpu().numpy()
    ref = K.matrix(curve, tau, p, R)
    assert np.array_equal(A, A.T)
    assert relmax(A, ref) < tol(p, N, R, tau)


def test_knots_points_and_rhs_match_oracle(ctx):
    from oracle import curves
    curve, p, N, R = synth.star(25), 3, 64, 2
    tau = knots(N, 7)
    xy = ctx.rhs_points(curve, p, N, "wq", n_ref=R, knots=tau).cpu().numpy()
    x, y = curves.evaluate(curve, K.nodes(tau, R))[:2]
    assert np.abs(xy[:, 0] - x).max() < 1e-14 and np.abs(xy[:, 1] - y).max() < 1e-14
    beta = ctx.rhs(curve, p, N, synth.g_exp_cos, "wq", n_ref=R, knots=tau).cpu().numpy()
    assert relmax(beta, K.rhs(curve, tau, p, R, synth.g_exp_cos)) < 1e-13


def test_knots_larger_matrix_matches_oracle(ctx):
    """Several tiles in both directions, ragged last tile (N = 300, 24-entry tiles)."""
    curve, p, N, R = synth.ellipse_bspline_nonuniform(3), 3, 300, 1
    tau = graded(N, 0.4)
    A = ctx.assemble(curve, p, N, "wq", n_ref=R, knots=tau).cpu().numpy()
    assert relmax(A, K.matrix(curve, tau, p, R)) < 1e-12


def test_uniform_knot_vector_matches_the_uniform_path(ctx):
    """The general kernel (per-row rules, full singular table, K2 from the node
    parameters) on an explicitly uniform knot vector reproduces the
    translation-invariant path to rounding."""
    curve, p, N, R = synth.star(26), 3, 128, 1
    A_u = ctx.assemble(curve, p, N, "wq", n_ref=R).cpu().numpy()
    A_k = ctx.assemble(curve, p, N, "wq", n_ref=R, knots=np.arange(N + 1) / N).cpu().numpy()
    assert relmax(A_k, A_u) < 1e-13


def test_knots_solution_converges_on_graded_mesh(ctx):
    """Galerkin solution on the circle with graded knots, assembled, right-hand
    side and solved on the device: order p + 1 towards the exact density."""
    r, p = 0.5, 2
    t = (np.arange(4000) + 0.5) / 4000
    ex = circle.density_x2_minus_y2(r, t)
    errs = []
    for N in (16, 32, 64):
        tau = graded(N)
        A = ctx.assemble(synth.circle(r), p, N, "wq", knots=tau)
        beta = ctx.rhs(synth.circle(r), p, N, synth.g_x2_minus_y2, "wq", knots=tau)
        x, info = ctx.solve(A, beta)
        al = x.cpu().numpy()
        phi = sum(al[j] * K.basis(tau, p, j, t) for j in range(N))
        errs.append(np.sqrt(np.mean((phi - ex) ** 2) / np.mean(ex ** 2)))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(2.6 < q < 4.0 for q in rates), (errs, rates)


def test_knots_unsupported_paths(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    curve, p, N = synth.star(27), 3, 40
    tau = knots(N, 9)
    rules = ctx.rules(p, N, 1, tau)
    A = torch.zeros((N, N), dtype=torch.float64, device="cuda")
    A32 = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    for args in [(S.SGBEM_EBE, 4, S.SGBEM_FP64, A), (S.SGBEM_WQ, 0, S.SGBEM_FP32, A32)]:
        with pytest.raises(S.SgbemError) as e:
            S.sgbem_assemble(ctx.ctx, curve, rules, args[0], args[1], args[2], args[3].data_ptr(), N)
        assert e.value.status == S.SGBEM_E_UNSUPPORTED
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_assemble_noalloc(ctx.ctx, curve, rules, S.SGBEM_FP64, A.data_ptr(), N)
    assert e.value.status == S.SGBEM_E_UNSUPPORTED
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_batch_create(ctx.ctx, [curve], [rules], S.SGBEM_FP64, [A.data_ptr()], [N])
    assert e.value.status == S.SGBEM_E_UNSUPPORTED
    with pytest.raises(S.SgbemError) as e:       # n_ref = 3: no kernel compiled
        r3 = S.sgbem_weights(ctx.ctx, 2, 12, 3, knots(12, 10))
        S.sgbem_assemble(ctx.ctx, curve, r3, S.SGBEM_WQ, 0, S.SGBEM_FP64, A.data_ptr(), N)
    assert e.value.status == S.SGBEM_E_UNSUPPORTED
    with pytest.raises(S.SgbemError) as e:       # beyond the full singular table's limit
        S.sgbem_weights(ctx.ctx, 2, 4097, 1, np.linspace(0, 1, 4098))
    assert e.value.status == S.SGBEM_E_UNSUPPORTED
