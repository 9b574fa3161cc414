"""The boundary's geometry and memory contract on an MI355X, through the C ABI:

* closed B-spline curves on non-uniform periodic knots (Section 3: control
  points plus the knot vector of one period): the fast and the plain form, the
  right-hand side and the library's points against the oracle, inline and
  device-resident control nets, the batched and the allocation-free launches;
* the context's HBM budget: a call whose allocation would exceed it fails with
  E_NOMEM before allocating anything, and sgbem_memory_need states exactly
  what each call takes.

Tolerances as in the parity tests: FP64 within 1e-12 of the oracle
(max-norm relative), FP32 within 2e-5."""
import numpy as np
import pytest

import synth
from oracle import curves, ebe, wq

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


NONUNIFORM = [
    ("ellipse-knots", synth.ellipse_bspline_nonuniform(0), 3, 96, 1),
    ("ellipse-knots-R2", synth.ellipse_bspline_nonuniform(1), 2, 50, 2),
    ("net80-knots", synth.ellipse_bspline_nonuniform(3, n_ctrl=80, jitter=0.6), 4, 64, 1),
]


@pytest.mark.parametrize("name,curve,p,N,R", NONUNIFORM, ids=[c[0] for c in NONUNIFORM])
def test_nonuniform_knot_curve_fast_form_matches_oracle(ctx, name, curve, p, N, R):
    print(f"case {name}: p={p} N={N} n_ref={R}", flush=True)
    ref = wq.matrix(curve, p, N, R)
    A = ctx.assemble(curve, p, N, "wq", n_ref=R).cpu().numpy()
    assert relmax(A, ref) < 1e-12
    A32 = ctx.assemble(curve, p, N, "wq", n_ref=R, precision="fp32").cpu().numpy()
    assert relmax(A32.astype(np.float64), ref) < 2e-5


def test_nonuniform_knot_curve_plain_form_matches_oracle(ctx):
    curve, p, N, G = synth.ellipse_bspline_nonuniform(2), 2, 60, 4
    ref = ebe.matrix(curve, p, N, G)
    A = ctx.assemble(curve, p, N, "ebe", n_gauss=G).cpu().numpy()
    assert relmax(A, ref) < 1e-12


def test_nonuniform_knot_points_and_rhs_match_oracle(ctx):
    curve, p, N, R = synth.ellipse_bspline_nonuniform(0), 3, 96, 1
    xy = ctx.rhs_points(curve, p, N, "wq", n_ref=R).cpu().numpy()
    x, y = curves.evaluate(curve, np.arange(2 * R * N) / (2 * R * N))[:2]
    assert np.abs(xy[:, 0] - x).max() < 1e-14 and np.abs(xy[:, 1] - y).max() < 1e-14
    beta = ctx.rhs(curve, p, N, synth.g_exp_cos, "wq", n_ref=R).cpu().numpy()
    ref = wq.rhs(curve, p, N, R, synth.g_exp_cos)
    assert relmax(beta, ref) < 1e-13


def test_nonuniform_knot_curve_in_batch_and_noalloc(ctx):
    """A non-uniform-knot curve travels inline in the batched and the
    allocation-free launches: both equal the single-curve assembly."""
    import torch
    from paper_1703_10016_amd import sgbem as S
    cases = [(synth.ellipse_bspline_nonuniform(4), 3, 130), (synth.star(2), 2, 70),
             (synth.ellipse_bspline_nonuniform(5), 2, 64)]
    outs = [torch.full((N, N), float("nan"), dtype=torch.float64, device="cuda") for (_, _, N) in cases]
    rules = [ctx.rules(p, N, 1) for (_, p, N) in cases]
    b = S.sgbem_batch_create(ctx.ctx, [c for (c, _, _) in cases], rules, S.SGBEM_FP64,
                             [o.data_ptr() for o in outs], [o.stride(0) for o in outs])
    S.sgbem_batch_assemble(ctx.ctx, b)
    torch.cuda.synchronize()
    for (curve, p, N), o, r in zip(cases, outs, rules):
        ref = ctx.assemble(curve, p, N, "wq").cpu().numpy()
        assert np.array_equal(o.cpu().numpy(), ref)
        o.fill_(float("nan"))
        S.sgbem_assemble_noalloc(ctx.ctx, curve, r, S.SGBEM_FP64, o.data_ptr(), o.stride(0))
        assert np.array_equal(o.cpu().numpy(), ref)
    S.sgbem_batch_free(ctx.ctx, b)


def test_budget_rejects_before_allocating():
    import torch
    from paper_1703_10016_amd import sgbem as S
    from paper_1703_10016_amd.runtime import Context
    curve, p, N = synth.ellipse_bspline_nonuniform(0), 3, 256
    need_r = S.sgbem_memory_need(S.SGBEM_MEM_RULES, p, N, 1)
    need_a = S.sgbem_memory_need(S.SGBEM_MEM_ASSEMBLE_WQ, p, N, 1)
    need_s = S.sgbem_memory_need(S.SGBEM_MEM_SOLVE, p, N)
    # one byte short of the rule block: nothing allocated
    with Context(0, hbm_budget_bytes=need_r - 1) as c:
        with pytest.raises(S.SgbemError) as e:
            c.rules(p, N, 1)
        assert e.value.status == S.SGBEM_E_NOMEM
        assert S.sgbem_ctx_memory(c.ctx) == (0, need_r - 1)
    # rules + assembly fit exactly; the solve does not, and leaves the context as it was
    with Context(0, hbm_budget_bytes=need_r + need_a) as c:
        A = c.assemble(curve, p, N, "wq")
        assert S.sgbem_ctx_memory(c.ctx)[0] == need_r + need_a
        beta = c.rhs(curve, p, N, synth.g_exp_cos, "wq")
        with pytest.raises(S.SgbemError) as e:
            c.solve(A, beta)
        assert e.value.status == S.SGBEM_E_NOMEM
        assert S.sgbem_ctx_memory(c.ctx)[0] == need_r + need_a
        # the matrix is still right after the rejected call
        assert relmax(A.cpu().numpy(), wq.matrix(curve, p, N, 1)) < 1e-12
    # the solve's stated need is exactly enough
    with Context(0, hbm_budget_bytes=need_r + need_a + need_s) as c:
        A = c.assemble(curve, p, N, "wq")
        beta = c.rhs(curve, p, N, synth.g_exp_cos, "wq")
        x, info = c.solve(A, beta)
        held, budget = S.sgbem_ctx_memory(c.ctx)
        assert held == budget == need_r + need_a + need_s
        xr = np.linalg.solve(A.cpu().numpy(), beta.cpu().numpy())
        assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
        # freeing the rules gives their bytes back
        S.sgbem_rules_free(c.ctx, c._rules.pop((p, N, 1)))
        assert S.sgbem_ctx_memory(c.ctx)[0] == need_a + need_s
    torch.cuda.synchronize()


def test_budget_counts_plain_form_and_batches():
    from paper_1703_10016_amd import sgbem as S
    from paper_1703_10016_amd.runtime import Context
    curve, p, N, G = synth.star(3), 2, 120, 5
    need_r = S.sgbem_memory_need(S.SGBEM_MEM_RULES, p, N, 1)
    need_e = S.sgbem_memory_need(S.SGBEM_MEM_ASSEMBLE_EBE, p, N, 1, G)
    with Context(0, hbm_budget_bytes=need_r + need_e) as c:
        A = c.assemble(curve, p, N, "ebe", n_gauss=G)
        c.rhs(curve, p, N, synth.g_exp_cos, "ebe", n_gauss=G)
        assert S.sgbem_ctx_memory(c.ctx)[0] == need_r + need_e
        assert relmax(A.cpu().numpy(), ebe.matrix(curve, p, N, G)) < 1e-12
        # a batch description does not fit in what is left
        import torch
        out = torch.empty((N, N), dtype=torch.float64, device="cuda")
        with pytest.raises(S.SgbemError) as e:
            S.sgbem_batch_create(c.ctx, [curve], [c.rules(p, N, 1)], S.SGBEM_FP64, [out.data_ptr()], [N])
        assert e.value.status == S.SGBEM_E_NOMEM
        assert S.sgbem_ctx_memory(c.ctx)[0] == need_r + need_e
