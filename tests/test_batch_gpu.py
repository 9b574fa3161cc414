"""Batched persistent assembly (fast form) on an MI355X: every matrix of a
mixed-degree, ragged-size batch equals its single-curve assembly, before and
after autotuning, and a HIP-graph capture replays to the same result."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_1703_10016_amd.runtime import Context
    c = Context(0)
    yield c
    c.close()


CASES = [(synth.star(40 + k), p, N) for k, (p, N) in enumerate(
    [(2, 37), (3, 64), (4, 100), (2, 129), (3, 256), (4, 300), (2, 513), (3, 8), (4, 10), (2, 700), (3, 1000), (4, 31)])]


def _batch(ctx, prec):
    import torch
    from paper_1703_10016_amd import sgbem as S
    dt = torch.float64 if prec == "fp64" else torch.float32
    outs = [torch.full((N, N), float("nan"), dtype=dt, device="cuda") for (_, _, N) in CASES]
    rules = [ctx.rules(p, N, 1) for (_, p, N) in CASES]
    b = S.sgbem_batch_create(ctx.ctx, [c for (c, _, _) in CASES], rules,
                             S.SGBEM_FP64 if prec == "fp64" else S.SGBEM_FP32,
                             [o.data_ptr() for o in outs], [o.stride(0) for o in outs])
    return b, outs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_single_curve(ctx, prec):
    import torch
    from paper_1703_10016_amd import sgbem as S
    b, outs = _batch(ctx, prec)
    S.sgbem_batch_assemble(ctx.ctx, b)
    torch.cuda.synchronize()
    for (curve, p, N), o in zip(CASES, outs):
        ref = ctx.assemble(curve, p, N, "wq", precision=prec).cpu().numpy()
        got = o.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, got.T)
        assert np.abs(got - ref).max() <= (1e-15 if prec == "fp64" else 1e-6) * np.abs(ref).max()
    cfg, ms = S.sgbem_batch_tune(ctx.ctx, b, 2)
    assert 0 <= cfg < 4 and ms > 0
    for o in outs:
        o.fill_(float("nan"))
    S.sgbem_batch_assemble(ctx.ctx, b)
    torch.cuda.synchronize()
    for (curve, p, N), o in zip(CASES, outs):
        ref = ctx.assemble(curve, p, N, "wq", precision=prec).cpu().numpy()
        got = o.cpu().numpy()
        assert np.abs(got - ref).max() <= (1e-15 if prec == "fp64" else 1e-6) * np.abs(ref).max()
    S.sgbem_batch_free(ctx.ctx, b)


def test_batch_graph_replay(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    b, outs = _batch(ctx, "fp32")
    S.sgbem_batch_assemble(ctx.ctx, b)
    torch.cuda.synchronize()
    eager = [o.cpu().numpy().copy() for o in outs]
    g = torch.cuda.CUDAGraph()
    S.sgbem_ctx_set_stream(ctx.ctx, torch.cuda.current_stream().cuda_stream)
    s = torch.cuda.Stream()
    S.sgbem_ctx_set_stream(ctx.ctx, s.cuda_stream)
    with torch.cuda.graph(g, stream=s):
        S.sgbem_batch_assemble(ctx.ctx, b)
    S.sgbem_ctx_set_stream(ctx.ctx, ctx.stream.cuda_stream)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, o in zip(eager, outs):
            assert np.array_equal(o.cpu().numpy(), e), rep
    del g
    S.sgbem_batch_free(ctx.ctx, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_members_match_oracle(ctx, prec):
    """Batch members against the oracle (eqs. IK1e2 / IK1e2_bis, Alg. 3), not
    against the library's own single-curve path: full matrices for three
    members of different degree, sampled rows (upper part from the row, lower
    part through the mirror) for two members with N >= 700.  1e-12 in FP64,
    2e-5 in FP32, max-norm relative."""
    import torch
    from oracle import wq
    from paper_1703_10016_amd import sgbem as S
    b, outs = _batch(ctx, prec)
    S.sgbem_batch_assemble(ctx.ctx, b)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "fp64" else 2e-5
    for k in (1, 2, 5):                   # (p, N) = (3, 64), (4, 100), (4, 300)
        curve, p, N = CASES[k]
        got = outs[k].double().cpu().numpy()
        ref = wq.matrix(curve, p, N, 1)
        assert np.abs(got - ref).max() < tol * np.abs(ref).max(), (k, p, N)
    for k in (9, 10):                     # (2, 700), (3, 1000)
        curve, p, N = CASES[k]
        got = outs[k].double().cpu().numpy()
        rows = [0, 1, N // 2 + 1, N - 1]
        ref = wq.full_rows(curve, p, N, 1, rows)
        for r, i in enumerate(rows):
            assert np.abs(got[i, i:] - ref[r, i:]).max() < tol * np.abs(ref[r]).max(), (k, i)
            assert np.array_equal(got[i, :i], got[:i, i])
    S.sgbem_batch_free(ctx.ctx, b)
