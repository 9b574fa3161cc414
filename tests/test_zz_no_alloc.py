"""The allocation-free fast-form assembly (sgbem_assemble_noalloc) on an
MI355X, called through the C ABI: its matrices equal those of sgbem_assemble
with the same rules bit for bit (same kernels, same inputs), on consecutive
calls that reuse the fixed geometry array with a smaller input the second
time, and sizes beyond the array are rejected before any launch."""
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


def _pair(ctx, curve, p, N, n_ref, prec):
    """(noalloc result, sgbem_assemble result) as host arrays; the noalloc
    output starts as NaN so that an unwritten entry cannot pass."""
    import torch
    from paper_1703_10016_amd import sgbem as S
    dt = torch.float64 if prec == "fp64" else torch.float32
    pc = S.SGBEM_FP64 if prec == "fp64" else S.SGBEM_FP32
    rules = ctx.rules(p, N, n_ref)
    out = torch.full((N, N + 3), float("nan"), dtype=dt, device="cuda")   # lda > N
    print(f"noalloc: p={p} N={N} n_ref={n_ref} {prec}", flush=True)
    S.sgbem_assemble_noalloc(ctx.ctx, curve, rules, pc, out.data_ptr(), out.stride(0))
    got = out[:, :N].cpu().numpy()
    ref = ctx.assemble(curve, p, N, "wq", n_ref=n_ref, precision=prec).cpu().numpy()
    return got, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_assemble_on_two_calls_smaller_second(ctx, prec):
    # first call: the ellipse at p = 3, N = 1024; second: a smaller star, other degree
    for curve, p, N in [(synth.ellipse_bspline(), 3, 1024), (synth.star(7), 2, 200)]:
        got, ref = _pair(ctx, curve, p, N, 1, prec)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref)


def test_noalloc_matches_oracle_small(ctx):
    from oracle import wq
    curve, p, N = synth.star(3), 4, 48
    got, ref = _pair(ctx, curve, p, N, 1, "fp64")
    assert np.array_equal(got, ref)
    o = wq.matrix(curve, p, N, 1)
    assert np.abs(got - o).max() <= 1e-12 * np.abs(o).max()


def test_noalloc_refined_rules_then_smaller(ctx):
    for curve, p, N, n_ref in [(synth.star(11), 3, 700, 2), (synth.circle(0.5), 2, 64, 1)]:
        got, ref = _pair(ctx, curve, p, N, n_ref, "fp64")
        assert np.array_equal(got, ref)


def test_noalloc_limits(ctx):
    import torch
    from paper_1703_10016_amd import sgbem as S
    # 2 n_ref N beyond the fixed array: rejected before any launch
    N = S.SGBEM_NOALLOC_MAX_NODES // 2 + 1
    rules = ctx.rules(2, N, 1)
    out = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_assemble_noalloc(ctx.ctx, synth.star(1), rules, S.SGBEM_FP64, out.data_ptr(), N)
    assert e.value.status == S.SGBEM_E_INVAL
    # a control net that does not travel inline
    big = synth.ellipse_bspline(n_ctrl=65)
    r2 = ctx.rules(2, 32, 1)
    A = torch.zeros((32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_assemble_noalloc(ctx.ctx, big, r2, S.SGBEM_FP64, A.data_ptr(), 32)
    assert e.value.status == S.SGBEM_E_UNSUPPORTED
    # the largest accepted size still assembles (sampled rows against sgbem_assemble)
    Nmax = S.SGBEM_NOALLOC_MAX_NODES // 2
    rm = ctx.rules(2, Nmax, 1)
    rows = torch.zeros((Nmax, Nmax), dtype=torch.float32, device="cuda")
    S.sgbem_assemble_noalloc(ctx.ctx, synth.star(2), rm, S.SGBEM_FP32, rows.data_ptr(), Nmax)
    pick = [0, 1, 777, Nmax // 2, Nmax - 1]
    got = rows[pick].cpu().numpy()
    ctx.assemble(synth.star(2), 2, Nmax, "wq", precision="fp32", out=rows)
    assert np.array_equal(got, rows[pick].cpu().numpy())
    del rows
    torch.cuda.empty_cache()
