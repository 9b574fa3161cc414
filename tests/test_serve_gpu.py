"""Serving loop (continuous batching of independent solves) through the C ABI.

Each request is assembled by the fast form, its right-hand side formed and its
system solved by the mixed-precision solve, on one of several streams.  Every
kernel on the path reduces in a fixed order (no atomics), so a request's alpha
must be bit-for-bit the same whether it runs alone or among others.
"""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _S():
    from paper_1703_10016_amd import sgbem as S
    return S


def _requests(specs):
    """(curve, p, N, g) for star curves, g = exp(x1) cos(x2) at the node points."""
    S = _S()
    out = []
    for idx, (p, N) in enumerate(specs):
        curve = synth.star(40000 + idx)
        xy = S.sgbem_node_points_host(curve, N, 1)
        out.append((curve, p, N, synth.g_exp_cos(xy[:, 0], xy[:, 1])))
    return out


def _drain(S, srv, n, timeout=120.0):
    got = []
    t_end = time.time() + timeout
    while len(got) < n and time.time() < t_end:
        got += S.sgbem_server_poll(srv, 64, 0.5)
    assert len(got) == n, f"only {len(got)} of {n} completions"
    return {c.tag: c for c in got}


def _run_server(reqs, arrivals=None, **cfg):
    S = _S()
    srv = S.sgbem_server_create(**cfg)
    try:
        xs = [np.zeros(r[2]) for r in reqs]
        for i, (curve, p, N, g) in enumerate(reqs):
            S.sgbem_server_submit(srv, curve, p, N, g, xs[i], 0.0 if arrivals is None else arrivals[i], i)
        comp = _drain(S, srv, len(reqs))
        stats = S.sgbem_server_stats(srv)
    finally:
        S.sgbem_server_destroy(srv)
    return xs, comp, stats


MIX = [(2, 256), (3, 300), (4, 512), (3, 777), (2, 1024), (4, 1500), (3, 2048), (2, 640), (3, 512), (4, 1024),
       (3, 256), (2, 2048)]


def test_each_result_is_the_same_alone_and_in_the_mix():
    S = _S()
    reqs = _requests(MIX)
    xs_mix, comp, stats = _run_server(reqs, workers=6, budget_bytes=2 << 30, max_N=2048, max_rules=64)
    assert all(c.status == 0 for c in comp.values()), [c.message for c in comp.values() if c.status]
    assert stats["completed"] == len(MIX) and stats["failed"] == 0 and stats["peak_in_flight"] > 1
    for i, r in enumerate(reqs):
        xs_solo, comp1, _ = _run_server([r], workers=1, budget_bytes=1 << 30, max_N=2048, max_rules=3)
        assert comp1[0].status == 0
        assert np.array_equal(xs_solo[0], xs_mix[i]), f"request {i} (p, N) = {MIX[i]} differs alone / in the mix"


def test_server_matches_the_single_call_path():
    """The served alpha equals assemble + rhs + solve through a context, up to
    the last bits of the host node points (g sampled at host vs device points)."""
    import torch
    from paper_1703_10016_amd.runtime import Context
    S = _S()
    reqs = _requests([(3, 700), (2, 1200)])
    xs, comp, _ = _run_server(reqs, workers=2, budget_bytes=1 << 30, max_N=2048, max_rules=8)
    ctx = Context()
    for (curve, p, N, g), x in zip(reqs, xs):
        A = ctx.assemble(curve, p, N, "wq", precision="fp64")
        beta = ctx.rhs(curve, p, N, synth.g_exp_cos, "wq")
        ref, info = ctx.solve(A, beta, tol=1e-12)
        ref = ref.cpu().numpy()
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()
    torch.cuda.synchronize()


def test_admission_never_exceeds_the_budget():
    S = _S()
    specs = [(3, 1024)] * 6 + [(2, 512)] * 4
    reqs = _requests(specs)
    f1024 = S.sgbem_server_footprint(1024, S.SGBEM_FP64)
    budget = 2 * f1024 + f1024 // 2      # two N = 1024 requests, or one with some smaller ones
    xs, comp, stats = _run_server(reqs, workers=4, budget_bytes=budget, max_N=1024, max_rules=16)
    assert all(c.status == 0 for c in comp.values())
    assert stats["peak_bytes"] <= budget
    # replay the admission intervals: the footprints held at any instant fit the budget
    ev = sorted([(c.t_admit, c.footprint) for c in comp.values()] + [(c.t_done, -c.footprint) for c in comp.values()],
                key=lambda e: (e[0], e[1]))
    held = 0
    for _, d in ev:
        held += d
        assert held <= budget
    for c in comp.values():
        assert c.t_arrival <= c.t_admit <= c.t_done


def test_oversized_request_is_rejected_without_a_completion():
    S = _S()
    srv = S.sgbem_server_create(workers=1, budget_bytes=S.sgbem_server_footprint(512), max_N=4096, max_rules=3)
    try:
        (curve, p, N, g), = _requests([(2, 1024)])
        with pytest.raises(S.SgbemError) as e:
            S.sgbem_server_submit(srv, curve, p, N, g, np.zeros(N), 0.0, 7)
        assert e.value.status == S.SGBEM_E_NOMEM
        with pytest.raises(S.SgbemError) as e:   # N above max_N
            S.sgbem_server_submit(srv, curve, p, 8192, np.zeros(16384), np.zeros(8192), 0.0, 8)
        assert e.value.status == S.SGBEM_E_INVAL
        assert S.sgbem_server_poll(srv, 8, 0.2) == []
        st = S.sgbem_server_stats(srv)
        assert st["rejected"] == 1 and st["submitted"] == 0
    finally:
        S.sgbem_server_destroy(srv)


def test_arrival_times_are_respected_and_rules_are_cached():
    S = _S()
    srv = S.sgbem_server_create(workers=2, budget_bytes=1 << 30, max_N=1024, max_rules=5)
    try:
        reqs = _requests([(3, 512)] * 3 + [(2, 256 + 16 * k) for k in range(6)])
        t0 = S.sgbem_server_clock(srv)
        xs = [np.zeros(r[2]) for r in reqs]
        for i, (curve, p, N, g) in enumerate(reqs):
            S.sgbem_server_submit(srv, curve, p, N, g, xs[i], t0 + 0.3 + 0.02 * i, i)
        comp = _drain(S, srv, len(reqs))
        st = S.sgbem_server_stats(srv)
    finally:
        S.sgbem_server_destroy(srv)
    for i, c in comp.items():
        assert c.status == 0 and c.t_admit >= c.t_arrival >= t0 + 0.3 + 0.02 * i - 1e-9
    # 7 distinct (p, N) with room for 5: hits for the repeated N = 512, evictions for the rest
    assert st["rules_hits"] >= 2 and st["rules_misses"] >= 7 and st["rules_cached"] <= 5
    # results after evictions and rebuilds equal a fresh run
    xs2, comp2, _ = _run_server(reqs[-2:], workers=1, budget_bytes=1 << 30, max_N=1024, max_rules=3)
    assert np.array_equal(xs2[0], xs[-2]) and np.array_equal(xs2[1], xs[-1])


def test_refinement_limit_reports_noconv_per_request():
    S = _S()
    reqs = _requests([(3, 300), (2, 400)])
    xs, comp, stats = _run_server(reqs, workers=2, budget_bytes=1 << 30, max_N=512, max_rules=8, max_iter=0)
    assert all(c.status == S.SGBEM_E_NOCONV for c in comp.values())
    assert stats["failed"] == 2 and stats["completed"] == 2


def test_destroy_drops_requests_not_yet_admitted():
    S = _S()
    srv = S.sgbem_server_create(workers=1, budget_bytes=1 << 28, max_N=512, max_rules=3)
    reqs = _requests([(2, 256)] * 4)
    xs = [np.zeros(256) for _ in reqs]
    t0 = S.sgbem_server_clock(srv)
    for i, (curve, p, N, g) in enumerate(reqs):
        S.sgbem_server_submit(srv, curve, p, N, g, xs[i], t0 + 3600.0, i)
    st = S.sgbem_server_stats(srv)
    assert st["waiting"] == 4 and st["in_flight"] == 0
    t = time.time()
    S.sgbem_server_destroy(srv)
    assert time.time() - t < 10.0


def test_served_solution_matches_oracle_solve():
    """Served alpha against LAPACK's FP64 solve of the oracle's matrix and
    right-hand side (eqs. IK1e2 / IK1e2_bis, eq. final_b1), not against the
    library's own single-call path.  The served matrix is within 1e-12
    (max-norm relative) of the oracle's and the refinement stops at 1e-12, so
    the relative solution error is bounded by cond_2(A) times a small multiple
    of 1e-12: the test allows 1e-10 + 4 cond_2(A) 1e-12."""
    from oracle import wq
    reqs = _requests([(3, 300), (2, 256)])
    xs, comp, _ = _run_server(reqs, workers=2, budget_bytes=1 << 30, max_N=512, max_rules=8)
    for (curve, p, N, _), x, c in zip(reqs, xs, [comp[0], comp[1]]):
        assert c.status == 0, c.message
        A = wq.matrix(curve, p, N, 1)
        beta = wq.rhs(curve, p, N, 1, synth.g_exp_cos)
        ref = np.linalg.solve(A, beta)
        err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        assert err < 1e-10 + 4 * np.linalg.cond(A) * 1e-12, (p, N, err, np.linalg.cond(A))
