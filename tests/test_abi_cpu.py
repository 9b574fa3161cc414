"""The C ABI library loads, exports every declared entry point, and its host
planner agrees with the oracle (CPU only, no device calls)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1703_10016_amd import sgbem as S
    if not os.path.exists(S.LIB_PATH):
        from paper_1703_10016_amd import build
        build.build()
    return S


def _declared():
    txt = open(os.path.join(ROOT, "include", "sgbem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgbem_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    S = _lib()
    L = S.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(S.exported_symbols()) == set(names)
    assert b"gfx950" in L.sgbem_version()


@pytest.mark.parametrize("p,N,R", [(2, 16, 1), (3, 20, 2), (4, 12, 1), (2, 9, 3), (3, 8, 4)])
def test_planner_matches_oracle_rules(p, N, R):
    """Alg. 1 weights and the singular-weight tables of the library's host
    planner (Householder QR, Gauss-log moments, bordered cyclic Cholesky) against
    the oracle's dense least-squares route."""
    S = _lib()
    from oracle import wq
    w0, bv, ws = S.sgbem_weights_host(p, N, R)
    nset, wref = wq.regular_weights(p, N, R, rows=[0])[0]
    from oracle import bspline
    eta = wq.nodes(N, R)
    Bloc = np.stack([bspline.periodic(p, R * N, k, eta[nset]) for k in wq.exactness_set(p, N, R, 0)])
    # two minimum-norm routes (QR vs SVD) agree to the conditioning of the local system
    tol = 4 * np.finfo(float).eps * np.linalg.cond(Bloc)
    assert np.abs(w0 - wref).max() < tol * np.abs(wref).max()
    Ws = wq.singular_weights(p, N, R)
    M2 = 2 * R * N
    m = np.arange(M2)
    lib_full = ws[m[:, None] % 2, (m[None, :] - m[:, None]) % M2]
    assert np.abs(lib_full - Ws).max() < 2e-14 * np.abs(Ws).max()
    from oracle import bspline
    assert np.abs(bv - bspline.periodic(p, N, 0, wq.nodes(N, R)[nset])).max() < 1e-15


def test_planner_nearfield_matches_oracle():
    S = _lib()
    from oracle import nearfield
    u, w, mco, madj = S.sgbem_nearfield_host()
    uo, wo, Mco, Madj = nearfield.reference_matrices(16)
    assert np.abs(u - uo).max() < 1e-15 and np.abs(w - wo).max() < 1e-15
    assert np.abs(mco - Mco).max() < 1e-15
    assert np.abs(madj - Madj).max() < 1e-15


@pytest.mark.parametrize("args", [(0, 16, 1), (7, 64, 1), (3, 7, 1), (2, 16, 0), (2, 16, 5)])
def test_planner_rejects_bad_arguments(args):
    S = _lib()
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_weights_host(*args)
    assert e.value.status == S.SGBEM_E_INVAL


def test_python_binding_has_no_compute_fallback():
    """The binding only marshals arguments: it must not import the oracle or
    numerical libraries beyond numpy / ctypes."""
    src = open(os.path.join(ROOT, "paper_1703_10016_amd", "sgbem.py")).read()
    src += open(os.path.join(ROOT, "paper_1703_10016_amd", "runtime.py")).read()
    assert "oracle" not in src and "scipy" not in src


@pytest.mark.parametrize("which", ["circle", "ellipse", "star", "ellipse-nonuniform", "nonuniform-80"])
def test_node_points_host_match_oracle_curve(which):
    """The host node points f(n / 2 n_ref N) agree with the oracle's curve
    evaluation (de Boor / polar form, Section 3) to rounding."""
    import synth
    from oracle import curves
    S = _lib()
    curve = {"circle": synth.circle(0.5), "ellipse": synth.ellipse_bspline(), "star": synth.star(7),
             "ellipse-nonuniform": synth.ellipse_bspline_nonuniform(0),
             "nonuniform-80": synth.ellipse_bspline_nonuniform(3, n_ctrl=80, jitter=0.6)}[which]
    for N, R in [(37, 1), (64, 2)]:
        xy = S.sgbem_node_points_host(curve, N, R)
        t = np.arange(2 * R * N) / (2 * R * N)
        x, y = curves.evaluate(curve, t)[:2]
        assert np.abs(xy[:, 0] - x).max() < 1e-14 and np.abs(xy[:, 1] - y).max() < 1e-14


def test_server_footprint_formula():
    """A request holds A (N^2 words of the matrix precision), the solve
    workspace (4 N^2 bytes of FP32 LU plus O(N)), and g, beta, x (O(N))."""
    S = _lib()
    for N in (16, 256, 1000, 4099, 8192):
        f64 = S.sgbem_server_footprint(N, S.SGBEM_FP64)
        f32 = S.sgbem_server_footprint(N, S.SGBEM_FP32)
        ws = S.sgbem_memory_need(S.SGBEM_MEM_SOLVE, 1, N)
        assert 12 * N * N <= f64 <= 8 * N * N + ws + 32 * N + 1024
        assert 8 * N * N <= f32 <= 4 * N * N + ws + 32 * N + 1024
        assert abs((f64 - f32) - 4 * N * N) < 256 and f64 % 256 == 0 and f32 % 256 == 0
    for bad in [(0, 0), (70000, 0), (64, 2)]:
        with pytest.raises(S.SgbemError) as e:
            S.sgbem_server_footprint(*bad)
        assert e.value.status == S.SGBEM_E_INVAL


@pytest.mark.parametrize("kw", [dict(workers=0), dict(workers=65), dict(budget_bytes=0), dict(precision=3),
                                dict(max_N=2), dict(workers=4, max_rules=8), dict(max_iter=-1), dict(tol=-1.0)])
def test_server_rejects_bad_config_before_touching_the_device(kw):
    S = _lib()
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_server_create(**kw)
    assert e.value.status == S.SGBEM_E_INVAL


def test_node_points_host_nonuniform_knots_with_derivative_at_breakpoints():
    """Node points on a knot vector with clustered knots, where many nodes fall
    on or next to breakpoints (the span search's boundary cases)."""
    import synth
    from oracle import curves
    S = _lib()
    tau = np.array([0.0, 0.125, 0.25, 0.26, 0.27, 0.5, 0.625, 0.75, 0.875, 1.0])
    ctrl = np.stack([np.cos(2 * np.pi * np.arange(9) / 9), 0.6 * np.sin(2 * np.pi * np.arange(9) / 9)], 1)
    for d in (1, 2, 3, 5):
        curve = synth.BSplineCurve(degree=d, ctrl=ctrl, knots=tau)
        xy = S.sgbem_node_points_host(curve, 16, 2)
        x, y = curves.evaluate(curve, np.arange(64) / 64)[:2]
        assert np.abs(xy[:, 0] - x).max() < 1e-14 and np.abs(xy[:, 1] - y).max() < 1e-14


@pytest.mark.parametrize("knots", [np.array([0.0, 0.3, 0.3, 0.6, 1.0]), np.array([0.1, 0.3, 0.5, 0.7, 1.0]),
                                   np.array([0.0, 0.3, 0.5, 0.7, 0.99]), np.array([0.0, 0.5, 0.4, 0.7, 1.0])])
def test_bad_knot_vectors_are_rejected(knots):
    """Knots of one period must run from 0 to 1 and increase strictly."""
    import synth
    S = _lib()
    ctrl = np.stack([np.cos(np.arange(4)), np.sin(np.arange(4))], 1)
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_node_points_host(synth.BSplineCurve(degree=2, ctrl=ctrl, knots=knots), 8, 1)
    assert e.value.status == S.SGBEM_E_INVAL


def _al256(b):
    return (b + 255) // 256 * 256


def _buf(b):
    return max(4096, (b + 4095) // 4096 * 4096)


def test_memory_need_formulas():
    """Device bytes per call kind, as the header states them: rule block
    72 M (+ alignment), node geometry 48 M, solve workspace 4 N^2 + O(N) (plus
    8 MiB per 1024 rows beyond N = 4096), each buffer rounded up to 4096 bytes,
    control nets beyond 64 points added."""
    S = _lib()
    for p, N, R in [(3, 1024, 1), (2, 16384, 1), (4, 700, 2), (6, 14, 4)]:
        M = R * N
        n = 2 * M
        rules = _al256(8 * n) + _al256(16 * n) + _al256(512) + _al256(4 * n) + _al256(8 * n)
        assert S.sgbem_memory_need(S.SGBEM_MEM_RULES, p, N, R) == _buf(rules)
        assert abs(_buf(rules) - 72 * M) <= 4096 + 5 * 256
        assert S.sgbem_memory_need(S.SGBEM_MEM_ASSEMBLE_WQ, p, N, R) == _buf(48 * M)
        assert S.sgbem_memory_need(S.SGBEM_MEM_ASSEMBLE_WQ, p, N, R, n_ctrl=64) == _buf(48 * M)
        assert S.sgbem_memory_need(S.SGBEM_MEM_ASSEMBLE_WQ, p, N, R, n_ctrl=100) == _buf(48 * M) + _buf(8 * 301)
    for N in (16, 1000, 4096, 4099, 16384):
        sv = S.sgbem_memory_need(S.SGBEM_MEM_SOLVE, 1, N)
        Np = (N + 63) // 64 * 64
        # beyond N = 4096: the inverted 1024-row diagonal blocks of L and U, 8 MiB per 1024 rows
        inv = 8 * 1024 * 1024 * ((N + 1023) // 1024) if N > 4096 else 0
        assert 4 * N * N + inv <= sv <= 4 * Np * Np + inv + 1900 * Np + 65536 and sv % 4096 == 0
    p, N, G = 3, 200, 5
    ebe = S.sgbem_memory_need(S.SGBEM_MEM_ASSEMBLE_EBE, p, N, 1, G)
    assert ebe == _buf(24 * N * G) + _buf(24 * N * 16) + _buf(16 * N * (p + 1) ** 2) + _buf(8 * (544 + 16 * (p + 1))) \
        + _buf(8 * G * (p + 1))
    d = S.sgbem_memory_need(S.SGBEM_MEM_RHS_DIRECT, p, N, 1, 4)
    assert d >= _buf(48 * N) + _buf(8 * (5 * N * 4 + 2 * 2 * N))
    for bad in [dict(what=9), dict(what=0, N=0), dict(what=0, n_ref=5), dict(what=1, p=0), dict(what=2, n_gauss=0),
                dict(what=3, n_gauss=3), dict(what=1, n_ctrl=-1)]:
        kw = dict(p=3, N=64, n_ref=1, n_gauss=4, n_ctrl=0)
        kw.update(bad)
        with pytest.raises(S.SgbemError) as e:
            S.sgbem_memory_need(kw.pop("what"), **kw)
        assert e.value.status == S.SGBEM_E_INVAL


def _knots(N, seed, spread=0.6):
    rng = np.random.default_rng(seed)
    u = (np.arange(N + 1) + spread * (rng.uniform(0, 1, N + 1) - 0.5)) / N
    u[0], u[-1] = 0.0, 1.0
    return u


@pytest.mark.parametrize("p,N,R,seed", [(2, 10, 1, 0), (3, 9, 2, 1), (4, 12, 1, 2), (1, 8, 1, 3), (6, 14, 1, 4)])
def test_knot_planner_matches_oracle(p, N, R, seed):
    """Rules on non-uniform knots from the library's host planner (Householder QR
    per row, local Cox-de Boor pieces, general cyclic banded Cholesky) against
    the oracle's dense least-squares route (O6)."""
    from oracle import wq_knots as K
    S = _lib()
    tau = _knots(N, seed)
    W, Bv, Ws, eta = S.sgbem_weights_host_knots(p, N, R, tau)
    assert np.array_equal(eta, K.nodes(tau, R))
    tb = K.refine(tau, R)
    rules = K.regular_weights(tau, p, R)
    for i, (nset, w) in rules.items():
        Bloc = np.stack([K.basis(tb, p, int(k), eta[nset]) for k in K.exactness_set(p, N, R, i)])
        tol = 20 * np.finfo(float).eps * np.linalg.cond(Bloc) * np.abs(w).max()
        assert np.abs(W[i] - w).max() < tol, (i, np.abs(W[i] - w).max(), tol)
        assert np.abs(Bv[i] - K.basis(tau, p, i, eta[nset])).max() < 4e-15   # (the oracle wraps by t + 1)
    Wso = K.singular_weights(tau, p, R)
    assert np.abs(Ws - Wso).max() < 2e-13 * np.abs(Wso).max(), np.abs(Ws - Wso).max() / np.abs(Wso).max()


def test_knot_planner_on_uniform_knots_matches_uniform_tables():
    S = _lib()
    p, N, R = 3, 16, 2
    W, Bv, Ws, eta = S.sgbem_weights_host_knots(p, N, R, np.arange(N + 1) / N)
    w0, bv, ws = S.sgbem_weights_host(p, N, R)
    assert np.abs(W - w0[None, :]).max() < 1e-13 and np.abs(Bv - bv[None, :]).max() < 1e-15
    M2 = 2 * R * N
    m = np.arange(M2)
    full = ws[m[:, None] % 2, (m[None, :] - m[:, None]) % M2]
    assert np.abs(Ws - full).max() < 1e-13 * np.abs(full).max()


@pytest.mark.parametrize("args,status", [((3, 10, 1, np.linspace(0, 1, 10)), -1),
                                         ((3, 10, 1, np.r_[0, 0.5, 0.4, np.linspace(0.5, 1, 8)]), -1),
                                         ((2, 4096, 2, np.linspace(0, 1, 4097)), -6)])
def test_knot_planner_rejects(args, status):
    S = _lib()
    p, N, R, tau = args
    with pytest.raises((S.SgbemError, ValueError)) as e:
        S.sgbem_weights_host_knots(p, N, R, tau)
    if isinstance(e.value, S.SgbemError):
        assert e.value.status == status


# ---------------------------------------------------------------- open arcs
def _breaks(n, seed, a=-1.0, b=1.0, spread=0.6):
    rng = np.random.default_rng([1703, 80000 + seed])
    u = (np.arange(n + 1) + spread * (rng.uniform(0, 1, n + 1) - 0.5)) / n
    u[0], u[-1] = 0.0, 1.0
    return a + (b - a) * u


@pytest.mark.parametrize("p,n,R,seed", [(2, 10, 1, 0), (3, 7, 2, 1), (1, 5, 1, 2), (6, 9, 1, 3), (4, 3, 2, 4),
                                        (2, 1, 2, 5), (5, 12, 2, 6), (1, 2, 1, 7)])
def test_open_planner_matches_oracle(p, n, R, seed):
    """Open-arc rules from the library's host planner (Householder QR per row, clamped Cox-de Boor pieces,
    banded Cholesky of the Gram matrix) against the oracle's dense least-squares route (O7)."""
    from oracle import wq_open as O
    S = _lib()
    br = _breaks(n, seed)
    n0, cnt, W, Bv, Ws, eta = S.sgbem_weights_host_open(p, br, R)
    assert np.array_equal(eta, O.nodes(br, p, R))
    assert W.shape[1] == 2 * R * (p + 1) - 1 + 2 * p
    T = O.knot_vector(br, p)
    Tb = O.knot_vector(O.refine(br, R), p)
    for i, (nset, w) in O.regular_weights(br, p, R).items():
        assert n0[i] == nset[0] and cnt[i] == nset.size and np.array_equal(nset, n0[i] + np.arange(cnt[i]))
        Bloc = np.stack([O.basis(Tb, p, int(k), eta[nset]) for k in O.exactness_set(br, p, R, i)])
        tol = 20 * np.finfo(float).eps * np.linalg.cond(Bloc) * np.abs(w).max()
        assert np.abs(W[i, :cnt[i]] - w).max() < tol, (i, np.abs(W[i, :cnt[i]] - w).max(), tol)
        assert np.all(W[i, cnt[i]:] == 0) and np.all(Bv[i, cnt[i]:] == 0)
        assert np.abs(Bv[i, :cnt[i]] - O.basis(T, p, i, eta[nset])).max() < 2e-15
    Wso = O.singular_weights(br, p, R)
    assert np.abs(Ws - Wso).max() < 2e-13 * np.abs(Wso).max(), np.abs(Ws - Wso).max() / np.abs(Wso).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("R", [1, 2])
def test_open_tile_windows_fit_the_kernel(p, R):
    """The assembly kernel's node window per 24-row tile is P (T - 1) + (p - 1) + QM: the row starts n0 grow
    by 2R per row except once by 2R + p - 1 (after the rows whose support holds the first element)."""
    S = _lib()
    P, T = 2 * R, 24
    QM = P * (p + 1) - 1 + 2 * p
    for n in [1, 2, 3, p + 1, 23, 24, 25, 47, 60, 101]:
        if R * n < 2:
            continue
        n0, cnt = S.sgbem_weights_host_open(p, np.linspace(0.0, 1.0, n + 1), R)[:2]
        assert cnt.max() <= QM and np.all(np.diff(n0) >= 0)
        N = n + p
        for I0 in range(0, N, T):
            assert n0[min(I0 + T - 1, N - 1)] - n0[I0] + QM <= P * (T - 1) + (p - 1) + QM


def test_open_memory_need():
    S = _lib()
    for p, n, R in [(2, 640, 1), (3, 100, 2), (6, 5, 4)]:
        N, QM, nq = n + p, 2 * R * (p + 1) - 1 + 2 * p, 2 * p + 2 * R * n - 1
        want = 2 * _al256(8 * N * QM) + _al256(8 * nq * nq) + _al256(8 * nq) + 2 * _al256(4 * N)
        assert S.sgbem_memory_need(S.SGBEM_MEM_RULES_OPEN, p, n, R) == _buf(want)


@pytest.mark.parametrize("args,status", [((2, np.array([0.0, 0.5, 0.5, 1.0]), 1), -1),
                                         ((2, np.array([1.0, 0.0]), 1), -1),
                                         ((2, np.array([0.0, 1.0]), 1), -1),
                                         ((7, np.linspace(0, 1, 5), 1), -1),
                                         ((2, np.linspace(0, 1, 5), 5), -1),
                                         ((2, np.array([0.0, np.nan, 1.0]), 1), -1),
                                         ((2, np.linspace(0, 1, 4096), 1), -6)])
def test_open_planner_rejects(args, status):
    S = _lib()
    p, br, R = args
    with pytest.raises(S.SgbemError) as e:
        S.sgbem_weights_host_open(p, br, R)
    assert e.value.status == status
