"""ctypes binding of libsgbem (include/sgbem.h): argument marshalling only.

Every numerical step runs inside the library's HIP kernels; PyTorch only
provides device memory and the stream.  The library must have been built
(``python -m paper_1703_10016_amd.build`` or ``__graft_entry__.build()``);
there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgbem.so")

SGBEM_OK, SGBEM_E_INVAL, SGBEM_E_NOMEM, SGBEM_E_SINGULAR = 0, -1, -2, -3
SGBEM_E_NOCONV, SGBEM_E_DEVICE, SGBEM_E_UNSUPPORTED = -4, -5, -6
SGBEM_CURVE_BSPLINE, SGBEM_CURVE_POLAR, SGBEM_CURVE_BSPLINE_OPEN = 0, 1, 2
SGBEM_WQ, SGBEM_EBE = 0, 1
SGBEM_FP64, SGBEM_FP32 = 0, 1
SGBEM_NOALLOC_MAX_NODES = 65536

_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_SINGULAR", -4: "E_NOCONV", -5: "E_DEVICE",
          -6: "E_UNSUPPORTED"}


class SgbemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class sgbem_curve(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("degree", ctypes.c_int32), ("n_ctrl", ctypes.c_int32),
                ("ctrl_xy", ctypes.POINTER(ctypes.c_double)), ("knots", ctypes.POINTER(ctypes.c_double)),
                ("r0", ctypes.c_double),
                ("n_modes", ctypes.c_int32), ("a", ctypes.POINTER(ctypes.c_double)),
                ("phi", ctypes.POINTER(ctypes.c_double))]


class sgbem_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_update", ctypes.c_double),
                ("backward_err", ctypes.c_double), ("pivoted", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sgbem_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("workers", ctypes.c_int32), ("budget_bytes", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("max_N", ctypes.c_int32), ("max_rules", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double)]


class sgbem_request(ctypes.Structure):
    _fields_ = [("curve", sgbem_curve), ("p", ctypes.c_int32), ("N", ctypes.c_int32),
                ("g", ctypes.POINTER(ctypes.c_double)), ("x", ctypes.POINTER(ctypes.c_double)),
                ("arrival_s", ctypes.c_double), ("tag", ctypes.c_uint64)]


class sgbem_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("backward_err", ctypes.c_double), ("footprint", ctypes.c_int64), ("message", ctypes.c_char * 96)]


class sgbem_server_info(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("rejected", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("waiting", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("peak_in_flight", ctypes.c_int32), ("rules_cached", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("rules_hits", ctypes.c_int64), ("rules_misses", ctypes.c_int64)]


_lib = None


def lib():
    """Load libsgbem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1703_10016_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(sgbem_curve)
        sig = {
            "sgbem_ctx_create": [i32, vp, ctypes.c_uint64, ctypes.POINTER(vp)],
            "sgbem_ctx_memory": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)],
            "sgbem_memory_need": [i32, i32, i32, i32, i32, i32, ctypes.POINTER(i64)],
            "sgbem_ctx_destroy": [vp],
            "sgbem_ctx_set_stream": [vp, vp],
            "sgbem_ctx_set_timing": [vp, i32],
            "sgbem_ctx_kernel_time": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
            "sgbem_weights": [vp, i32, i32, i32, dp, ctypes.POINTER(vp)],
            "sgbem_weights_host_knots": [i32, i32, i32, dp, dp, dp, dp, dp],
            "sgbem_weights_open": [vp, i32, i32, i32, dp, ctypes.POINTER(vp)],
            "sgbem_weights_host_open": [i32, i32, i32, dp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32), dp, dp, dp, dp],
            "sgbem_rules_free": [vp, vp],
            "sgbem_weights_host": [i32, i32, i32, dp, dp, dp],
            "sgbem_nearfield_host": [dp, dp, dp, dp],
            "sgbem_rhs_points": [vp, cp, vp, i32, i32, vp, i64, ctypes.POINTER(i64)],
            "sgbem_assemble": [vp, cp, vp, i32, i32, i32, vp, i64],
            "sgbem_assemble_noalloc": [vp, cp, vp, i32, vp, i64],
            "sgbem_rhs": [vp, cp, vp, i32, i32, vp, vp],
            "sgbem_solve": [vp, i32, vp, i64, i32, vp, vp, dbl, i32, ctypes.POINTER(sgbem_solve_info)],
            "sgbem_batch_create": [vp, i32, cp, ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                   ctypes.POINTER(vp)],
            "sgbem_batch_assemble": [vp, vp],
            "sgbem_batch_tune": [vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)],
            "sgbem_batch_free": [vp, vp],
            "sgbem_node_points_host": [cp, i32, i32, dp],
            "sgbem_rhs_direct": [vp, cp, vp, i32, vp, vp, vp, vp],
            "sgbem_assemble_collocation": [vp, cp, vp, vp, i64],
            "sgbem_collocation_rhs": [vp, vp, vp, vp],
            "sgbem_server_footprint": [i32, i32, ctypes.POINTER(i64)],
            "sgbem_server_create": [ctypes.POINTER(sgbem_server_config), ctypes.POINTER(vp)],
            "sgbem_server_submit": [vp, ctypes.POINTER(sgbem_request)],
            "sgbem_server_poll": [vp, ctypes.POINTER(sgbem_completion), i32, dbl, ctypes.POINTER(i32)],
            "sgbem_server_clock": [vp, ctypes.POINTER(dbl)],
            "sgbem_server_stats": [vp, ctypes.POINTER(sgbem_server_info)],
            "sgbem_server_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.sgbem_last_error.restype = ctypes.c_char_p
        L.sgbem_last_error.argtypes = []
        L.sgbem_version.restype = ctypes.c_char_p
        L.sgbem_version.argtypes = []
        _lib = L
    return _lib


def _check(st):
    if st != SGBEM_OK:
        raise SgbemError(st, lib().sgbem_last_error().decode())


def exported_symbols():
    """Names of the ABI functions (for the load / export check)."""
    return ["sgbem_ctx_create", "sgbem_ctx_destroy", "sgbem_ctx_set_stream", "sgbem_ctx_set_timing",
            "sgbem_ctx_kernel_time", "sgbem_last_error", "sgbem_version",
            "sgbem_weights", "sgbem_rules_free", "sgbem_weights_host", "sgbem_nearfield_host", "sgbem_rhs_points",
            "sgbem_assemble", "sgbem_rhs", "sgbem_solve", "sgbem_batch_create", "sgbem_batch_assemble",
            "sgbem_batch_tune", "sgbem_batch_free", "sgbem_node_points_host", "sgbem_server_footprint",
            "sgbem_server_create", "sgbem_server_submit", "sgbem_server_poll", "sgbem_server_clock",
            "sgbem_server_stats", "sgbem_server_destroy", "sgbem_rhs_direct",
            "sgbem_assemble_collocation", "sgbem_collocation_rhs", "sgbem_assemble_noalloc",
            "sgbem_ctx_memory", "sgbem_memory_need", "sgbem_weights_host_knots", "sgbem_weights_open",
            "sgbem_weights_host_open"]


# ------------------------------------------------------------------ curve marshalling
class Curve:
    """A curve description kept alive next to its C struct."""

    def __init__(self, curve):
        self._keep = []
        c = sgbem_curve()
        kind = getattr(curve, "kind", None)
        if kind == "polar":
            c.kind = SGBEM_CURVE_POLAR
            c.r0 = float(curve.r0)
            a = np.ascontiguousarray(curve.a, dtype=np.float64)
            ph = np.ascontiguousarray(curve.phi, dtype=np.float64)
            c.n_modes = a.size
            self._keep += [a, ph]
            c.a = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            c.phi = ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        elif kind == "bspline":
            c.kind = SGBEM_CURVE_BSPLINE
            c.degree = int(curve.degree)
            q = np.ascontiguousarray(curve.ctrl, dtype=np.float64)
            c.n_ctrl = q.shape[0]
            self._keep.append(q)
            c.ctrl_xy = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            kn = getattr(curve, "knots", None)
            if kn is not None:
                kn = np.ascontiguousarray(kn, dtype=np.float64)
                if kn.shape != (q.shape[0] + 1,):
                    raise ValueError("knots must hold n_ctrl + 1 breakpoints")
                self._keep.append(kn)
                c.knots = kn.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        elif kind == "bspline_open":
            c.kind = SGBEM_CURVE_BSPLINE_OPEN
            c.degree = int(curve.degree)
            q = np.ascontiguousarray(curve.ctrl, dtype=np.float64)
            c.n_ctrl = q.shape[0]
            kn = np.ascontiguousarray(curve.knots, dtype=np.float64)
            if kn.shape != (q.shape[0] + c.degree + 1,):
                raise ValueError("an open arc's knots must hold n_ctrl + degree + 1 values")
            self._keep += [q, kn]
            c.ctrl_xy = q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            c.knots = kn.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            raise ValueError("curve must have kind 'polar', 'bspline' or 'bspline_open'")
        self.c = c

    def ref(self):
        return ctypes.byref(self.c)


def _as_curve(curve):
    return curve if isinstance(curve, Curve) else Curve(curve)


# ------------------------------------------------------------------ ABI functions
def sgbem_ctx_create(device=0, stream=None, hbm_budget_bytes=0):
    h = ctypes.c_void_p()
    _check(lib().sgbem_ctx_create(int(device), ctypes.c_void_p(stream or 0), int(hbm_budget_bytes), ctypes.byref(h)))
    return h


def sgbem_ctx_memory(ctx):
    """(bytes held, budget) of a context."""
    held, budget = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().sgbem_ctx_memory(ctx, ctypes.byref(held), ctypes.byref(budget)))
    return held.value, budget.value


SGBEM_MEM_RULES, SGBEM_MEM_ASSEMBLE_WQ, SGBEM_MEM_ASSEMBLE_EBE, SGBEM_MEM_RHS_DIRECT, SGBEM_MEM_SOLVE = 0, 1, 2, 3, 4
SGBEM_MEM_RULES_KNOTS, SGBEM_MEM_RULES_OPEN = 5, 6


def sgbem_memory_need(what, p=1, N=1, n_ref=1, n_gauss=0, n_ctrl=0):
    b = ctypes.c_int64()
    _check(lib().sgbem_memory_need(int(what), int(p), int(N), int(n_ref), int(n_gauss), int(n_ctrl), ctypes.byref(b)))
    return b.value


def sgbem_ctx_destroy(ctx):
    _check(lib().sgbem_ctx_destroy(ctx))


def sgbem_ctx_set_stream(ctx, stream):
    _check(lib().sgbem_ctx_set_stream(ctx, ctypes.c_void_p(stream or 0)))


def sgbem_ctx_set_timing(ctx, on):
    _check(lib().sgbem_ctx_set_timing(ctx, int(bool(on))))


def sgbem_ctx_kernel_time(ctx):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().sgbem_ctx_kernel_time(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _knots_ptr(knots, N):
    """(pointer, keep-alive array) for an optional knot vector of N + 1 breakpoints."""
    if knots is None:
        return None, None
    k = np.ascontiguousarray(knots, dtype=np.float64)
    if k.shape != (N + 1,):
        raise ValueError("knots must hold N + 1 breakpoints")
    return k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k


def sgbem_weights(ctx, p, N, n_ref=1, knots=None):
    h = ctypes.c_void_p()
    kp, keep = _knots_ptr(knots, N)
    _check(lib().sgbem_weights(ctx, int(p), int(N), int(n_ref), kp, ctypes.byref(h)))
    del keep
    return h


def sgbem_weights_host_knots(p, N, n_ref, knots):
    """(W[N, Q], Bv[N, Q], Ws[2M, 2M], eta[2M]) of the rules on non-uniform knots."""
    Q, M = 2 * n_ref * (p + 1) - 1, n_ref * N
    W, Bv, Ws, eta = np.zeros(N * Q), np.zeros(N * Q), np.zeros(4 * M * M), np.zeros(2 * M)
    kp, keep = _knots_ptr(knots, N)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().sgbem_weights_host_knots(int(p), int(N), int(n_ref), kp, P(W), P(Bv), P(Ws), P(eta)))
    del keep
    return W.reshape(N, Q), Bv.reshape(N, Q), Ws.reshape(2 * M, 2 * M), eta


def _breaks_ptr(breaks):
    b = np.ascontiguousarray(breaks, dtype=np.float64)
    if b.ndim != 1 or b.size < 2:
        raise ValueError("breaks must hold n_el + 1 breakpoints")
    return b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), b


def sgbem_weights_open(ctx, p, breaks, n_ref=1):
    """Rules of an open arc on the breakpoints breaks[0] = a < ... < breaks[n_el] = b."""
    h = ctypes.c_void_p()
    bp, keep = _breaks_ptr(breaks)
    _check(lib().sgbem_weights_open(ctx, int(p), keep.size - 1, int(n_ref), bp, ctypes.byref(h)))
    return h


def sgbem_weights_host_open(p, breaks, n_ref=1):
    """(n0[N], cnt[N], W[N, QM], Bv[N, QM], Ws[nq, nq], eta[nq]) of the open-arc rules."""
    bp, keep = _breaks_ptr(breaks)
    n_el = keep.size - 1
    N, nq = n_el + p, 2 * p + 2 * n_ref * n_el - 1
    qm = ctypes.c_int32()
    I = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    D = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().sgbem_weights_host_open(int(p), n_el, int(n_ref), bp, ctypes.byref(qm), None, None, None, None, None,
                                         None))
    QM = qm.value
    n0, cnt = np.zeros(N, dtype=np.int32), np.zeros(N, dtype=np.int32)
    W, Bv, Ws, eta = np.zeros(N * QM), np.zeros(N * QM), np.zeros(nq * nq), np.zeros(nq)
    _check(lib().sgbem_weights_host_open(int(p), n_el, int(n_ref), bp, ctypes.byref(qm), I(n0), I(cnt), D(W), D(Bv),
                                         D(Ws), D(eta)))
    return n0, cnt, W.reshape(N, QM), Bv.reshape(N, QM), Ws.reshape(nq, nq), eta


def sgbem_rules_free(ctx, rules):
    _check(lib().sgbem_rules_free(ctx, rules))


def sgbem_weights_host(p, N, n_ref=1):
    """(w0[Q], bvals[Q], ws[2, 2M]) from the library's host planner."""
    Q = max(1, 2 * n_ref * (p + 1) - 1)
    M = max(1, n_ref * N)
    w0, bv, ws = np.zeros(Q), np.zeros(Q), np.zeros(4 * M)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().sgbem_weights_host(int(p), int(N), int(n_ref), P(w0), P(bv), P(ws)))
    return w0, bv, ws.reshape(2, 2 * M)


def sgbem_nearfield_host():
    u, w, mco, madj = np.zeros(16), np.zeros(16), np.zeros(256), np.zeros(256)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().sgbem_nearfield_host(P(u), P(w), P(mco), P(madj)))
    return u, w, mco.reshape(16, 16), madj.reshape(16, 16)


def sgbem_rhs_points(ctx, curve, rules, method, n_gauss, d_xy_ptr, cap):
    cnt = ctypes.c_int64()
    c = _as_curve(curve)
    _check(lib().sgbem_rhs_points(ctx, c.ref(), rules, int(method), int(n_gauss), ctypes.c_void_p(d_xy_ptr),
                                  int(cap), ctypes.byref(cnt)))
    return cnt.value


def sgbem_assemble(ctx, curve, rules, method, n_gauss, precision, d_A_ptr, lda):
    c = _as_curve(curve)
    _check(lib().sgbem_assemble(ctx, c.ref(), rules, int(method), int(n_gauss), int(precision),
                                ctypes.c_void_p(d_A_ptr), int(lda)))


def sgbem_assemble_noalloc(ctx, curve, rules, precision, d_A_ptr, lda):
    c = _as_curve(curve)
    _check(lib().sgbem_assemble_noalloc(ctx, c.ref(), rules, int(precision), ctypes.c_void_p(d_A_ptr), int(lda)))


def sgbem_rhs(ctx, curve, rules, method, n_gauss, d_g_ptr, d_beta_ptr):
    c = _as_curve(curve)
    _check(lib().sgbem_rhs(ctx, c.ref(), rules, int(method), int(n_gauss), ctypes.c_void_p(d_g_ptr),
                           ctypes.c_void_p(d_beta_ptr)))


def sgbem_solve(ctx, N, d_A_ptr, lda, a_prec, d_beta_ptr, d_x_ptr, tol=1e-12, max_iter=30, check=True):
    info = sgbem_solve_info()
    st = lib().sgbem_solve(ctx, int(N), ctypes.c_void_p(d_A_ptr), int(lda), int(a_prec), ctypes.c_void_p(d_beta_ptr),
                           ctypes.c_void_p(d_x_ptr), float(tol), int(max_iter), ctypes.byref(info))
    if check:
        _check(st)
    return st, info


def sgbem_batch_create(ctx, curves, rules, precision, d_A_ptrs, ldas):
    """curves: list of curve descriptions; rules: list of handles; d_A_ptrs / ldas: lists."""
    n = len(curves)
    cs = [_as_curve(c) for c in curves]
    arr = (sgbem_curve * n)(*[c.c for c in cs])
    rl = (ctypes.c_void_p * n)(*[r.value for r in rules])
    ptrs = (ctypes.c_void_p * n)(*d_A_ptrs)
    ld = (ctypes.c_int64 * n)(*ldas)
    h = ctypes.c_void_p()
    _check(lib().sgbem_batch_create(ctx, n, arr, rl, int(precision), ptrs, ld, ctypes.byref(h)))
    h._keep = (cs, arr)
    return h


def sgbem_batch_assemble(ctx, batch):
    _check(lib().sgbem_batch_assemble(ctx, batch))


def sgbem_batch_tune(ctx, batch, reps=3):
    cfg, ms = ctypes.c_int32(), ctypes.c_double()
    _check(lib().sgbem_batch_tune(ctx, batch, int(reps), ctypes.byref(cfg), ctypes.byref(ms)))
    return cfg.value, ms.value


def sgbem_batch_free(ctx, batch):
    _check(lib().sgbem_batch_free(ctx, batch))


# ------------------------------------------------------------------ host node points, serving
def sgbem_node_points_host(curve, N, n_ref=1):
    """f(n / (2 n_ref N)) as an array [2 n_ref N, 2] (host evaluation)."""
    c = _as_curve(curve)
    xy = np.zeros((2 * n_ref * N, 2))
    _check(lib().sgbem_node_points_host(c.ref(), int(N), int(n_ref),
                                        xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return xy


def sgbem_server_footprint(N, precision=SGBEM_FP64):
    b = ctypes.c_int64()
    _check(lib().sgbem_server_footprint(int(N), int(precision), ctypes.byref(b)))
    return b.value


def sgbem_server_create(device=0, workers=4, budget_bytes=8 << 30, precision=SGBEM_FP64, max_N=8192,
                        max_rules=256, max_iter=30, tol=1e-12):
    cfg = sgbem_server_config(int(device), int(workers), int(budget_bytes), int(precision), int(max_N),
                              int(max_rules), int(max_iter), float(tol))
    h = ctypes.c_void_p()
    _check(lib().sgbem_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def sgbem_server_submit(server, curve, p, N, g, x, arrival_s, tag):
    """g: float64 host array [2N] (copied by the call); x: float64 host array [N]
    that receives alpha and must stay alive until the request's completion."""
    c = _as_curve(curve)
    g = np.ascontiguousarray(g, dtype=np.float64)
    if g.size != 2 * N or x.dtype != np.float64 or x.size != N or not x.flags["C_CONTIGUOUS"]:
        raise ValueError("g must have 2N and x N contiguous float64 entries")
    dp = ctypes.POINTER(ctypes.c_double)
    r = sgbem_request(c.c, int(p), int(N), g.ctypes.data_as(dp), x.ctypes.data_as(dp), float(arrival_s),
                      int(tag))
    _check(lib().sgbem_server_submit(server, ctypes.byref(r)))


def sgbem_server_poll(server, cap=64, timeout_s=0.0):
    buf = (sgbem_completion * cap)()
    n = ctypes.c_int32()
    _check(lib().sgbem_server_poll(server, buf, int(cap), float(timeout_s), ctypes.byref(n)))
    return [buf[i] for i in range(n.value)]


def sgbem_server_clock(server):
    t = ctypes.c_double()
    _check(lib().sgbem_server_clock(server, ctypes.byref(t)))
    return t.value


def sgbem_server_stats(server):
    info = sgbem_server_info()
    _check(lib().sgbem_server_stats(server, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in sgbem_server_info._fields_}


def sgbem_server_destroy(server):
    _check(lib().sgbem_server_destroy(server))


def sgbem_rhs_direct(ctx, curve, rules, n_gauss, d_g_nodes_ptr, d_g_gauss_ptr, d_F_ptr, d_b2_ptr=None):
    c = _as_curve(curve)
    _check(lib().sgbem_rhs_direct(ctx, c.ref(), rules, int(n_gauss), ctypes.c_void_p(d_g_nodes_ptr),
                                  ctypes.c_void_p(d_g_gauss_ptr), ctypes.c_void_p(d_F_ptr),
                                  ctypes.c_void_p(d_b2_ptr) if d_b2_ptr else None))


def sgbem_assemble_collocation(ctx, curve, rules, d_A_ptr, lda):
    c = _as_curve(curve)
    _check(lib().sgbem_assemble_collocation(ctx, c.ref(), rules, ctypes.c_void_p(d_A_ptr), int(lda)))


def sgbem_collocation_rhs(ctx, rules, d_g_nodes_ptr, d_b_ptr):
    _check(lib().sgbem_collocation_rhs(ctx, rules, ctypes.c_void_p(d_g_nodes_ptr), ctypes.c_void_p(d_b_ptr)))
