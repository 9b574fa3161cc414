"""O2: element-by-element Galerkin assembly, eq. elbyelint (test infrastructure only).

Python side: geometry at the Gauss points (``curves``), the reference
matrices of the log part (``nearfield``) and a ctypes call into the plain C
loop ``ebe_oracle.c``.  The right-hand side of eq. final_b1 is integrated with
the same G-point Gauss rule per element.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import bspline, curves, nearfield

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ebe_oracle.c")
_LIB = os.path.join(_HERE, "libebe_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no device code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        ci = ctypes.c_int
        lib.oracle_ebe_entries.restype = ci
        lib.oracle_ebe_entries.argtypes = [ci, ci,
                                           ci, d, d, d, d, d,
                                           ci, d, d, d, d, d,
                                           ci, d, d, d,
                                           d, d,
                                           ctypes.c_int64, i32, i32, d, ci]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


class EBEProblem:
    """Geometry sampled once for (curve, N, G, Gn, Gs)."""

    def __init__(self, curve, p: int, N: int, G: int, Gn: int = 16, Gs: int = 16):
        self.p, self.N, self.G, self.Gn, self.Gs = p, N, G, Gn, Gs
        e = np.arange(N)[:, None]
        self.gu, self.gw = gauss01(G)
        self.nu, self.nw = gauss01(Gn)
        self.su, self.sw, self.Mco, self.Madj = nearfield.reference_matrices(Gs)
        x, y, _, _, J = curves.evaluate(curve, ((e + self.gu[None, :]) / N).ravel())
        self.gx, self.gy, self.gJ = [np.ascontiguousarray(v) for v in (x, y, J)]
        x, y, _, _, J = curves.evaluate(curve, ((e + self.nu[None, :]) / N).ravel())
        self.nx, self.ny, self.nJ = [np.ascontiguousarray(v) for v in (x, y, J)]
        _, _, _, _, J = curves.evaluate(curve, ((e + self.su[None, :]) / N).ravel())
        self.sJ = np.ascontiguousarray(J)
        self.curve = curve

    def entries(self, ii, jj, nthreads: int | None = None):
        """A_{ii[k], jj[k]}; returns (values, threads used)."""
        ii = np.ascontiguousarray(ii, dtype=np.int32).ravel()
        jj = np.ascontiguousarray(jj, dtype=np.int32).ravel()
        out = np.empty(ii.size, dtype=np.float64)
        if nthreads is None:
            nthreads = os.cpu_count() or 1
        lib = _load()
        used = lib.oracle_ebe_entries(
            self.p, self.N,
            self.G, _ptr(self.gu), _ptr(self.gw), _ptr(self.gx), _ptr(self.gy), _ptr(self.gJ),
            self.Gn, _ptr(self.nu), _ptr(self.nw), _ptr(self.nx), _ptr(self.ny), _ptr(self.nJ),
            self.Gs, _ptr(self.su), _ptr(self.sw), _ptr(self.sJ),
            _ptr(np.ascontiguousarray(self.Mco)), _ptr(np.ascontiguousarray(self.Madj)),
            ii.size, ii.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            jj.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(out), int(nthreads))
        self.threads_used = used
        return out

    def rows(self, rows, nthreads: int | None = None) -> np.ndarray:
        rows = np.asarray(rows, dtype=np.int32)
        ii = np.repeat(rows, self.N)
        jj = np.tile(np.arange(self.N, dtype=np.int32), rows.size)
        return self.entries(ii, jj, nthreads).reshape(rows.size, self.N)

    def matrix(self, nthreads: int | None = None) -> np.ndarray:
        return self.rows(np.arange(self.N), nthreads)

    def rhs(self, g) -> np.ndarray:
        """beta_i = int B_i J g(f) ds by the G-point Gauss rule on each element."""
        p, N = self.p, self.N
        x, y, J = (self.gx.reshape(N, self.G), self.gy.reshape(N, self.G), self.gJ.reshape(N, self.G))
        gv = g(x, y)
        beta = np.zeros(N)
        for i in range(N):
            for a in range(p + 1):
                e = (i + a) % N
                beta[i] += np.sum(self.gw * bspline.cardinal(p, a + self.gu) * J[e] * gv[e]) / N
        return beta


def matrix(curve, p, N, G, Gn=16, Gs=16, nthreads=None):
    return EBEProblem(curve, p, N, G, Gn, Gs).matrix(nthreads)
