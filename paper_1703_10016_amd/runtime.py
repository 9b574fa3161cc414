"""Torch-side convenience wrapper over the C ABI: device buffers come from
torch, every computation is a libsgbem call on the context's stream."""
from __future__ import annotations

import numpy as np

from . import sgbem as S

_METHODS = {"wq": S.SGBEM_WQ, "ebe": S.SGBEM_EBE}
_PREC = {"fp64": S.SGBEM_FP64, "fp32": S.SGBEM_FP32}


class Context:
    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = S.sgbem_ctx_create(device, self.stream.cuda_stream, hbm_budget_bytes)
        self._rules = {}

    def close(self):
        if self.ctx is not None:
            S.sgbem_ctx_destroy(self.ctx)
            self.ctx = None
            self._rules = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def rules(self, p: int, N: int, n_ref: int = 1, knots=None):
        """Rules handle of (p, N, n_ref) on uniform knots, or on the given knot
        vector of N + 1 breakpoints (cached per knot vector)."""
        key = (p, N, n_ref) if knots is None else (p, N, n_ref, np.asarray(knots, dtype=np.float64).tobytes())
        if key not in self._rules:
            self._rules[key] = S.sgbem_weights(self.ctx, p, N, n_ref, knots)
        return self._rules[key]

    def assemble(self, curve, p, N, method="wq", n_ref=1, n_gauss=6, precision="fp64", out=None, knots=None):
        dt = self.torch.float64 if precision == "fp64" else self.torch.float32
        if out is None:
            out = self.torch.empty((N, N), dtype=dt, device=self.device)
        assert out.dtype == dt and out.is_cuda and out.stride(1) == 1 and out.shape[0] >= N
        S.sgbem_assemble(self.ctx, curve, self.rules(p, N, n_ref, knots), _METHODS[method], n_gauss, _PREC[precision],
                         out.data_ptr(), out.stride(0))
        return out

    def rhs_points(self, curve, p, N, method="wq", n_ref=1, n_gauss=6, knots=None):
        count = 2 * n_ref * N if method == "wq" else N * n_gauss
        xy = self.torch.empty((count, 2), dtype=self.torch.float64, device=self.device)
        S.sgbem_rhs_points(self.ctx, curve, self.rules(p, N, n_ref, knots), _METHODS[method], n_gauss, xy.data_ptr(),
                           count)
        return xy

    def sample(self, g, xy):
        """The Dirichlet datum at the library's points (evaluated by the caller)."""
        self.stream.synchronize()
        h = xy.cpu().numpy()
        return self.torch.from_numpy(np.ascontiguousarray(g(h[:, 0], h[:, 1]), dtype=np.float64)).to(self.device)

    def rhs(self, curve, p, N, g, method="wq", n_ref=1, n_gauss=6, knots=None):
        gv = self.sample(g, self.rhs_points(curve, p, N, method, n_ref, n_gauss, knots))
        beta = self.torch.empty(N, dtype=self.torch.float64, device=self.device)
        S.sgbem_rhs(self.ctx, curve, self.rules(p, N, n_ref, knots), _METHODS[method], n_gauss, gv.data_ptr(),
                    beta.data_ptr())
        return beta

    # ---- open arcs (exterior problem, indirect form): N = n_el + p unknowns
    def rules_open(self, p: int, breaks, n_ref: int = 1):
        """Open-arc rules on the breakpoints breaks[0] = a < ... < breaks[n_el] = b (cached)."""
        b = np.ascontiguousarray(breaks, dtype=np.float64)
        key = ("open", p, n_ref, b.tobytes())
        if key not in self._rules:
            self._rules[key] = S.sgbem_weights_open(self.ctx, p, b, n_ref)
        return self._rules[key]

    def assemble_arc(self, curve, p, breaks, n_ref=1, out=None):
        N = len(breaks) - 1 + p
        if out is None:
            out = self.torch.empty((N, N), dtype=self.torch.float64, device=self.device)
        assert out.dtype == self.torch.float64 and out.is_cuda and out.stride(1) == 1 and out.shape[0] >= N
        S.sgbem_assemble(self.ctx, curve, self.rules_open(p, breaks, n_ref), S.SGBEM_WQ, 0, S.SGBEM_FP64,
                         out.data_ptr(), out.stride(0))
        return out

    def rhs_points_arc(self, curve, p, breaks, n_ref=1):
        count = 2 * p + 2 * n_ref * (len(breaks) - 1) - 1
        xy = self.torch.empty((count, 2), dtype=self.torch.float64, device=self.device)
        S.sgbem_rhs_points(self.ctx, curve, self.rules_open(p, breaks, n_ref), S.SGBEM_WQ, 0, xy.data_ptr(), count)
        return xy

    def rhs_arc(self, curve, p, breaks, uD, n_ref=1):
        """F_i = int B_i J u_D on the arc (indirect form) by the regular rule."""
        gv = self.sample(uD, self.rhs_points_arc(curve, p, breaks, n_ref))
        beta = self.torch.empty(len(breaks) - 1 + p, dtype=self.torch.float64, device=self.device)
        S.sgbem_rhs(self.ctx, curve, self.rules_open(p, breaks, n_ref), S.SGBEM_WQ, 0, gv.data_ptr(), beta.data_ptr())
        return beta

    def rhs_direct(self, curve, p, N, g, n_gauss=4, n_ref=1, with_b2=False):
        """F = b1/2 - b2/(2 pi) of the direct formulation (and b2 when asked)."""
        gn = self.sample(g, self.rhs_points(curve, p, N, "wq", n_ref))
        gg = self.sample(g, self.rhs_points(curve, p, N, "ebe", n_ref, n_gauss))
        F = self.torch.empty(N, dtype=self.torch.float64, device=self.device)
        b2 = self.torch.empty(N, dtype=self.torch.float64, device=self.device) if with_b2 else None
        S.sgbem_rhs_direct(self.ctx, curve, self.rules(p, N, n_ref), n_gauss, gn.data_ptr(), gg.data_ptr(),
                           F.data_ptr(), b2.data_ptr() if with_b2 else None)
        return (F, b2) if with_b2 else F

    def assemble_collocation(self, curve, p, N, n_ref=1, out=None):
        """The collocation matrix (FP64, not symmetric) at the Greville abscissae."""
        if out is None:
            out = self.torch.empty((N, N), dtype=self.torch.float64, device=self.device)
        S.sgbem_assemble_collocation(self.ctx, curve, self.rules(p, N, n_ref), out.data_ptr(), out.stride(0))
        return out

    def collocation_rhs(self, curve, p, N, g, n_ref=1):
        gn = self.sample(g, self.rhs_points(curve, p, N, "wq", n_ref))
        b = self.torch.empty(N, dtype=self.torch.float64, device=self.device)
        S.sgbem_collocation_rhs(self.ctx, self.rules(p, N, n_ref), gn.data_ptr(), b.data_ptr())
        return b

    def solve(self, A, beta, tol=1e-12, max_iter=30, check=True):
        N = A.shape[0]
        prec = S.SGBEM_FP64 if A.dtype == self.torch.float64 else S.SGBEM_FP32
        x = self.torch.empty(N, dtype=self.torch.float64, device=self.device)
        st, info = S.sgbem_solve(self.ctx, N, A.data_ptr(), A.stride(0), prec, beta.data_ptr(), x.data_ptr(),
                                 tol, max_iter, check=check)
        return x, info
