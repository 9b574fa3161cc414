#!/usr/bin/env python3
"""Galerkin entries/s of the weighted-quadrature row assembly against the
element-by-element Gauss assembly at equal solution error, on one MI355X.

Workload: the ellipse with semi-axes (1, 0.5) as a closed cubic B-spline of 32
control points, periodic B-splines p = 3 on N = 1024 elements, FP64,
g = exp(x1) cos(x2).  A step is one assembly of the full 1024 x 1024 matrix by
the fast form (node-grid geometry kernel + fused sweep-and-contract kernel),
with the curve and the quadrature rules resident on the device.  K steps are
captured in one HIP graph and replayed once inside the timed region.

Also measured in the same run (reported beside the headline value):
 * the element-by-element form at the smallest Gauss order whose solution
   error is not larger than the fast form's (errors of the coefficient vector
   against an element-by-element G = 8 solution), and the speedup;
 * latency of a solve request (assemble + right-hand side + mixed-precision
   solve: FP32 explicit inverse by Gauss-Jordan, FP64 refinement), p50 / p99
   over repeated requests;
 * the fused kernel's duration from HIP events on its stream -> roofline;
 * FP32 and FP64 throughput at N = 16384 (a star curve, one assembly each);
 * a grid of star curves, 8 per point, p in {2, 3, 4} and N in {4096, 16384}:
   FP32 assembly, then FP32 LU + FP64 refinement of that matrix to 1e-10;
 * the direct formulation's right-hand side (double-layer sweep, eq. final_b2)
   at the workload and at N = 16384;
 * collocation BEM with the same rules at the workload and at N = 16384;
 * a batch of 256 star curves (N in [128, 2048], p in {2, 3}, FP32) in one
   autotuned persistent launch replayed from a HIP graph, against 256
   sequential single-curve launches;
 * the CPU oracle (element-by-element, FP64, C + OpenMP) on a sample of rows,
   and the oracle's G = 24 solution as a second reference of the equal-error
   comparison;
 * a serving sweep (Poisson arrivals at 10 .. 1000 req/s, about 10 s of
   arrivals per rate, 100 to 2000 requests);
 * the general-rule paths: the parabola test on an open arc (Table 2's largest
   case, DoF 642, and the largest singular table, 8191 nodes) and a closed
   curve on graded non-uniform periodic knots (N = 1024 and 4096): rule
   construction on the host, the assembly kernel, right-hand side and solve,
   and for the arc E_R / E_M against the exact density.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12          # MI355X FP64 vector, FLOP/s
PEAK_FP32 = 157.3e12         # MI355X FP32, vector and dense MFMA alike, FLOP/s
PEAK_HBM = 8.0e12            # bytes/s
FLOPS_PER_LOG = 20           # cost model of one FP64 logarithm (the table-free series: ~20 FP64 operations)
DL_FLOPS_PER_EVAL = 11       # double-layer kernel value: 2 differences, numerator and denominator (3 each), 1 division, 1 multiply-add


def wq_flops_per_entry(p: int, R: int) -> float:
    """Algorithmic flops per matrix entry of the fast form: stage 1 and stage 2
    contractions, (4R + 1) Q multiply-adds, Q = 2R(p+1) - 1 (2 flops each), and
    4R^2 kernel evaluations on the node grid (difference, squared distance,
    scaling: 6 flops + one logarithm)."""
    Q = 2 * R * (p + 1) - 1
    return 2.0 * (4 * R + 1) * Q + 4.0 * R * R * (6 + FLOPS_PER_LOG)


def ebe_flops_per_entry(p: int, G: int) -> float:
    """Element-by-element far part: G^2 kernel evaluations (5 flops + log) and
    (p+1) G^2 + (p+1) G multiply-adds per entry (sum factorised)."""
    return G * G * (5 + FLOPS_PER_LOG) + 2.0 * ((p + 1) * G * G + (p + 1) * G)


def kernel_source_hash() -> str:
    """Hash of the sources of the headline kernel: the tile kernel's headers and
    the dispatch line of its instance (p = 3, n_ref = 1 in FP64)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1703_10016_amd", "csrc")
    for f in ("tile_kernel.hpp", "kernels.hpp", "log_table.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "asm_wq_f64.hip"), "rb") as fh:
        h.update(b"".join(l for l in fh.read().splitlines(True) if l.lstrip().startswith(b"case 50:")))
    return h.hexdigest()[:16]


def write_traffic(fetch_csv: str, write_csv: str, path: str | None = None) -> dict:
    """HBM bytes per launch of the fused kernel from two counter runs of
    `--profile-run`: each counter (KiB per dispatch) is scaled by the ratio of the
    256 MiB that the run's copy kernel moves to what the counter reads for it."""
    import csv
    copy_kib = 32 * 1024 * 1024 * 8 / 1024.0

    def per_dispatch(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
        fused = [v for (d, n), v in vals.items() if "tile_kernel<2, 7, 1, true, double, double" in n]
        # the copy is the run's last dispatch (the fill of its source, before it, writes as much)
        big = sorted((int(d), v) for (d, n), v in vals.items() if "tile_kernel" not in n and v > 0.25 * copy_kib)
        if not fused or not big:
            raise SystemExit(f"{path}: {len(fused)} fused dispatches, no 256 MiB copy")
        return sum(fused) / len(fused), big[-1][1]

    f_kib, f_copy = per_dispatch(fetch_csv, "FETCH_SIZE")
    w_kib, w_copy = per_dispatch(write_csv, "WRITE_SIZE")
    fs, ws = copy_kib / f_copy, copy_kib / w_copy
    out = {"bytes_per_launch": (f_kib * fs + w_kib * ws) * 1024.0, "fetch_kib_scaled": f_kib * fs,
           "write_kib_scaled": w_kib * ws, "fetch_scale": fs, "write_scale": ws,
           "fetch_kib_raw": f_kib, "write_kib_raw": w_kib, "copy_fetch_kib_raw": f_copy, "copy_write_kib_raw": w_copy,
           "source_hash": kernel_source_hash()}
    path = path or os.path.join(ROOT, "profiles", "wq_fp64_ellipse_N1024_traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))
    return out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def requests_for_rate(rate, n_req, seconds):
    """Requests sent at one arrival rate: n_req if given, else the rate times an
    arrival window of `seconds`, between 100 and 2000 (at least 1000 completions
    from 100 req/s up, so that p99 is a percentile and not the largest sample)."""
    if n_req > 0:
        return n_req
    return int(min(2000, max(100, round(rate * seconds))))


def serve_sweep(S, rates, n_req, workers, seconds=10.0, one_at_a_time=True):
    """Open-loop serving: for each rate, star requests with Poisson arrivals
    (N log-uniform in [256, 8192], p in {2, 3, 4}) go to one server; each is
    assembled (fast form, FP64), its right-hand side formed and solved (FP32
    factor + FP64 refinement).  Latency runs from the request's arrival to
    alpha in host memory; solves/s is completions over the span from the
    first arrival to the last completion."""
    import synth
    budget = 24 << 30
    out = {"workers": workers, "budget_bytes": budget,
           "requests_per_rate": {str(r): requests_for_rate(r, n_req, seconds) for r in rates},
           "matrix_precision": "fp64"}
    out["rates"] = []
    rows_by_workers = {}
    for w in ([workers, 1] if one_at_a_time else [workers]):
        out_w = _serve_rates(S, rates if w == workers else rates[-1:], n_req, w, budget, seconds)
        rows_by_workers[w] = out_w
    out["rates"] = rows_by_workers[workers]
    if one_at_a_time:
        one = rows_by_workers[1][0]
        top = rows_by_workers[workers][-1]
        out["one_at_a_time"] = one
        out["speedup_vs_one_at_a_time"] = top["solves_per_s"] / one["solves_per_s"]
        log(f"[bench] serving at {one['rate']:g} req/s: {workers} slots {top['solves_per_s']:.1f} solves/s vs one at a "
            f"time {one['solves_per_s']:.1f} solves/s -> {out['speedup_vs_one_at_a_time']:.2f}x (same results: "
            f"every kernel reduces in a fixed order)")
    return out


def _serve_rates(S, rates, n_req, workers, budget, seconds):
    import synth
    rows = []
    srv = S.sgbem_server_create(workers=workers, budget_bytes=budget, precision=S.SGBEM_FP64, max_N=8192,
                                max_rules=512, max_iter=30, tol=1e-12)
    try:
        # warm every kernel the path launches (one request per degree), untimed
        warm = [(synth.star(1), p, 512) for p in (2, 3, 4)]
        xw = [np.zeros(512) for _ in warm]
        for i, (cv, p, N) in enumerate(warm):
            xy = S.sgbem_node_points_host(cv, N, 1)
            S.sgbem_server_submit(srv, cv, p, N, synth.g_exp_cos(xy[:, 0], xy[:, 1]), xw[i], 0.0, i)
        _serve_drain(S, srv, len(warm))
        for rate in rates:
            arrivals, probs = synth.config_serving(rate, requests_for_rate(rate, n_req, seconds))
            gs = []
            for pb in probs:   # the client's boundary data at the fast form's node points
                xy = S.sgbem_node_points_host(pb.curve, pb.N, 1)
                gs.append(pb.g(xy[:, 0], xy[:, 1]))
            xs = [np.zeros(pb.N) for pb in probs]
            before = S.sgbem_server_stats(srv)
            t0 = S.sgbem_server_clock(srv) + 0.05
            for i, pb in enumerate(probs):
                S.sgbem_server_submit(srv, pb.curve, pb.p, pb.N, gs[i], xs[i], t0 + float(arrivals[i]), i)
            comp = _serve_drain(S, srv, len(probs))
            after = S.sgbem_server_stats(srv)
            ok = [c for c in comp if c.status == 0]
            lat = np.array([c.t_done - c.t_arrival for c in ok]) * 1e3
            span = max(c.t_done for c in comp) - t0
            row = {"rate": rate, "completed": len(comp), "ok": len(ok),
                   "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "solves_per_s": len(comp) / span,
                   "mean_entries": float(np.mean([pb.N ** 2 for pb in probs])),
                   "mean_queue_ms": float(np.mean([(c.t_admit - c.t_arrival) * 1e3 for c in ok])),
                   "peak_in_flight": after["peak_in_flight"], "peak_bytes": after["peak_bytes"],
                   "rules_misses": after["rules_misses"] - before["rules_misses"]}
            rows.append(row)
            log(f"[bench] serving ({workers} slot{'s' if workers > 1 else ''}) rate {rate:g}/s x {len(probs)}: "
                f"p50 {row['p50_ms']:.2f} ms p99 {row['p99_ms']:.2f} ms, "
                f"{row['solves_per_s']:.1f} solves/s, queue {row['mean_queue_ms']:.1f} ms, "
                f"{len(ok)}/{len(comp)} ok")
    finally:
        S.sgbem_server_destroy(srv)
    return rows


def _serve_drain(S, srv, n, timeout=900.0):
    got = []
    t_end = time.time() + timeout
    t_log = time.time() + 30.0
    while len(got) < n:
        if time.time() > t_end:
            raise RuntimeError(f"serving: {len(got)} of {n} completions before the time limit")
        got += S.sgbem_server_poll(srv, 256, 1.0)
        if time.time() > t_log:     # progress of long sweeps (2000 requests at 10 req/s take 200 s)
            log(f"[bench] serving: {len(got)} of {n} requests completed")
            t_log = time.time() + 30.0
    return got


def _timed_kernel(S, ctx, fn, reps):
    """Average duration of the assembly kernel of fn() (HIP events of its own dispatch)."""
    fn()
    S.sgbem_ctx_set_timing(ctx.ctx, 1)
    for _ in range(reps):
        fn()
    tms, cnt = S.sgbem_ctx_kernel_time(ctx.ctx)
    S.sgbem_ctx_set_timing(ctx.ctx, 0)
    return tms / cnt


def general_rules(ctx, S, synth, torch, stream):
    """Open arcs (the parabola test of Section 6) and non-uniform periodic knots: per-row rules and the
    full singular table.  Flops per entry as for the uniform fast form (wq_flops_per_entry); the arc
    computes every entry (N^2), the closed curve the upper triangle (N(N+1)/2)."""
    from scipy.interpolate import BSpline

    def arc_errors(br, d, alpha):
        """E_R (relative L2 error, 8-point Gauss per element) and E_M (maximum on 500 uniform points) of
        phi_h = sum_j alpha_j B_j against the exact density sqrt(1 + 4 t^2) of the parabola test."""
        T = np.concatenate([np.full(d, br[0]), br, np.full(d, br[-1])])
        phi_h = BSpline(T, alpha, d)
        gu, gw = np.polynomial.legendre.leggauss(8)
        h = np.diff(br)
        tq = (br[:-1, None] + h[:, None] * (gu[None, :] + 1) / 2).ravel()
        wq = (h[:, None] * gw[None, :] / 2).ravel()
        e = phi_h(tq) - synth.parabola_phi(tq)
        tu = np.linspace(br[0], br[-1], 500)
        return (math.sqrt(np.sum(wq * e * e) / np.sum(wq * synth.parabola_phi(tq) ** 2)),
                float(np.abs(phi_h(tu) - synth.parabola_phi(tu)).max()))

    out = {"open_arc": [], "knots": []}
    for d, n in ((2, 640), (2, 4094)):
        br = np.linspace(-1.0, 1.0, n + 1)
        cur = synth.parabola()
        Nd = n + d
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.rules_open(d, br)
        t_rules = time.perf_counter() - t0
        A = torch.empty((Nd, Nd), dtype=torch.float64, device="cuda")
        kms = _timed_kernel(S, ctx, lambda: ctx.assemble_arc(cur, d, br, out=A), 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.assemble_arc(cur, d, br, out=A)
        beta = ctx.rhs_arc(cur, d, br, synth.parabola_uD)
        x, info = ctx.solve(A, beta, tol=1e-12, max_iter=30)
        torch.cuda.synchronize()
        t_req = time.perf_counter() - t0
        ER, EM = arc_errors(br, d, x.cpu().numpy())
        fl = float(Nd) * Nd * wq_flops_per_entry(d, 1)
        row = {"workload": f"parabola x2 = 1 - x1^2, d={d}, n_el={n} (DoF {Nd}, {2 * d + 2 * n - 1} nodes), n_ref=1",
               "rules_build_ms": t_rules * 1e3, "assembly_kernel_us": kms * 1e3,
               "entries_per_s": Nd * Nd / (kms * 1e-3), "tflops": fl / (kms * 1e-3) / 1e12,
               "frac_of_fp64_peak": fl / (kms * 1e-3) / PEAK_FP64,
               "request_ms": t_req * 1e3, "request": "assemble + rhs (host-sampled u_D) + solve",
               "solve_pivoted": int(info.pivoted), "E_R": ER, "E_M": EM}
        out["open_arc"].append(row)
        log(f"[bench] open arc {row['workload']}: rules {t_rules*1e3:.1f} ms, kernel {kms*1e3:.1f} us "
            f"({row['entries_per_s']:.3e} entries/s, {row['tflops']:.2f} TFLOP/s), request {t_req*1e3:.2f} ms, "
            f"E_R {ER:.3e}, E_M {EM:.3e}")
        del A
        S.sgbem_rules_free(ctx.ctx, ctx._rules.pop(("open", d, 1, np.ascontiguousarray(br).tobytes())))
    for Nk in (1024, 4096):
        u = np.arange(Nk + 1) / Nk
        tau = u + 0.3 * np.sin(2 * math.pi * u) / (2 * math.pi)
        tau[0], tau[-1] = 0.0, 1.0
        crv, pk = synth.ellipse_bspline_nonuniform(0), 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.rules(pk, Nk, 1, tau)
        t_rules = time.perf_counter() - t0
        A = torch.empty((Nk, Nk), dtype=torch.float64, device="cuda")
        kms = _timed_kernel(S, ctx, lambda: ctx.assemble(crv, pk, Nk, "wq", out=A, knots=tau), 10)
        fl = Nk * (Nk + 1) / 2 * wq_flops_per_entry(pk, 1)
        row = {"workload": f"ellipse on graded periodic knots (32-point cubic net), p={pk}, N={Nk}, n_ref=1",
               "rules_build_ms": t_rules * 1e3, "assembly_kernel_us": kms * 1e3,
               "entries_per_s": Nk * Nk / (kms * 1e-3), "tflops": fl / (kms * 1e-3) / 1e12,
               "frac_of_fp64_peak": fl / (kms * 1e-3) / PEAK_FP64}
        out["knots"].append(row)
        log(f"[bench] knots {row['workload']}: rules {t_rules*1e3:.1f} ms, kernel {kms*1e3:.1f} us "
            f"({row['entries_per_s']:.3e} entries/s, {row['tflops']:.2f} TFLOP/s)")
        del A
        S.sgbem_rules_free(ctx.ctx, ctx._rules.pop((pk, Nk, 1, np.asarray(tau, dtype=np.float64).tobytes())))
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="skip the N = 16384 points")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-curve batch")
    ap.add_argument("--no-stars", action="store_true",
                    help="skip the star grid (8 curves per p in {2, 3, 4} and N in {4096, 16384}, FP32)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop sweep")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests per arrival rate (0: the rate times --serve-seconds, within [100, 2000])")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="arrival window per rate when --serve-requests is 0")
    ap.add_argument("--serve-rates", type=str, default="10,30,100,300,1000", help="arrival rates, req/s")
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--solves", type=int, default=60)
    ap.add_argument("--no-general", action="store_true", help="skip the open-arc and non-uniform-knot paths")
    ap.add_argument("--profile-run", action="store_true",
                    help="only K direct WQ assemblies of the workload and one 256 MiB device copy "
                         "(the copy calibrates the byte counters of a profiler run)")
    ap.add_argument("--profile-n", type=int, default=0,
                    help="with --profile-run: assemble the star curve (p = 3) at this N instead of the workload")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="no GPU work: turn the counter CSVs of two profiler runs of --profile-run (FETCH_SIZE, "
                         "then WRITE_SIZE) into profiles/wq_fp64_ellipse_N1024_traffic.json, scaling each "
                         "counter by what it reads for the run's 256 MiB copy")
    ap.add_argument("--profile-solve", type=int, default=0,
                    help="profiling only: assemble the star curve (p = 3) at this N in FP32 and solve it W + K times")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (the matrix would be "
              "sharded by row blocks of tiles, each GPU assembling and factoring its own rows).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1703_10016_amd import sgbem as S
    from paper_1703_10016_amd.runtime import Context

    assert torch.cuda.is_available(), "no GPU visible"
    K, W = args.steps, args.warmup
    prob = synth.config_ellipse()
    curve, p, N, g = prob.curve, prob.p, prob.N, prob.g
    R = 1
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = Context(0, stream=stream)

    t0 = time.perf_counter()
    ctx.rules(p, N, R)
    t_rules = time.perf_counter() - t0
    if args.profile_solve:
        Ns = args.profile_solve
        star = synth.star(0)
        A = torch.empty((Ns, Ns), dtype=torch.float32, device="cuda")
        ctx.assemble(star, p, Ns, "wq", n_ref=R, precision="fp32", out=A)
        bb = ctx.rhs(star, p, Ns, g, method="wq", n_ref=R)
        for _ in range(W + K):
            xb, sinfo = ctx.solve(A, bb, tol=1e-10, max_iter=30)
        torch.cuda.synchronize()
        log(f"[bench] profile run: {W + K} solves of the N={Ns} star (FP32 matrix), {sinfo.iters} refinement steps")
        ctx.close()
        return
    if args.profile_run:
        if args.profile_n:
            curve, N = synth.star(0), args.profile_n
        A = torch.empty((N, N), dtype=torch.float64, device="cuda")
        for _ in range(W + K):
            ctx.assemble(curve, p, N, "wq", n_ref=R, out=A)
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                      # 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        log(f"[bench] profile run: {W + K} WQ assemblies, one copy of {src.numel() * 8} bytes")
        ctx.close()
        return
    log(f"[bench] rules (p={p}, N={N}, n_ref={R}) built in {t_rules*1e3:.1f} ms")

    # ---------------------------------------------------------------- equal error
    def solve_coeffs(method, **kw):
        A = ctx.assemble(curve, p, N, method, **kw)
        beta = ctx.rhs(curve, p, N, g, method=method, **kw)
        x, info = ctx.solve(A, beta, tol=1e-12, max_iter=30)
        return x.cpu().numpy()

    # Interior potential u_h(x) = sum_j alpha_j int B_j(t) (-1/2pi) ln|x - f(t)| J(t) dt: the
    # right-hand side routine (8-point Gauss per element, far from x) applied to the kernel as datum.
    # u = g inside the curve, so |u_h - g| at interior points measures the error without a reference.
    th = 2.0 * math.pi * np.arange(8) / 8
    xin = np.concatenate([0.3 * np.cos(th), 0.6 * np.cos(th + 0.2)])
    yin = np.concatenate([0.15 * np.sin(th), 0.3 * np.sin(th + 0.2)])
    g_in = g(xin, yin)
    cols = np.stack([ctx.rhs(curve, p, N, (lambda x, y, a=a, b=b: -np.log(np.hypot(x - a, y - b)) / (2 * math.pi)),
                             method="ebe", n_gauss=8).cpu().numpy() for a, b in zip(xin, yin)])
    interior_err = lambda a: float(np.abs(cols @ a - g_in).max() / np.abs(g_in).max())

    a_ref = solve_coeffs("ebe", n_gauss=8)
    err = lambda a: float(np.linalg.norm(a - a_ref) / np.linalg.norm(a_ref))
    sol_wq = {r: solve_coeffs("wq", n_ref=r) for r in (1, 2, 3, 4)}
    sol_ebe = {G: solve_coeffs("ebe", n_gauss=G) for G in (1, 2, 3, 4, 5, 6)}
    sol_ebe[8] = a_ref
    err_wq = err(sol_wq[R])
    err_ebe = {G: err(a) for G, a in sol_ebe.items() if G != 8}
    G_eq = next((G for G in sorted(err_ebe) if err_ebe[G] <= err_wq), 6)
    log(f"[bench] solution error vs EBE(G=8): WQ " + " ".join(f"n_ref={r}:{err(a):.3e}" for r, a in sol_wq.items()) +
        "; EBE " + " ".join(f"G={G}:{e:.3e}" for G, e in err_ebe.items()) + f" -> equal-error G = {G_eq}")
    log(f"[bench] interior potential error (16 points): WQ " +
        " ".join(f"n_ref={r}:{interior_err(a):.3e}" for r, a in sol_wq.items()) + "; EBE " +
        " ".join(f"G={G}:{interior_err(a):.3e}" for G, a in sorted(sol_ebe.items())))

    # ---------------------------------------------------------------- timed steps (graph replay)
    def graph_rate(method, steps, precision="fp64", **kw):
        A = torch.empty((N, N), dtype=torch.float64 if precision == "fp64" else torch.float32, device="cuda")
        kw = dict(kw, precision=precision)
        for _ in range(W):
            ctx.assemble(curve, p, N, method, out=A, **kw)
        torch.cuda.synchronize()
        gph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gph, stream=stream):
            for _ in range(steps):
                ctx.assemble(curve, p, N, method, out=A, **kw)
        gph.replay()                      # warm replay
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        gph.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        del gph
        return ms / steps, A

    ms_wq, A_wq = graph_rate("wq", K, n_ref=R)
    value = N * N / (ms_wq * 1e-3)
    log(f"[bench] WQ FP64 step {ms_wq*1e3:.2f} us -> {value:.3e} entries/s")
    ms_ebe, _ = graph_rate("ebe", max(10, K // 4), n_gauss=G_eq)
    ebe_rate = N * N / (ms_ebe * 1e-3)
    log(f"[bench] EBE FP64 G={G_eq} step {ms_ebe*1e3:.2f} us -> {ebe_rate:.3e} entries/s")

    # error-vs-time front of both forms, speedup at matched error by log-log interpolation
    front_steps = max(10, K // 4)
    t_wq = {r: (ms_wq if r == R else graph_rate("wq", front_steps, n_ref=r)[0]) for r in (1, 2, 3, 4)}
    t_ebe = {G: (ms_ebe if G == G_eq else graph_rate("ebe", front_steps, n_gauss=G)[0]) for G in (2, 3, 4, 6, 8)}
    front = {"wq": [{"n_ref": r, "us_per_step": t_wq[r] * 1e3, "solution_err": err(sol_wq[r]),
                     "interior_err": interior_err(sol_wq[r])} for r in t_wq],
             "ebe": [{"n_gauss": G, "us_per_step": t_ebe[G] * 1e3,
                      "solution_err": err_ebe.get(G), "interior_err": interior_err(sol_ebe[G])} for G in t_ebe]}

    def matched(key, e):
        """EBE step time at error e, log-log interpolated between the bracketing Gauss orders."""
        pts = [(row[key], row["us_per_step"]) for row in front["ebe"] if row[key]]   # by rising order
        for (e0, t0), (e1, t1) in zip(pts, pts[1:]):
            if e1 <= e <= e0:
                f = math.log(e / e0) / math.log(e1 / e0)
                return math.exp(math.log(t0) + f * math.log(t1 / t0))
        return None

    speedup_interp = {}
    for key in ("solution_err", "interior_err"):
        t_m = matched(key, front["wq"][R - 1][key])
        speedup_interp[key] = t_m / front["wq"][R - 1]["us_per_step"] if t_m else None
    for row in front["wq"]:
        log(f"[bench] front WQ n_ref={row['n_ref']}: {row['us_per_step']:.2f} us, solution err {row['solution_err']:.2e}, "
            f"interior err {row['interior_err']:.2e}")
    for row in front["ebe"]:
        se = f"{row['solution_err']:.2e}" if row["solution_err"] else "(reference)"
        log(f"[bench] front EBE G={row['n_gauss']}: {row['us_per_step']:.2f} us, solution err {se}, "
            f"interior err {row['interior_err']:.2e}")
    log(f"[bench] WQ vs EBE at matched error (log-interpolated): {speedup_interp}")

    # FP32 kernel evaluation and contraction (FP64 node differences and rule tables): rate and
    # error against the FP64 matrix (itself within 1e-12 of the oracle) and of the solution
    ms_wq32, A_wq32 = graph_rate("wq", K, precision="fp32", n_ref=R)
    A64h = A_wq.cpu().numpy()
    mat_err32 = float(np.abs(A_wq32.double().cpu().numpy() - A64h).max() / np.abs(A64h).max())
    beta_h = ctx.rhs(curve, p, N, g, method="wq", n_ref=R)
    x64, _ = ctx.solve(A_wq, beta_h, tol=1e-12, max_iter=30)
    x32, _ = ctx.solve(A_wq32, beta_h, tol=1e-12, max_iter=30)
    sol_err32 = float(np.linalg.norm((x32 - x64).cpu().numpy()) / np.linalg.norm(x64.cpu().numpy()))
    fp32 = {"ms_per_step": ms_wq32, "entries_per_s": N * N / (ms_wq32 * 1e-3),
            "matrix_rel_err_vs_fp64": mat_err32, "solution_rel_err_vs_fp64": sol_err32,
            "solution_err_vs_ebe8": err(x32.cpu().numpy())}
    log(f"[bench] WQ FP32 step {ms_wq32*1e3:.2f} us -> {N*N/(ms_wq32*1e-3):.3e} entries/s; matrix error vs FP64 "
        f"{mat_err32:.2e}, solution {sol_err32:.2e} (vs EBE G=8 reference {fp32['solution_err_vs_ebe8']:.2e})")
    del A_wq32

    # direct launches (host enqueue included), for reference
    A = torch.empty((N, N), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.assemble(curve, p, N, "wq", n_ref=R, out=A)
    torch.cuda.synchronize()
    ms_direct = (time.perf_counter() - t0) * 1e3 / K

    # ---------------------------------------------------------------- roofline of the fused kernel
    S.sgbem_ctx_set_timing(ctx.ctx, 1)
    for _ in range(K):
        ctx.assemble(curve, p, N, "wq", n_ref=R, out=A)
    tot_ms, cnt = S.sgbem_ctx_kernel_time(ctx.ctx)
    S.sgbem_ctx_set_timing(ctx.ctx, 0)
    kern_ms = tot_ms / cnt
    upper = N * (N + 1) / 2
    flops = upper * wq_flops_per_entry(p, R)
    achieved = flops / (kern_ms * 1e-3)
    log(f"[bench] fused WQ kernel {kern_ms*1e3:.2f} us avg over {cnt}: {achieved/1e12:.3f} TFLOP/s "
        f"({achieved/PEAK_FP64:.4f} of FP64 peak), write {8*N*N/(kern_ms*1e-3)/1e9:.1f} GB/s")
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "wq_fp64_ellipse_N1024_traffic.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tj = json.load(f)
        if tj.get("source_hash") == kernel_source_hash():   # counters only count for the kernel they measured
            traffic = tj.get("bytes_per_launch")

    # ---------------------------------------------------------------- solve latency
    xy = ctx.rhs_points(curve, p, N, "wq", n_ref=R)
    gv = ctx.sample(g, xy)
    beta = torch.empty(N, dtype=torch.float64, device="cuda")
    lat_req, lat_solve = [], []
    for it in range(args.solves + 3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.assemble(curve, p, N, "wq", n_ref=R, out=A)
        S.sgbem_rhs(ctx.ctx, curve, ctx.rules(p, N, R), S.SGBEM_WQ, 0, gv.data_ptr(), beta.data_ptr())
        t1 = time.perf_counter()
        x, info = ctx.solve(A, beta, tol=1e-12, max_iter=30)
        t2 = time.perf_counter()
        if it >= 3:
            lat_req.append((t2 - t0) * 1e3)
            lat_solve.append((t2 - t1) * 1e3)
    pct = lambda v, q: float(np.percentile(np.array(v), q))
    log(f"[bench] request latency p50 {pct(lat_req, 50):.3f} ms p99 {pct(lat_req, 99):.3f} ms; "
        f"solve p50 {pct(lat_solve, 50):.3f} p99 {pct(lat_solve, 99):.3f} ms ({info.iters} refinement steps)")

    # ---------------------------------------------------------------- N = 16384 scale points
    scale = {}
    if not args.no_scale:
        star = synth.star(0)
        Nb = 16384
        for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
            Ab = torch.empty((Nb, Nb), dtype=dt, device="cuda")
            ctx.assemble(star, p, Nb, "wq", n_ref=R, precision=prec, out=Ab)
            torch.cuda.synchronize()
            S.sgbem_ctx_set_timing(ctx.ctx, 1)
            reps = 3
            for _ in range(reps):
                ctx.assemble(star, p, Nb, "wq", n_ref=R, precision=prec, out=Ab)
            tms, c2 = S.sgbem_ctx_kernel_time(ctx.ctx)
            S.sgbem_ctx_set_timing(ctx.ctx, 0)
            kms = tms / c2
            fl = Nb * (Nb + 1) / 2 * wq_flops_per_entry(p, R)
            pk = PEAK_FP32 if prec == "fp32" else PEAK_FP64
            scale[prec] = {"N": Nb, "kernel_ms": round(kms, 4), "entries_per_s": Nb * Nb / (kms * 1e-3),
                           "tflops": fl / (kms * 1e-3) / 1e12, "frac_of_vector_peak": fl / (kms * 1e-3) / pk}
            log(f"[bench] star N={Nb} WQ {prec}: {kms:.3f} ms -> {Nb*Nb/(kms*1e-3):.3e} entries/s, "
                f"{fl/(kms*1e-3)/1e12:.2f} TFLOP/s")
            # FP32 LU (without interchanges for this symmetric matrix unless that attempt fails) +
            # FP64 refinement to 1e-10; the LU is (2/3) N^3 flop, reported against the FP32 MFMA
            # peak over the whole solve's wall time
            bb = ctx.rhs(star, p, Nb, g, method="wq", n_ref=R)
            ctx.solve(Ab, bb, tol=1e-10, max_iter=30)                  # warm: workspace, code objects
            sms = []
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xb, sinfo = ctx.solve(Ab, bb, tol=1e-10, max_iter=30)
                torch.cuda.synchronize()
                sms.append((time.perf_counter() - t0) * 1e3)
            lu_fl = 2.0 / 3.0 * Nb ** 3
            scale[prec].update({"solve_ms": min(sms), "solve_iters": sinfo.iters, "solve_pivoted": int(sinfo.pivoted),
                                "solve_backward_err": sinfo.backward_err,
                                "lu_tflops_over_solve": lu_fl / (min(sms) * 1e-3) / 1e12,
                                "lu_frac_of_fp32_peak": lu_fl / (min(sms) * 1e-3) / PEAK_FP32})
            log(f"[bench] star N={Nb} solve ({prec} matrix): {min(sms):.1f} ms, {sinfo.iters} refinement steps, "
                f"pivoted {sinfo.pivoted}, backward err {sinfo.backward_err:.1e}; "
                f"LU {lu_fl/(min(sms)*1e-3)/1e12:.1f} TFLOP/s over the solve")
            del Ab, bb, xb
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- star grid: 8 curves per (p, N)
    # FP32 kernel values and contraction (FP64 rule tables), then FP32 LU + FP64
    # refinement of the FP32 matrix to 1e-10; per point the median assembly
    # kernel time and the median / max solve time over the curves
    stars = {}
    if not args.no_stars:
        stars = {"curves_per_point": 8, "seeds": "star(idx), idx = 0..7", "precision": "fp32 matrix, fp64 refinement",
                 "tol": 1e-10, "points": []}
        for Ng in (4096, 16384):
            Ag = torch.empty((Ng, Ng), dtype=torch.float32, device="cuda")
            for pg in (2, 3, 4):
                kt, st, its, piv, bwd = [], [], [], 0, 0.0
                for idx in range(8):
                    crv = synth.star(idx)
                    ctx.assemble(crv, pg, Ng, "wq", precision="fp32", out=Ag)      # rules, code objects
                    torch.cuda.synchronize()
                    S.sgbem_ctx_set_timing(ctx.ctx, 1)
                    ctx.assemble(crv, pg, Ng, "wq", precision="fp32", out=Ag)
                    tms, c2 = S.sgbem_ctx_kernel_time(ctx.ctx)
                    S.sgbem_ctx_set_timing(ctx.ctx, 0)
                    kt.append(tms / c2)
                    bg = ctx.rhs(crv, pg, Ng, g, method="wq")
                    if idx == 0:
                        ctx.solve(Ag, bg, tol=1e-10, max_iter=30)               # workspace, code objects
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    xg, sg = ctx.solve(Ag, bg, tol=1e-10, max_iter=30)
                    torch.cuda.synchronize()
                    st.append((time.perf_counter() - t0) * 1e3)
                    its.append(int(sg.iters))
                    piv += int(sg.pivoted)
                    bwd = max(bwd, float(sg.backward_err))
                    del xg, bg
                km = float(np.median(kt))
                pt = {"p": pg, "N": Ng, "assembly_kernel_ms_median": round(km, 4),
                      "entries_per_s": Ng * Ng / (km * 1e-3),
                      "tflops": Ng * (Ng + 1) / 2 * wq_flops_per_entry(pg, 1) / (km * 1e-3) / 1e12,
                      "solve_ms_median": round(float(np.median(st)), 3), "solve_ms_max": round(max(st), 3),
                      "refinement_steps": its, "pivoted": piv, "max_backward_err": bwd}
                stars["points"].append(pt)
                log(f"[bench] stars p={pg} N={Ng} (8 curves, FP32): assembly {km:.3f} ms median, solve "
                    f"{pt['solve_ms_median']:.1f} ms median / {pt['solve_ms_max']:.1f} max, steps {its}, pivoted {piv}, "
                    f"backward err <= {bwd:.1e}")
            del Ag
            torch.cuda.empty_cache()

    # ---------------------------------------------------------------- direct formulation: double-layer sweep
    direct_rhs = {}
    if not args.no_scale:
        for label, crv, pd, Nd in (("ellipse", curve, p, N), ("star", synth.star(0), 3, 16384)):
            G = 4
            gn = ctx.sample(g, ctx.rhs_points(crv, pd, Nd, "wq"))
            gg = ctx.sample(g, ctx.rhs_points(crv, pd, Nd, "ebe", 1, G))
            Fd = torch.empty(Nd, dtype=torch.float64, device="cuda")
            rl = ctx.rules(pd, Nd, 1)
            S.sgbem_rhs_direct(ctx.ctx, crv, rl, G, gn.data_ptr(), gg.data_ptr(), Fd.data_ptr())
            torch.cuda.synchronize()
            S.sgbem_ctx_set_timing(ctx.ctx, 1)
            reps = 20 if Nd <= 4096 else 3
            t0 = time.perf_counter()
            for _ in range(reps):
                S.sgbem_rhs_direct(ctx.ctx, crv, rl, G, gn.data_ptr(), gg.data_ptr(), Fd.data_ptr())
            torch.cuda.synchronize()
            call_ms = (time.perf_counter() - t0) * 1e3 / reps
            tms, c2 = S.sgbem_ctx_kernel_time(ctx.ctx)
            S.sgbem_ctx_set_timing(ctx.ctx, 0)
            kms = tms / c2
            evals = 2.0 * Nd * Nd * G            # 2N nodes x N G Gauss points
            fl = evals * DL_FLOPS_PER_EVAL
            direct_rhs[label] = {"N": Nd, "p": pd, "n_gauss": G, "sweep_us": kms * 1e3, "call_ms": call_ms,
                                 "kernel_evals_per_s": evals / (kms * 1e-3), "tflops": fl / (kms * 1e-3) / 1e12,
                                 "frac_of_fp64_peak": fl / (kms * 1e-3) / PEAK_FP64}
            log(f"[bench] direct RHS ({label}, N={Nd}, G={G}): double-layer sweep {kms*1e3:.1f} us "
                f"({evals/(kms*1e-3):.3e} kernel values/s, {fl/(kms*1e-3)/1e12:.2f} TFLOP/s FP64), whole call {call_ms:.3f} ms")

    # ---------------------------------------------------------------- collocation BEM with the same rules
    colloc = {}
    if not args.no_scale:
        for label, crv, pc, Nc in (("ellipse", curve, p, N), ("star", synth.star(0), 3, 16384)):
            Ac = torch.empty((Nc, Nc), dtype=torch.float64, device="cuda")
            ctx.assemble_collocation(crv, pc, Nc, out=Ac)
            torch.cuda.synchronize()
            S.sgbem_ctx_set_timing(ctx.ctx, 1)
            reps = 20 if Nc <= 4096 else 3
            for _ in range(reps):
                ctx.assemble_collocation(crv, pc, Nc, out=Ac)
            tms, c2 = S.sgbem_ctx_kernel_time(ctx.ctx)
            S.sgbem_ctx_set_timing(ctx.ctx, 0)
            kms = tms / c2
            Qc = 2 * (pc + 1) - 1
            fl = float(Nc) * Nc * (2 * (6 + FLOPS_PER_LOG) + 4 * Qc)
            colloc[label] = {"N": Nc, "p": pc, "kernel_us": kms * 1e3, "entries_per_s": Nc * Nc / (kms * 1e-3),
                             "tflops": fl / (kms * 1e-3) / 1e12, "frac_of_fp64_peak": fl / (kms * 1e-3) / PEAK_FP64}
            log(f"[bench] collocation ({label}, N={Nc}, p={pc}): {kms*1e3:.1f} us -> {Nc*Nc/(kms*1e-3):.3e} entries/s, "
                f"{fl/(kms*1e-3)/1e12:.2f} TFLOP/s FP64")
            del Ac
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- batched persistent launch (256 stars)
    batch = None
    if not args.no_batch:
        probs = synth.config_batch(256)
        t0 = time.perf_counter()
        brules = [ctx.rules(pb.p, pb.N, 1) for pb in probs]
        t_brules = time.perf_counter() - t0
        bouts = [torch.empty((pb.N, pb.N), dtype=torch.float32, device="cuda") for pb in probs]
        hb = S.sgbem_batch_create(ctx.ctx, [pb.curve for pb in probs], brules, S.SGBEM_FP32,
                                  [o.data_ptr() for o in bouts], [o.stride(0) for o in bouts])
        cfg, tune_ms = S.sgbem_batch_tune(ctx.ctx, hb, 2)
        entries = float(sum(pb.N * pb.N for pb in probs))
        gb = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gb, stream=stream):
            S.sgbem_batch_assemble(ctx.ctx, hb)
        gb.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            gb.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_batch = e0.elapsed_time(e1) / reps
        del gb
        # 256 sequential single-curve launches: with a synchronisation after each, and back to back
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pb, o in zip(probs, bouts):
            ctx.assemble(pb.curve, pb.p, pb.N, "wq", precision="fp32", out=o)
            torch.cuda.synchronize()
        ms_seq_sync = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        for pb, o in zip(probs, bouts):
            ctx.assemble(pb.curve, pb.p, pb.N, "wq", precision="fp32", out=o)
        torch.cuda.synchronize()
        ms_seq = (time.perf_counter() - t0) * 1e3
        S.sgbem_batch_free(ctx.ctx, hb)
        del bouts
        torch.cuda.empty_cache()
        cfgs = [(28, 7), (32, 8), (24, 6), (16, 4)]   # the library's batched tile configurations, in order
        batch = {"curves": len(probs), "entries": entries, "precision": "fp32",
                 "batched_graph_ms": ms_batch, "entries_per_s": entries / (ms_batch * 1e-3),
                 "sequential_sync_ms": ms_seq_sync, "sequential_ms": ms_seq,
                 "speedup_vs_sequential_sync": ms_seq_sync / ms_batch, "speedup_vs_sequential": ms_seq / ms_batch,
                 "tuned_tile": {"T": cfgs[cfg][0], "S": cfgs[cfg][1]}, "rules_build_s": t_brules}
        log(f"[bench] batch of {len(probs)} stars ({entries:.3e} entries, FP32): one graph-replayed persistent launch "
            f"{ms_batch:.3f} ms ({entries/(ms_batch*1e-3):.3e} entries/s), tuned T={cfgs[cfg][0]} S={cfgs[cfg][1]}; "
            f"256 sequential launches {ms_seq:.3f} ms, with a sync each {ms_seq_sync:.3f} ms")

    # ---------------------------------------------------------------- general rules: open arc, non-uniform knots
    general = None
    if not args.no_general:
        general = general_rules(ctx, S, synth, torch, stream)

    # ---------------------------------------------------------------- serving loop (Poisson arrivals)
    serving = None
    if not args.no_serving:
        serving = serve_sweep(S, [float(r) for r in args.serve_rates.split(",")], args.serve_requests,
                              args.serve_workers, args.serve_seconds)

    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import ebe as oebe
        P = oebe.EBEProblem(curve, p, N, G_eq)
        nthreads = min(os.cpu_count() or 1, 16)
        t0 = time.perf_counter()
        P.rows(np.arange(16), nthreads)
        dt1 = time.perf_counter() - t0
        # rows of the matrix, cycled, for about --cpu-seconds of oracle work
        nrows = int(max(16, 16 * args.cpu_seconds / max(dt1, 1e-4)))
        rows = np.arange(nrows) % N
        t0 = time.perf_counter()
        done = 0
        while done < nrows:
            chunk = rows[done:done + N]
            P.rows(chunk, nthreads)
            done += chunk.size
        dt = time.perf_counter() - t0
        cpu = {"value": nrows * N / dt, "unit": "entries/s", "cores": int(P.threads_used), "kind": "oracle",
               "sample": f"element-by-element oracle (FP64, G={G_eq}, 16x16 near rule) on {nrows} rows of the "
                         f"N={N} ellipse matrix taken cyclically ({nrows*N} entries, {dt:.1f} s)"}
        log(f"[bench] CPU oracle: {cpu['value']:.3e} entries/s on {cpu['cores']} threads ({dt:.1f} s)")
        # The survey's reference for the equal-error comparison: alpha from the oracle's plain
        # form at G = 24 (FP64, upper triangle, mirrored), solved by LAPACK on the host.
        t0 = time.perf_counter()
        P24 = oebe.EBEProblem(curve, p, N, 24)
        iu, ju = np.triu_indices(N)
        v24 = P24.entries(iu, ju, nthreads)
        A24 = np.zeros((N, N))
        A24[iu, ju] = v24
        A24[ju, iu] = v24
        a24 = np.linalg.solve(A24, P24.rhs(g))
        err24 = lambda a: float(np.linalg.norm(a - a24) / np.linalg.norm(a24))
        for row in front["wq"]:
            row["solution_err_oracle_g24"] = err24(sol_wq[row["n_ref"]])
        for row in front["ebe"]:
            row["solution_err_oracle_g24"] = err24(sol_ebe[row["n_gauss"]])
        t_m = matched("solution_err_oracle_g24", front["wq"][R - 1]["solution_err_oracle_g24"])
        speedup_interp["solution_err_oracle_g24"] = t_m / front["wq"][R - 1]["us_per_step"] if t_m else None
        cpu["reference_g24_s"] = time.perf_counter() - t0
        log(f"[bench] equal error against the oracle's G=24 solution ({cpu['reference_g24_s']:.1f} s on the host): WQ " +
            " ".join(f"n_ref={row['n_ref']}:{row['solution_err_oracle_g24']:.2e}" for row in front["wq"]) + "; EBE " +
            " ".join(f"G={row['n_gauss']}:{row['solution_err_oracle_g24']:.2e}" for row in front["ebe"]) +
            f" -> log-interpolated speedup {speedup_interp['solution_err_oracle_g24']}")

    out = {
        "metric": "Galerkin entries/sec, WQ row vs element-by-element at equal err; p99 solve latency",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_wq,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ellipse (1, 0.5) as closed cubic B-spline of 32 control points; periodic "
                               "B-splines p=3, N=1024; weighted-quadrature row assembly n_ref=1, FP64",
                   "p": p, "N": N, "n_ref": R, "step": "geometry + fused WQ assembly, HIP graph replay"},
        "equal_error": {"wq_solution_err": err_wq, "ebe_solution_err": err_ebe, "ebe_gauss_order": G_eq,
                        "reference": "element-by-element G=8 solution (FP64, this GPU); solution_err_oracle_g24: "
                                     "against the CPU oracle's element-by-element G=24 solution",
                        "interior_points": "16 points inside the ellipse, error of u_h against g",
                        "front": front, "speedup_log_interpolated": speedup_interp},
        "ebe": {"entries_per_s": ebe_rate, "ms_per_step": ms_ebe, "n_gauss": G_eq},
        "speedup_wq_vs_ebe_equal_err": value / ebe_rate,
        "direct_launch_ms_per_step": ms_direct,
        "rules_build_ms": t_rules * 1e3,
        "solve_latency_ms": {"p50": pct(lat_solve, 50), "p99": pct(lat_solve, 99)},
        "request_latency_ms": {"p50": pct(lat_req, 50), "p99": pct(lat_req, 99),
                               "request": "assemble + rhs + mixed solve, N=1024"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64, "traffic": traffic,
                     "kernel": "fused WQ sweep-and-contract (FP64)", "kernel_us": kern_ms * 1e3,
                     "flops_per_launch": flops},
        "scale_N16384": scale,
        "stars_grid": stars,
        "fp32_fast_form": fp32,
        "direct_rhs": direct_rhs,
        "collocation": colloc,
        "batch_256_stars": batch,
        "serving": serving,
        "general_rules": general,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
