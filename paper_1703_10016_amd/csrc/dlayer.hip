// Right-hand side of the direct formulation (eq. final_b2 by the rule of
// Section 5; F = b1/2 - b2/(2 pi), eq. seconda_BIE in the weak form eq. weakpb).
//
//   v_n = sum over the composite Gauss points xi of w(xi) Kbar(eta_n, xi) u_D(xi),
//   Kbar(s, t) = [(f1(t) - f1(s)) f2'(t) - (f2(t) - f2(s)) f1'(t)] / |f(s) - f(t)|^2
//
// (the outward normal derivative of ln|x - y| at y = f(t), times J(t), for a
// counter-clockwise curve), then h_n = u_D(eta_n)/2 - v_n/(2 pi) is contracted
// with the regular weighted rule exactly as b1 (the rule is linear), giving F.
// With an even number of Gauss points per element no Gauss point falls on a
// node, so Kbar is never evaluated at coincident points.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "curve_eval.hpp"
#include "dlayer.hpp"

namespace sgbem {

__global__ void geometry_d_kernel(CurveDev c, GridDesc g, GaussW gw, const double *gval, double *X, double *Y,
                                  double *DX, double *DY, double *coef)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.npts) return;
    const int e = n / g.P, q = n - e * g.P;
    const double t = (double(e) + g.off[q]) / double(g.N);
    double x, y, dx, dy;
    eval_curve_d(c, t, x, y, dx, dy);
    X[n] = x;
    Y[n] = y;
    DX[n] = dx;
    DY[n] = dy;
    coef[n] = gw.w[q] * gval[n];   // composite Gauss weight w_q / N times u_D
}

// FP64 quotient a / b, b > 0: reciprocal by v_rcp_f64 and one Newton step,
// quotient corrected once by its residual.
__device__ __forceinline__ double quot(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    const double q = a * r;
    return fma(r, fma(-q, b, a), q);
}

// part[c][n] = sum over the Gauss points of chunk c of coef * Kbar(eta_n, xi):
// one node per thread, the chunk's points staged through LDS 256 at a time.
__global__ __launch_bounds__(256) void dl_sweep_kernel(int nn, const double *X1, const double *Y1, int np,
                                                       const double *X2, const double *Y2, const double *DX2,
                                                       const double *DY2, const double *coef, int chunk,
                                                       double *part)
{
    __shared__ double sx[256], sy[256], sdx[256], sdy[256], sc[256];
    const int tid = threadIdx.x;
    const int n = blockIdx.x * 256 + tid;
    const double x1 = n < nn ? X1[n] : 0.0, y1 = n < nn ? Y1[n] : 0.0;
    const int p0 = blockIdx.y * chunk, p1 = min(np, p0 + chunk);
    double acc = 0.0;
    for (int b = p0; b < p1; b += 256) {
        const int k = b + tid;
        if (k < p1) {
            sx[tid] = X2[k];
            sy[tid] = Y2[k];
            sdx[tid] = DX2[k];
            sdy[tid] = DY2[k];
            sc[tid] = coef[k];
        }
        __syncthreads();
        const int cnt = min(256, p1 - b);
        for (int j = 0; j < cnt; ++j) {
            const double ax = sx[j] - x1, ay = sy[j] - y1;
            const double num = fma(ax, sdy[j], -ay * sdx[j]);
            const double den = fma(ax, ax, ay * ay);
            acc = fma(sc[j], quot(num, den), acc);
        }
        __syncthreads();
    }
    if (n < nn) part[int64_t(blockIdx.y) * nn + n] = acc;
}

// ---------------------------------------------------------------- near terms
// For a Gauss point t close to the node s (h = t - s small), f(t) - f(s) is
// nearly tangent to f'(t) and the sweep's FP64 Kbar loses ~log10(1/|h|)
// digits to cancellation.  With E = f(t - h) - f(t) + f'(t) h (second order in
// h) the chord is f(t) - f(s) = f'(t) h - E and the numerator is -E x f'(t):
// no cancellation once E and f'(t) come from one representation of the curve.
//  polar: f = r(theta) e(theta), theta = 2 pi t, phi = 2 pi h,
//    E = r cm1(phi) e - r sm(phi) e_perp - r' phi cm1(phi) e + r' phi sin(phi) e_perp + rho e(theta - phi),
//    rho = r(theta - phi) - r(theta) + r'(theta) phi
//        = r0 sum_k a_k [cos A_k cm1(k phi) + sin A_k sm(k phi)], A_k = k theta + phi_k,
//    with cm1(x) = cos x - 1 = -2 sin^2(x/2) and sm(x) = sin x - x (series near 0);
//  B-spline (periodic): from t to t - h span by span (segment lengths that sum
//    to -h exactly: t - h itself is never formed); on a segment of length
//    delta starting at u, E gains sum_{k>=2} f^(k)(u) delta^k / k! +
//    (f'(u) - f'(t)) delta, and f'(u) - f'(t) gains sum_{k>=2} f^(k)(u)
//    delta^(k-1) / (k-1)! (every term second order, the first derivative carried
//    across the knots), f^(k)(u) by de Boor on the span's derivative curves.
__device__ __forceinline__ double cosm1(double x)
{
    const double s = sin(0.5 * x);
    return -2.0 * s * s;
}

__device__ __forceinline__ double sinmx(double x)
{
    if (fabs(x) < 0.25) {   // -x^3/3! + x^5/5! - ... + x^15/15! (next term below 1e-22 x)
        const double x2 = x * x;
        double p = -1.0 / 1307674368000.0;
        p = fma(p, x2, 1.0 / 6227020800.0);
        p = fma(p, x2, -1.0 / 39916800.0);
        p = fma(p, x2, 1.0 / 362880.0);
        p = fma(p, x2, -1.0 / 5040.0);
        p = fma(p, x2, 1.0 / 120.0);
        p = fma(p, x2, -1.0 / 6.0);
        return x * x2 * p;
    }
    return sin(x) - x;
}

// knot k of the periodic extension (uniform k / n_ctrl, or breakpoints + whole periods)
__device__ __forceinline__ double ext_knot(const CurveDev &c, const double *tk, int k)
{
    const int nc = c.n_ctrl;
    if (!c.nonuniform) return double(k) / nc;
    const int q = k >= 0 ? k / nc : -((-k + nc - 1) / nc), j = k - q * nc;
    return tk[j] + q;
}

// f^(k)(u), k = 0 .. d, of the polynomial of span l (periodic B-spline of degree d <= 7)
__device__ void span_derivs(const CurveDev &c, const double *tk, const double *cq, int l, double u, double *Dx, double *Dy)
{
    const int d = c.degree, nc = c.n_ctrl;
    double T[16], cx[8], cy[8];
    for (int i = 0; i <= 2 * d + 1; ++i) T[i] = ext_knot(c, tk, l - d + i);
    for (int i = 0; i <= d; ++i) {
        const int j = ((l - d + i) % nc + nc) % nc;
        cx[i] = cq[2 * j];
        cy[i] = cq[2 * j + 1];
    }
    for (int k = 0; k <= d; ++k) {
        if (k > 0)   // level-k control points from level k - 1 (degree d - k + 1 -> d - k)
            for (int i = d; i >= k; --i) {
                const double sc = double(d - k + 1) / (T[i + d - k + 1] - T[i]);
                cx[i] = sc * (cx[i] - cx[i - 1]);
                cy[i] = sc * (cy[i] - cy[i - 1]);
            }
        const int q = d - k;
        double wx[8], wy[8];
        for (int i = k; i <= d; ++i) {
            wx[i] = cx[i];
            wy[i] = cy[i];
        }
        for (int r = 1; r <= q; ++r)
            for (int i = d; i >= k + r; --i) {
                const double al = (u - T[i]) / (T[i + q + 1 - r] - T[i]);
                wx[i] = (1.0 - al) * wx[i - 1] + al * wx[i];
                wy[i] = (1.0 - al) * wy[i - 1] + al * wy[i];
            }
        Dx[k] = wx[d];
        Dy[k] = wy[d];
    }
}

// Kbar(t - h, t) without cancellation (see above); t the Gauss point, h = t - s.
__device__ double kbar_near(const CurveDev &c, double t, double h)
{
    double Ex, Ey, Fx, Fy;   // E and f'(t), from one representation
    if (c.kind == 1) {
        const double *ca = c.inline_data ? c.inl : c.a;
        const double *cphi = c.inline_data ? c.inl + 64 : c.phi;
        constexpr double TWO_PI = 6.283185307179586476925286766559;
        double sn, cs;
        sincos_pi(2.0 * t, &sn, &cs);
        const double th = TWO_PI * t, phi = TWO_PI * h;
        double r = 1.0, dr = 0.0, rho = 0.0;
        for (int k = 1; k <= c.n_modes; ++k) {
            double sk, ck;
            sin_cos(k * th + cphi[k - 1], &sk, &ck);
            r += ca[k - 1] * ck;
            dr -= k * ca[k - 1] * sk;
            const double B = k * phi;
            rho += ca[k - 1] * (ck * cosm1(B) + sk * sinmx(B));
        }
        r *= c.r0;
        dr *= c.r0;
        rho *= c.r0;
        const double c1 = cosm1(phi), s1 = sinmx(phi), sp = s1 + phi, cp = 1.0 + c1;
        // e = (cs, sn), e_perp = (-sn, cs), e(theta - phi) = cp e - sp e_perp
        const double ex2 = cp * cs + sp * sn, ey2 = cp * sn - sp * cs;
        Ex = r * c1 * cs + r * s1 * sn - dr * phi * c1 * cs - dr * phi * sp * sn + rho * ex2;
        Ey = r * c1 * sn - r * s1 * cs - dr * phi * c1 * sn + dr * phi * sp * cs + rho * ey2;
        Fx = TWO_PI * (dr * cs - r * sn);
        Fy = TWO_PI * (dr * sn + r * cs);
    } else {
        const double *tk = c.inline_data ? c.inl + 128 : c.knots;
        const double *cq = c.inline_data ? c.inl : c.ctrl;
        const int d = c.degree, nc = c.n_ctrl;
        double Dx[8], Dy[8];
        // rem: the signed distance still to go (exactly -h at the start; a segment that
        // ends on a knot has the exact length knot - u, so the lengths sum to -h)
        double u = t, rem = -h, gx = 0.0, gy = 0.0;   // g = f'(u) - f'(t)
        Ex = Ey = 0.0;
        Fx = Fy = 0.0;
        for (int seg = 0; seg < nc + 2 && rem != 0.0; ++seg) {
            const bool left = rem < 0.0;
            // the span holding the open segment from u in the direction of travel
            int l = int(floor(u * nc));
            if (c.nonuniform) {
                const double fl = floor(u);
                const double w = u - fl;
                int lo = 0, hi = nc - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (tk[mid] <= w) lo = mid;
                    else hi = mid - 1;
                }
                l = int(fl) * nc + lo;
            }
            while (ext_knot(c, tk, l + 1) <= u) ++l;
            while (ext_knot(c, tk, l) > u) --l;
            if (left && ext_knot(c, tk, l) >= u) --l;   // u on a knot, moving left
            const double bound = left ? ext_knot(c, tk, l) : ext_knot(c, tk, l + 1);
            const double dist = bound - u;
            const bool last = fabs(rem) <= fabs(dist);
            const double delta = last ? rem : dist;
            span_derivs(c, tk, cq, l, u, Dx, Dy);
            if (seg == 0) {
                Fx = Dx[1];
                Fy = Dy[1];
            } else if (d == 1) {   // piecewise linear: the derivative jumps at the knot
                gx = Dx[1] - Fx;
                gy = Dy[1] - Fy;
            }
            // sum_{k>=2} D_k delta^k / k! and sum_{k>=2} D_k delta^(k-1) / (k-1)!, by Horner from k = d
            double ex = 0.0, ey = 0.0, fx = 0.0, fy = 0.0;
            for (int k = d; k >= 2; --k) {
                ex = (ex + Dx[k]) * delta / k;
                ey = (ey + Dy[k]) * delta / k;
                fx = (fx + Dx[k]) * delta / (k - 1);
                fy = (fy + Dy[k]) * delta / (k - 1);
            }
            Ex += ex * delta + gx * delta;
            Ey += ey * delta + gy * delta;
            gx += fx;
            gy += fy;
            if (last) break;
            rem -= delta;
            u = bound;
        }
    }
    const double ax = Fx * h - Ex, ay = Fy * h - Ey;
    return -(Ex * Fy - Ey * Fx) / (ax * ax + ay * ay);
}

// part[n] += sum over the near Gauss points of coef (Kbar_near - Kbar_sweep): the
// Gauss points of node n's element and its two neighbours (element e = n / P1,
// P1 nodes per element), the sweep's own value recomputed from the same arrays
// and operations.  h from the integer indices: h = (P1 e' - n + P1 u_q) / (P1 N)
// with e' the element index taken periodically nearest to the node.
// gu.w[q]: the Gauss nodes u_q on [0, 1] (not the weights).
// One thread per (node, near Gauss point): a workgroup takes blockDim / (3G)
// nodes (3G <= 24); the differences meet in LDS and one thread per node adds
// them in the order (element -1, 0, +1; Gauss point 0 .. G-1).
__device__ __forceinline__ bool dl_near_skip(int N, int en, int de)
{
    if (N < 3 && de == 1 && ((en + 1) % N) == ((en - 1 + N) % N)) return true;   // N = 2: one neighbour
    return N < 2 && de != 0;
}

__global__ __launch_bounds__(256) void dl_near_kernel(CurveDev c, int N, int P1, int G, GaussW gu, int nn,
                                                      const double *X1, const double *Y1, const double *X2,
                                                      const double *Y2, const double *DX2, const double *DY2,
                                                      const double *coef, double *part)
{
    __shared__ double diff[256];
    const int per = 3 * G, npw = int(blockDim.x) / per;
    const int tid = threadIdx.x, ln = tid / per, it = tid - ln * per;
    const int n = int(blockIdx.x) * npw + ln;
    const bool node = ln < npw && n < nn;
    const int en = node ? n / P1 : 0;
    if (node) {
        const int de = it / G - 1, q = it - (it / G) * G;
        double v = 0.0;
        if (!dl_near_skip(N, en, de)) {
            const int e = ((en + de) % N + N) % N, ee = en + de;   // periodic index, and its unwrapped position
            const int k = e * G + q;
            const double ax = X2[k] - X1[n], ay = Y2[k] - Y1[n];
            const double num = fma(ax, DY2[k], -ay * DX2[k]);
            const double den = fma(ax, ax, ay * ay);
            const double kd = quot(num, den);
            const double t = (double(e) + gu.w[q]) / double(N);
            const double h = (double(P1 * ee - n) + P1 * gu.w[q]) / double(P1 * N);
            v = kbar_near(c, t, h) - kd;
        }
        diff[tid] = v;
    }
    __syncthreads();
    if (node && it == 0) {
        double corr = 0.0;
        for (int de = -1; de <= 1; ++de) {
            if (dl_near_skip(N, en, de)) continue;
            const int e = ((en + de) % N + N) % N;
            for (int q = 0; q < G; ++q) corr = fma(coef[e * G + q], diff[tid + (de + 1) * G + q], corr);
        }
        part[n] += corr;
    }
}

hipError_t launch_dl_near(const CurveDev &c, int N, int P1, int G, const GaussW &gu, int nn, const double *X1,
                          const double *Y1, const double *X2, const double *Y2, const double *DX2, const double *DY2,
                          const double *coef, double *part, hipStream_t s)
{
    if (G < 1 || 3 * G > 256) return hipErrorInvalidValue;
    const int npw = 256 / (3 * G);
    hipLaunchKernelGGL(dl_near_kernel, dim3((nn + npw - 1) / npw), dim3(256), 0, s, c, N, P1, G, gu, nn, X1, Y1, X2, Y2,
                       DX2, DY2, coef, part);
    return hipGetLastError();
}

// h_n = g_n / 2 - v_n / (2 pi), v_n the chunk partials summed in chunk order;
// v_n itself when vout is given.
__global__ void dl_reduce_kernel(int nn, int nchunk, const double *part, const double *g, double *h, double *vout)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += part[int64_t(c) * nn + n];
    h[n] = 0.5 * g[n] - v * 0.15915494309189533577;   // 1 / (2 pi)
    if (vout) vout[n] = v;
}

hipError_t launch_dl_geometry(const CurveDev &c, const GridDesc &g, const GaussW &gw, const double *gval,
                              double *X, double *Y, double *DX, double *DY, double *coef, hipStream_t s)
{
    hipLaunchKernelGGL(geometry_d_kernel, dim3((g.npts + 255) / 256), dim3(256), 0, s, c, g, gw, gval, X, Y, DX, DY,
                       coef);
    return hipGetLastError();
}

int dl_chunks(int nn, int np)
{
    const int gx = (nn + 255) / 256;
    int c = (2048 + gx - 1) / gx;                 // aim at >= 2048 workgroups
    const int maxc = (np + 255) / 256;            // at least 256 points per chunk
    if (c > maxc) c = maxc;
    if (c > 64) c = 64;
    return c < 1 ? 1 : c;
}

hipError_t launch_dl_sweep(int nn, const double *X1, const double *Y1, int np, const double *X2, const double *Y2,
                           const double *DX2, const double *DY2, const double *coef, int nchunk, double *part,
                           hipStream_t s, const KernelEvents *ev)
{
    int chunk = (np + nchunk - 1) / nchunk;
    chunk = (chunk + 255) / 256 * 256;
    const dim3 grid((nn + 255) / 256, nchunk);
    if (ev)
        hipExtLaunchKernelGGL(dl_sweep_kernel, grid, dim3(256), 0, s, ev->start, ev->stop, 0, nn, X1, Y1, np, X2, Y2,
                              DX2, DY2, coef, chunk, part);
    else
        hipLaunchKernelGGL(dl_sweep_kernel, grid, dim3(256), 0, s, nn, X1, Y1, np, X2, Y2, DX2, DY2, coef, chunk,
                           part);
    return hipGetLastError();
}

hipError_t launch_dl_reduce(int nn, int nchunk, const double *part, const double *g, double *h, double *vout,
                            hipStream_t s)
{
    hipLaunchKernelGGL(dl_reduce_kernel, dim3((nn + 255) / 256), dim3(256), 0, s, nn, nchunk, part, g, h, vout);
    return hipGetLastError();
}

}  // namespace sgbem
