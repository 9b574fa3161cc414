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
