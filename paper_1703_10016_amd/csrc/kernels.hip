// Geometry, element-by-element near pairs, band correction and right-hand
// side kernels; dispatch of the tile kernels.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "curve_eval.hpp"

namespace sgbem {

// ------------------------------------------------------------------ geometry
// f, f' and J = |f'| (eq. J) at the grid points.
//  polar:   f = r(theta) (cos theta, sin theta), theta = 2 pi t, closed-form derivative;
//  B-spline (periodic uniform knots, Section 3): de Boor's algorithm on the span
//           containing n_ctrl t, and on the derivative curve with control points
//           n_ctrl (Q_j - Q_{j-1}) at degree d-1.
__global__ void geometry_kernel(CurveDev c, GridDesc g, double *X, double *Y, double *J)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.npts) return;
    double t;
    if (g.tpar) {
        t = g.tpar[n];
    } else if (g.P == 0) {
        t = double(n) / double(g.npts);
    } else {
        const int e = n / g.P, q = n - e * g.P;
        t = (double(e) + g.off[q]) / double(g.N);
    }
    eval_curve(c, t, X[n], Y[n], J[n]);
}

hipError_t launch_geometry(const CurveDev &c, const GridDesc &g, double *X, double *Y, double *J, hipStream_t s)
{
    const int bs = 64;   // small launches (2048 points at N = 1024): more workgroups, faster ramp (1 % of the step)
    hipLaunchKernelGGL(geometry_kernel, dim3((g.npts + bs - 1) / bs), dim3(bs), 0, s, c, g, X, Y, J);
    return hipGetLastError();
}

__global__ void points_xy_kernel(const double *X, const double *Y, int npts, double *xy)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= npts) return;
    xy[2 * n] = X[n];
    xy[2 * n + 1] = Y[n];
}

hipError_t launch_points_xy(const double *X, const double *Y, int npts, double *xy, hipStream_t s)
{
    hipLaunchKernelGGL(points_xy_kernel, dim3((npts + 255) / 256), dim3(256), 0, s, X, Y, npts, xy);
    return hipGetLastError();
}

// ------------------------------------------------------------------ EBE near pairs
// For element e and its right neighbour (type 1) or itself (type 0):
//   L[a][b] = h^2 sum_{g1,g2} M_p(a+u1) J1 Kt(g1,g2) J2 M_p(b+u2),
//   Kt = w1 w2 (1/2 ln|f1 - f2|^2 - ln|u1 - u2 - dd|) + Mhat(g1, g2),
// the regular part [ln|f(s)-f(t)| - ln|s-t|] by 16 x 16 Gauss plus the exactly
// integrated ln|s-t| part of the interpolated B J (reference matrices Mhat);
// coincident diagonal points take ln(J h) (eq. F1_lim).
__global__ __launch_bounds__(256) void near_kernel(NearArgs a)
{
    const int e = blockIdx.x >> 1, type = blockIdx.x & 1;
    const int N = a.N, p = a.p, np = p + 1;
    const int e2 = type ? (e + 1) % N : e;
    const double h = 1.0 / N;
    __shared__ double Kt[16][17];
    __shared__ double C[16][8];
    const int t = threadIdx.x;
    {
        const int g1 = t >> 4, g2 = t & 15;
        const int k1 = e * 16 + g1, k2 = e2 * 16 + g2;
        const double w12 = a.w16[g1] * a.w16[g2];
        double kt;
        if (type == 0 && g1 == g2) {
            kt = w12 * log(a.J16[k1] * h) + a.mco[g1 * 16 + g2];
        } else {
            const double dx = a.X16[k1] - a.X16[k2], dy = a.Y16[k1] - a.Y16[k2];
            const double du = fabs(a.u16[g1] - a.u16[g2] - double(type));
            kt = w12 * (0.5 * log(dx * dx + dy * dy) - log(du)) + (type ? a.madj[g1 * 16 + g2] : a.mco[g1 * 16 + g2]);
        }
        Kt[g1][g2] = kt;
    }
    __syncthreads();
    if (t < 16 * np) {
        const int g1 = t / np, b = t - g1 * np;
        double s = 0.0;
        for (int g2 = 0; g2 < 16; ++g2) s += Kt[g1][g2] * a.J16[e2 * 16 + g2] * a.bv16[b * 16 + g2];
        C[g1][b] = s;
    }
    __syncthreads();
    if (t < np * np) {
        const int ia = t / np, b = t - ia * np;
        double s = 0.0;
        for (int g1 = 0; g1 < 16; ++g1) s += a.bv16[ia * 16 + g1] * a.J16[e * 16 + g1] * C[g1][b];
        a.L[(int64_t(e) * 2 + type) * np * np + ia * np + b] = h * h * s;
    }
}

hipError_t launch_near(const NearArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(near_kernel, dim3(2 * a.N), dim3(256), 0, s, a);
    return hipGetLastError();
}

// A[i][j] += scale sum_{a,b} L(i+a, j+b)[a][b] over the coincident / adjacent
// element pairs of supp B_i x supp B_j; (i, j) and (j, i) get the same value.
template <typename OutT>
__global__ void band_kernel(int N, int p, const double *L, double scale, OutT *out, int64_t lda)
{
    const int np = p + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * (p + 2)) return;
    const int i = idx / (p + 2), o = idx - i * (p + 2);
    if (2 * o == N && i >= N / 2) return;      // same unordered pair reached from i - N/2
    const int j = (i + o) % N;
    double s = 0.0;
    for (int ia = 0; ia <= p; ++ia) {
        const int e1 = (i + ia) % N;
        for (int b = 0; b <= p; ++b) {
            const int e2 = (j + b) % N;
            int de = e2 - e1;
            if (de < 0) de += N;
            if (de == 0)
                s += L[(int64_t(e1) * 2 + 0) * np * np + ia * np + b];
            else if (de == 1)
                s += L[(int64_t(e1) * 2 + 1) * np * np + ia * np + b];
            else if (de == N - 1)
                s += L[(int64_t(e2) * 2 + 1) * np * np + b * np + ia];
        }
    }
    // (i, j) and (j, i) hold the same value before the update; compute the
    // new value once so that the matrix stays exactly symmetric.
    const OutT v = OutT(double(out[int64_t(i) * lda + j]) + scale * s);
    out[int64_t(i) * lda + j] = v;
    if (i != j) out[int64_t(j) * lda + i] = v;
}

hipError_t launch_band(int prec, int N, int p, const double *L, double scale, void *out, int64_t lda, hipStream_t s)
{
    const int n = N * (p + 2);
    if (prec == 0)
        hipLaunchKernelGGL(band_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, s, N, p, L, scale,
                           reinterpret_cast<double *>(out), lda);
    else
        hipLaunchKernelGGL(band_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, N, p, L, scale,
                           reinterpret_cast<float *>(out), lda);
    return hipGetLastError();
}

// ------------------------------------------------------------------ right-hand side
__global__ void rhs_kernel(int N, int npts, int P, int s0, int Q, const double *coef, double scale,
                           const double *J, const double *g, double *beta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int q = 0; q < Q; ++q) {
        const int n = (P * i + s0 + q) % npts;
        s += coef[q] * J[n] * g[n];
    }
    beta[i] = scale * s;
}

hipError_t launch_rhs(int N, int npts, int P, int s0, int Q, const double *coef, double scale, const double *J,
                      const double *g, double *beta, hipStream_t s)
{
    hipLaunchKernelGGL(rhs_kernel, dim3((N + 127) / 128), dim3(128), 0, s, N, npts, P, s0, Q, coef, scale, J, g, beta);
    return hipGetLastError();
}

}  // namespace sgbem
