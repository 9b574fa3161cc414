// Sum-factorised Galerkin tile kernel (fused kernel sweep + banded contraction).
//
// Both assembly forms share one structure.  A point grid carries P points per
// element (WQ: the 2 n_ref nodes of Section 4 per element; EBE: the G Gauss
// points), basis function j owns the Q points n = P j + S0 + q of its
// support, and
//
//   stage 1   C1[n1][j] = sum_q J(n2) (coefA[q] U(n1,n2) + coefB[q] V(n1,n2)),  n2 = P j + S0 + q
//   stage 2   A[i][j]   = scale sum_q coefA[q] J(n1) C1[n1][j],                 n1 = P i + S0 + q
//
// WQ (eqs. IK1e2, IK1e2_bis, Alg. 3):  U = K1(n1,n2) = 1/2 ln(|f1-f2|^2 (pi/sin(pi d/npts))^2)
//     (diagonal: ln J, eq. F1_lim), V = singular weight w_{n2}^{(eta_n1)}, coefA = regular
//     weights, coefB = B_j at the nodes;
// EBE far part (eq. elbyelint):  U = ln|f1-f2| for element pairs that are neither
//     coincident nor adjacent (0 otherwise), V = 0, coefA = h w_g M_p(a + u_g).
//
// One workgroup owns a T x T tile of A in the upper triangle.  The node
// coordinates of its two point windows and the slices of the translation-
// invariant tables sit in LDS; every thread of stage 1 sweeps one n1 row
// against a strip of S columns, evaluating each kernel value once and
// accumulating it into the S column sums in registers; stage 2 contracts
// C1 from LDS.  The tile is written row-major (coalesced) and mirrored through
// LDS, so the matrix is exactly symmetric (rows i <= j are the computed ones).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sgbem {

// FP64 natural logarithm for positive normal arguments, table driven (Tang's scheme):
// x = 2^e m with m in [1, 2); j = the top 6 fraction bits of m;
// c_j = 1 / (1 + (j + 1/2)/64), r = m c_j - 1 (|r| < 1/128, one rounding by the fma);
// log x = e ln2 + log(1/c_j) + log1p(r), log1p by its Taylor series to r^8
// (truncation |r|^9/9 < 1e-20).  tab[2j] = c_j, tab[2j+1] = log(1/c_j); ln 2 is
// split into a 32-bit head (e ln2_hi exact) and a tail.  Absolute error a few
// units in the last place of the result's scale.
__device__ __forceinline__ void build_log_tab(double *tab)
{
    for (int j = threadIdx.x; j < 64; j += blockDim.x) {
        const double c = 1.0 / (1.0 + (j + 0.5) / 64.0);
        tab[2 * j] = c;
        tab[2 * j + 1] = -log(c);
    }
}
__device__ __forceinline__ double log_tab64(double x, const double *tab)
{
    constexpr double ln2_hi = 0.69314718036912381649017333984375;
    constexpr double ln2_lo = 1.9082149292705877000220e-10;
    int e = __builtin_amdgcn_frexp_exp(x) - 1;              // x = m 2^e, m in [1, 2)
    const double m = 2.0 * __builtin_amdgcn_frexp_mant(x);
    const int j = (__double2hiint(m) >> 14) & 63;
    const double c = tab[2 * j], lc = tab[2 * j + 1];
    const double r = fma(m, c, -1.0);
    double p = -0.125;
    p = fma(p, r, 1.0 / 7.0);
    p = fma(p, r, -1.0 / 6.0);
    p = fma(p, r, 0.2);
    p = fma(p, r, -0.25);
    p = fma(p, r, 1.0 / 3.0);
    p = fma(p, r, -0.5);
    p = fma(p, r, 1.0);
    const double ed = double(e);
    return fma(ed, ln2_hi, lc + fma(ed, ln2_lo, p * r));
}

// FP64 natural logarithm without tables: x = 2^e m, m in [sqrt(1/2), sqrt(2)),
// s = (m - 1)/(m + 1) (|s| <= 0.1716; reciprocal by v_rcp_f64 and one Newton
// step, quotient corrected once by its residual, which leaves s exact to
// rounding whenever the reciprocal carries more than ~27 bits),
// log m = 2 atanh(s) = 2 sum_k s^(2k+1)/(2k+1) to k = 10 (first omitted term
// 2 s^23/23 < 2.2e-19).
__device__ __forceinline__ double log_atanh64(double x)
{
    constexpr double ln2_hi = 0.69314718036912381649017333984375;   // ln 2 truncated to 32 fraction bits
    constexpr double ln2_lo = 1.9082149292705877000220e-10;         // ln 2 - ln2_hi
    int e = __builtin_amdgcn_frexp_exp(x);
    double m = __builtin_amdgcn_frexp_mant(x);               // [1/2, 1)
    const bool lo = m < 0.70710678118654752440;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double num = m - 1.0, den = m + 1.0;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    double s = num * r;
    s = fma(r, fma(-s, den, num), s);
    const double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double t = 2.0 * s;
    const double lm = fma(t * s2, p, t);
    const double ed = double(e);
    return fma(ed, ln2_hi, fma(ed, ln2_lo, lm));
}

// Logarithm of the kernel sweep (choices measured on MI355X): FP64 weighted
// quadrature uses the table-free series above (1.4x faster than the device
// library's log there; the sweep's LDS already carries the node windows and
// rule tables), the FP64 element-by-element sweep the table-driven log (2x
// faster than the library's there).  FP32: v_log_f32.
template <typename Real, bool TableLog>
__device__ __forceinline__ Real k_log(Real x, const double *tab);
template <>
__device__ __forceinline__ double k_log<double, true>(double x, const double *tab) { return log_tab64(x, tab); }
template <>
__device__ __forceinline__ double k_log<double, false>(double x, const double *) { return log_atanh64(x); }
template <>
__device__ __forceinline__ float k_log<float, true>(float x, const double *) { return __logf(x); }
template <>
__device__ __forceinline__ float k_log<float, false>(float x, const double *) { return __logf(x); }

struct TileArgsF {          // FP32 copies of the per-support coefficients
    float coefA[64];
    float coefB[64];
};

template <typename Real, typename Args, typename ArgsF>
__device__ __forceinline__ Real coef_a(const Args &a, const ArgsF &f, int q)
{
    if constexpr (sizeof(Real) == 8) return a.coefA[q];
    else return f.coefA[q];
}
template <typename Real, typename Args, typename ArgsF>
__device__ __forceinline__ Real coef_b(const Args &a, const ArgsF &f, int q)
{
    if constexpr (sizeof(Real) == 8) return a.coefB[q];
    else return f.coefB[q];
}

__device__ __forceinline__ void tile_coords(int nb, int b, int &bi, int &bj)
{
    // linear index b over the upper-triangle tiles, row by row
    const double tn = 2.0 * nb + 1.0;
    int r = int((tn - sqrt(tn * tn - 8.0 * b)) * 0.5);
    if (r < 0) r = 0;
    while (r > 0 && r * nb - (r * (r - 1)) / 2 > b) --r;
    while ((r + 1) * nb - ((r + 1) * r) / 2 <= b) ++r;
    bi = r;
    bj = r + (b - (r * nb - (r * (r - 1)) / 2));
}

// One T x T tile (bi <= bj) of one matrix: the whole sweep-and-contract.
template <int P, int Q, int S0, bool WQ, typename Real, typename OutT, int T, int S, typename Args, typename ArgsF>
__device__ __forceinline__ void tile_body(const Args &a, const ArgsF &af, int bi, int bj)
{
    constexpr int L = P * (T - 1) + Q;     // points in each window
    constexpr int LT = 2 * L - 1;          // table slice for n2 - n1
    constexpr int NSTRIP = T / S;
    constexpr int W2 = P * (S - 1) + Q;    // n2 points swept by one strip
    static_assert(T % S == 0, "strip must divide tile");

    __shared__ double sx1[L], sy1[L], sx2[L], sy2[L];
    __shared__ Real sJ1[L], sJ2[L];
    __shared__ int se1[WQ ? 1 : L], se2[WQ ? 1 : L];
    __shared__ Real sinv[WQ ? LT : 1], sw[WQ ? 2 * LT : 1];   // sw[par * LT + dl]
    __shared__ Real C1[L][T + 1];
    __shared__ Real tileo[T][T + 1];
    constexpr bool kTableLog = !WQ && sizeof(Real) == 8;
    __shared__ double ltab[kTableLog ? 128 : 1];
    if constexpr (kTableLog) build_log_tab(ltab);

    const int N = a.N, npts = a.npts;
    const int I0 = bi * T, J0 = bj * T;
    const int start1 = (P * I0 + S0) % npts;
    const int start2 = (P * J0 + S0) % npts;

    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        const int g1 = (start1 + r) % npts;
        const int g2 = (start2 + r) % npts;
        sx1[r] = a.X[g1];
        sy1[r] = a.Y[g1];
        sJ1[r] = Real(a.J[g1]);
        sx2[r] = a.X[g2];
        sy2[r] = a.Y[g2];
        sJ2[r] = Real(a.J[g2]);
        if constexpr (!WQ) {
            se1[r] = g1 / P;
            se2[r] = g2 / P;
        }
    }
    if constexpr (WQ) {
        // slice index dl <-> d = (start2 - start1 + dl - (L - 1)) mod npts
        int dbase = (start2 - start1 - (L - 1)) % npts;
        if (dbase < 0) dbase += npts;
        for (int dl = threadIdx.x; dl < LT; dl += blockDim.x) {
            const int d = (dbase + dl) % npts;
            if constexpr (sizeof(Real) == 8) {
                sinv[dl] = Real(a.inv_s2[d]);
                sw[dl] = Real(a.ws[d]);
                sw[LT + dl] = Real(a.ws[npts + d]);
            } else {
                sinv[dl] = Real(a.inv_s2f[d]);
                sw[dl] = Real(a.wsf[d]);
                sw[LT + dl] = Real(a.wsf[npts + d]);
            }
        }
    }
    __syncthreads();

    // ---------------- stage 1: kernel sweep and contraction over the n2 supports
    for (int item = threadIdx.x; item < L * NSTRIP; item += blockDim.x) {
        const int r = item % L;
        const int st = item / L;
        const double x1 = sx1[r], y1 = sy1[r];
        const Real J1 = sJ1[r];
        const int par = (start1 + r) % npts & 1;
        const Real *swp = WQ ? sw + par * LT : sw;     // singular weights of this row's node class
        const int e1 = WQ ? 0 : se1[r];
        Real acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = Real(0);
#pragma unroll
        for (int k2 = 0; k2 < W2; ++k2) {
            const int c2 = st * S * P + k2;
            const double dx = x1 - sx2[c2], dy = y1 - sy2[c2];
            Real r2;
            if constexpr (sizeof(Real) == 8) {
                r2 = dx * dx + dy * dy;
            } else {
                const float fx = float(dx), fy = float(dy);
                r2 = fx * fx + fy * fy;
            }
            Real U, V = Real(0);
            if constexpr (WQ) {
                const int dl = c2 - r + (L - 1);
                const Real inv = sinv[dl];
                const Real ratio = (inv == Real(0)) ? J1 * J1 : r2 * inv;
                U = Real(0.5) * k_log<Real, kTableLog>(ratio, ltab);
                V = swp[dl];
            } else {
                int de = se2[c2] - e1;
                if (de < 0) de += N;
                const bool near = (de == 0) | (de == 1) | (de == N - 1);
                U = near ? Real(0) : Real(0.5) * k_log<Real, kTableLog>(r2, ltab);
            }
            const Real J2 = sJ2[c2];
            const Real JU = J2 * U, JV = J2 * V;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int q = k2 - s * P;
                if (q >= 0 && q < Q) {
                    acc[s] = fma(coef_a<Real>(a, af, q), JU, acc[s]);
                    if constexpr (WQ) acc[s] = fma(coef_b<Real>(a, af, q), JV, acc[s]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) C1[r][st * S + s] = J1 * acc[s];
    }
    __syncthreads();

    // ---------------- stage 2: contraction over the n1 supports
    const Real scale = Real(a.scale);
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int il = e / T, jl = e % T;
        Real v = Real(0);
#pragma unroll
        for (int q = 0; q < Q; ++q) v += coef_a<Real>(a, af, q) * C1[P * il + q][jl];
        tileo[il][jl] = v * scale;
    }
    __syncthreads();

    OutT *out = reinterpret_cast<OutT *>(a.out);
    const int64_t lda = a.lda;
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int il = e / T, jl = e % T;
        const int i = I0 + il, j = J0 + jl;
        if (i < N && j < N) {
            const Real v = (bi == bj && il > jl) ? tileo[jl][il] : tileo[il][jl];
            out[int64_t(i) * lda + j] = OutT(v);
        }
    }
    if (bi != bj) {
        for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
            const int rl = e / T, cl = e % T;          // output row J0 + rl, column I0 + cl
            const int i = J0 + rl, j = I0 + cl;
            if (i < N && j < N) out[int64_t(i) * lda + j] = OutT(tileo[cl][rl]);
        }
    }
    __syncthreads();   // LDS is reused by the next tile of a persistent block
}

// WPE: minimum waves per SIMD the register allocation must allow (1: no
// constraint).  Large matrices gain from 4 (more waves to hide the latency of
// the logarithm's dependent chain), small ones lose to the extra spills.
template <int P, int Q, int S0, bool WQ, typename Real, typename OutT, int T, int S, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void tile_kernel(TileArgs a, TileArgsF af)
{
    const int nb = (a.N + T - 1) / T;
    int bi, bj;
    tile_coords(nb, blockIdx.x, bi, bj);
    tile_body<P, Q, S0, WQ, Real, OutT, T, S>(a, af, bi, bj);
}

template <int P, int Q, int S0, bool WQ, typename Real, int T, int S, int WPE = 1>
hipError_t launch_tile(const TileArgs &a, hipStream_t s, const KernelEvents *ev = nullptr)
{
    TileArgsF af;
    for (int q = 0; q < 64; ++q) {
        af.coefA[q] = float(a.coefA[q]);
        af.coefB[q] = float(a.coefB[q]);
    }
    const int nb = (a.N + T - 1) / T;
    const int blocks = nb * (nb + 1) / 2;
    using OutT = Real;
    if (ev)
        hipExtLaunchKernelGGL((tile_kernel<P, Q, S0, WQ, Real, OutT, T, S, WPE>), dim3(blocks), dim3(256), 0, s,
                              ev->start, ev->stop, 0, a, af);
    else
        hipLaunchKernelGGL((tile_kernel<P, Q, S0, WQ, Real, OutT, T, S, WPE>), dim3(blocks), dim3(256), 0, s, a, af);
    return hipGetLastError();
}

}  // namespace sgbem
