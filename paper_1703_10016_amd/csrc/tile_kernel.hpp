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
#include <type_traits>
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "log_table.hpp"

namespace sgbem {

// FP64 natural logarithm for positive normal arguments, table driven (Tang's scheme):
// x = 2^e m with m in [1/2, 1) (frexp); j = the top 8 fraction bits of x;
// c_j = 2 / (1 + (j + 1/2)/256), r = m c_j - 1 (|r| < 2^-9, one rounding by the
// fma); log x = e ln2 + log(1/c_j) + log1p(r), log1p(r) = r + r^2 q(r) with q
// the Taylor series to r^5/5 (truncation |r|^6/6 < 1e-17).  tab[j] =
// (c_j, log(1/c_j)) from log_table.hpp, copied to LDS per workgroup; ln 2 is
// split into a 32-bit head (e ln2_hi exact) and a tail.  Absolute error
// <= 1.2e-16 over [4e-18, 2e17] (arithmetic checked against 50-digit values).
__device__ __forceinline__ void load_log_tab(double2 *tab)
{
    for (int j = threadIdx.x; j < 256; j += blockDim.x) tab[j] = make_double2(kLogTab256[2 * j], kLogTab256[2 * j + 1]);
}
// The LDS copy of the table: one per kernel, whichever tile variants it inlines.
__device__ __forceinline__ double2 *log_tab_lds()
{
    __shared__ double2 tab[256];
    return tab;
}
__device__ __forceinline__ double log_tab64(double x, const double2 *tab)
{
    constexpr double ln2_hi = 0.69314718036912381649017333984375;
    constexpr double ln2_lo = 1.9082149292705877000220e-10;
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
    const uint32_t hi = uint32_t(__double_as_longlong(x) >> 32);
    const double2 cl = tab[(hi >> 12) & 255];
    const double r = fma(m, cl.x, -1.0);
    double q = 0.2;
    q = fma(q, r, -0.25);
    q = fma(q, r, 1.0 / 3.0);
    q = fma(q, r, -0.5);
    const double ed = double(e);
    return fma(ed, ln2_hi, cl.y + fma(ed, ln2_lo, fma(q, r * r, r)));
}

// Logarithm of the kernel sweep (choices measured on MI355X): FP64 uses the
// table-driven log above (a 64-entry version cost 23 FP64-operation
// equivalents per log against 41 for a table-free atanh series and 91 for the
// device library's log, measured as throughput on independent chains; the
// 256-entry table shortens the polynomial by three more FMAs); FP32: v_log_f32.
template <typename Real>
__device__ __forceinline__ Real k_log(Real x, const double2 *tab);
template <>
__device__ __forceinline__ double k_log<double>(double x, const double2 *tab) { return log_tab64(x, tab); }
template <>
__device__ __forceinline__ float k_log<float>(float x, const double2 *) { return __logf(x); }

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
    // linear index b over the upper-triangle tiles, row by row; the FP32 estimate
    // of the row is corrected by the two integer loops below
    const float tn = 2.0f * float(nb) + 1.0f;
    int r = int((tn - __builtin_sqrtf(fmaxf(tn * tn - 8.0f * float(b), 0.0f))) * 0.5f);
    if (r < 0) r = 0;
    while (r > 0 && r * nb - (r * (r - 1)) / 2 > b) --r;
    while ((r + 1) * nb - ((r + 1) * r) / 2 <= b) ++r;
    bi = r;
    bj = r + (b - (r * nb - (r * (r - 1)) / 2));
}

// The LDS of one tile: the two node windows, the table slices (WQ) or element
// indices (plain form), the stage-1 sums and the output tile.
template <int P, int Q, bool WQ, typename Real, int T>
struct TileLds {
    static constexpr int L = P * (T - 1) + Q;     // points in each window
    static constexpr int LT = 2 * L - 1;          // table slice for n2 - n1
    static constexpr int TW = (T % 2 == 0) ? T + 2 : T + 1;   // row pitch: even for paired columns
    using Real2 = typename std::conditional<sizeof(Real) == 8, double2, float2>::type;
    double *sx1, *sy1, *sx2, *sy2;
    Real *sJ1, *sJ2;
    int *se1, *se2;
    // sinvz[dl] = ((pi / sin(pi d / npts))^2, 1 if d = 0 else 0) of the slice; sw[par * LT + dl]
    Real2 *sinvz;
    Real *sw;
    Real (*C1)[TW];
    Real (*tileo)[TW];
    // bytes of the arrays carved one after another, each on 16 bytes
    static constexpr size_t al(size_t b) { return (b + 15) & ~size_t(15); }
    static constexpr size_t bytes()
    {
        return 4 * al(8 * L) + 2 * al(sizeof(Real) * L) + 2 * al(4 * (WQ ? 1 : L)) + al(sizeof(Real2) * (WQ ? LT : 1)) +
               al(sizeof(Real) * (WQ ? 2 * LT : 1)) + al(sizeof(Real) * L * TW) + al(sizeof(Real) * T * TW);
    }
};

// Where a tile's LDS lives: static arrays per instantiation (a kernel that
// inlines one tile variant), or, with DYN, the kernel's dynamic LDS, which every
// variant a kernel inlines then shares (the launch gives TileLds::bytes() of
// the largest).
template <int P, int Q, bool WQ, typename Real, int T, bool DYN>
__device__ __forceinline__ TileLds<P, Q, WQ, Real, T> tile_lds()
{
    using M = TileLds<P, Q, WQ, Real, T>;
    constexpr int L = M::L, LT = M::LT, TW = M::TW;
    using Real2 = typename M::Real2;
    M m;
    if constexpr (DYN) {
        extern __shared__ __align__(16) char tile_dyn_lds[];
        char *p = tile_dyn_lds;
        auto take = [&p](size_t b) { char *q = p; p += M::al(b); return q; };
        m.sx1 = reinterpret_cast<double *>(take(8 * L));
        m.sy1 = reinterpret_cast<double *>(take(8 * L));
        m.sx2 = reinterpret_cast<double *>(take(8 * L));
        m.sy2 = reinterpret_cast<double *>(take(8 * L));
        m.sJ1 = reinterpret_cast<Real *>(take(sizeof(Real) * L));
        m.sJ2 = reinterpret_cast<Real *>(take(sizeof(Real) * L));
        m.se1 = reinterpret_cast<int *>(take(4 * (WQ ? 1 : L)));
        m.se2 = reinterpret_cast<int *>(take(4 * (WQ ? 1 : L)));
        m.sinvz = reinterpret_cast<Real2 *>(take(sizeof(Real2) * (WQ ? LT : 1)));
        m.sw = reinterpret_cast<Real *>(take(sizeof(Real) * (WQ ? 2 * LT : 1)));
        m.C1 = reinterpret_cast<Real(*)[TW]>(take(sizeof(Real) * L * TW));
        m.tileo = reinterpret_cast<Real(*)[TW]>(take(sizeof(Real) * T * TW));
    } else {
        __shared__ double sx1[L], sy1[L], sx2[L], sy2[L];
        __shared__ Real sJ1[L], sJ2[L];
        __shared__ int se1[WQ ? 1 : L], se2[WQ ? 1 : L];
        __shared__ Real2 sinvz[WQ ? LT : 1];
        __shared__ Real sw[WQ ? 2 * LT : 1];
        __shared__ __align__(16) Real C1[L][TW];
        __shared__ __align__(16) Real tileo[T][TW];
        m.sx1 = sx1; m.sy1 = sy1; m.sx2 = sx2; m.sy2 = sy2;
        m.sJ1 = sJ1; m.sJ2 = sJ2; m.se1 = se1; m.se2 = se2;
        m.sinvz = sinvz; m.sw = sw; m.C1 = C1; m.tileo = tileo;
    }
    return m;
}

// One T x T tile (bi <= bj) of one matrix: the whole sweep-and-contract.
template <int P, int Q, int S0, bool WQ, typename Real, typename OutT, int T, int S, bool DYN = false, typename Args,
          typename ArgsF>
__device__ __forceinline__ void tile_body(const Args &a, const ArgsF &af, int bi, int bj)
{
    using M = TileLds<P, Q, WQ, Real, T>;
    constexpr int L = M::L;
    constexpr int LT = M::LT;
    constexpr int NSTRIP = T / S;
    constexpr int W2 = P * (S - 1) + Q;    // n2 points swept by one strip
    static_assert(T % S == 0, "strip must divide tile");

    const M m = tile_lds<P, Q, WQ, Real, T, DYN>();
    double *const sx1 = m.sx1, *const sy1 = m.sy1, *const sx2 = m.sx2, *const sy2 = m.sy2;
    Real *const sJ1 = m.sJ1, *const sJ2 = m.sJ2;
    int *const se1 = m.se1, *const se2 = m.se2;
    using Real2 = typename M::Real2;
    Real2 *const sinvz = m.sinvz;
    Real *const sw = m.sw;
    Real(*const C1)[M::TW] = m.C1;
    Real(*const tileo)[M::TW] = m.tileo;
    constexpr bool kTableLog = sizeof(Real) == 8;
    double2 *ltab = nullptr;
    if constexpr (kTableLog) {
        ltab = log_tab_lds();
        load_log_tab(ltab);
    }

    const int N = a.N, npts = a.npts;
    const int I0 = bi * T, J0 = bj * T;
    const int start1 = (P * I0 + S0) % npts;
    const int start2 = (P * J0 + S0) % npts;

    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        // start + r < 2 npts whenever the window is not longer than the grid
        int g1 = start1 + r, g2 = start2 + r;
        if (L <= npts) {
            g1 = g1 >= npts ? g1 - npts : g1;
            g2 = g2 >= npts ? g2 - npts : g2;
        } else {
            g1 %= npts;
            g2 %= npts;
        }
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
            int d = dbase + dl;
            if (LT <= npts) d = d >= npts ? d - npts : d;
            else d %= npts;
            const Real z = d == 0 ? Real(1) : Real(0);
            if constexpr (sizeof(Real) == 8) {
                sinvz[dl] = Real2{Real(a.inv_s2[d]), z};
                sw[dl] = Real(a.ws[d]);
                sw[LT + dl] = Real(a.ws[npts + d]);
            } else {
                sinvz[dl] = Real2{Real(a.inv_s2f[d]), z};
                sw[dl] = Real(a.wsf[d]);
                sw[LT + dl] = Real(a.wsf[npts + d]);
            }
        }
    }
    __syncthreads();

    // halved regular weights of stage 1 (exact: a power of two)
    Real ah[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) ah[q] = Real(0.5) * coef_a<Real>(a, af, q);

    // ---------------- stage 1: kernel sweep and contraction over the n2 supports
    for (int item = threadIdx.x; item < L * NSTRIP; item += blockDim.x) {
        const int r = item % L;
        const int st = item / L;
        const double x1 = sx1[r], y1 = sy1[r];
        const Real J1 = sJ1[r];
        const Real J1sq = J1 * J1;
        const int par = (start1 + r) & 1;     // npts is even: the parity of the node index
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
            // U = 2 K1 (the 1/2 of K1 = 1/2 ln(...) sits in the halved weights ah[q])
            Real U, V = Real(0);
            if constexpr (WQ) {
                // the diagonal (d = 0, z = 1, inv = 0) is the same node: r2 = 0 exactly, and
                // the ratio is J1^2; elsewhere z = 0 and the ratio is r2 * inv.  No
                // conditional on r2, so that the node loads are not sunk into a branch per
                // kernel value.
                const int dl = c2 - r + (L - 1);
                const Real2 iz = sinvz[dl];
                const Real ratio = fma(J1sq, iz.y, r2 * iz.x);
                U = k_log<Real>(ratio, ltab);
                V = swp[dl];
            } else {
                int de = se2[c2] - e1;
                if (de < 0) de += N;
                const bool near = (de == 0) | (de == 1) | (de == N - 1);
                U = near ? Real(0) : k_log<Real>(r2, ltab);
            }
            const Real J2 = sJ2[c2];
            const Real JU = J2 * U, JV = J2 * V;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int q = k2 - s * P;
                if (q >= 0 && q < Q) {
                    acc[s] = fma(ah[q], JU, acc[s]);
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
    if constexpr (T % 2 == 0) {
        // two adjacent columns per work item (one paired LDS read per support point)
        constexpr int TP = T / 2;
        for (int e = threadIdx.x; e < T * TP; e += blockDim.x) {
            const int il = e / TP, jl = 2 * (e - (e / TP) * TP);
            Real v0 = Real(0), v1 = Real(0);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const Real2 c = *reinterpret_cast<const Real2 *>(&C1[P * il + q][jl]);
                const Real w = coef_a<Real>(a, af, q);
                v0 += w * c.x;
                v1 += w * c.y;
            }
            *reinterpret_cast<Real2 *>(&tileo[il][jl]) = Real2{v0 * scale, v1 * scale};
        }
    } else {
        for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
            const int il = e / T, jl = e % T;
            Real v = Real(0);
#pragma unroll
            for (int q = 0; q < Q; ++q) v += coef_a<Real>(a, af, q) * C1[P * il + q][jl];
            tileo[il][jl] = v * scale;
        }
    }
    __syncthreads();

    OutT *out = reinterpret_cast<OutT *>(a.out);
    const int64_t lda = a.lda;
    // an off-diagonal tile inside the matrix, with every pair of columns (j even from J0)
    // aligned for one paired store: no per-entry checks
    using OutT2 = typename std::conditional<sizeof(OutT) == 8, double2, float2>::type;
    const bool paired = (T % 2 == 0) && bi != bj && I0 + T <= N && J0 + T <= N &&
                        ((reinterpret_cast<uintptr_t>(out) | uintptr_t(lda) * sizeof(OutT)) % (2 * sizeof(OutT))) == 0;
    if (paired) {
        constexpr int TP = T / 2;
        for (int e = threadIdx.x; e < T * TP; e += blockDim.x) {
            const int rl = e / TP, cl = 2 * (e - (e / TP) * TP);
            const Real2 v = *reinterpret_cast<const Real2 *>(&tileo[rl][cl]);
            *reinterpret_cast<OutT2 *>(out + int64_t(I0 + rl) * lda + J0 + cl) = OutT2{OutT(v.x), OutT(v.y)};
            // mirror: row J0 + rl, columns I0 + cl, I0 + cl + 1
            *reinterpret_cast<OutT2 *>(out + int64_t(J0 + rl) * lda + I0 + cl) =
                OutT2{OutT(tileo[cl][rl]), OutT(tileo[cl + 1][rl])};
        }
        __syncthreads();   // LDS is reused by the next tile of a persistent block
        return;
    }
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
// NT: threads per workgroup (a multiple of 64; the sweep's L T/S items are
// spread over them).
template <int P, int Q, int S0, bool WQ, typename Real, typename OutT, int T, int S, int WPE, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void tile_kernel(TileArgs a, TileArgsF af)
{
    const int nb = (a.N + T - 1) / T;
    // workgroups go round-robin to the 8 XCDs; give each XCD a contiguous run of tiles
    // (row by row), so that neighbouring tiles writing the same output lines share an L2
    const int ntiles = nb * (nb + 1) / 2;
    const int q = ntiles >> 3, rem = ntiles & 7;
    const int x = int(blockIdx.x & 7), k = int(blockIdx.x >> 3);
    int bi, bj;
    tile_coords(nb, x * q + min(x, rem) + k, bi, bj);
    tile_body<P, Q, S0, WQ, Real, OutT, T, S>(a, af, bi, bj);
}

template <int P, int Q, int S0, bool WQ, typename Real, int T, int S, int WPE = 1, int NT = 256>
hipError_t launch_tile(const TileArgs &a, hipStream_t s, const KernelEvents *ev = nullptr)
{
    static_assert(NT % 64 == 0 && NT <= 1024, "workgroup size");
    TileArgsF af;
    for (int q = 0; q < 64; ++q) {
        af.coefA[q] = float(a.coefA[q]);
        af.coefB[q] = float(a.coefB[q]);
    }
    const int nb = (a.N + T - 1) / T;
    const int blocks = nb * (nb + 1) / 2;
    using OutT = Real;
    if (ev)
        hipExtLaunchKernelGGL((tile_kernel<P, Q, S0, WQ, Real, OutT, T, S, WPE, NT>), dim3(blocks), dim3(NT), 0, s,
                              ev->start, ev->stop, 0, a, af);
    else
        hipLaunchKernelGGL((tile_kernel<P, Q, S0, WQ, Real, OutT, T, S, WPE, NT>), dim3(blocks), dim3(NT), 0, s, a, af);
    return hipGetLastError();
}

}  // namespace sgbem
