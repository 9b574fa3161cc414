// Fast-form assembly on an open arc (Section 2, exterior problem in indirect
// form; eqs. IK1e2, IK1e2_bis with the rules of Alg. 1 and Alg. 2 on the node
// vector of Section 4).
//
// The non-uniform-knot tile kernel without the periodic wrap: row i's rule
// lives on the nodes n0[i] .. n0[i] + QM - 1 (zero-padded, n0 non-decreasing),
// so a tile's rows and columns each read one contiguous window of nodes; the
// singular weights come from the full table Ws[npts][npts]; the kernel split is
// the printed one:
//   K1(n1, n2) = 1/2 ln(|f1 - f2|^2 / (eta_n1 - eta_n2)^2),  K1(n, n) = ln J(n).
// Every tile of the matrix is computed (the rows of eq. IK1e2_bis are not mirrored).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "arc.hpp"
#include "tile_kernel.hpp"

namespace sgbem {

namespace {

template <int QM, int T, int S, int L>
__global__ __launch_bounds__(256) void arc_tile_kernel(ArcArgs a)
{
    static_assert(T % S == 0, "strip must divide tile");
    constexpr int NSTRIP = T / S;
    __shared__ double sx1[L], sy1[L], st1[L], sJ1[L], sx2[L], sy2[L], st2[L], sJ2[L];
    __shared__ int sg1[L], sg2[L];
    __shared__ int off1[T], off2[T];
    __shared__ double sW1[T][QM], sW2[T][QM], sB2[T][QM];
    __shared__ double C1[L][T + 1];
    double2 *ltab = log_tab_lds();
    load_log_tab(ltab);

    const int N = a.N, npts = a.npts;
    const int nb = (N + T - 1) / T;
    const int bi = blockIdx.x / nb, bj = blockIdx.x - (blockIdx.x / nb) * nb;
    const int I0 = bi * T, J0 = bj * T;
    const int base1 = a.n0[I0], base2 = a.n0[J0];
    for (int l = threadIdx.x; l < T; l += blockDim.x) {
        // rows / columns past N: the last row's offsets (never stored)
        off1[l] = a.n0[min(I0 + l, N - 1)] - base1;
        off2[l] = a.n0[min(J0 + l, N - 1)] - base2;
    }
    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        // window positions past the last node: the last node (weights there are zero)
        const int g1 = min(base1 + r, npts - 1), g2 = min(base2 + r, npts - 1);
        sg1[r] = g1;
        sx1[r] = a.X[g1];
        sy1[r] = a.Y[g1];
        sJ1[r] = a.J[g1];
        st1[r] = a.eta[g1];
        sg2[r] = g2;
        sx2[r] = a.X[g2];
        sy2[r] = a.Y[g2];
        sJ2[r] = a.J[g2];
        st2[r] = a.eta[g2];
    }
    for (int e = threadIdx.x; e < T * QM; e += blockDim.x) {
        const int l = e / QM, q = e - (e / QM) * QM;
        const int i = min(I0 + l, N - 1), j = min(J0 + l, N - 1);
        sW1[l][q] = a.W[int64_t(i) * QM + q];
        sW2[l][q] = a.W[int64_t(j) * QM + q];
        sB2[l][q] = a.Bv[int64_t(j) * QM + q];
    }
    __syncthreads();

    // rows of the first window actually used: up to the last row's support
    const int L1 = off1[T - 1] + QM;
    // ---------------- stage 1: kernel sweep and contraction over the n2 supports
    for (int item = threadIdx.x; item < L1 * NSTRIP; item += blockDim.x) {
        const int r = item % L1;
        const int st = item / L1;
        const double x1 = sx1[r], y1 = sy1[r], t1 = st1[r], J1 = sJ1[r];
        const int g1 = sg1[r];
        const double *wsrow = a.Ws + int64_t(g1) * npts;
        int o[S];
#pragma unroll
        for (int s = 0; s < S; ++s) o[s] = off2[st * S + s];
        double acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = 0.0;
        const int c_lo = o[0], c_hi = o[S - 1] + QM;
        for (int c2 = c_lo; c2 < c_hi; ++c2) {
            const int g2 = sg2[c2];
            const double dx = x1 - sx2[c2], dy = y1 - sy2[c2];
            // diagonal: the same node, |f1 - f2|^2 = 0 exactly; the parameter difference is
            // replaced by 1 there so that the quotient stays finite (no branch per value)
            const bool diag = g2 == g1;
            const double dt = diag ? 1.0 : t1 - st2[c2];
            const double ratio = (dx * dx + dy * dy) / (dt * dt) + (diag ? J1 * J1 : 0.0);
            const double U = 0.5 * log_tab64(ratio, ltab);
            const double V = wsrow[g2];
            const double J2 = sJ2[c2];
            const double JU = J2 * U, JV = J2 * V;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int q = c2 - o[s];
                if (q >= 0 && q < QM) {
                    const int jl = st * S + s;
                    acc[s] = fma(sW2[jl][q], JU, acc[s]);
                    acc[s] = fma(sB2[jl][q], JV, acc[s]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) C1[r][st * S + s] = J1 * acc[s];
    }
    __syncthreads();

    // ---------------- stage 2: contraction over the n1 supports, stored row by row
    double *out = a.out;
    const int64_t lda = a.lda;
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int il = e / T, jl = e % T;
        const int i = I0 + il, j = J0 + jl;
        if (i >= N || j >= N) continue;
        const int o1 = off1[il];
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < QM; ++q) v += sW1[il][q] * C1[o1 + q][jl];
        out[int64_t(i) * lda + j] = v * a.scale;
    }
}

template <int p, int P>
hipError_t launch_arc_tiles(const ArcArgs &a, hipStream_t s, const KernelEvents *ev)
{
    constexpr int T = kArcTile, S = 6;
    constexpr int QM = arc_qm(p, P), L = arc_window(p, P);
    const int nb = (a.N + T - 1) / T;
    const int blocks = nb * nb;
    if (ev)
        hipExtLaunchKernelGGL((arc_tile_kernel<QM, T, S, L>), dim3(blocks), dim3(256), 0, s, ev->start, ev->stop, 0, a);
    else
        hipLaunchKernelGGL((arc_tile_kernel<QM, T, S, L>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void rhs_arc_kernel(int N, int QM, const int32_t *n0, const int32_t *cnt, const double *W, const double *J,
                               const double *g, double *beta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    const int c = cnt[i], b = n0[i];
    for (int q = 0; q < c; ++q) s += W[int64_t(i) * QM + q] * J[b + q] * g[b + q];
    beta[i] = s;
}

}  // namespace

bool assemble_arc_supported(int p, int P) { return p >= 1 && p <= 6 && (P == 2 || P == 4); }

hipError_t launch_assemble_arc(int p, const ArcArgs &a, hipStream_t s, const KernelEvents *ev)
{
    switch (p * 16 + a.P) {
    case 18: return launch_arc_tiles<1, 2>(a, s, ev);
    case 20: return launch_arc_tiles<1, 4>(a, s, ev);
    case 34: return launch_arc_tiles<2, 2>(a, s, ev);
    case 36: return launch_arc_tiles<2, 4>(a, s, ev);
    case 50: return launch_arc_tiles<3, 2>(a, s, ev);
    case 52: return launch_arc_tiles<3, 4>(a, s, ev);
    case 66: return launch_arc_tiles<4, 2>(a, s, ev);
    case 68: return launch_arc_tiles<4, 4>(a, s, ev);
    case 82: return launch_arc_tiles<5, 2>(a, s, ev);
    case 84: return launch_arc_tiles<5, 4>(a, s, ev);
    case 98: return launch_arc_tiles<6, 2>(a, s, ev);
    case 100: return launch_arc_tiles<6, 4>(a, s, ev);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rhs_arc(int N, int QM, const int32_t *n0, const int32_t *cnt, const double *W, const double *J,
                          const double *g, double *beta, hipStream_t s)
{
    hipLaunchKernelGGL(rhs_arc_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, QM, n0, cnt, W, J, g, beta);
    return hipGetLastError();
}

}  // namespace sgbem
