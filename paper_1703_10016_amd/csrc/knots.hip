// Fast-form assembly on non-uniform periodic knots (Section 3; eqs. IK1e2,
// IK1e2_bis with the rules of Alg. 1 and Alg. 2 in their general form).
//
// The structure of the uniform tile kernel (tile_kernel.hpp) without its
// translation invariance: the regular weights and the B_j values come per row
// from W[N][Q] and Bv[N][Q] (staged in LDS for the tile's rows and columns),
// the singular weights from the full table Ws[2M][2M] (read once per kernel
// value), and the periodic kernel split from the node parameters:
//   K1(n1, n2) = 1/2 ln(|f1 - f2|^2 (pi / sin(pi (eta_n1 - eta_n2)))^2),  K1(n, n) = ln J(n).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "knots.hpp"
#include "tile_kernel.hpp"

namespace sgbem {

namespace {

constexpr double kPiK = 3.14159265358979323846264338327950288;

template <int P, int Q, int T, int S>
__global__ __launch_bounds__(256) void knot_tile_kernel(KnotArgs a)
{
    constexpr int L = P * (T - 1) + Q;     // nodes in each window
    constexpr int NSTRIP = T / S;
    constexpr int W2 = P * (S - 1) + Q;    // column-window nodes swept by one strip
    static_assert(T % S == 0, "strip must divide tile");
    __shared__ double sx1[L], sy1[L], st1[L], sJ1[L], sx2[L], sy2[L], st2[L], sJ2[L];
    __shared__ int sg1[L], sg2[L];
    __shared__ double sW1[T][Q], sW2[T][Q], sB2[T][Q];
    __shared__ double C1[L][T + 1];
    double2 *ltab = log_tab_lds();
    load_log_tab(ltab);
    __shared__ double tileo[T][T + 1];

    const int N = a.N, npts = a.npts;
    const int nb = (N + T - 1) / T;
    int bi, bj;
    tile_coords(nb, blockIdx.x, bi, bj);
    const int I0 = bi * T, J0 = bj * T;
    const int start1 = (P * I0 + 1) % npts, start2 = (P * J0 + 1) % npts;
    for (int r = threadIdx.x; r < L; r += blockDim.x) {
        const int g1 = (start1 + r) % npts, g2 = (start2 + r) % npts;
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
    for (int e = threadIdx.x; e < T * Q; e += blockDim.x) {
        const int l = e / Q, q = e - (e / Q) * Q;
        const int i = min(I0 + l, N - 1), j = min(J0 + l, N - 1);   // rows / columns past N: never stored
        sW1[l][q] = a.W[int64_t(i) * Q + q];
        sW2[l][q] = a.W[int64_t(j) * Q + q];
        sB2[l][q] = a.Bv[int64_t(j) * Q + q];
    }
    __syncthreads();

    // ---------------- stage 1: kernel sweep and contraction over the n2 supports
    for (int item = threadIdx.x; item < L * NSTRIP; item += blockDim.x) {
        const int r = item % L;
        const int st = item / L;
        const double x1 = sx1[r], y1 = sy1[r], t1 = st1[r], J1 = sJ1[r];
        const int g1 = sg1[r];
        const double *wsrow = a.Ws + int64_t(g1) * npts;
        double acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = 0.0;
        // not unrolled: each kernel value carries a sine and a division, and the
        // unrolled sweep held one wavefront per SIMD (380 registers)
#pragma unroll 1
        for (int k2 = 0; k2 < W2; ++k2) {
            const int c2 = st * S * P + k2;
            const int g2 = sg2[c2];
            const double dx = x1 - sx2[c2], dy = y1 - sy2[c2];
            const double r2 = dx * dx + dy * dy;
            double d = t1 - st2[c2];
            d -= rint(d);
            // diagonal: the same node, r2 = 0 exactly; sin replaced by 1 there so that the
            // product stays finite (no branch per kernel value around the node loads)
            const bool diag = g2 == g1;
            const double sp = diag ? 1.0 : sinpi(d);
            const double isp = kPiK / sp;
            const double ratio = fma(r2, isp * isp, diag ? J1 * J1 : 0.0);
            const double U = 0.5 * log_tab64(ratio, ltab);
            const double V = wsrow[g2];
            const double J2 = sJ2[c2];
            const double JU = J2 * U, JV = J2 * V;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int q = k2 - s * P;
                if (q >= 0 && q < Q) {
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

    // ---------------- stage 2: contraction over the n1 supports
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int il = e / T, jl = e % T;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) v += sW1[il][q] * C1[P * il + q][jl];
        tileo[il][jl] = v * a.scale;
    }
    __syncthreads();

    double *out = a.out;
    const int64_t lda = a.lda;
    for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
        const int il = e / T, jl = e % T;
        const int i = I0 + il, j = J0 + jl;
        if (i < N && j < N) out[int64_t(i) * lda + j] = (bi == bj && il > jl) ? tileo[jl][il] : tileo[il][jl];
    }
    if (bi != bj) {
        for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
            const int rl = e / T, cl = e % T;
            const int i = J0 + rl, j = I0 + cl;
            if (i < N && j < N) out[int64_t(i) * lda + j] = tileo[cl][rl];
        }
    }
}

template <int P, int Q>
hipError_t launch_knot_tiles(const KnotArgs &a, hipStream_t s, const KernelEvents *ev)
{
    constexpr int T = 24, S = 6;
    const int nb = (a.N + T - 1) / T;
    const int blocks = nb * (nb + 1) / 2;
    if (ev)
        hipExtLaunchKernelGGL((knot_tile_kernel<P, Q, T, S>), dim3(blocks), dim3(256), 0, s, ev->start, ev->stop, 0, a);
    else
        hipLaunchKernelGGL((knot_tile_kernel<P, Q, T, S>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void rhs_knots_kernel(int N, int npts, int P, int Q, const double *W, const double *J, const double *g,
                                 double *beta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int q = 0; q < Q; ++q) {
        const int n = int((int64_t(P) * i + 1 + q) % npts);
        s += W[int64_t(i) * Q + q] * J[n] * g[n];
    }
    beta[i] = s;
}

}  // namespace

bool assemble_knots_supported(int p, int P) { return p >= 1 && p <= 6 && (P == 2 || P == 4); }

hipError_t launch_assemble_knots(int p, const KnotArgs &a, hipStream_t s, const KernelEvents *ev)
{
    switch (p * 16 + a.P) {
    case 18: return launch_knot_tiles<2, 3>(a, s, ev);
    case 20: return launch_knot_tiles<4, 7>(a, s, ev);
    case 34: return launch_knot_tiles<2, 5>(a, s, ev);
    case 36: return launch_knot_tiles<4, 11>(a, s, ev);
    case 50: return launch_knot_tiles<2, 7>(a, s, ev);
    case 52: return launch_knot_tiles<4, 15>(a, s, ev);
    case 66: return launch_knot_tiles<2, 9>(a, s, ev);
    case 68: return launch_knot_tiles<4, 19>(a, s, ev);
    case 82: return launch_knot_tiles<2, 11>(a, s, ev);
    case 84: return launch_knot_tiles<4, 23>(a, s, ev);
    case 98: return launch_knot_tiles<2, 13>(a, s, ev);
    case 100: return launch_knot_tiles<4, 27>(a, s, ev);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rhs_knots(int N, int npts, int P, int Q, const double *W, const double *J, const double *g,
                            double *beta, hipStream_t s)
{
    hipLaunchKernelGGL(rhs_knots_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, npts, P, Q, W, J, g, beta);
    return hipGetLastError();
}

}  // namespace sgbem
