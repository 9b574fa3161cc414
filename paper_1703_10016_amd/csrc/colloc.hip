// Collocation BEM with the weighted quadrature rules (the paper's Conclusions:
// the outer collocation node fixed, the new rules for the inner integral).
//
//   A_ij = scale * [ sum_q w0_q J(eta_n) K1(x_i, eta_n) + sum_q B_j(eta_n) J(eta_n) w_n^(x_i) ],
//   n = P j + 1 + q (the support nodes of B_j), x_i = node P i + R (p+1) (the
//   Greville abscissa of B_i, a node of eta), scale = -1/(2 pi),
//
// i.e. the first-stage column sums of the Galerkin row assembly (eqs. IK1e2,
// IK1e2_bis) at the collocation nodes, without the outer rule.  The matrix is not
// symmetric; every tile of it is computed.
#include <hip/hip_runtime.h>

#include "colloc.hpp"
#include "tile_kernel.hpp"

namespace sgbem {

template <int P, int Q, int TR, int TC, int S>
__global__ __launch_bounds__(256) void colloc_kernel(TileArgs a)
{
    constexpr int L2 = P * (TC - 1) + Q;       // column window points
    constexpr int SPAN1 = P * (TR - 1) + 1;    // nodes spanned by the tile's collocation nodes
    constexpr int LT = L2 + SPAN1 - 1;         // table slice for n2 - n1
    constexpr int NSTRIP = TC / S;
    constexpr int W2 = P * (S - 1) + Q;        // window points swept by one strip
    static_assert(TC % S == 0, "strip must divide tile");
    __shared__ double sx1[TR], sy1[TR], sJ1[TR];
    __shared__ double sx2[L2], sy2[L2], sJ2[L2];
    // sinvz[dl] = ((pi / sin(pi d / npts))^2, 1 if d = 0 else 0); sw[par * LT + dl]
    __shared__ double2 sinvz[LT];
    __shared__ double sw[2 * LT];
    double2 *ltab = log_tab_lds();
    load_log_tab(ltab);
    __shared__ double tileo[TR][TC + 1];

    const int N = a.N, npts = a.npts;
    const int nbc = (N + TC - 1) / TC;
    const int bi = blockIdx.x / nbc, bj = blockIdx.x - (blockIdx.x / nbc) * nbc;
    const int I0 = bi * TR, J0 = bj * TC;
    const int r0 = (P * I0 + (Q + 1) / 2) % npts;   // collocation node of row I0: P I0 + R (p + 1)
    const int start2 = (P * J0 + 1) % npts;         // first support node of column J0
    for (int r = threadIdx.x; r < TR; r += blockDim.x) {
        const int g1 = (r0 + P * r) % npts;
        sx1[r] = a.X[g1];
        sy1[r] = a.Y[g1];
        sJ1[r] = a.J[g1];
    }
    for (int r = threadIdx.x; r < L2; r += blockDim.x) {
        const int g2 = (start2 + r) % npts;
        sx2[r] = a.X[g2];
        sy2[r] = a.Y[g2];
        sJ2[r] = a.J[g2];
    }
    // slice index dl <-> d = (n2 - n1) mod npts with n2 = start2 + c, n1 = r0 + P r: dl = c - P r + SPAN1 - 1
    int dbase = (start2 - r0 - (SPAN1 - 1)) % npts;
    if (dbase < 0) dbase += npts;
    for (int dl = threadIdx.x; dl < LT; dl += blockDim.x) {
        const int d = (dbase + dl) % npts;
        sinvz[dl] = make_double2(a.inv_s2[d], d == 0 ? 1.0 : 0.0);
        sw[dl] = a.ws[d];
        sw[LT + dl] = a.ws[npts + d];
    }
    __syncthreads();

    // halved regular weights: the 1/2 of K1 = 1/2 ln(...) (exact: a power of two)
    double ah[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) ah[q] = 0.5 * a.coefA[q];
    for (int item = threadIdx.x; item < TR * NSTRIP; item += blockDim.x) {
        const int r = item % TR, st = item / TR;
        const double x1 = sx1[r], y1 = sy1[r], J1 = sJ1[r];
        const double J1sq = J1 * J1;
        const int par = (r0 + P * r) & 1;        // npts is even: the parity of the node index
        const double *swp = sw + par * LT;      // singular weights of this collocation node's class
        double acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = 0.0;
#pragma unroll
        for (int k2 = 0; k2 < W2; ++k2) {
            const int c2 = st * S * P + k2;
            const double dx = x1 - sx2[c2], dy = y1 - sy2[c2];
            const double r2 = dx * dx + dy * dy;
            const int dl = c2 - P * r + SPAN1 - 1;
            // the diagonal (z = 1, inv = 0) is the same node, r2 = 0 exactly: K1(s, s) = ln J(s)
            // (eq. F1_lim); U = 2 K1, the 1/2 sits in ah[q]
            const double2 iz = sinvz[dl];
            const double ratio = fma(J1sq, iz.y, r2 * iz.x);
            const double U = log_tab64(ratio, ltab);
            const double J2 = sJ2[c2];
            const double JU = J2 * U, JV = J2 * swp[dl];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int q = k2 - s * P;
                if (q >= 0 && q < Q) acc[s] = fma(ah[q], JU, fma(a.coefB[q], JV, acc[s]));
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) tileo[r][st * S + s] = a.scale * acc[s];
    }
    __syncthreads();
    double *out = static_cast<double *>(a.out);
    for (int e = threadIdx.x; e < TR * TC; e += blockDim.x) {
        const int il = e / TC, jl = e - (e / TC) * TC;
        const int i = I0 + il, j = J0 + jl;
        if (i < N && j < N) out[int64_t(i) * a.lda + j] = tileo[il][jl];
    }
}

__global__ void colloc_gather_kernel(int N, int npts, int P, int c0, const double *g, double *b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) b[i] = g[(P * i + c0) % npts];
}

namespace {
template <int P, int Q>
hipError_t launch_one(const TileArgs &a, hipStream_t s, const KernelEvents *ev)
{
    constexpr int TR = 64, TC = 32, S = 8;
    const int blocks = ((a.N + TR - 1) / TR) * ((a.N + TC - 1) / TC);
    if (ev)
        hipExtLaunchKernelGGL((colloc_kernel<P, Q, TR, TC, S>), dim3(blocks), dim3(256), 0, s, ev->start, ev->stop, 0, a);
    else
        hipLaunchKernelGGL((colloc_kernel<P, Q, TR, TC, S>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}
}  // namespace

bool colloc_supported(int p, int P) { return p >= 1 && p <= 6 && (P == 2 || P == 4); }

hipError_t launch_colloc(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev)
{
    switch (p * 16 + P) {
    case 18: return launch_one<2, 3>(a, s, ev);
    case 34: return launch_one<2, 5>(a, s, ev);
    case 50: return launch_one<2, 7>(a, s, ev);
    case 66: return launch_one<2, 9>(a, s, ev);
    case 82: return launch_one<2, 11>(a, s, ev);
    case 98: return launch_one<2, 13>(a, s, ev);
    case 20: return launch_one<4, 7>(a, s, ev);
    case 36: return launch_one<4, 11>(a, s, ev);
    case 52: return launch_one<4, 15>(a, s, ev);
    case 68: return launch_one<4, 19>(a, s, ev);
    case 84: return launch_one<4, 23>(a, s, ev);
    case 100: return launch_one<4, 27>(a, s, ev);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_colloc_gather(int N, int npts, int P, int c0, const double *g, double *b, hipStream_t s)
{
    hipLaunchKernelGGL(colloc_gather_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, npts, P, c0, g, b);
    return hipGetLastError();
}

}  // namespace sgbem
