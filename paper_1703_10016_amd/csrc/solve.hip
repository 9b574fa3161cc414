// Mixed-precision solve of the Galerkin system A alpha = beta (eq. sistlin):
// FP32 LU with partial pivoting (blocked right-looking; panel on one
// workgroup, trailing update on FP32 MFMA), FP64 iterative refinement with the
// stored matrix.  The factor is kept column-major in the workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "solve.hpp"

namespace sgbem {

namespace {

constexpr int NB = 64;            // widest panel (register panels); longer panels use 32 columns
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct WS {
    float *LU;
    int *piv, *perm, *info;
    double *r;
    float *v, *v2;
    double *red;     // reduction outputs
    float *DI;       // inverted diagonal blocks
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

WS carve(void *base, int N)
{
    char *p = static_cast<char *>(base);
    WS w;
    w.LU = reinterpret_cast<float *>(p);
    p += align_up(size_t(N) * N * sizeof(float));
    w.piv = reinterpret_cast<int *>(p);
    p += align_up(size_t(N) * sizeof(int));
    w.perm = reinterpret_cast<int *>(p);
    p += align_up(size_t(N) * sizeof(int));
    w.info = reinterpret_cast<int *>(p);
    p += align_up(sizeof(int) * 4);
    w.r = reinterpret_cast<double *>(p);
    p += align_up(size_t(N) * sizeof(double));
    w.v = reinterpret_cast<float *>(p);
    p += align_up(size_t(N) * sizeof(float));
    w.v2 = reinterpret_cast<float *>(p);
    p += align_up(size_t(N) * sizeof(float));
    w.red = reinterpret_cast<double *>(p);
    p += align_up(64 * sizeof(double)) + align_up(size_t(N) * sizeof(double));
    w.DI = reinterpret_cast<float *>(p);
    return w;
}

__global__ void zero_int_kernel(int *p)
{
    if (threadIdx.x == 0) *p = 0;
}

// ---------------------------------------------------------------- copy / transpose
template <typename InT>
__global__ void to_colmajor_kernel(int N, const InT *A, int64_t lda, float *LU)
{
    __shared__ float t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int i = by + k, j = bx + tx;
        if (i < N && j < N) t[k][tx] = float(A[int64_t(i) * lda + j]);
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int j = bx + k, i = by + tx;     // LU column j, row i
        if (i < N && j < N) LU[int64_t(j) * N + i] = t[tx][k];
    }
}

// ---------------------------------------------------------------- panel
// Factor LU[k0:N, k0:k0+w] in place (one workgroup): for every column the
// pivot is the entry of largest magnitude (lowest row on ties), rows are
// swapped inside the panel, the column is scaled and the rest of the panel
// receives the rank-1 update.
__global__ __launch_bounds__(1024) void panel_kernel(int N, float *LU, int k0, int w, int *piv, int *info)
{
    __shared__ float smax[32];
    __shared__ int sidx[32];
    __shared__ float urow[NB];
    __shared__ int spiv;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    for (int j = k0; j < k0 + w; ++j) {
        float* colj = LU + int64_t(j) * N;
        float best = -1.0f;
        int bidx = N;
        for (int i = j + tid; i < N; i += blockDim.x) {
            const float v = fabsf(colj[i]);
            if (v > best || (v == best && i < bidx)) {
                best = v;
                bidx = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(best, off);
            const int oi = __shfl_xor(bidx, off);
            if (ov > best || (ov == best && oi < bidx)) {
                best = ov;
                bidx = oi;
            }
        }
        if (lane == 0) {
            smax[wid] = best;
            sidx[wid] = bidx;
        }
        __syncthreads();
        if (tid == 0) {
            float b = smax[0];
            int bi = sidx[0];
            for (int q = 1; q < nw; ++q)
                if (smax[q] > b || (smax[q] == b && sidx[q] < bi)) {
                    b = smax[q];
                    bi = sidx[q];
                }
            if (!(b > 0.0f)) {
                if (*info == 0) *info = j + 1;
                bi = j;
            }
            spiv = bi;
            piv[j] = bi;
        }
        __syncthreads();
        const int pr = spiv;
        if (pr != j) {
            for (int c = k0 + tid; c < k0 + w; c += blockDim.x) {
                float *col = LU + int64_t(c) * N;
                const float a = col[j];
                col[j] = col[pr];
                col[pr] = a;
            }
        }
        __syncthreads();
        for (int c = j + tid; c < k0 + w; c += blockDim.x) urow[c - k0] = LU[int64_t(c) * N + j];
        __syncthreads();
        const float d = urow[j - k0];
        if (d != 0.0f) {
            const float inv = 1.0f / d;
            for (int i = j + 1 + tid; i < N; i += blockDim.x) {
                const float l = colj[i] * inv;
                colj[i] = l;
                for (int c = j + 1; c < k0 + w; ++c) LU[int64_t(c) * N + i] -= l * urow[c - k0];
            }
        }
        __syncthreads();
    }
}

// Wavefront-wide max / min of a 32-bit unsigned value by DPP row operations
// (quad permutes, row shifts by 4 and 8, row broadcasts 15 and 31: lane 63
// ends with the result), returned uniform.  Every lane of the wavefront must be
// active.
template <bool MAX>
__device__ __forceinline__ unsigned wave_reduce_u32(unsigned v)
{
    auto op = [](unsigned a, unsigned b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
    v = op(v, unsigned(__builtin_amdgcn_update_dpp(int(v), int(v), 0xb1, 0xf, 0xf, false)));
    v = op(v, unsigned(__builtin_amdgcn_update_dpp(int(v), int(v), 0x4e, 0xf, 0xf, false)));
    v = op(v, unsigned(__builtin_amdgcn_update_dpp(int(v), int(v), 0x114, 0xf, 0xe, false)));
    v = op(v, unsigned(__builtin_amdgcn_update_dpp(int(v), int(v), 0x118, 0xf, 0xc, false)));
    v = op(v, unsigned(__builtin_amdgcn_update_dpp(int(v), int(v), 0x142, 0xa, 0xf, false)));
    v = op(v, unsigned(__builtin_amdgcn_update_dpp(int(v), int(v), 0x143, 0xc, 0xf, false)));
    return unsigned(__builtin_amdgcn_readlane(int(v), 63));
}

// Register-resident panel factorisation (one workgroup of 1024 threads, RT rows
// per thread, W <= 32 columns): thread t owns the panel rows k0 + r*1024 + t
// with all W columns in registers.  The column loop is unrolled, so every
// register index is a compile-time constant.  Per column: pivot = largest
// magnitude at or below the diagonal, lowest row on ties.  Each wavefront finds
// its own candidate (two DPP reductions: the largest magnitude, then the lowest
// row holding it) and publishes it with the candidate row's values; the owner
// of the diagonal row publishes that row.  After the column's one barrier every
// thread reduces the 16 candidates the same way (the winning wavefront is the
// owner of the pivot row), interchanges the two rows in registers (earlier L
// multipliers included: a row interchange of the panel), scales and updates
// the rows below.  The published values are double-buffered by column parity:
// a wavefront can write a buffer again only after the next column's barrier,
// which every wavefront reaches after its last read of it.  Global memory is
// touched only to load the panel and to store it, the pivots and info.
template <int RT, int W>
__global__ __launch_bounds__(1024) void panel_reg_kernel(int N, float *LU, int k0, int w, int *piv, int *info)
{
    __shared__ unsigned smag[2][16];
    __shared__ int srow[2][16];
    __shared__ float crow[2][16][W];     // each wavefront's candidate row
    __shared__ float jrow[2][W];         // the diagonal row
    __shared__ int pivs[W];
    __shared__ int sinfo;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) sinfo = 0;
    float a[RT][W];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int i = k0 + r * 1024 + tid;
#pragma unroll
        for (int c = 0; c < W; ++c) a[r][c] = (i < N && c < w) ? LU[int64_t(k0 + c) * N + i] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        if (j < w) {
            const int gj = k0 + j, buf = j & 1;
            // this thread's candidate: magnitude bits (monotone for non-negative floats), lowest row on ties
            unsigned mag = 0u;
            int row = 0x7fffffff;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int i = k0 + r * 1024 + tid;
                const unsigned m = __float_as_uint(fabsf(a[r][j]));
                if (i >= gj && i < N && (m > mag || (m == mag && i < row))) {
                    mag = m;
                    row = i;
                }
            }
            const unsigned wmag = wave_reduce_u32<true>(mag);
            const int wrow = int(wave_reduce_u32<false>(mag == wmag ? unsigned(row) : 0x7fffffffu));
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int i = k0 + r * 1024 + tid;
                if (i == wrow) {
#pragma unroll
                    for (int c = 0; c < W; ++c) crow[buf][wid][c] = a[r][c];
                }
                if (i == gj) {
#pragma unroll
                    for (int c = 0; c < W; ++c) jrow[buf][c] = a[r][c];
                }
            }
            if (lane == 0) {
                smag[buf][wid] = wmag;
                srow[buf][wid] = wrow;
            }
            __syncthreads();
            const unsigned cm = smag[buf][lane & 15], cr = unsigned(srow[buf][lane & 15]);
            const unsigned gm = wave_reduce_u32<true>(lane < 16 ? cm : 0u);
            const int gr = int(wave_reduce_u32<false>(lane < 16 && cm == gm ? cr : 0x7fffffffu));
            const float b = __uint_as_float(gm);
            const bool ok = b > 0.0f;
            const int pr = ok ? gr : gj;
            const float *prow = ok ? crow[buf][((pr - k0) & 1023) >> 6] : jrow[buf];
            if (tid == 0) {
                if (!ok && sinfo == 0) sinfo = gj + 1;
                pivs[j] = pr;
            }
            const float d = prow[j];
            const float inv = ok ? 1.0f / d : 0.0f;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int i = k0 + r * 1024 + tid;
                if (i == gj) {
#pragma unroll
                    for (int c = 0; c < W; ++c) a[r][c] = prow[c];
                } else if (i == pr) {
#pragma unroll
                    for (int c = 0; c < W; ++c) a[r][c] = jrow[buf][c];
                }
                if (i > gj && i < N && ok) {
                    const float l = a[r][j] * inv;
                    a[r][j] = l;
#pragma unroll
                    for (int c = j + 1; c < W; ++c) a[r][c] -= l * prow[c];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int i = k0 + r * 1024 + tid;
#pragma unroll
        for (int c = 0; c < W; ++c)
            if (i < N && c < w) LU[int64_t(k0 + c) * N + i] = a[r][c];
    }
    __syncthreads();
    if (tid < w) piv[k0 + tid] = pivs[tid];
    if (tid == 0 && sinfo != 0 && *info == 0) *info = sinfo;
}

// Apply the panel's interchanges to the columns outside it.
__global__ void laswp_kernel(int N, float *LU, int k0, int w, const int *piv)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N - w) return;
    if (c >= k0) c += w;
    float *col = LU + int64_t(c) * N;
    for (int j = k0; j < k0 + w; ++j) {
        const int pr = piv[j];
        if (pr != j) {
            const float a = col[j];
            col[j] = col[pr];
            col[pr] = a;
        }
    }
}

// For the narrow panel at k0 (w <= 64 columns), on the block columns
// [cb, ce) outside the panel: apply the panel's row interchanges, then for the
// columns right of the panel solve U12 = L11^{-1} A12.  One wavefront per
// column: lane 0 applies the interchanges in order, the workgroup barrier makes
// them visible, then lane r holds row k0 + r for the solve.
__global__ __launch_bounds__(256) void swap_trsm_kernel(int N, float *LU, int k0, int w, const int *piv, int cb, int ce)
{
    __shared__ float L[NB][NB + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += blockDim.x) {
        const int r = e % w, c = e / w;
        L[r][c] = LU[int64_t(k0 + c) * N + k0 + r];
    }
    const int lane = tid & 63;
    int col = cb + blockIdx.x * 4 + (tid >> 6);
    if (col >= k0) col += w;
    const bool valid = col < ce;
    float *cp = LU + int64_t(valid ? col : 0) * N;
    if (valid && lane == 0) {
        for (int j = k0; j < k0 + w; ++j) {
            const int pr = piv[j];
            if (pr != j) {
                const float a = cp[j];
                cp[j] = cp[pr];
                cp[pr] = a;
            }
        }
    }
    __syncthreads();
    if (!valid || col < k0) return;
    cp += k0;
    float x = lane < w ? cp[lane] : 0.0f;
    for (int s = 0; s < w; ++s) {
        const float xs = __shfl(x, s);
        if (lane > s && lane < w) x -= L[lane][s] * xs;
    }
    if (lane < w) cp[lane] = x;
}

// U12 = L11^{-1} A12 for a block of bk <= 128 factored columns at K0, on the
// columns [c0, N): L11 (unit lower) in LDS; each wavefront solves two columns
// at once (their dependent chains interleave), lane l holding rows K0 + l and
// K0 + 64 + l of both, the solved value of each step broadcast by readlane.
__global__ __launch_bounds__(1024) void trsm_block_kernel(int N, float *LU, int K0, int bk, int c0)
{
    __shared__ float L[128][129];
    const int tid = threadIdx.x;
    for (int e = tid; e < bk * bk; e += blockDim.x) {
        const int r = e % bk, c = e / bk;
        L[r][c] = LU[int64_t(K0 + c) * N + K0 + r];
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int ca = c0 + blockIdx.x * 32 + 2 * wave, cb = ca + 1;
    if (ca >= N) return;
    const bool hb = cb < N;
    float *pa = LU + int64_t(ca) * N + K0;
    float *pb = LU + int64_t(hb ? cb : ca) * N + K0;
    float x0a = lane < bk ? pa[lane] : 0.0f, x1a = lane + 64 < bk ? pa[lane + 64] : 0.0f;
    float x0b = lane < bk ? pb[lane] : 0.0f, x1b = lane + 64 < bk ? pb[lane + 64] : 0.0f;
    for (int s = 0; s < bk; ++s) {
        const float xa = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s < 64 ? x0a : x1a), s & 63));
        const float xb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s < 64 ? x0b : x1b), s & 63));
        if (lane > s && lane < bk) {
            const float l = L[lane][s];
            x0a -= l * xa;
            x0b -= l * xb;
        }
        if (lane + 64 > s && lane + 64 < bk) {
            const float l = L[lane + 64][s];
            x1a -= l * xa;
            x1b -= l * xb;
        }
    }
    if (lane < bk) pa[lane] = x0a;
    if (lane + 64 < bk) pa[lane + 64] = x1a;
    if (hb) {
        if (lane < bk) pb[lane] = x0b;
        if (lane + 64 < bk) pb[lane + 64] = x1b;
    }
}

// C -= L21 U12 on FP32 MFMA (16x16x4) for C = LU[r0:N, c0:cend],
// L21 = LU[r0:N, kb:kb+klen], U12 = LU[kb:kb+klen, c0:cend]: the workgroup owns a
// 64 x 64 block of C, each wavefront a 32 x 32 quarter as 2 x 2 MFMA tiles; K
// runs in chunks of 32 staged through LDS (zero-padded past klen).  The MFMA
// "rows" index the columns of C and its "columns" the rows of C, so each lane's
// results are contiguous in the column-major factor.
__global__ __launch_bounds__(256) void gemm_update_kernel(int N, float *LU, int r0, int c0, int cend, int kb, int klen)
{
    __shared__ float As[64][33];   // L21 chunk: [row][k]
    __shared__ float Bs[64][33];   // U12 chunk transposed: [col][k]
    const int m0 = r0 + blockIdx.x * 64;    // first row of C
    const int n0 = c0 + blockIdx.y * 64;    // first column of C
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wc = (wave >> 1) * 32;    // C columns of this wave
    const int wr = (wave & 1) * 32;     // C rows of this wave
    floatx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kc = 0; kc < klen; kc += 32) {
        const int kl = min(32, klen - kc);
        for (int e = tid; e < 64 * 32; e += blockDim.x) {
            const int r = e & 63, k = e >> 6;
            As[r][k] = (m0 + r < N && k < kl) ? LU[int64_t(kb + kc + k) * N + m0 + r] : 0.0f;
        }
        for (int e = tid; e < 64 * 32; e += blockDim.x) {
            const int k = e & 31, c = e >> 5;
            Bs[c][k] = (n0 + c < cend && k < kl) ? LU[int64_t(n0 + c) * N + kb + kc + k] : 0.0f;
        }
        __syncthreads();
        for (int k = 0; k < kl; k += 4) {
            const int kk = k + (lane >> 4);
            for (int a = 0; a < 2; ++a) {
                const float av = Bs[wc + a * 16 + (lane & 15)][kk];   // MFMA A: [C column][k]
                for (int b = 0; b < 2; ++b) {
                    const float bv = As[wr + b * 16 + (lane & 15)][kk]; // MFMA B: [k][C row]
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[a][b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int i = 0; i < 4; ++i) {
                const int c = n0 + wc + a * 16 + 4 * (lane >> 4) + i;
                const int r = m0 + wr + b * 16 + (lane & 15);
                if (r < N && c < cend) LU[int64_t(c) * N + r] -= acc[a][b][i];
            }
}

// ---------------------------------------------------------------- triangular solves
// One launch per 64-row block; every workgroup solves the diagonal block
// (the same arithmetic in each) and then updates its own rows.
// Inverses of the 64 x 64 diagonal blocks of L (unit lower) and U, kept so
// that every block step of the triangular solves is a plain matrix-vector
// product.  DI[b][0] = inv(L_bb), DI[b][1] = inv(U_bb), row-major 64 x 64;
// a partial last block is padded with the identity.
__global__ __launch_bounds__(64) void invert_diag_kernel(int N, const float *LU, float *DI)
{
    __shared__ float T[64][65];
    __shared__ float X[64][65];
    const int b0 = blockIdx.x * 64, bw = min(64, N - b0);
    const int c = threadIdx.x;
    for (int r = 0; r < 64; ++r) T[r][c] = (r < bw && c < bw) ? LU[int64_t(b0 + c) * N + b0 + r] : (r == c ? 1.0f : 0.0f);
    __syncthreads();
    // L X = I, column c: X[r][c] = delta_rc - sum_{k<r} L[r][k] X[k][c]
    for (int r = 0; r < 64; ++r) {
        float s = (r == c) ? 1.0f : 0.0f;
        for (int k = 0; k < r; ++k) s -= T[r][k] * X[k][c];
        X[r][c] = s;
    }
    for (int r = 0; r < 64; ++r) DI[(int64_t(blockIdx.x) * 2 + 0) * 4096 + r * 64 + c] = X[r][c];
    __syncthreads();
    // U X = I, column c: X[r][c] = (delta_rc - sum_{k>r} U[r][k] X[k][c]) / U[r][r]
    for (int r = 63; r >= 0; --r) {
        float s = (r == c) ? 1.0f : 0.0f;
        for (int k = r + 1; k < 64; ++k) s -= T[r][k] * X[k][c];
        X[r][c] = s / T[r][r];
    }
    for (int r = 0; r < 64; ++r) DI[(int64_t(blockIdx.x) * 2 + 1) * 4096 + r * 64 + c] = X[r][c];
}

// Forward step for the 64-row block at b0: x_b = inv(L_bb) y_b (computed by
// every workgroup), written to yout by workgroup 0; rows below are updated in
// y (rows of the block itself are only read in this launch).
__global__ __launch_bounds__(256) void trsv_lower_kernel(int N, const float *LU, const float *DI, float *y, float *yout, int b0)
{
    __shared__ float yb[64], xb[64];
    const int bw = min(64, N - b0);
    const int tid = threadIdx.x;
    if (tid < 64) yb[tid] = tid < bw ? y[b0 + tid] : 0.0f;
    __syncthreads();
    if (tid < 64) {
        const float *row = DI + (int64_t(b0 / 64) * 2 + 0) * 4096 + tid * 64;
        float s = 0.0f;
        for (int k = 0; k < 64; ++k) s += row[k] * yb[k];
        xb[tid] = s;
        if (blockIdx.x == 0 && tid < bw) yout[b0 + tid] = s;
    }
    __syncthreads();
    const int r = b0 + bw + blockIdx.x * blockDim.x + tid;
    if (r < N) {
        float s = 0.0f;
        for (int k = 0; k < bw; ++k) s += LU[int64_t(b0 + k) * N + r] * xb[k];
        y[r] -= s;
    }
}

__global__ __launch_bounds__(256) void trsv_upper_kernel(int N, const float *LU, const float *DI, float *y, float *yout, int b0, int bw)
{
    __shared__ float yb[64], xb[64];
    const int tid = threadIdx.x;
    if (tid < 64) yb[tid] = tid < bw ? y[b0 + tid] : 0.0f;
    __syncthreads();
    if (tid < 64) {
        const float *row = DI + (int64_t(b0 / 64) * 2 + 1) * 4096 + tid * 64;
        float s = 0.0f;
        for (int k = 0; k < 64; ++k) s += row[k] * yb[k];
        xb[tid] = s;
        if (blockIdx.x == 0 && tid < bw) yout[b0 + tid] = s;
    }
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + tid;
    if (r < b0) {
        float s = 0.0f;
        for (int k = 0; k < bw; ++k) s += LU[int64_t(b0 + k) * N + r] * xb[k];
        y[r] -= s;
    }
}

__global__ void permute_kernel(int N, const int *perm, const double *src, float *dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dst[i] = float(src[perm[i]]);
}

// ---------------------------------------------------------------- refinement pieces
// r = beta - A x (FP64), one wavefront per row; A row-major as stored.
template <typename InT>
__global__ __launch_bounds__(256) void residual_kernel(int N, const InT *A, int64_t lda, const double *x,
                                                       const double *beta, double *r)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const InT *a = A + int64_t(row) * lda;
    double s = 0.0;
    for (int j = lane; j < N; j += 64) s += double(a[j]) * x[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) r[row] = beta[row] - s;
}

template <typename InT>
__global__ __launch_bounds__(256) void rowabs_kernel(int N, const InT *A, int64_t lda, double *rs)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const InT *a = A + int64_t(row) * lda;
    double s = 0.0;
    for (int j = lane; j < N; j += 64) s += fabs(double(a[j]));
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) rs[row] = s;
}

// x += d (d FP32), and max-norms: red[0] = |d|_inf, red[1] = |x|_inf, red[2] = |r|_inf, red[3] = |beta|_inf
__global__ __launch_bounds__(1024) void update_norms_kernel(int N, double *x, const float *d, const double *r,
                                                            const double *beta, int add, double *red)
{
    __shared__ double s[4][16];
    double m[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double xi = add ? x[i] + double(d[i]) : double(d[i]);
        x[i] = xi;
        m[0] = fmax(m[0], fabs(double(d[i])));
        m[1] = fmax(m[1], fabs(xi));
        m[2] = fmax(m[2], fabs(r[i]));
        m[3] = fmax(m[3], fabs(beta[i]));
    }
    for (int q = 0; q < 4; ++q) {
        for (int off = 32; off > 0; off >>= 1) m[q] = fmax(m[q], __shfl_xor(m[q], off));
        if ((threadIdx.x & 63) == 0) s[q][threadIdx.x >> 6] = m[q];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) v = fmax(v, s[threadIdx.x][k]);
        red[threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(1024) void max_kernel(int N, const double *v, double *out)
{
    __shared__ double s[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) m = fmax(m, fabs(v[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v2 = 0.0;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) v2 = fmax(v2, s[k]);
        *out = v2;
    }
}

template <typename InT>
void launch_residual(int N, const void *A, int64_t lda, const double *x, const double *beta, double *r, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel<InT>, dim3((N + 3) / 4), dim3(256), 0, s, N, static_cast<const InT *>(A), lda,
                       x, beta, r);
}

}  // namespace

size_t solve_workspace_bytes(int N)
{
    const size_t nblk = size_t(N + 63) / 64;
    return align_up(size_t(N) * N * sizeof(float)) + 2 * align_up(size_t(N) * sizeof(int)) + align_up(16) +
           align_up(size_t(N) * sizeof(double)) + 2 * align_up(size_t(N) * sizeof(float)) + align_up(64 * sizeof(double)) +
           align_up(size_t(N) * sizeof(double)) + align_up(nblk * 2 * 4096 * sizeof(float));
}

hipError_t lu_factor_f32(int N, float *LU, int *piv, int *info, void *diag_inv, hipStream_t s)
{
    // Two levels: blocks of BK columns, each factored by narrow register panels
    // whose triangular solves and updates stay inside the block; then one
    // triangular solve for the block's U12 and one rank-BK update of the
    // trailing matrix (the MFMA-bound part).  Row interchanges always go to
    // the full rows.  Up to N = 4096 one block spans the matrix (every narrow
    // panel updates the whole trailing matrix): there the launches saved
    // outweigh the traffic of the narrow updates (measured).
    const int BK = N <= 4096 ? N : 128;
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, info);
    for (int K0 = 0; K0 < N; K0 += BK) {
        const int KE = std::min(N, K0 + BK);
        for (int k0 = K0; k0 < KE;) {
            const int m = N - k0;
            int w;
            // register panels while the rows fit (1, 2, 4, 8 rows per thread), narrower as they grow
            if (m <= 1024) {
                w = std::min(32, KE - k0);
                hipLaunchKernelGGL((panel_reg_kernel<1, 32>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
            } else if (m <= 2048) {
                w = std::min(16, KE - k0);
                hipLaunchKernelGGL((panel_reg_kernel<2, 16>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
            } else if (m <= 4096) {
                w = std::min(8, KE - k0);
                hipLaunchKernelGGL((panel_reg_kernel<4, 8>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
            } else if (m <= 8192) {
                w = std::min(8, KE - k0);
                hipLaunchKernelGGL((panel_reg_kernel<8, 8>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
            } else {
                w = std::min(32, KE - k0);
                hipLaunchKernelGGL(panel_kernel, dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
            }
            // the panel's interchanges on the other block columns, U12 right of it
            const int others = KE - K0 - w;
            if (others > 0)
                hipLaunchKernelGGL(swap_trsm_kernel, dim3((others + 3) / 4), dim3(256), 0, s, N, LU, k0, w, piv, K0, KE);
            const int rin = KE - k0 - w;   // block columns right of the narrow panel
            if (rin > 0)
                hipLaunchKernelGGL(gemm_update_kernel, dim3((N - k0 - w + 63) / 64, (rin + 63) / 64), dim3(256), 0, s,
                                   N, LU, k0 + w, k0 + w, KE, k0, w);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            k0 += w;
        }
        // the block's interchanges on the columns outside it (left: L of earlier blocks; right: A12, A22)
        if (N - (KE - K0) > 0)
            hipLaunchKernelGGL(laswp_kernel, dim3((N - (KE - K0) + 255) / 256), dim3(256), 0, s, N, LU, K0, KE - K0, piv);
        const int rest = N - KE;
        if (rest > 0) {
            hipLaunchKernelGGL(trsm_block_kernel, dim3((rest + 31) / 32), dim3(1024), 0, s, N, LU, K0, KE - K0, KE);
            const int nbk = (rest + 63) / 64;
            hipLaunchKernelGGL(gemm_update_kernel, dim3(nbk, nbk), dim3(256), 0, s, N, LU, KE, KE, N, K0, KE - K0);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (diag_inv) hipLaunchKernelGGL(invert_diag_kernel, dim3((N + 63) / 64), dim3(64), 0, s, N, LU, static_cast<float *>(diag_inv));
    return hipGetLastError();
}

hipError_t lu_solve_f32(int N, const float *LU, const float *diag_inv, float *b, float *tmp, hipStream_t s)
{
    // b is already permuted (b := P b).
    // forward: b is updated below each block, solved blocks go to tmp;
    // backward: tmp is updated above each block, solved blocks go to b.
    for (int b0 = 0; b0 < N; b0 += 64) {
        const int rest = std::max(0, N - b0 - 64);
        hipLaunchKernelGGL(trsv_lower_kernel, dim3(std::max(1, (rest + 255) / 256)), dim3(256), 0, s, N, LU, diag_inv,
                           b, tmp, b0);
    }
    const int nblk = (N + 63) / 64;
    for (int bk = nblk - 1; bk >= 0; --bk) {
        const int b0 = bk * 64, bw = std::min(64, N - b0);
        hipLaunchKernelGGL(trsv_upper_kernel, dim3(std::max(1, (b0 + 255) / 256)), dim3(256), 0, s, N, LU, diag_inv,
                           tmp, b, b0, bw);
    }
    return hipGetLastError();
}

int mixed_solve(int N, const void *d_A, int64_t lda, int a_prec, const double *d_beta, double *d_x, double tol,
                int max_iter, void *ws_base, hipStream_t s, SolveResult &res, std::string &msg)
{
    WS w = carve(ws_base, N);
    auto fail = [&](int st, const char *m, hipError_t e) {
        msg = std::string(m) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
        return st;
    };
    dim3 tg((N + 31) / 32, (N + 31) / 32);
    if (a_prec == 0)
        hipLaunchKernelGGL(to_colmajor_kernel<double>, tg, dim3(256), 0, s, N, static_cast<const double *>(d_A), lda, w.LU);
    else
        hipLaunchKernelGGL(to_colmajor_kernel<float>, tg, dim3(256), 0, s, N, static_cast<const float *>(d_A), lda, w.LU);
    hipError_t e = lu_factor_f32(N, w.LU, w.piv, w.info, w.DI, s);
    if (e != hipSuccess) return fail(-5, "LU factorisation launch", e);
    // ||A||_inf for the backward error (one read of A)
    if (a_prec == 0)
        hipLaunchKernelGGL(rowabs_kernel<double>, dim3((N + 3) / 4), dim3(256), 0, s, N, static_cast<const double *>(d_A), lda, w.red + 8);
    else
        hipLaunchKernelGGL(rowabs_kernel<float>, dim3((N + 3) / 4), dim3(256), 0, s, N, static_cast<const float *>(d_A), lda, w.red + 8);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, w.red + 8, w.red + 4);
    // permutation from the interchange sequence (host, O(N))
    std::vector<int> piv(N), perm(N);
    int info = 0;
    double normA = 0.0;
    if ((e = hipMemcpyAsync(piv.data(), w.piv, N * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&normA, w.red + 4, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(-5, "LU factorisation", e);
    if (info != 0) return fail(-3, "zero pivot in the FP32 LU factorisation", hipSuccess);
    for (int i = 0; i < N; ++i) perm[i] = i;
    for (int j = 0; j < N; ++j) std::swap(perm[j], perm[piv[j]]);
    if ((e = hipMemcpyAsync(w.perm, perm.data(), N * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
        return fail(-5, "permutation upload", e);

    auto residual = [&]() {
        if (a_prec == 0) launch_residual<double>(N, d_A, lda, d_x, d_beta, w.r, s);
        else launch_residual<float>(N, d_A, lda, d_x, d_beta, w.r, s);
    };
    double red[4];
    // x0 = LU \ beta
    hipLaunchKernelGGL(permute_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, w.perm, d_beta, w.v);
    (void)lu_solve_f32(N, w.LU, w.DI, w.v, w.v2, s);
    hipLaunchKernelGGL(update_norms_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.v, d_beta, d_beta, 0, w.red);
    res.iters = 0;
    res.rel_update = 1.0;
    res.backward_err = 1.0;
    int status = -4;
    double prev = 1e300;
    // Refinement: stop when ||d|| <= tol ||x||, or when the corrections stop
    // shrinking (||d_k|| > ||d_{k-1}|| / 2: the FP64 residual has reached the
    // cond(A) eps floor) with a backward error at the FP64 level.
    for (int it = 0; it < max_iter; ++it) {
        residual();
        hipLaunchKernelGGL(permute_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, w.perm, w.r, w.v);
        (void)lu_solve_f32(N, w.LU, w.DI, w.v, w.v2, s);
        hipLaunchKernelGGL(update_norms_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.v, w.r, d_beta, 1, w.red);
        if ((e = hipMemcpyAsync(red, w.red, sizeof red, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail(-5, "refinement step", e);
        res.iters = it + 1;
        res.rel_update = red[1] > 0 ? red[0] / red[1] : 0.0;
        res.backward_err = red[2] / (normA * red[1] + red[3]);   // of the iterate before this step
        if (res.rel_update <= tol) {
            status = 0;
            break;
        }
        if (res.rel_update > 0.5 * prev && res.backward_err <= 64 * 1.1102230246251565e-16) {
            status = 0;
            break;
        }
        prev = res.rel_update;
    }
    // backward error of the returned x: ||beta - A x||_inf / (||A||_inf ||x||_inf + ||beta||_inf)
    residual();
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, w.r, w.red + 5);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.red + 6);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, d_beta, w.red + 7);
    double nr[4];
    if ((e = hipMemcpyAsync(nr, w.red + 4, sizeof nr, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(-5, "backward error", e);
    res.backward_err = nr[1] / (nr[0] * nr[2] + nr[3]);
    if (status != 0) return fail(-4, "iterative refinement did not reach the tolerance", hipSuccess);
    return 0;
}

}  // namespace sgbem
