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

// Register-resident panel factorisation (one workgroup of 1024 threads, RT rows
// per thread, W <= 32 columns): thread t owns the panel rows k0 + r*1024 + t
// with all W columns in registers.  The column loop is unrolled, so every
// register index is a compile-time constant.  Per column: pivot = largest
// magnitude at or below the diagonal (lowest row on ties); the pivot row and
// the diagonal row exchange their register rows through LDS (earlier L
// multipliers included: a row interchange of the panel) -- only the two
// owning wavefronts execute that copy; the rows below are scaled and updated.
// Global memory is touched only to load the panel and to store it, the
// pivots and info at the end; two barriers per column.
template <int RT, int W>
__global__ __launch_bounds__(1024) void panel_reg_kernel(int N, float *LU, int k0, int w, int *piv, int *info)
{
    __shared__ unsigned long long skey[16];
    __shared__ float prow[W], jrow[W];
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
            const int gj = k0 + j;
            // pivot key: |value| bits (monotone for non-negative floats) high, inverted row low,
            // so the largest key is the largest magnitude with the lowest row on ties
            unsigned long long key = 0ull;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int i = k0 + r * 1024 + tid;
                if (i >= gj && i < N) {
                    const unsigned long long k = (static_cast<unsigned long long>(__float_as_uint(fabsf(a[r][j]))) << 32) |
                                                 static_cast<unsigned int>(0x7fffffff - i);
                    key = k > key ? k : key;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(key, off);
                key = o > key ? o : key;
            }
            if (lane == 0) skey[wid] = key;
            __syncthreads();
            key = skey[lane & 15];
            for (int off = 8; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(key, off);
                key = o > key ? o : key;
            }
            const float b = __uint_as_float(static_cast<unsigned int>(key >> 32));
            int pr = 0x7fffffff - static_cast<int>(key & 0xffffffffull);
            if (!(b > 0.0f)) pr = gj;
            if (tid == 0) {
                if (!(b > 0.0f) && sinfo == 0) sinfo = gj + 1;
                pivs[j] = pr;
            }
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int i = k0 + r * 1024 + tid;
                if (i == pr) {
#pragma unroll
                    for (int c = 0; c < W; ++c) prow[c] = a[r][c];
                }
                if (i == gj) {
#pragma unroll
                    for (int c = 0; c < W; ++c) jrow[c] = a[r][c];
                }
            }
            __syncthreads();
            const float d = prow[j];
            const float inv = d != 0.0f ? 1.0f / d : 0.0f;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const int i = k0 + r * 1024 + tid;
                if (i == gj) {
#pragma unroll
                    for (int c = 0; c < W; ++c) a[r][c] = prow[c];
                } else if (i == pr) {
#pragma unroll
                    for (int c = 0; c < W; ++c) a[r][c] = jrow[c];
                }
                if (i > gj && i < N && d != 0.0f) {
                    const float l = a[r][j] * inv;
                    a[r][j] = l;
#pragma unroll
                    for (int c = j + 1; c < W; ++c) a[r][c] -= l * prow[c];
                }
            }
            // No third barrier: skey/prow/jrow of the next column are written only
            // after the next column's first barrier, which every wavefront reaches
            // after its last read of this column's values.
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

// U12 = L11^{-1} A12: one wavefront per column of A12, lane r holds row k0 + r.
__global__ __launch_bounds__(256) void trsm_kernel(int N, float *LU, int k0, int w)
{
    __shared__ float L[NB][NB + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < w * w; e += blockDim.x) {
        const int r = e % w, c = e / w;
        L[r][c] = LU[int64_t(k0 + c) * N + k0 + r];
    }
    __syncthreads();
    const int lane = tid & 63;
    const int col = k0 + w + blockIdx.x * 4 + (tid >> 6);
    if (col >= N) return;
    float *cp = LU + int64_t(col) * N + k0;
    float x = lane < w ? cp[lane] : 0.0f;
    for (int s = 0; s < w; ++s) {
        const float xs = __shfl(x, s);
        if (lane > s && lane < w) x -= L[lane][s] * xs;
    }
    if (lane < w) cp[lane] = x;
}

// C -= L21 U12 on FP32 MFMA (16x16x4): the workgroup owns a 64 x 64 block of
// the trailing matrix; each wavefront a 32 x 32 quarter as 2 x 2 MFMA tiles.
// The MFMA "rows" index the columns of C and its "columns" the rows of C, so
// each lane's results are contiguous in the column-major factor.
__global__ __launch_bounds__(256) void gemm_update_kernel(int N, float *LU, int k0, int w)
{
    __shared__ float As[64][NB + 1];   // L21 block: [row][k]
    __shared__ float Bs[64][NB + 1];   // U12 block transposed: [col][k]
    const int m0 = k0 + w + blockIdx.x * 64;    // first row of C
    const int n0 = k0 + w + blockIdx.y * 64;    // first column of C
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * w; e += blockDim.x) {
        const int r = e & 63, k = e >> 6;
        As[r][k] = (m0 + r < N) ? LU[int64_t(k0 + k) * N + m0 + r] : 0.0f;
    }
    for (int e = tid; e < 64 * w; e += blockDim.x) {
        const int k = e % w, c = e / w;
        Bs[c][k] = (n0 + c < N) ? LU[int64_t(n0 + c) * N + k0 + k] : 0.0f;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int wc = (wave >> 1) * 32;    // C columns of this wave
    const int wr = (wave & 1) * 32;     // C rows of this wave
    floatx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k = 0; k < w; k += 4) {
        const int kk = k + (lane >> 4);
        for (int a = 0; a < 2; ++a) {
            const float av = Bs[wc + a * 16 + (lane & 15)][kk];   // MFMA A: [C column][k]
            for (int b = 0; b < 2; ++b) {
                const float bv = As[wr + b * 16 + (lane & 15)][kk]; // MFMA B: [k][C row]
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[a][b], 0, 0, 0);
            }
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int i = 0; i < 4; ++i) {
                const int c = n0 + wc + a * 16 + 4 * (lane >> 4) + i;
                const int r = m0 + wr + b * 16 + (lane & 15);
                if (r < N && c < N) LU[int64_t(c) * N + r] -= acc[a][b][i];
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
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, info);
    for (int k0 = 0; k0 < N;) {
        const int m = N - k0;
        int w;
        // register panels while the rows fit (1, 2, 4, 8 rows per thread), narrower as they grow
        if (m <= 1024) {
            w = std::min(32, m);
            hipLaunchKernelGGL((panel_reg_kernel<1, 32>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
        } else if (m <= 2048) {
            w = 16;
            hipLaunchKernelGGL((panel_reg_kernel<2, 16>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
        } else if (m <= 4096) {
            w = 8;
            hipLaunchKernelGGL((panel_reg_kernel<4, 8>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
        } else if (m <= 8192) {
            w = 8;
            hipLaunchKernelGGL((panel_reg_kernel<8, 8>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
        } else {
            w = 32;
            hipLaunchKernelGGL(panel_kernel, dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
        }
        if (N - w > 0) hipLaunchKernelGGL(laswp_kernel, dim3((N - w + 255) / 256), dim3(256), 0, s, N, LU, k0, w, piv);
        const int rest = N - k0 - w;
        if (rest > 0) {
            hipLaunchKernelGGL(trsm_kernel, dim3((rest + 3) / 4), dim3(256), 0, s, N, LU, k0, w);
            const int nbk = (rest + 63) / 64;
            hipLaunchKernelGGL(gemm_update_kernel, dim3(nbk, nbk), dim3(256), 0, s, N, LU, k0, w);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k0 += w;
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
