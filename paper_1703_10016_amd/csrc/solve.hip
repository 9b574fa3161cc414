// Mixed-precision solve of the Galerkin system A alpha = beta (eq. sistlin):
// FP32 LU, FP64 iterative refinement with the stored matrix.  An exactly
// symmetric A (the Galerkin matrix) is first factored without row
// interchanges (blocked right-looking: diagonal block on one workgroup, the
// blocks below and right of it by triangular solves or products with its
// inverses, trailing update on FP32 MFMA) and that factor is kept only if the
// refinement converges; otherwise, and for any other A, LU with partial
// pivoting (register panels on one workgroup, the same MFMA update).  The
// factor is kept column-major in the workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "solve.hpp"

namespace sgbem {

namespace {

constexpr int NB = 64;            // widest panel (register panels); longer panels use 32 columns
constexpr int kGJMaxN = 4096;     // up to this order: the explicit inverse (block Gauss-Jordan)
// Beyond kGJMaxN the triangular solves go by super-blocks of kSB rows with the
// inverses of L's and U's kSB x kSB diagonal super-blocks formed once per factor.
constexpr int kSB = 1024;
int superblocks(int N) { return (N + kSB - 1) / kSB; }
size_t blkinv_floats(int N) { return N > kGJMaxN ? size_t(2) * superblocks(N) * kSB * kSB : 0; }
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

struct WS {
    float *LU;       // the FP32 factor (column-major, ld N) or the Gauss-Jordan inverse (row-major, ld Np)
    int *piv, *perm, *info;
    double *r;
    float *v, *v2;
    double *red;     // reduction outputs
    float *DI;       // inverted diagonal blocks
    float *DI2;      // off-diagonal blocks of the inverses of pairs of diagonal blocks
    float *GR, *GC, *GP;   // Gauss-Jordan panels: row blocks [2][nt][64][64], column blocks [2][nt][64][64], pivot inverses [2][64][64]
    float *INV;      // beyond kGJMaxN: [super-block][L, U][kSB x kSB] inverted diagonal super-blocks (column-major), else null
};

// Order padded to whole 64 x 64 tiles (the Gauss-Jordan inverse works on tiles).
int padded64(int N) { return (N + 63) / 64 * 64; }

// Control block of the batched refinement (doubles, written by the device):
//  [0] max |A_ij - A_ji|   [1] ||A||_inf   [2] previous ||d|| / ||x||   [3] stop reason
//  (0 running, 1 converged, 2 stalled, 3 not finite, 4 zero pivot, 5 not symmetric)
//  [4] steps taken   [5] last ||d|| / ||x||   [6] last backward error
//  [7] 1 when the last correction did not halve (the first slow step)
enum { CTL_ASYM = 0, CTL_NORMA = 1, CTL_PREV = 2, CTL_STOP = 3, CTL_ITERS = 4, CTL_REL = 5, CTL_BWD = 6, CTL_SLOW = 7,
       CTL_SIZE = 8 };

// True when a batched refinement has stopped (or the matrix is not symmetric):
// the remaining kernels of the batch return at once.
__device__ __forceinline__ bool ctl_stopped(const double *ctl) { return ctl && (ctl[CTL_STOP] != 0.0 || ctl[CTL_ASYM] != 0.0); }


size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

WS carve(void *base, int N)
{
    char *p = static_cast<char *>(base);
    WS w;
    const size_t Np = size_t(padded64(N));
    w.LU = reinterpret_cast<float *>(p);
    p += align_up(Np * Np * sizeof(float));
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
    p += align_up(size_t(N + 63) / 64 * 2 * 4096 * sizeof(float));
    w.DI2 = reinterpret_cast<float *>(p);
    p += align_up(std::max<size_t>(size_t(N + 63) / 64 / 2, 1) * 2 * 4096 * sizeof(float));
    const size_t nt = Np / 64;
    w.GR = reinterpret_cast<float *>(p);
    p += align_up(2 * nt * 4096 * sizeof(float));
    w.GC = reinterpret_cast<float *>(p);
    p += align_up(2 * nt * 4096 * sizeof(float));
    w.GP = reinterpret_cast<float *>(p);
    p += align_up(2 * 4096 * sizeof(float));
    w.INV = N > kGJMaxN ? reinterpret_cast<float *>(p) : nullptr;
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

// The FP32 factor's starting copy of an exactly symmetric A: column j of the
// column-major copy is row j of A (equal to the transpose's column), so the
// copy streams rows and needs no transpose.  With VEC (rows of A 16-byte
// aligned, N % 4 == 0) four entries per thread move as one vector.
template <typename InT, bool VEC>
__global__ __launch_bounds__(256) void copy_rows_kernel(int N, const InT *A, int64_t lda, float *LU)
{
    const int j = blockIdx.y, i0 = (blockIdx.x * 256 + threadIdx.x) * 4;
    if (i0 >= N) return;
    const InT *a = A + int64_t(j) * lda + i0;
    float *o = LU + int64_t(j) * N + i0;
    if (VEC && i0 + 4 <= N) {
        float4 v;
        if constexpr (sizeof(InT) == 4) {
            v = *reinterpret_cast<const float4 *>(a);
        } else {
            const double2 lo = *reinterpret_cast<const double2 *>(a), hi = *reinterpret_cast<const double2 *>(a + 2);
            v = make_float4(float(lo.x), float(lo.y), float(hi.x), float(hi.y));
        }
        *reinterpret_cast<float4 *>(o) = v;
    } else {
        for (int e = 0; e < 4 && i0 + e < N; ++e) o[e] = float(a[e]);
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

// Register-resident panel factorisation: one workgroup of NT threads (NT / 64
// wavefronts), RT slots per thread, W <= 64 columns.  Slot r of thread t holds
// one panel row, all W columns, in registers, and the row's current position
// pos[r] (initially k0 + r NT + t).  Every loop over r and over the columns is
// unrolled, so every register index is a compile-time constant.
//
// Row interchanges are lazy: the interchange of rows gj and pr at column j only
// swaps the two positions (the slot holding position pr takes gj and the slot
// holding gj takes pr, found by comparing positions), and the final store
// writes every slot to the row of its position.  The result is the same as
// moving the rows, L multipliers included, without moving data in registers.
//
// Per column j (gj = k0 + j; the active slots are those with pos >= gj):
//  * each thread holds its candidate, the active slot of largest magnitude in
//    column j, lowest position on ties; each wavefront reduces the candidates
//    by two DPP reductions (largest magnitude, then lowest position holding
//    it) and the owner of the winning slot publishes its columns j..W-1;
//  * one barrier; every thread picks the winner among the NT / 64 published
//    candidates the same way, so all agree on the pivot position pr;
//  * positions are swapped as above; the active rows (now pos > gj) are
//    scaled and updated with the pivot row held in registers, branch-free
//    (inactive slots are updated with a zero multiplier), and in the same pass
//    each thread takes its candidate for column j + 1.
// Slots past N hold zeros at a position no real row has: they never become the
// pivot (a zero magnitude only wins when every candidate is zero, and then
// the lowest position, a real row, wins and the column is singular: no
// interchange, no update).  Published values are double-buffered by column
// parity: a buffer is written again two columns later, after a barrier that
// every wavefront reaches only when done reading it.  Global memory is touched
// only to load and store the panel, the pivots and info.
template <int RT, int W, int NT>
__global__ __launch_bounds__(NT) void panel_reg_kernel(int N, float *LU, int k0, int w, int *piv, int *info)
{
    constexpr int NWV = NT / 64;
    constexpr int NONE = 0x7fffffff, PAD = 0x7ffffff0;
    static_assert(NT % 64 == 0 && NWV <= 16 && W <= 64, "panel shape");
    __shared__ unsigned smag[2][NWV];
    __shared__ int spos[2][NWV];
    __shared__ float crow[2][NWV][W];    // each wavefront's candidate row, columns j..W-1
    __shared__ int pivs[W];
    __shared__ int sinfo;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) sinfo = 0;
    // Every load is unconditional, from a clamped (valid, finite) entry, and is
    // multiplied by 1 or 0: its result is always used, so the loads are all in
    // flight together instead of each in its own branch followed by a wait.
    float a[RT][W];
    int pos[RT];
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const float *col = LU + int64_t(k0 + min(c, w - 1)) * N;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int i = k0 + r * NT + tid;
            a[r][c] = col[min(i, N - 1)] * ((i < N && c < w) ? 1.0f : 0.0f);
        }
    }
    // pin every value here (an empty statement that reads and writes it), so that the
    // loads are all issued before the column loop rather than each sunk to its first use
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int r = 0; r < RT; ++r) asm volatile("" : "+v"(a[r][c]));
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int i = k0 + r * NT + tid;
        pos[r] = i < N ? i : PAD;
    }
    // candidate for column 0: every slot is active
    float best = -1.0f;
    int bpos = NONE, bslot = 0;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const float m = fabsf(a[r][0]);
        const bool take = (m > best) | ((m == best) & (pos[r] < bpos));
        best = take ? m : best;
        bpos = take ? pos[r] : bpos;
        bslot = take ? r : bslot;
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        // no branch on j < w either: columns past w are zero in every row, so their
        // pass finds no pivot and changes nothing (only the singular flag is guarded)
        {
            const int gj = k0 + j, buf = j & 1;
            const bool has = best >= 0.0f;
            const unsigned mag = has ? __float_as_uint(best) : 0u;   // monotone for non-negative floats
            const int key = has ? bpos : NONE;
            const unsigned wmag = wave_reduce_u32<true>(mag);
            const int wpos = int(wave_reduce_u32<false>(mag == wmag ? unsigned(key) : unsigned(NONE)));
            // publish the wavefront's candidate (its owner lane and slot made uniform)
            const unsigned long long own = __ballot(key == wpos);
            const int wl = int(__builtin_ctzll(own | (1ull << 63)));
            const int rw = __builtin_amdgcn_readlane(bslot, wl);
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (r == rw && lane == wl) {
#pragma unroll
                    for (int c = 0; c < W; ++c)
                        if (c >= j) crow[buf][wid][c] = a[r][c];
                }
            if (lane == 0) {
                smag[buf][wid] = wmag;
                spos[buf][wid] = wpos;
            }
            __syncthreads();
            // the winner among the wavefronts' candidates (position gj is one of the
            // active slots, so a candidate exists)
            unsigned gm = 0u;
            int gp = NONE, gw = 0;
#pragma unroll
            for (int q = 0; q < NWV; ++q) {
                const unsigned m = smag[buf][q];
                const int p = spos[buf][q];
                if (m > gm || (m == gm && p < gp)) {
                    gm = m;
                    gp = p;
                    gw = q;
                }
            }
            const bool ok = __uint_as_float(gm) > 0.0f;
            const int pr = ok ? gp : gj;
            if (tid == 0) {
                if (!ok && j < w && sinfo == 0) sinfo = gj + 1;
                pivs[j] = pr;
            }
            // interchange of rows gj and pr: swap the two positions
#pragma unroll
            for (int r = 0; r < RT; ++r) pos[r] = pos[r] == pr ? gj : (pos[r] == gj ? pr : pos[r]);
            // One branch-free pass (a branch here would make the compiler copy the whole
            // panel at the join): the active rows are scaled and updated with the pivot
            // row held in registers; inactive slots, and every slot when the column is
            // singular, get a zero multiplier.  Candidates for column j + 1 on the way.
            float pv[W];
#pragma unroll
            for (int c = 0; c < W; ++c) pv[c] = c >= j ? crow[buf][gw][c] : 0.0f;   // constant trip count
            const float inv = ok ? 1.0f / pv[j] : 0.0f;
            best = -1.0f;
            bpos = NONE;
            bslot = 0;
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const bool act = pos[r] > gj;
                const float lr = a[r][j] * inv;
                const float l = act ? lr : 0.0f;
                a[r][j] = act ? lr : a[r][j];
#pragma unroll
                for (int c = 0; c < W; ++c)
                    if (c > j) a[r][c] -= l * pv[c];
                if (j + 1 < W) {
                    const float m = fabsf(a[r][j + 1]);
                    const bool take = act & ((m > best) | ((m == best) & (pos[r] < bpos)));
                    best = take ? m : best;
                    bpos = take ? pos[r] : bpos;
                    bslot = take ? r : bslot;
                }
            }
        }
    }
    // an opaque copy of the base pointer: the store addresses are formed anew here
    // instead of being kept live, in registers, from the loads at the start
    float *LUs = LU;
    asm volatile("" : "+s"(LUs));
#pragma unroll
    for (int c = 0; c < W; ++c) {
        if (c < w) {
            float *col = LUs + int64_t(k0 + c) * N;
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (pos[r] < N) col[pos[r]] = a[r][c];
        }
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
    {
        // unconditional loads from clamped entries, unrolled: all in flight together
        float v[16];
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + it * 1024, r = e & 127, c = e >> 7;
            v[it] = LU[int64_t(K0 + min(c, bk - 1)) * N + K0 + min(r, bk - 1)];
        }
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + it * 1024;
            L[e & 127][e >> 7] = v[it];
        }
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
    __builtin_amdgcn_s_setprio(3);   // panel work: ahead of the trailing update's MFMA waves on a shared SIMD
    __shared__ float As[64][33];   // L21 chunk: [row][k]
    __shared__ float Bs[64][33];   // U12 chunk transposed: [col][k]
    const int m0 = r0 + blockIdx.x * 64;    // first row of C
    const int n0 = c0 + blockIdx.y * 64;    // first column of C
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wc = (wave >> 1) * 32;    // C columns of this wave
    const int wr = (wave & 1) * 32;     // C rows of this wave
    // this lane's 16 entries of C, loaded before the K loop (clamped addresses)
    // so that their HBM latency overlaps the multiplications
    float cpre[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = n0 + wc + a * 16 + 4 * (lane >> 4) + i;
                const int r = m0 + wr + b * 16 + (lane & 15);
                cpre[a][b][i] = LU[int64_t(min(c, cend - 1)) * N + min(r, N - 1)];
            }
    floatx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kc = 0; kc < klen; kc += 32) {
        const int kl = min(32, klen - kc);
        // unconditional loads from clamped entries, masked, unrolled: all in flight together
        float va[8], vb[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = tid + it * 256, r = e & 63, k = e >> 6;
            va[it] = LU[int64_t(kb + kc + min(k, kl - 1)) * N + min(m0 + r, N - 1)] * ((m0 + r < N && k < kl) ? 1.0f : 0.0f);
        }
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = tid + it * 256, k = e & 31, c = e >> 5;
            vb[it] = LU[int64_t(min(n0 + c, cend - 1)) * N + kb + kc + min(k, kl - 1)] * ((n0 + c < cend && k < kl) ? 1.0f : 0.0f);
        }
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = tid + it * 256;
            As[e & 63][e >> 6] = va[it];
        }
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = tid + it * 256;
            Bs[e >> 5][e & 31] = vb[it];
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
                if (r < N && c < cend) LU[int64_t(c) * N + r] = cpre[a][b][i] - acc[a][b][i];
            }
}

// One 128 x 128 block at (m0, n0) of the trailing update C -= L21 U12 of the
// blocked LU (same operands as gemm_update_kernel) for N % 4 == 0,
// m0 % 4 == 0, klen % 4 == 0, on v_mfma_f32_32x32x2_f32: a 64 x 64 quarter
// (2 x 2 MFMA blocks, accumulators in AGPRs) per wavefront, K in chunks of 16
// double-buffered in LDS (one barrier per chunk; the next chunk's loads are in
// flight during the current chunk's products, and their 0/1 edge masks are
// applied only when they go to LDS, so no wait sits before the products).
// L21 is staged as [k][m] (its column-major layout; the row pitch 160 puts the
// two k of a 32x32x2 step in disjoint banks).  U12 is staged as [n][k] (pitch
// 18: conflict-free reads), or, with SYM (a symmetric matrix factored without
// interchanges, where U = D L^T), formed on the fly as U12(k, n) = D_k L(n, k)
// from the rows n of the column panel and staged as [k][n] like L21.  Each
// lane's results are four runs of four rows of one column of C, so C moves in
// 16-byte accesses.
constexpr int kUpdKC = 16, kUpdSA = 160, kUpdSB = 18;
constexpr int kUpdBFloats = 2 * kUpdKC * kUpdSA;   // >= 2 * 128 * kUpdSB
template <bool SYM>
__device__ __forceinline__ void update128_tile(float (&As)[2][kUpdKC][kUpdSA], float *Bsm, int m0, int n0, int N, float *LU,
                                               int cend, int kb, int klen)
{
    constexpr int KC = kUpdKC;
    auto &Bs = *reinterpret_cast<float (*)[2][128][kUpdSB]>(Bsm);
    auto &Bt = *reinterpret_cast<float (*)[2][kUpdKC][kUpdSA]>(Bsm);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int mw = (wave & 1) * 64, nw = (wave >> 1) * 64, li = lane & 31, lg = lane >> 5;
    floatx16 acc[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[mb][nb][i] = 0.0f;
    // staging: two float4 of L21 (4 rows of one k) and two of U12 (4 k of one column) per thread,
    // loaded from clamped addresses; the 0/1 masks scale them on the way to LDS
    float4 ra[2], rb[2];
    float sa[2], sb[2];
    auto gload = [&](int kc) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 256 * i, k = e >> 5, m4 = (e & 31) * 4;
            sa[i] = (kc + k < klen && m0 + m4 < N) ? 1.0f : 0.0f;
            ra[i] = *reinterpret_cast<const float4 *>(LU + int64_t(kb + min(kc + k, klen - 1)) * N + min(m0 + m4, N - 4));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            if (SYM) {   // L(n0 + n4 .. + 3, kb + kc + k), scaled by the pivot D_k on the way to LDS
                const int e = tid + 256 * i, k = e >> 5, n4 = (e & 31) * 4, kk = kb + min(kc + k, klen - 1);
                sb[i] = (kc + k < klen && n0 + n4 < cend) ? LU[int64_t(kk) * N + kk] : 0.0f;
                rb[i] = *reinterpret_cast<const float4 *>(LU + int64_t(kk) * N + min(n0 + n4, cend - 4));
            } else {
                const int e = tid + 256 * i, n = e >> 2, k4 = (e & 3) * 4;
                sb[i] = (n0 + n < cend && kc + k4 < klen) ? 1.0f : 0.0f;
                rb[i] = *reinterpret_cast<const float4 *>(LU + int64_t(min(n0 + n, cend - 1)) * N + kb + min(kc + k4, klen - 4));
            }
        }
    };
    auto swrite = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 256 * i;
            const float4 v = ra[i];
            *reinterpret_cast<float4 *>(&As[buf][e >> 5][(e & 31) * 4]) = make_float4(v.x * sa[i], v.y * sa[i], v.z * sa[i], v.w * sa[i]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float4 v = rb[i];
            if (SYM) {
                const int e = tid + 256 * i;
                *reinterpret_cast<float4 *>(&Bt[buf][e >> 5][(e & 31) * 4]) = make_float4(v.x * sb[i], v.y * sb[i], v.z * sb[i], v.w * sb[i]);
            } else {
                const int e = tid + 256 * i, n = e >> 2, k4 = (e & 3) * 4;
                *reinterpret_cast<float2 *>(&Bs[buf][n][k4]) = make_float2(v.x * sb[i], v.y * sb[i]);
                *reinterpret_cast<float2 *>(&Bs[buf][n][k4 + 2]) = make_float2(v.z * sb[i], v.w * sb[i]);
            }
        }
    };
    const int nc = (klen + KC - 1) / KC;
    gload(0);
    swrite(0);
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
        const int buf = c & 1;
        if (c + 1 < nc) gload((c + 1) * KC);
        // 32x32x2: lanes 0-31 carry k = 2s, lanes 32-63 k = 2s + 1; A lane i holds row i of the
        // 32-row block, B lane j column j of the 32-column block
#pragma unroll
        for (int s = 0; s < KC / 2; ++s) {
            const int k = 2 * s + lg;
            float a[2], b[2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) a[mb] = As[buf][k][mw + mb * 32 + li];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) b[nb] = SYM ? Bt[buf][k][nw + nb * 32 + li] : Bs[buf][nw + nb * 32 + li][k];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
        }
        if (c + 1 < nc) swrite(buf ^ 1);
        __syncthreads();
    }
    // result (i, j) of a 32x32 block sits in lane j + 32 * ((i / 4) % 2), entry 4 * (i / 8) + i % 4
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int row = m0 + mw + mb * 32 + 8 * qq + 4 * lg, col = n0 + nw + nb * 32 + li;
                if (row < N && col < cend) {
                    float4 *p = reinterpret_cast<float4 *>(LU + int64_t(col) * N + row);
                    float4 cv = *p;
                    cv.x -= acc[mb][nb][4 * qq + 0];
                    cv.y -= acc[mb][nb][4 * qq + 1];
                    cv.z -= acc[mb][nb][4 * qq + 2];
                    cv.w -= acc[mb][nb][4 * qq + 3];
                    *p = cv;
                }
            }
}

// Block coordinates.  Rectangle: ntr x ntc blocks numbered in bands 16 blocks
// wide (row by row within a band), so that a run of consecutive blocks shares
// the band's U12 columns while the L21 rows stream through.  Lower: the blocks
// of an nt x nt grid that lie in 256 x 256 blocks on or below the diagonal
// (tr / 2 >= tc / 2), column by column; columns 2j and 2j + 1 hold nt - 2j
// blocks each, 2j (nt + 1 - j) blocks come before them.
__device__ __forceinline__ void band_coords(int t, int ntr, int ntc, int &tr, int &tc)
{
    const int band = t / (16 * ntr), tb = t - band * 16 * ntr, wb = min(16, ntc - band * 16);
    tr = tb / wb;
    tc = band * 16 + tb % wb;
}

__device__ __forceinline__ void lower256_coords(int t, int nt, int &tr, int &tc)
{
    int j = max(0, int(((nt + 1) - sqrtf(float((nt + 1) * (nt + 1) - 2 * t))) * 0.5f));
    while (j > 0 && 2 * j * (nt + 1 - j) > t) --j;
    while (2 * (j + 1) * (nt - j) <= t) ++j;
    const int u = t - 2 * j * (nt + 1 - j), h = nt - 2 * j;
    tr = 2 * j + u % h;
    tc = 2 * j + u / h;
}

// Number of blocks of the lower order for an nt x nt grid.
inline int lower256_count(int nt) { return 2 * (nt / 2) * (nt + 1 - nt / 2) + (nt % 2); }

// The update over ntiles blocks of 128 x 128 (rectangle or lower order).
// Workgroup ids go round-robin over the eight XCDs; XCD x takes a contiguous
// run of the block numbers, and its per_xcd workgroups stride through that
// run, so one launch of 8 * ceil(blocks / 8) workgroups does one block each
// and a smaller grid is persistent (it leaves CU slots free for other work on
// the device).
template <bool SYM, bool LOWER>
__global__ __launch_bounds__(256) void update128_kernel(int N, float *LU, int r0, int c0, int cend, int kb, int klen,
                                                        int ntr, int ntc, int ntiles, int per_xcd)
{
    __shared__ __align__(16) float As[2][kUpdKC][kUpdSA];
    __shared__ __align__(16) float Bsm[kUpdBFloats];
    const int q = ntiles >> 3, rem = ntiles & 7;
    const int x = int(blockIdx.x & 7), cnt = q + (x < rem ? 1 : 0), base = x * q + min(x, rem);
    if (SYM && !LOWER) __builtin_amdgcn_s_setprio(2);   // the next block's panel: ahead of the rest update
    for (int lt = int(blockIdx.x >> 3); lt < cnt; lt += per_xcd) {
        int tr, tc;
        if (LOWER) lower256_coords(base + lt, ntr, tr, tc);
        else band_coords(base + lt, ntr, ntc, tr, tc);
        update128_tile<SYM>(As, Bsm, r0 + 128 * tr, c0 + 128 * tc, N, LU, cend, kb, klen);
    }
}

// U above the diagonal 256 x 256 blocks of a symmetric matrix factored
// without interchanges: U(r, c) = D_r L(c, r) for c >= 256 (r / 256 + 1), by
// blocks of 64 rows x 128 columns of U transposed through LDS (from 128-entry,
// 512-byte runs of L's columns); blocks left of that line return at once.
__global__ __launch_bounds__(256) void fill_upper_kernel(int N, float *LU)
{
    __shared__ float T[64][129];
    const int I = blockIdx.y, J = blockIdx.x;   // U rows 64 I.., columns 128 J..
    if (2 * J < (I / 4 + 1) * 4) return;
    const int tid = threadIdx.x, r0 = 64 * I, c0 = 128 * J;
    float v[32];
#pragma unroll
    for (int it = 0; it < 32; ++it) {   // L(c0 + i, r0 + j): i fastest (contiguous)
        const int e = tid + 256 * it, i = e & 127, j = e >> 7;
        v[it] = LU[int64_t(min(r0 + j, N - 1)) * N + min(c0 + i, N - 1)];
    }
#pragma unroll
    for (int it = 0; it < 32; ++it) {
        const int e = tid + 256 * it;
        T[e >> 7][e & 127] = v[it];   // T[j][i] = L(c0 + i, r0 + j)
    }
    __syncthreads();
    const int j = tid & 63, r = r0 + j;
    const float d = LU[int64_t(min(r, N - 1)) * N + min(r, N - 1)];
#pragma unroll
    for (int it = 0; it < 32; ++it) {   // U(r0 + j, c0 + i): j fastest (contiguous)
        const int i = (tid >> 6) + 4 * it, c = c0 + i;
        if (r < N && c < N) LU[int64_t(c) * N + r] = d * T[j][i];
    }
}

// ---------------------------------------------------------------- blocked LU without interchanges
// Without interchanges, every 64-column diagonal block is factored by one
// wavefront and inverted by two, and L21, U12 become plain products with the
// inverses (no dependent chain).
//
// diag64_kernel: wavefront 0 factors the bk x bk block (bk <= 64, padded with
// the identity) with lane l holding row l in registers: per column j the
// pivot row's entries come from lane j by readlane (every index a
// compile-time constant: the loops are unrolled); then, from the factor staged
// in LDS, wavefront 0 forms inv(L) and wavefront 1 inv(U), lane c holding
// column c (forward / backward substitution against the identity, the factor
// read by broadcast).  The inverses go to DI (the inverted diagonal blocks of
// the triangular solves, column-major); a zero or non-finite pivot is
// reported in info like a singular column.
__global__ __launch_bounds__(128) void diag64_kernel(int N, float *LU, int K0, int bk, float *DI, int *info)
{
    __builtin_amdgcn_s_setprio(3);   // panel work: ahead of the trailing update's MFMA waves on a shared SIMD
    __shared__ float F[64][65];      // the factor: unit-lower L below the diagonal, U on and above
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (wave == 0) {
        float e[64];
        const int lr = min(lane, bk - 1);
#pragma unroll
        for (int c = 0; c < 64; ++c) {
            const bool in = lane < bk && c < bk;
            e[c] = LU[int64_t(K0 + min(c, bk - 1)) * N + K0 + lr] * (in ? 1.0f : 0.0f) + ((!in && lane == c) ? 1.0f : 0.0f);
        }
#pragma unroll
        for (int c = 0; c < 64; ++c) asm volatile("" : "+v"(e[c]));
        int bad = 0;
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e[j]), j));
            const bool ok = fabsf(d) > 0.0f && fabsf(d) <= 3.402823466e38f;
            if (!ok && j < bk && bad == 0) bad = K0 + j + 1;
            const float inv = ok ? 1.0f / d : 0.0f;
            const float l = lane > j ? e[j] * inv : 0.0f;
            e[j] = lane > j ? l : e[j];
#pragma unroll
            for (int c = j + 1; c < 64; ++c)
                e[c] -= l * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e[c]), j));
        }
#pragma unroll
        for (int c = 0; c < 64; ++c) F[lane][c] = e[c];
        float *LUs = LU;
        asm volatile("" : "+s"(LUs));
#pragma unroll
        for (int c = 0; c < 64; ++c)
            if (c < bk && lane < bk) LUs[int64_t(K0 + c) * N + K0 + lane] = e[c];
        if (lane == 0 && bad != 0 && *info == 0) *info = bad;
    }
    __syncthreads();
    float x[64];
    // (each sum in four interleaved partial sums: four short dependent chains
    // instead of one long one, on a wavefront that has its SIMD to itself)
    if (wave == 0) {
        // inv(L), column lane: x_r = delta_{r,lane} - sum_{k<r} L_rk x_k
#pragma unroll
        for (int r = 0; r < 64; ++r) {
            float p4[4] = {r == lane ? 1.0f : 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < r; ++k) p4[k & 3] -= F[r][k] * x[k];
            x[r] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        }
    } else {
        // inv(U), column lane: x_r = (delta_{r,lane} - sum_{k>r} U_rk x_k) / U_rr
#pragma unroll
        for (int r = 63; r >= 0; --r) {
            float p4[4] = {r == lane ? 1.0f : 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k = r + 1; k < 64; ++k) p4[k & 3] -= F[r][k] * x[k];
            x[r] = ((p4[0] + p4[1]) + (p4[2] + p4[3])) / F[r][r];
        }
    }
    float *out = DI + (int64_t(K0 / 64) * 2 + wave) * 4096 + lane * 64;   // column lane, entries r
#pragma unroll
    for (int r = 0; r < 64; r += 4) *reinterpret_cast<float4 *>(out + r) = make_float4(x[r], x[r + 1], x[r + 2], x[r + 3]);
}

// After diag64_kernel: workgroups [0, nrb) form L21 = A21 inv(U11) on 64-row
// blocks below the diagonal block, workgroups [nrb, 2 nrb) form
// U12 = inv(L11) A12 on 64-column blocks right of it (a block of 64 x bk or
// bk x 64 entries in LDS with the 64 x 64 inverse, one product, written back in
// place: every workgroup reads and writes only its own entries).
__global__ __launch_bounds__(256) void panel_mul_kernel(int N, float *LU, int K0, int bk, int KE, const float *DI, int nrb)
{
    __builtin_amdgcn_s_setprio(3);   // panel work: ahead of the trailing update's MFMA waves on a shared SIMD
    __shared__ float X[64][65], V[64][65];
    const int tid = threadIdx.x;
    const bool rows = int(blockIdx.x) < nrb;
    const int blk = rows ? blockIdx.x : blockIdx.x - nrb;
    const int b0 = KE + 64 * blk, nb = min(64, N - b0);
    // the inverse: V[r][k] = entry (r, k), DI column-major (entry (r, k) at k * 64 + r)
    const float *inv = DI + (int64_t(K0 / 64) * 2 + (rows ? 1 : 0)) * 4096;
    float v[16], xv[16];
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + it * 256;
        v[it] = inv[e];                                              // entry (e % 64, e / 64)
        const int i = e & 63, j = e >> 6;
        // rows: X[i][j] = A21(b0 + i, K0 + j); columns: X[i][j] = A12(K0 + i, b0 + j)
        const int64_t a = rows ? int64_t(K0 + min(j, bk - 1)) * N + min(b0 + i, N - 1)
                               : int64_t(min(b0 + j, N - 1)) * N + K0 + min(i, bk - 1);
        const bool in = rows ? (i < nb && j < bk) : (i < bk && j < nb);
        xv[it] = LU[a] * (in ? 1.0f : 0.0f);
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + it * 256;
        V[e & 63][e >> 6] = v[it];
        X[e & 63][e >> 6] = xv[it];
    }
    __syncthreads();
    // Y = P Q (rows: P = X, Q = V; columns: P = V, Q = X) on v_mfma_f32_16x16x4_f32,
    // a 32 x 32 block of Y per wavefront, with the operand layout of
    // gemm_update_kernel: the first operand runs over Y's columns and the second
    // over its rows, so 16 consecutive lanes hold 16 consecutive rows of a
    // column of Y (one contiguous store).
    const int wave = tid >> 6, lane = tid & 63;
    const int wc = (wave >> 1) * 32, wr = (wave & 1) * 32;
    float (*P)[65] = rows ? X : V;
    float (*Q)[65] = rows ? V : X;
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 64; k += 4) {
        const int kk = k + (lane >> 4);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const float av = Q[kk][wc + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const float bv = P[wr + b * 16 + (lane & 15)][kk];
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[a][b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = wc + a * 16 + 4 * (lane >> 4) + q, i = wr + b * 16 + (lane & 15);
                if (rows) {
                    if (i < nb && j < bk) LU[int64_t(K0 + j) * N + b0 + i] = acc[a][b][q];
                } else {
                    if (i < bk && j < nb) LU[int64_t(b0 + j) * N + K0 + i] = acc[a][b][q];
                }
            }
}

// ---------------------------------------------------------------- triangular solves
// One launch per 64-row block; every workgroup solves the diagonal block
// (the same arithmetic in each) and then updates its own rows.
// Inverses of the 64 x 64 diagonal blocks of L (unit lower) and U, kept so
// that every block step of the triangular solves is a plain matrix-vector
// product.  DI[b][0] = inv(L_bb), DI[b][1] = inv(U_bb), column-major 64 x 64
// (entry (r, k) at k * 64 + r: a wavefront reading row r = lane of column k is
// coalesced); a partial last block is padded with the identity.
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
    for (int r = 0; r < 64; ++r) DI[(int64_t(blockIdx.x) * 2 + 0) * 4096 + c * 64 + r] = X[r][c];
    __syncthreads();
    // U X = I, column c: X[r][c] = (delta_rc - sum_{k>r} U[r][k] X[k][c]) / U[r][r]
    for (int r = 63; r >= 0; --r) {
        float s = (r == c) ? 1.0f : 0.0f;
        for (int k = r + 1; k < 64; ++k) s -= T[r][k] * X[k][c];
        X[r][c] = s / T[r][r];
    }
    for (int r = 0; r < 64; ++r) DI[(int64_t(blockIdx.x) * 2 + 1) * 4096 + c * 64 + r] = X[r][c];
}

// Forward step for the 64-row block at b0: x_b = inv(L_bb) y_b (computed by
// every workgroup), written to yout by workgroup 0; rows below are updated in
// y (rows of the block itself are only read in this launch).  Both products
// issue their 64 loads unconditionally (clamped addresses, the solved block
// padded with zeros), so the loads are in flight together, and sum in four
// interleaved partial sums (short dependent chains).
__global__ __launch_bounds__(256) void trsv_lower_kernel(int N, const float *LU, const float *DI, float *y, float *yout, int b0)
{
    __shared__ float yb[64], xb[64];
    const int bw = min(64, N - b0);
    const int tid = threadIdx.x;
    if (tid < 64) yb[tid] = tid < bw ? y[b0 + tid] : 0.0f;
    __syncthreads();
    if (tid < 64) {
        const float *blk = DI + (int64_t(b0 / 64) * 2 + 0) * 4096 + tid;
        float d[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) d[k] = blk[k * 64];
        float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 64; ++k) p4[k & 3] += d[k] * yb[k];
        const float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        xb[tid] = tid < bw ? s : 0.0f;
        if (blockIdx.x == 0 && tid < bw) yout[b0 + tid] = s;
    }
    __syncthreads();
    const int r = b0 + bw + blockIdx.x * blockDim.x + tid;
    const float *col = LU + int64_t(b0) * N + min(r, N - 1);
    float v[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) v[k] = col[int64_t(min(k, bw - 1)) * N];
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 64; ++k) p4[k & 3] += v[k] * xb[k];
    const float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    if (r < N) y[r] -= s;
}

__global__ __launch_bounds__(256) void trsv_upper_kernel(int N, const float *LU, const float *DI, float *y, float *yout, int b0, int bw)
{
    __shared__ float yb[64], xb[64];
    const int tid = threadIdx.x;
    if (tid < 64) yb[tid] = tid < bw ? y[b0 + tid] : 0.0f;
    __syncthreads();
    if (tid < 64) {
        const float *blk = DI + (int64_t(b0 / 64) * 2 + 1) * 4096 + tid;
        float d[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) d[k] = blk[k * 64];
        float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 64; ++k) p4[k & 3] += d[k] * yb[k];
        const float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        xb[tid] = tid < bw ? s : 0.0f;
        if (blockIdx.x == 0 && tid < bw) yout[b0 + tid] = s;
    }
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + tid;
    const float *col = LU + int64_t(b0) * N + min(r, max(b0 - 1, 0));
    float v[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) v[k] = col[int64_t(min(k, bw - 1)) * N];
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 64; ++k) p4[k & 3] += v[k] * xb[k];
    const float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    if (r < b0) y[r] -= s;
}

// Pairs of 64-row blocks for the triangular solves: with the inverses A^-1,
// B^-1 of two consecutive diagonal blocks, the inverse of the 128 x 128 block
// they form has one more 64 x 64 block,
//   unit lower  [[A, 0], [C, B]]:  -B^-1 C A^-1 (bottom left),
//   upper       [[A, D], [0, B]]:  -A^-1 D B^-1 (top right),
// which pair_inverse_kernel forms (two 64 x 64 x 64 products, one workgroup
// per pair and triangle) into DI2[pair][0 / 1], column-major like DI.  Rows
// past N (a partial last block) take no part: C and D are zero there.
__global__ __launch_bounds__(256) void pair_inverse_kernel(int N, const float *LU, const float *DI, float *DI2)
{
    __shared__ float M[64][65], V[64][65], T[64][65];
    const int tid = threadIdx.x, pr = blockIdx.x >> 1, up = blockIdx.x & 1;
    const int b0 = 128 * pr;
    const float *iA = DI + (int64_t(2 * pr) * 2 + up) * 4096;       // inverse of block 2 pr
    const float *iB = DI + (int64_t(2 * pr + 1) * 2 + up) * 4096;   // inverse of block 2 pr + 1
    // M = C (lower: rows of block B, columns of block A) or D (upper: rows of A, columns of B)
    float v[16];
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + it * 256, i = e & 63, k = e >> 6;
        const int row = up ? b0 + i : b0 + 64 + i, col = up ? b0 + 64 + k : b0 + k;
        v[it] = LU[int64_t(min(col, N - 1)) * N + min(row, N - 1)] * ((row < N && col < N) ? 1.0f : 0.0f);
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + it * 256;
        M[e & 63][e >> 6] = v[it];
    }
    // first product with the inverse on M's right (lower: A^-1) or left... done as
    // lower: T = M iA, X = -iB T;  upper: T = M iB, Y = -iA T
    const float *right = up ? iB : iA, *left = up ? iA : iB;
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + it * 256;
        V[e & 63][e >> 6] = right[e];                                // entry (e % 64, e / 64)
    }
    __syncthreads();
    const int i = tid & 63, j0 = (tid >> 6) * 16;
    float y[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) y[q] = 0.0f;
#pragma unroll 8
    for (int k = 0; k < 64; ++k) {
        const float mk = M[i][k];
#pragma unroll
        for (int q = 0; q < 16; ++q) y[q] += mk * V[k][j0 + q];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) T[i][j0 + q] = y[q];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + it * 256;
        V[e & 63][e >> 6] = left[e];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) y[q] = 0.0f;
#pragma unroll 8
    for (int k = 0; k < 64; ++k) {
        const float vk = V[i][k];
#pragma unroll
        for (int q = 0; q < 16; ++q) y[q] += vk * T[k][j0 + q];
    }
    float *out = DI2 + (int64_t(pr) * 2 + up) * 4096;
#pragma unroll
    for (int q = 0; q < 16; ++q) out[(j0 + q) * 64 + i] = -y[q];    // entry (i, j0 + q), column-major
}

// Forward step for the 128 rows of pair pr: x_A = A^-1 y_A, x_B = X y_A + B^-1 y_B
// (every workgroup; workgroup 0 writes them to yout), then the rows below take
// the pair's 128 columns of L.  A workgroup owns 64 rows and splits the 128
// columns in four quarters, one per wave, whose sums meet in LDS in a fixed
// order.  Every load (the wave's quarter of L, the pair's y and inverse blocks)
// is issued before the first wait: y reaches the lanes by readlane, not through
// LDS, so the only barrier is the one that hands x to the four waves.  Loads
// unconditional, sums in partial sums.
__global__ __launch_bounds__(256) void trsv_lower2_kernel(int N, const float *LU, const float *DI, const float *DI2,
                                                          float *y, float *yout, int pr)
{
    __shared__ float xb[128], part[4][64];
    const int b0 = 128 * pr, bw = min(128, N - b0);
    const int tid = threadIdx.x, lr = tid & 63, q = tid >> 6;
    const int r = b0 + bw + blockIdx.x * 64 + lr;
    const float *col = LU + int64_t(b0) * N + min(r, N - 1);
    float v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = col[int64_t(min(q * 32 + k, bw - 1)) * N];
    if (tid < 128) {
        // lane k of waves 0 and 1 holds y_A[k] and y_B[k]; readlane broadcasts them
        const float yA = y[b0 + min(lr, bw - 1)] * (lr < bw ? 1.0f : 0.0f);
        const float yB = y[b0 + min(64 + lr, bw - 1)] * (64 + lr < bw ? 1.0f : 0.0f);
        const float ys = tid < 64 ? yA : yB;
        const int blk = tid < 64 ? 2 * pr : 2 * pr + 1;
        const float *inv = DI + (int64_t(blk) * 2 + 0) * 4096 + lr;
        const float *x2 = DI2 + (int64_t(pr) * 2 + 0) * 4096 + lr;
        float d[64], e2[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) d[k] = inv[k * 64];
#pragma unroll
        for (int k = 0; k < 64; ++k) e2[k] = x2[k * 64] * (tid < 64 ? 0.0f : 1.0f);   // unconditional loads
        float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 64; ++k)
            p4[k & 3] += d[k] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ys), k)) +
                         e2[k] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yA), k));
        const float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        xb[tid] = tid < bw ? s : 0.0f;
        if (blockIdx.x == 0 && tid < bw) yout[b0 + tid] = s;
    }
    __syncthreads();
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 32; ++k) p4[k & 3] += v[k] * xb[q * 32 + k];
    part[q][lr] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    __syncthreads();
    if (q == 0 && r < N) y[r] -= (part[0][lr] + part[1][lr]) + (part[2][lr] + part[3][lr]);
}

// Backward step for the 128 rows of pair pr: x_B = B^-1 y_B, x_A = A^-1 y_A + Y y_B,
// then the rows above take the pair's 128 columns of U (64 rows per workgroup,
// column quarters per wave, as in the forward step).
__global__ __launch_bounds__(256) void trsv_upper2_kernel(int N, const float *LU, const float *DI, const float *DI2,
                                                          float *y, float *yout, int pr)
{
    __shared__ float xb[128], part[4][64];
    const int b0 = 128 * pr, bw = min(128, N - b0);
    const int tid = threadIdx.x, lr = tid & 63, q = tid >> 6;
    const int r = blockIdx.x * 64 + lr;
    const float *col = LU + int64_t(b0) * N + min(r, max(b0 - 1, 0));
    float v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = col[int64_t(min(q * 32 + k, bw - 1)) * N];
    if (tid < 128) {
        const float yA = y[b0 + min(lr, bw - 1)] * (lr < bw ? 1.0f : 0.0f);
        const float yB = y[b0 + min(64 + lr, bw - 1)] * (64 + lr < bw ? 1.0f : 0.0f);
        const float ys = tid < 64 ? yA : yB;
        const int blk = tid < 64 ? 2 * pr : 2 * pr + 1;
        const float *inv = DI + (int64_t(blk) * 2 + 1) * 4096 + lr;
        const float *x2 = DI2 + (int64_t(pr) * 2 + 1) * 4096 + lr;
        float d[64], e2[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) d[k] = inv[k * 64];
#pragma unroll
        for (int k = 0; k < 64; ++k) e2[k] = x2[k * 64] * (tid < 64 ? 1.0f : 0.0f);   // unconditional loads
        float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 64; ++k)
            p4[k & 3] += d[k] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ys), k)) +
                         e2[k] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yB), k));
        const float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        xb[tid] = tid < bw ? s : 0.0f;
        if (blockIdx.x == 0 && tid < bw) yout[b0 + tid] = s;
    }
    __syncthreads();
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 32; ++k) p4[k & 3] += v[k] * xb[q * 32 + k];
    part[q][lr] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    __syncthreads();
    if (q == 0 && r < b0) y[r] -= (part[0][lr] + part[1][lr]) + (part[2][lr] + part[3][lr]);
}

// ---------------------------------------------------------------- inverted diagonal super-blocks
// The inverses of L's (unit lower) and U's (upper) kSB x kSB diagonal blocks
// (rows beyond N padded with the identity), built by recursive doubling from
// the inverted 64 x 64 blocks: with a block split into halves P1, P2 of h rows,
//   inv(L) = [[inv(P1), 0], [-inv(P2) L21 inv(P1), inv(P2)]],
//   inv(U) = [[inv(P1), -inv(P1) U12 inv(P2)], [0, inv(P2)]],
// for h = 64, 128, 256, 512, the products of one level batched in two launches
// (T = L21 inv(P1) or inv(P1) U12, then the off-diagonal block from T; T sits in
// the unused triangle of the same kSB x kSB block, which every later read of an
// inverted block masks out).  Storage: INV + (sb * 2 + f)
// kSB^2, f = 0 for L, 1 for U, column-major with leading dimension kSB.

// The 64 x 64 diagonal blocks: DI's inverses (identity beyond N).
__global__ __launch_bounds__(256) void blkinv_diag_kernel(int N, const float *DI, float *INV)
{
    const int t = blockIdx.x, sb = blockIdx.y >> 1, f = blockIdx.y & 1, g = sb * (kSB / 64) + t;
    float *dst = INV + (int64_t(sb) * 2 + f) * kSB * kSB + int64_t(64 * t) * kSB + 64 * t;
    const float *src = DI + (int64_t(g) * 2 + f) * 4096;
    const bool in = 64 * g < N;
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = threadIdx.x + 256 * it, r = e & 63, c = e >> 6;
        dst[int64_t(c) * kSB + r] = in ? src[e] : (r == c ? 1.0f : 0.0f);
    }
}

// A view of a column-major matrix: entry (i, k) = base[(c0 + k) ld + r0 + i],
// read as 0 outside [0, rmax) x [0, cmax) (addresses clamped) and, for a view
// of an inverted block (tri 1: lower, 2: upper), outside its triangle: the
// other triangle holds the scratch products of the doubling.
struct MatView {
    const float *base;
    int64_t ld;
    int r0, c0, rmax, cmax, tri;
    __device__ float at(int i, int k) const
    {
        const int r = r0 + i, c = c0 + k;
        const float v = base[int64_t(min(c, cmax - 1)) * ld + min(r, rmax - 1)];
        const bool in = r < rmax && c < cmax && !(tri == 1 && r < c) && !(tri == 2 && r > c);
        return in ? v : 0.0f;
    }
};

// One level h of the doubling, stage 1 (T) or 2 (the off-diagonal block): the
// workgroup forms the 64 x 64 block (ti, tj) of C = alpha A B (h x h x h) for
// item z (factor f = z & 1, pair z >> 1 over super-blocks), on
// v_mfma_f32_16x16x4_f32 with the layout of gemm_update_kernel (K in chunks of
// 32 through LDS, a 32 x 32 quarter per wavefront).
template <int STAGE>
__global__ __launch_bounds__(256) void blkinv_gemm_kernel(int N, const float *LU, float *INV, int h)
{
    __shared__ float As[64][33];   // A chunk: [row][k]
    __shared__ float Bs[64][33];   // B chunk transposed: [col][k]
    const int npairs = kSB / (2 * h), z = blockIdx.z, f = z & 1, pl = z >> 1, sb = pl / npairs, a = 2 * h * (pl % npairs);
    const int a0 = sb * kSB, big = 1 << 30;
    float *IF = INV + (int64_t(sb) * 2 + f) * kSB * kSB;
    MatView A, B;
    int cr, cc;   // C block origin (local to IF)
    float alpha;
    if (STAGE == 1) {
        if (f == 0) {   // T = L21 inv(P1) -> IF(a.., a+h..)
            A = {LU, N, a0 + a + h, a0 + a, N, N, 0};
            B = {IF, kSB, a, a, big, big, 1};
            cr = a; cc = a + h;
        } else {        // T = inv(P1) U12 -> IF(a+h.., a..)
            A = {IF, kSB, a, a, big, big, 2};
            B = {LU, N, a0 + a, a0 + a + h, N, N, 0};
            cr = a + h; cc = a;
        }
        alpha = 1.0f;
    } else {
        if (f == 0) {   // inv(L)_21 = -inv(P2) T -> IF(a+h.., a..)
            A = {IF, kSB, a + h, a + h, big, big, 1};
            B = {IF, kSB, a, a + h, big, big, 0};
            cr = a + h; cc = a;
        } else {        // inv(U)_12 = -T inv(P2) -> IF(a.., a+h..)
            A = {IF, kSB, a + h, a, big, big, 0};
            B = {IF, kSB, a + h, a + h, big, big, 2};
            cr = a; cc = a + h;
        }
        alpha = -1.0f;
    }
    const int m0 = 64 * blockIdx.x, n0 = 64 * blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wc = (wave >> 1) * 32, wr = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kc = 0; kc < h; kc += 32) {
        float va[8], vb[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = tid + it * 256;
            va[it] = A.at(m0 + (e & 63), kc + (e >> 6));
            vb[it] = B.at(kc + (e & 31), n0 + (e >> 5));
        }
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = tid + it * 256;
            As[e & 63][e >> 6] = va[it];
            Bs[e >> 5][e & 31] = vb[it];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 32; k += 4) {
            const int kk = k + (lane >> 4);
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const float av = Bs[wc + x * 16 + (lane & 15)][kk];   // MFMA A: [C column][k]
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const float bv = As[wr + y * 16 + (lane & 15)][kk];   // MFMA B: [k][C row]
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[x][y], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = n0 + wc + x * 16 + 4 * (lane >> 4) + i, r = m0 + wr + y * 16 + (lane & 15);
                IF[int64_t(cc + c) * kSB + cr + r] = alpha * acc[x][y][i];
            }
}

// Forms the inverted super-blocks of the factor (after its 64 x 64 inverses DI).
void blkinv_build(int N, const float *LU, const float *DI, float *INV, hipStream_t s)
{
    const int nsb = superblocks(N);
    hipLaunchKernelGGL(blkinv_diag_kernel, dim3(kSB / 64, 2 * nsb), dim3(256), 0, s, N, DI, INV);
    for (int h = 64; 2 * h <= kSB; h *= 2) {
        const dim3 g(h / 64, h / 64, 2 * nsb * (kSB / (2 * h)));
        hipLaunchKernelGGL(blkinv_gemm_kernel<1>, g, dim3(256), 0, s, N, LU, INV, h);
        hipLaunchKernelGGL(blkinv_gemm_kernel<2>, g, dim3(256), 0, s, N, LU, INV, h);
    }
}

// out[r] = sum_c M(r, c) in[c] (or out[r] -= it) over the rows [r0, r1) and
// columns [c0, c1) (c1 - c0 <= 1024), in and out indexed like the rows and
// columns, M column-major with entry (r, c) at M[(c + mc0) ld + r + mr0] (the
// offsets map them into M's own indices): 64 rows per workgroup, lane i holding
// row i, the 16 wavefronts taking 64 columns each (32 loads of a column block
// in flight before their products), partial sums meeting in LDS in a fixed
// order.  TRI: 1 = only column blocks at or left of the row block (the
// lower triangle of an inverted L super-block), 2 = at or right of it (U), 0 =
// all.  ACC: out -= the sum (the updates), else out = the sum.
template <int TRI, bool ACC>
__global__ __launch_bounds__(1024) void blk_matvec_kernel(const float *M, int64_t ld, int r0, int r1, int c0, int c1,
                                                          int mr0, int mc0, const float *in, float *out)
{
    __shared__ float xs[1024];
    __shared__ float part[16][64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rb = blockIdx.x, r = r0 + 64 * rb + lane;
    if (c0 + tid < c1) xs[tid] = in[c0 + tid];
    __syncthreads();
    const int cb0 = 64 * wave, ncol = min(64, c1 - c0 - cb0);
    // the triangular kinds have r0 == c0: row block rb and column block wave, counted alike
    const bool skip = ncol <= 0 || (TRI == 1 && wave > rb) || (TRI == 2 && wave < rb);
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (!skip) {
        const float *m = M + int64_t(mc0 + c0 + cb0) * ld + mr0 + r0 + 64 * rb + min(lane, r1 - r0 - 64 * rb - 1);
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 32) {   // two halves of 32 loads in flight
            float v[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) v[k] = m[int64_t(min(k0 + k, ncol - 1)) * ld];
#pragma unroll
            for (int k = 0; k < 32; ++k) p4[k & 3] += (k0 + k < ncol ? v[k] : 0.0f) * xs[cb0 + min(k0 + k, ncol - 1)];
        }
    }
    part[wave][lane] = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    __syncthreads();
    if (wave == 0 && r < r1) {
        float t = 0.0f;
#pragma unroll
        for (int w = 0; w < 16; ++w) t += part[w][lane];
        if (ACC) out[r] -= t;
        else out[r] = t;
    }
}

// b := U^{-1} L^{-1} b for an already permuted b by super-blocks (tmp: N
// floats of scratch), with the inverted super-blocks INV: per super-block one
// product with its inverse and one update of the rows after (forward) or
// before (backward) it.
hipError_t lu_solve_blk(int N, const float *LU, const float *INV, float *b, float *tmp, hipStream_t s)
{
    const int nsb = superblocks(N);
    for (int sb = 0; sb < nsb; ++sb) {
        const int S0 = sb * kSB, bs = std::min(kSB, N - S0);
        const float *IL = INV + (int64_t(sb) * 2) * kSB * kSB;
        hipLaunchKernelGGL((blk_matvec_kernel<1, false>), dim3((bs + 63) / 64), dim3(1024), 0, s, IL, int64_t(kSB), S0,
                           S0 + bs, S0, S0 + bs, -S0, -S0, b, tmp);
        if (S0 + bs < N)
            hipLaunchKernelGGL((blk_matvec_kernel<0, true>), dim3((N - S0 - bs + 63) / 64), dim3(1024), 0, s, LU, int64_t(N),
                               S0 + bs, N, S0, S0 + bs, 0, 0, tmp, b);
    }
    for (int sb = nsb - 1; sb >= 0; --sb) {
        const int S0 = sb * kSB, bs = std::min(kSB, N - S0);
        const float *IU = INV + (int64_t(sb) * 2 + 1) * kSB * kSB;
        hipLaunchKernelGGL((blk_matvec_kernel<2, false>), dim3((bs + 63) / 64), dim3(1024), 0, s, IU, int64_t(kSB), S0,
                           S0 + bs, S0, S0 + bs, -S0, -S0, tmp, b);
        if (S0 > 0)
            hipLaunchKernelGGL((blk_matvec_kernel<0, true>), dim3((S0 + 63) / 64), dim3(1024), 0, s, LU, int64_t(N), 0, S0, S0,
                               S0 + bs, 0, 0, b, tmp);
    }
    return hipGetLastError();
}

__global__ void permute_kernel(int N, const int *perm, const double *src, float *dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dst[i] = float(src[perm[i]]);
}

// ---------------------------------------------------------------- Gauss-Jordan inverse (no interchanges)
// For an exactly symmetric A of moderate order the FP32 factor used by the
// refinement is the explicit inverse X, formed by block Gauss-Jordan
// elimination without interchanges on 64 x 64 tiles of the matrix padded
// with the identity to Np = 64 nt rows.  Sweep of pivot block k (P = A_kk^-1):
//   A_kk <- P,  A_kj <- P A_kj,  A_ik <- -A_ik P,  A_ij <- A_ij - A_ik P A_kj,
// with the old A_ik and A_kj on the right-hand sides; after the nt sweeps the
// matrix holds X = A^-1.  One launch per sweep, one workgroup per tile: the
// old row and column blocks of the sweep come from copies made by the
// previous launch (the tiles of row and column k are rewritten in the same
// launch), and the workgroup that updates the next pivot tile also inverts it.
// Every product runs on v_mfma_f32_16x16x4_f32.  A refinement step then needs
// one matrix-vector product with X instead of two triangular solves.
typedef float Tile64[64][65];

// acc[a][b][v] = (X Y)[wr + 16 a + 4 (lane >> 4) + v][wc + 16 b + (lane & 15)]:
// this wavefront's 32 x 32 quadrant of the product of two 64 x 64 LDS tiles.
__device__ __forceinline__ void mm64_acc(const float (*X)[65], const float (*Y)[65], floatx4 acc[2][2], int wr, int wc,
                                         int lane)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 64; k += 4) {
        const int kk = k + (lane >> 4);
        float av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = X[wr + 16 * a + (lane & 15)][kk];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Y[kk][wc + 16 * b + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
}

// Inverse of the 16 x 16 block B = T[q .. q+15][q .. q+15] by wavefront 0 into S:
// lane r (r < 16) holds row r in registers; per pivot the pivot row reaches
// every lane by readlane (scalar registers, no LDS) and each entry takes one
// FMA: with t = -B_rp / B_pp off the pivot row and t = 1 / B_pp - 1 on it,
// B_rc + t B_pc is the swept entry for c != p; column p becomes -B_rp / B_pp,
// and 1 / B_pp on the pivot.  Returns 1 on a zero or non-finite pivot.
__device__ __forceinline__ int invert16_wave(const float (*T)[65], int q, float (*S)[17], int lane)
{
    const int r = lane & 15;
    float e[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) e[c] = T[q + r][q + c];
    int bad = 0;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        float rp[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) rp[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e[c]), p));
        const float d = rp[p];
        const bool ok = fabsf(d) > 0.0f && fabsf(d) <= 3.402823466e38f;
        bad |= ok ? 0 : 1;
        const float ip = ok ? __builtin_amdgcn_rcpf(d) : 0.0f;
        const float f = e[p];
        const float t = (r == p) ? ip - 1.0f : -f * ip;
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c != p) e[c] = fmaf(t, rp[c], e[c]);
        e[p] = (r == p) ? ip : t;
    }
    if (lane < 16)
#pragma unroll
        for (int c = 0; c < 16; ++c) S[r][c] = e[c];
    return bad;
}

// In-place inverse of the 64 x 64 LDS tile T by four Gauss-Jordan sweeps of
// 16 x 16 pivot blocks (the same sweep as above, one level down).  Per sweep:
// wavefront 0 inverts the pivot block into S; then Uh = S T_q (the pivot
// block's rows, their own columns replaced by S) and, with V = T_{:q} (old),
// T <- T - V Uh outside the pivot rows and columns, -V Uh in the pivot
// columns, Uh in the pivot rows.  *bad (LDS, zeroed by the caller) is set on a
// zero or non-finite pivot.
__device__ __forceinline__ void invert64_lds(Tile64 &T, float (*S)[17], Tile64 &Uh, int *bad, int tid)
{
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
#pragma unroll
    for (int q = 0; q < 64; q += 16) {
        if (wave == 0) {
            if (invert16_wave(T, q, S, lane) && lane == 0) *bad = 1;
        }
        __syncthreads();
        {
            // Uh = S T[q .. q+15][:], wavefront w: columns 16 w .. 16 w + 15
            floatx4 u = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            const int c0 = 16 * wave;
#pragma unroll
            for (int k = 0; k < 16; k += 4) {
                const int kk = k + (lane >> 4);
                u = __builtin_amdgcn_mfma_f32_16x16x4f32(S[lane & 15][kk], T[q + kk][c0 + (lane & 15)], u, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = 4 * (lane >> 4) + v, j = c0 + (lane & 15);
                Uh[m][j] = (j >= q && j < q + 16) ? S[m][j - q] : u[v];
            }
        }
        // the old pivot columns of this wavefront's rows and its quadrant, read before any write
        float va[2][4], told[2][2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) va[a][ks] = T[wr + 16 * a + (lane & 15)][q + 4 * ks + (lane >> 4)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) told[a][b][v] = T[wr + 16 * a + 4 * (lane >> 4) + v][wc + 16 * b + (lane & 15)];
        __syncthreads();
        floatx4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = 4 * ks + (lane >> 4);
            float bv[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Uh[kk][wc + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va[a][ks], bv[b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = wr + 16 * a + 4 * (lane >> 4) + v, j = wc + 16 * b + (lane & 15);
                    const bool iq = i >= q && i < q + 16, jq = j >= q && j < q + 16;
                    T[i][j] = iq ? Uh[i - q][j] : (jq ? -acc[a][b][v] : told[a][b][v] - acc[a][b][v]);
                }
        __syncthreads();
    }
}

// Sweep k of the Gauss-Jordan inverse (k = -1: load A, FP64 or FP32 row-major,
// into the padded FP32 matrix W, row-major with ld Np).  Workgroup b owns tile
// (b / nt, b % nt).  Rin / Cin / Pin: the old row block k, column block k and
// the inverse of the pivot tile, made by the previous launch; the tiles of
// row and column k + 1 after this sweep go to Rout / Cout and the inverse of
// the new pivot tile to Pout (a zero or non-finite pivot sets *info).
template <typename InT>
__global__ __launch_bounds__(256) void gj_step_kernel(int N, int Np, int k, const InT *A, int64_t lda, float *W,
                                                      const float *Rin, const float *Cin, const float *Pin, float *Rout,
                                                      float *Cout, float *Pout, int *info, const double *ctl)
{
    __shared__ Tile64 T, L, R, P;
    if (ctl[CTL_ASYM] != 0.0) return;   // not symmetric: this inverse will not be used
    __shared__ float S[16][17];
    __shared__ int bad;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
    const int nt = Np / 64;
    const int bi = blockIdx.x / nt, bj = blockIdx.x - (blockIdx.x / nt) * nt;
    float *Wt = W + int64_t(bi) * 64 * Np + bj * 64;
    const bool ri = bi == k, cj = bj == k;
    if (k < 0) {
        float tv[16];
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + 256 * it, r = bi * 64 + (e >> 6), c = bj * 64 + (e & 63);
            const bool in = r < N && c < N;
            tv[it] = float(A[int64_t(min(r, N - 1)) * lda + min(c, N - 1)]) * (in ? 1.0f : 0.0f) +
                     ((!in && r == c) ? 1.0f : 0.0f);
        }
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + 256 * it;
            T[e >> 6][e & 63] = tv[it];
        }
    } else {
        float tv[16], pv[16], lv[16], rv[16];
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + 256 * it;
            tv[it] = Wt[int64_t(e >> 6) * Np + (e & 63)];
            pv[it] = Pin[e];
            lv[it] = Cin[int64_t(bi) * 4096 + e];
            rv[it] = Rin[int64_t(bj) * 4096 + e];
        }
#pragma unroll
        for (int it = 0; it < 16; ++it) {
            const int e = tid + 256 * it;
            T[e >> 6][e & 63] = tv[it];
            P[e >> 6][e & 63] = pv[it];
            L[e >> 6][e & 63] = lv[it];
            R[e >> 6][e & 63] = rv[it];
        }
    }
    __syncthreads();
    if (k >= 0) {
        floatx4 acc[2][2];
        if (ri && cj) {
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int e = tid + 256 * it;
                T[e >> 6][e & 63] = P[e >> 6][e & 63];
            }
        } else if (ri || cj) {
            // row k: P A_kj;  column k: -A_ik P
            if (ri) mm64_acc(P, T, acc, wr, wc, lane);
            else mm64_acc(T, P, acc, wr, wc, lane);
            __syncthreads();
            const float sg = ri ? 1.0f : -1.0f;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        T[wr + 16 * a + 4 * (lane >> 4) + v][wc + 16 * b + (lane & 15)] = sg * acc[a][b][v];
        } else {
            // A_ij - A_ik (P A_kj): first P A_kj into R, then the product with A_ik
            mm64_acc(P, R, acc, wr, wc, lane);
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) R[wr + 16 * a + 4 * (lane >> 4) + v][wc + 16 * b + (lane & 15)] = acc[a][b][v];
            __syncthreads();
            mm64_acc(L, R, acc, wr, wc, lane);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) T[wr + 16 * a + 4 * (lane >> 4) + v][wc + 16 * b + (lane & 15)] -= acc[a][b][v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = tid + 256 * it;
        Wt[int64_t(e >> 6) * Np + (e & 63)] = T[e >> 6][e & 63];
    }
    if (k + 1 < nt) {
        if (bi == k + 1)
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int e = tid + 256 * it;
                Rout[int64_t(bj) * 4096 + e] = T[e >> 6][e & 63];
            }
        if (bj == k + 1)
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int e = tid + 256 * it;
                Cout[int64_t(bi) * 4096 + e] = T[e >> 6][e & 63];
            }
        if (bi == k + 1 && bj == k + 1) {
            if (tid == 0) bad = 0;
            __syncthreads();
            invert64_lds(T, S, L, &bad, tid);
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int e = tid + 256 * it;
                Pout[e] = T[e >> 6][e & 63];
            }
            if (tid == 0 && bad && *info == 0) *info = 64 * (k + 1) + 1;
        }
    }
}

// v = X r: X the Gauss-Jordan inverse (row-major, ld Np; zero beyond column N
// in rows below N), r FP64; one wavefront per row, four columns per lane and
// step, two steps of loads in flight.
__global__ __launch_bounds__(256) void inv_apply_kernel(int N, int Np, const float *X, const double *r, float *v,
                                                        const double *ctl)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= N || ctl_stopped(ctl)) return;
    const float *x = X + int64_t(row) * Np;
    float p4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int j0 = 4 * lane; j0 < Np; j0 += 512) {
        const int j1 = j0 + 256;
        const float4 a0 = *reinterpret_cast<const float4 *>(x + j0);
        const float4 a1 = j1 < Np ? *reinterpret_cast<const float4 *>(x + j1) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float rv[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rv[q] = float(r[min(j0 + q, N - 1)]) * (j0 + q < N ? 1.0f : 0.0f);
            rv[4 + q] = float(r[min(j1 + q, N - 1)]) * (j1 + q < N ? 1.0f : 0.0f);
        }
        p4[0] += a0.x * rv[0];
        p4[1] += a0.y * rv[1];
        p4[2] += a0.z * rv[2];
        p4[3] += a0.w * rv[3];
        p4[0] += a1.x * rv[4];
        p4[1] += a1.y * rv[5];
        p4[2] += a1.z * rv[6];
        p4[3] += a1.w * rv[7];
    }
    float s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) v[row] = s;
}

// ---------------------------------------------------------------- refinement pieces
// r = beta - A x (FP64), one wavefront per row; A row-major as stored.
// Row access of A for the residual and the row sums: one wavefront per row;
// with VEC (rows 16-byte aligned) each lane takes 16-byte vectors (four FP32 or
// two FP64 entries), eight of them in flight, then the rest of the row entry
// by entry.
template <typename InT, bool VEC>
struct RowVec {
    static constexpr int V = VEC ? 16 / int(sizeof(InT)) : 1;
    // entries [V i, V i + V) of row a, as doubles
    __device__ static __forceinline__ void load(const InT *a, int i, double (&v)[V])
    {
        if constexpr (!VEC) {
            v[0] = double(a[i]);
        } else if constexpr (sizeof(InT) == 4) {
            const float4 f = *reinterpret_cast<const float4 *>(a + 4 * i);
            v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
        } else {
            const double2 f = *reinterpret_cast<const double2 *>(a + 2 * i);
            v[0] = f.x; v[1] = f.y;
        }
    }
};

// r = beta - A x, FP64 accumulation: each wavefront takes kResRows rows, so
// that every load of x serves all of them (x is re-read once per wavefront
// rather than once per row), two vectors per row in flight per step.
constexpr int kResRows = 4;
template <typename InT, bool VEC>
__global__ __launch_bounds__(256) void residual_kernel(int N, const InT *A, int64_t lda, const double *x,
                                                       const double *beta, double *r, const double *ctl)
{
    using R = RowVec<InT, VEC>;
    constexpr int V = R::V, RR = kResRows;
    const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RR;
    const int lane = threadIdx.x & 63;
    if (row0 >= N || ctl_stopped(ctl)) return;
    const InT *a[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) a[q] = A + int64_t(min(row0 + q, N - 1)) * lda;
    const int NV = N / V;
    double acc[RR][2];
#pragma unroll
    for (int q = 0; q < RR; ++q) acc[q][0] = acc[q][1] = 0.0;
    int i = lane;
    for (; i + 64 < NV; i += 2 * 64) {
        double av[2][RR][V], xv[2][V];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < RR; ++q) R::load(a[q], i + 64 * h, av[h][q]);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < V; ++e) xv[h][e] = x[V * (i + 64 * h) + e];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int e = 0; e < V; ++e) acc[q][h] += av[h][q][e] * xv[h][e];
    }
    for (; i < NV; i += 64) {
        double xv[V];
#pragma unroll
        for (int e = 0; e < V; ++e) xv[e] = x[V * i + e];
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            double av[V];
            R::load(a[q], i, av);
#pragma unroll
            for (int e = 0; e < V; ++e) acc[q][0] += av[e] * xv[e];
        }
    }
    for (int j = NV * V + lane; j < N; j += 64)
#pragma unroll
        for (int q = 0; q < RR; ++q) acc[q][0] += double(a[q][j]) * x[j];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        double s = acc[q][0] + acc[q][1];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0 && row0 + q < N) r[row0 + q] = beta[row0 + q] - s;
    }
}

// rs = the absolute row sums of A (the infinity norm's terms).
template <typename InT, bool VEC>
__global__ __launch_bounds__(256) void rowabs_kernel(int N, const InT *A, int64_t lda, double *rs)
{
    using R = RowVec<InT, VEC>;
    constexpr int V = R::V;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N) return;
    const InT *a = A + int64_t(row) * lda;
    const int NV = N / V;
    double p4[4] = {0.0, 0.0, 0.0, 0.0};
    int i = lane;
    for (; i + 7 * 64 < NV; i += 8 * 64) {
        double av[8][V];
#pragma unroll
        for (int u = 0; u < 8; ++u) R::load(a, i + 64 * u, av[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) p4[u & 3] += fabs(av[u][e]);
    }
    for (; i < NV; i += 64) {
        double av[V];
        R::load(a, i, av);
#pragma unroll
        for (int e = 0; e < V; ++e) p4[e & 3] += fabs(av[e]);
    }
    for (int j = NV * V + lane; j < N; j += 64) p4[0] += fabs(double(a[j]));
    double s = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) rs[row] = s;
}

// True when every row of A starts on a 16-byte boundary.
template <typename InT>
bool rows_aligned16(const void *A, int64_t lda)
{
    return reinterpret_cast<uintptr_t>(A) % 16 == 0 && (lda * int64_t(sizeof(InT))) % 16 == 0;
}

template <typename InT>
void launch_rowabs(int N, const void *A, int64_t lda, double *rs, hipStream_t s)
{
    if (rows_aligned16<InT>(A, lda))
        hipLaunchKernelGGL((rowabs_kernel<InT, true>), dim3((N + 3) / 4), dim3(256), 0, s, N, static_cast<const InT *>(A), lda, rs);
    else
        hipLaunchKernelGGL((rowabs_kernel<InT, false>), dim3((N + 3) / 4), dim3(256), 0, s, N, static_cast<const InT *>(A), lda, rs);
}

// Largest of two values that propagates NaN (fmax returns the other operand),
// so that a non-finite correction, residual or entry reaches the host's checks.
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

// x += d (d FP32), and max-norms: red[0] = |d|_inf, red[1] = |x|_inf, red[2] = |r|_inf, red[3] = |beta|_inf.
// With a control block (batched refinement): nothing once stopped; otherwise
// the step's decision, taken as the host would: converged when
// ||d|| <= tol ||x||, or when a correction does not halve
// (||d|| > ||d_prev|| / 2) with the backward error at the FP64 level; stalled
// above that level when a correction does not shrink at all or two in a row
// do not halve; not finite on NaN or overflow; a zero pivot (info) or an
// asymmetric matrix ends the attempt before the first step.
__global__ __launch_bounds__(1024) void update_norms_kernel(int N, double *x, const float *d, const double *r,
                                                            const double *beta, int add, double *red, double *ctl,
                                                            const int *info, double tol)
{
    __shared__ double s[4][16];
    if (ctl_stopped(ctl)) return;
    if (ctl && *info != 0) {
        if (threadIdx.x == 0) ctl[CTL_STOP] = 4.0;
        return;
    }
    double m[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double xi = add ? x[i] + double(d[i]) : double(d[i]);
        x[i] = xi;
        m[0] = nan_max(m[0], fabs(double(d[i])));
        m[1] = nan_max(m[1], fabs(xi));
        m[2] = nan_max(m[2], fabs(r[i]));
        m[3] = nan_max(m[3], fabs(beta[i]));
    }
    for (int q = 0; q < 4; ++q) {
        for (int off = 32; off > 0; off >>= 1) m[q] = nan_max(m[q], __shfl_xor(m[q], off));
        if ((threadIdx.x & 63) == 0) s[q][threadIdx.x >> 6] = m[q];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) v = nan_max(v, s[threadIdx.x][k]);
        red[threadIdx.x] = v;
        if (ctl) s[threadIdx.x][0] = v;
    }
    if (ctl) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const double dn = s[0][0], xn = s[1][0], rn = s[2][0], bn = s[3][0];
            const double rel = dn == 0.0 ? 0.0 : dn / xn;
            const double bwd = rn / (ctl[CTL_NORMA] * xn + bn);   // of the iterate before this step
            double stop = 0.0, slow = 0.0;
            if (rel <= tol) {
                stop = 1.0;
            } else if (rel > 0.5 * ctl[CTL_PREV]) {
                if (bwd <= 64 * 1.1102230246251565e-16) stop = 1.0;
                else if (rel >= ctl[CTL_PREV] || ctl[CTL_SLOW] != 0.0) stop = 2.0;
                else slow = 1.0;
            } else if (!(rel < 1e300)) {
                stop = 3.0;
            }
            ctl[CTL_SLOW] = slow;
            ctl[CTL_ITERS] += 1.0;
            ctl[CTL_REL] = rel;
            ctl[CTL_BWD] = bwd;
            ctl[CTL_PREV] = rel;
            ctl[CTL_STOP] = stop;
        }
    }
}

// End of a refinement batch, written straight to the caller's pinned host
// buffer: out[0 .. CTL_SIZE) = the control block, then |r|_inf, |x|_inf,
// |beta|_inf of the final iterate (its backward error) and the zero-pivot flag.
__global__ __launch_bounds__(1024) void final_norms_kernel(int N, const double *r, const double *x, const double *beta,
                                                           const double *ctl, const int *info, double *out)
{
    __shared__ double s[3][16];
    double m[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        m[0] = nan_max(m[0], fabs(r[i]));
        m[1] = nan_max(m[1], fabs(x[i]));
        m[2] = nan_max(m[2], fabs(beta[i]));
    }
    for (int q = 0; q < 3; ++q) {
        for (int off = 32; off > 0; off >>= 1) m[q] = nan_max(m[q], __shfl_xor(m[q], off));
        if ((threadIdx.x & 63) == 0) s[q][threadIdx.x >> 6] = m[q];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double v = 0.0;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) v = nan_max(v, s[threadIdx.x][k]);
        out[CTL_SIZE + threadIdx.x] = v;
    }
    if (threadIdx.x < CTL_SIZE) out[threadIdx.x] = ctl[threadIdx.x];
    if (threadIdx.x == 0) out[CTL_SIZE + 3] = double(*info);
}

__global__ void ctl_init_kernel(double *ctl)
{
    if (threadIdx.x == 0) {
        ctl[CTL_PREV] = 1e300;
        ctl[CTL_STOP] = 0.0;
        ctl[CTL_ITERS] = 0.0;
        ctl[CTL_REL] = 1.0;
        ctl[CTL_BWD] = 1.0;
        ctl[CTL_SLOW] = 0.0;
    }
}

__global__ __launch_bounds__(1024) void max_kernel(int N, const double *v, double *out)
{
    __shared__ double s[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) m = nan_max(m, fabs(v[i]));
    for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v2 = 0.0;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) v2 = nan_max(v2, s[k]);
        *out = v2;
    }
}

template <typename InT>
void launch_residual(int N, const void *A, int64_t lda, const double *x, const double *beta, double *r, hipStream_t s,
                     const double *ctl = nullptr)
{
    if (rows_aligned16<InT>(A, lda))
        hipLaunchKernelGGL((residual_kernel<InT, true>), dim3((N + 4 * kResRows - 1) / (4 * kResRows)), dim3(256), 0, s, N,
                           static_cast<const InT *>(A), lda, x, beta, r, ctl);
    else
        hipLaunchKernelGGL((residual_kernel<InT, false>), dim3((N + 4 * kResRows - 1) / (4 * kResRows)), dim3(256), 0, s, N,
                           static_cast<const InT *>(A), lda, x, beta, r, ctl);
}

// Exact symmetry test of A (row-major, leading dimension lda): each workgroup
// takes 32 x 32 tiles (ti, tj), ti <= tj, in a grid-stride loop, stages the
// mirror tile (tj, ti) in LDS and compares; out[blockIdx.x] = the largest
// |A_ij - A_ji| it saw.
template <typename InT>
__global__ __launch_bounds__(256) void asym_kernel(int N, const InT *A, int64_t lda, double *out)
{
    __shared__ InT T[32][33];
    __shared__ double s[4];
    const int nt = (N + 31) / 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double mx = 0.0;
    for (int64_t t = blockIdx.x; t < int64_t(nt) * nt; t += gridDim.x) {
        const int ti = int(t / nt), tj = int(t % nt);
        if (ti > tj) continue;                                   // uniform over the workgroup
        // loads from clamped addresses, all issued before any is used; entries
        // outside the matrix are masked by selection
        InT va[4], vb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int y = ty + 8 * q;
            va[q] = A[int64_t(min(tj * 32 + y, N - 1)) * lda + min(ti * 32 + tx, N - 1)];
            vb[q] = A[int64_t(min(ti * 32 + y, N - 1)) * lda + min(tj * 32 + tx, N - 1)];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) T[ty + 8 * q][tx] = va[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int y = ty + 8 * q, r = ti * 32 + y, c = tj * 32 + tx;
            const double d = fabs(double(vb[q]) - double(T[tx][y]));
            mx = (r < N && c < N) ? nan_max(mx, d) : mx;
        }
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) mx = nan_max(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = nan_max(nan_max(s[0], s[1]), nan_max(s[2], s[3]));
}

// Register panel for the rows k0..N-1 (m = N - k0 <= 16384) of the block
// [K0, KE): the shape (rows per thread, width, threads) is the fastest per
// column for that height (measured), the width shrinking as the rows per thread
// grow.  Returns the width used.
int launch_panel(int N, float *LU, int k0, int KE, int *piv, int *info, hipStream_t s)
{
    const int m = N - k0;
    int w;
    if (m <= 1024) {
        w = std::min(32, KE - k0);
        hipLaunchKernelGGL((panel_reg_kernel<4, 32, 256>), dim3(1), dim3(256), 0, s, N, LU, k0, w, piv, info);
    } else if (m <= 2048) {
        w = std::min(16, KE - k0);
        hipLaunchKernelGGL((panel_reg_kernel<4, 16, 512>), dim3(1), dim3(512), 0, s, N, LU, k0, w, piv, info);
    } else if (m <= 4096) {
        w = std::min(8, KE - k0);
        hipLaunchKernelGGL((panel_reg_kernel<8, 8, 512>), dim3(1), dim3(512), 0, s, N, LU, k0, w, piv, info);
    } else if (m <= 8192) {
        w = std::min(8, KE - k0);
        hipLaunchKernelGGL((panel_reg_kernel<8, 8, 1024>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
    } else {
        w = std::min(4, KE - k0);
        hipLaunchKernelGGL((panel_reg_kernel<16, 4, 1024>), dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
    }
    return w;
}

}  // namespace

size_t solve_workspace_bytes(int N)
{
    const size_t nblk = size_t(N + 63) / 64, Np = size_t(padded64(N));
    return align_up(Np * Np * sizeof(float)) + 2 * align_up(size_t(N) * sizeof(int)) + align_up(16) +
           align_up(size_t(N) * sizeof(double)) + 2 * align_up(size_t(N) * sizeof(float)) + align_up(64 * sizeof(double)) +
           align_up(size_t(N) * sizeof(double)) + align_up(nblk * 2 * 4096 * sizeof(float)) +
           align_up(std::max<size_t>(nblk / 2, 1) * 2 * 4096 * sizeof(float)) +
           2 * align_up(2 * nblk * 4096 * sizeof(float)) + align_up(2 * 4096 * sizeof(float)) +
           align_up(blkinv_floats(N) * sizeof(float));
}

bool lu_without_pivoting_supported(int N) { return N <= 16384; }

namespace {
// The rank-bk update of the trailing matrix [KE, N) x [KE, N).
void trailing_update(int N, float *LU, int KE, int K0, int bk, hipStream_t s)
{
    if (N % 4 == 0 && KE % 4 == 0 && bk % 4 == 0) {
        const int nt = (N - KE + 127) / 128, per = (nt * nt + 7) / 8;
        hipLaunchKernelGGL((update128_kernel<false, false>), dim3(8 * per), dim3(256), 0, s, N, LU, KE, KE, N, K0, bk, nt, nt,
                           nt * nt, per);
        return;
    }
    const int nb = (N - KE + 63) / 64;
    hipLaunchKernelGGL(gemm_update_kernel, dim3(nb, nb), dim3(256), 0, s, N, LU, KE, KE, N, K0, bk);
}

// C -= L U on rows [r0, rend) and columns [c0, cend) of the factor, L = its
// columns [kb, kb + klen), U = its rows [kb, kb + klen); rend - r0 is a
// multiple of 64 or rend = N (the launches cover whole 64- or 128-row blocks
// and mask only at N).  The 128 x 128 kernel for the rank-256 updates (at most
// max_per_xcd workgroups per XCD), the 64 x 64 one for the narrow strips of the
// panel work.
void update_region(int N, float *LU, int r0, int rend, int c0, int cend, int kb, int klen, hipStream_t s,
                   int max_per_xcd = 1 << 30)
{
    if (rend <= r0 || cend <= c0) return;
    if (klen > 64 && N % 4 == 0 && r0 % 4 == 0 && klen % 4 == 0 && ((rend - r0) % 128 == 0 || rend == N)) {
        const int ntr = (rend - r0 + 127) / 128, ntc = (cend - c0 + 127) / 128;
        const int per = std::min(max_per_xcd, (ntr * ntc + 7) / 8);
        hipLaunchKernelGGL((update128_kernel<false, false>), dim3(8 * per), dim3(256), 0, s, N, LU, r0, c0, cend, kb, klen,
                           ntr, ntc, ntr * ntc, per);
        return;
    }
    hipLaunchKernelGGL(gemm_update_kernel, dim3((rend - r0 + 63) / 64, (cend - c0 + 63) / 64), dim3(256), 0, s, N, LU, r0,
                       c0, cend, kb, klen);
}

// The symmetric update C -= L21 D L21^T (U12 = D L21^T formed from the column
// panel, columns [kb, kb + klen) of the factor) for N % 4 == 0: on the
// rectangle [r0, N) x [c0, cend) (whole 128-row blocks down to N), or, with
// lower, on the 256 x 256 blocks on or below the diagonal of [r0, N)^2.
void update_sym_region(int N, float *LU, int r0, int c0, int cend, int kb, int klen, bool lower, hipStream_t s,
                       int max_per_xcd = 1 << 30)
{
    if (r0 >= N || cend <= c0) return;
    const int ntr = (N - r0 + 127) / 128, ntc = lower ? ntr : (cend - c0 + 127) / 128;
    const int ntiles = lower ? lower256_count(ntr) : ntr * ntc, per = std::min(max_per_xcd, (ntiles + 7) / 8);
    if (lower)
        hipLaunchKernelGGL((update128_kernel<true, true>), dim3(8 * per), dim3(256), 0, s, N, LU, r0, r0, N, kb, klen, ntr,
                           ntr, ntiles, per);
    else
        hipLaunchKernelGGL((update128_kernel<true, false>), dim3(8 * per), dim3(256), 0, s, N, LU, r0, c0, cend, kb, klen, ntr,
                           ntc, ntiles, per);
}

}  // namespace

// The second stream and events of the look-ahead (default priority), owned by
// the caller's context: made on the first factorisation that uses them, kept
// until lookahead_free.
struct LookAhead {
    hipStream_t aux = nullptr;
    hipEvent_t ev_panel = nullptr, ev_rest[2] = {nullptr, nullptr};
};

void lookahead_free(void *p)
{
    LookAhead *la = static_cast<LookAhead *>(p);
    if (!la) return;
    if (la->aux) (void)hipStreamSynchronize(la->aux);
    for (hipEvent_t e : {la->ev_panel, la->ev_rest[0], la->ev_rest[1]})
        if (e) (void)hipEventDestroy(e);
    if (la->aux) (void)hipStreamDestroy(la->aux);
    delete la;
}

namespace {
// The caller's look-ahead resources (made in *slot on first use, on the
// current device); nullptr if they cannot be made: the updates then all go to
// the caller's stream, in the same order.
LookAhead *lookahead_get(void **slot)
{
    if (!slot) return nullptr;
    if (*slot) return static_cast<LookAhead *>(*slot);
    LookAhead *la = new LookAhead;
    if (hipStreamCreateWithFlags(&la->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&la->ev_panel, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&la->ev_rest[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&la->ev_rest[1], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        lookahead_free(la);
        return nullptr;
    }
    *slot = la;
    return la;
}
}  // namespace

hipError_t lu_factor_f32(int N, float *LU, int *piv, int *info, void *diag_inv, bool pivot, hipStream_t s,
                         void **lookahead)
{
    // Without pivoting (pivot false, N <= 16384, diag_inv required): blocked LU
    // in 64-column blocks up to N = 4096, 256-column blocks of four 64-column
    // quarters beyond (a quarter of the trailing matrix's traffic), the diagonal as pivot
    // and no interchange anywhere; the inverted 64 x 64 diagonal blocks go to
    // diag_inv.  With partial pivoting, two levels: blocks of BK columns, each
    // factored by narrow register panels whose triangular solves and updates
    // stay inside the block; then one triangular solve for the block's U12 and
    // one rank-BK update of the trailing matrix (the MFMA-bound part).  Row
    // interchanges always go to the full rows.  Up to N = 4096 one block spans
    // the matrix (every narrow panel updates the whole trailing matrix): there
    // the launches saved outweigh the traffic of the narrow updates (measured).
    if (!pivot && (!lu_without_pivoting_supported(N) || !diag_inv)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, info);
    if (!pivot && N <= 4096) {
        // 64-column blocks: diagonal block factored and inverted (its inverses are
        // the triangular solves' inverted diagonal blocks), then L21 and U12 as
        // products with the inverses, then the rank-64 update
        float *DI = static_cast<float *>(diag_inv);
        for (int K0 = 0; K0 < N; K0 += 64) {
            const int bk = std::min(64, N - K0), KE = K0 + bk, rest = N - KE;
            hipLaunchKernelGGL(diag64_kernel, dim3(1), dim3(128), 0, s, N, LU, K0, bk, DI, info);
            if (rest > 0) {
                const int nrb = (rest + 63) / 64;
                hipLaunchKernelGGL(panel_mul_kernel, dim3(2 * nrb), dim3(256), 0, s, N, LU, K0, bk, KE, DI, nrb);
                trailing_update(N, LU, KE, K0, bk, s);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipGetLastError();
    }
    if (!pivot) {
        // beyond N = 4096: blocks of 256 columns made of four 64-column quarters.
        // Each quarter is factored and inverted by diag64_kernel and gets its L21
        // and U12 from panel_mul_kernel; its rank-64 update then goes only to the
        // block's remaining columns (the column strip, every row below) and, for
        // a general A, to the block's remaining rows right of the block (the row
        // strip).  Each block's rank-256 trailing update is split in two: the
        // next block's columns (and rows) (the cross, on s, ahead of the next
        // block's panel work) and the rest, on a second stream, which runs while
        // s factors the next block (look-ahead of one block).  Every region is
        // written by one launch at a time: the cross of block b + 1 waits for the
        // rest of block b - 1, and the rest of block b for the panel work of
        // block b.
        //
        // The panel work on s (and the cross update) raise their wavefronts'
        // issue priority: on a SIMD shared with the rest update's MFMA waves
        // their short dependent chains would otherwise wait behind them.
        //
        // The matrices factored here are exactly symmetric (the caller's
        // symmetry test), so U = D L^T with D the pivots.  For N % 4 == 0 that
        // halves the work: only the 256 x 256 blocks on or below the diagonal are
        // updated, with U12 formed as D L21^T from the column panel; U12 is
        // formed by panel_mul_kernel only inside the diagonal block; no row
        // strips; and at the end U above the diagonal 256 x 256 blocks is filled
        // in as D L^T for the triangular solves.
        float *DI = static_cast<float *>(diag_inv);
        const bool sym = N % 4 == 0;
        LookAhead *la = lookahead_get(lookahead);
        hipStream_t aux = la ? la->aux : s;
        bool aux_used = false;
        int b = 0;
        for (int K0 = 0; K0 < N; K0 += 256, ++b) {
            const int KE = std::min(N, K0 + 256);
            if (K0 > 0) {
                // the cross of this block takes the previous block's rank-256 update
                if (la && b >= 2) {
                    if (hipError_t e = hipStreamWaitEvent(s, la->ev_rest[b & 1], 0); e != hipSuccess) return e;
                }
                const int Kp = K0 - 256;
                if (sym) {
                    update_sym_region(N, LU, K0, K0, KE, Kp, 256, false, s);
                } else {
                    update_region(N, LU, K0, N, K0, KE, Kp, 256, s);
                    if (KE < N) update_region(N, LU, K0, KE, KE, N, Kp, 256, s);
                }
            }
            for (int Kq = K0; Kq < KE; Kq += 64) {
                const int bq = std::min(64, N - Kq), KEq = Kq + bq;
                hipLaunchKernelGGL(diag64_kernel, dim3(1), dim3(128), 0, s, N, LU, Kq, bq, DI, info);
                if (KEq >= N) break;
                const int nr = (N - KEq + 63) / 64, nc = sym ? (KE - KEq + 63) / 64 : nr;
                hipLaunchKernelGGL(panel_mul_kernel, dim3(nr + nc), dim3(256), 0, s, N, LU, Kq, bq, KEq, DI, nr);
                if (KEq < KE) {
                    update_region(N, LU, KEq, N, KEq, KE, Kq, bq, s);
                    if (!sym && KE < N) update_region(N, LU, KEq, KE, KE, N, Kq, bq, s);
                }
            }
            // the rest of this block's trailing update, [KE + 256, N)^2
            if (KE + 256 < N) {
                if (la) {
                    hipError_t e;
                    if ((e = hipEventRecord(la->ev_panel, s)) != hipSuccess ||
                        (e = hipStreamWaitEvent(aux, la->ev_panel, 0)) != hipSuccess)
                        return e;
                }
                // two workgroups per CU (as fast as a full grid, measured): the
                // third slot stays free for the panel work on s
                if (sym) update_sym_region(N, LU, KE + 256, KE + 256, N, K0, 256, true, aux, la ? 64 : 1 << 30);
                else update_region(N, LU, KE + 256, N, KE + 256, N, K0, 256, aux, la ? 64 : 1 << 30);
                if (la) {
                    if (hipError_t e = hipEventRecord(la->ev_rest[b & 1], aux); e != hipSuccess) return e;
                    aux_used = true;
                }
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // s resumes after the last rest update
        if (aux_used) {
            hipError_t e;
            if ((e = hipEventRecord(la->ev_panel, aux)) != hipSuccess || (e = hipStreamWaitEvent(s, la->ev_panel, 0)) != hipSuccess)
                return e;
        }
        if (sym) {
            hipLaunchKernelGGL(fill_upper_kernel, dim3((N + 127) / 128, (N + 63) / 64), dim3(256), 0, s, N, LU);
        }
        return hipGetLastError();
    }
    const int BK = N <= 4096 ? N : 128;
    for (int K0 = 0; K0 < N; K0 += BK) {
        const int KE = std::min(N, K0 + BK);
        for (int k0 = K0; k0 < KE;) {
            int w;
            if (N - k0 > 16384) {
                w = std::min(32, KE - k0);
                hipLaunchKernelGGL(panel_kernel, dim3(1), dim3(1024), 0, s, N, LU, k0, w, piv, info);
            } else {
                w = launch_panel(N, LU, k0, KE, piv, info, s);
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
            trailing_update(N, LU, KE, K0, KE - K0, s);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (diag_inv) hipLaunchKernelGGL(invert_diag_kernel, dim3((N + 63) / 64), dim3(64), 0, s, N, LU, static_cast<float *>(diag_inv));
    return hipGetLastError();
}

hipError_t lu_solve_f32(int N, const float *LU, const float *diag_inv, const float *pair_inv, float *b, float *tmp,
                        hipStream_t s)
{
    // b is already permuted (b := P b).
    // forward: b is updated below each step, solved blocks go to tmp;
    // backward: tmp is updated above each step, solved blocks go to b.
    // One launch per pair of 64-row blocks (pair_inv: the off-diagonal blocks of
    // the pairs' inverses), one more for an odd last block.
    const int nblk = (N + 63) / 64, npair = nblk / 2;
    for (int pr = 0; pr < npair; ++pr) {
        const int rest = std::max(0, N - 128 * pr - 128);
        hipLaunchKernelGGL(trsv_lower2_kernel, dim3(std::max(1, (rest + 63) / 64)), dim3(256), 0, s, N, LU, diag_inv,
                           pair_inv, b, tmp, pr);
    }
    if (nblk & 1)
        hipLaunchKernelGGL(trsv_lower_kernel, dim3(1), dim3(256), 0, s, N, LU, diag_inv, b, tmp, (nblk - 1) * 64);
    if (nblk & 1) {
        const int b0 = (nblk - 1) * 64;
        hipLaunchKernelGGL(trsv_upper_kernel, dim3(std::max(1, (b0 + 255) / 256)), dim3(256), 0, s, N, LU, diag_inv,
                           tmp, b, b0, N - b0);
    }
    for (int pr = npair - 1; pr >= 0; --pr) {
        const int b0 = 128 * pr;
        hipLaunchKernelGGL(trsv_upper2_kernel, dim3(std::max(1, (b0 + 63) / 64)), dim3(256), 0, s, N, LU, diag_inv,
                           pair_inv, tmp, b, pr);
    }
    return hipGetLastError();
}

namespace {
// The Gauss-Jordan inverse of A (FP64 or FP32, row-major, lda) into w.LU
// (row-major, ld Np): one loading launch, then one launch per sweep.
hipError_t gj_inverse(int N, const void *A, int64_t lda, int a_prec, const WS &w, const double *ctl, hipStream_t s)
{
    const int Np = padded64(N), nt = Np / 64;
    float *GR[2] = {w.GR, w.GR + int64_t(nt) * 4096}, *GC[2] = {w.GC, w.GC + int64_t(nt) * 4096};
    float *GP[2] = {w.GP, w.GP + 4096};
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, w.info);
    if (a_prec == 0)
        hipLaunchKernelGGL(gj_step_kernel<double>, dim3(nt * nt), dim3(256), 0, s, N, Np, -1, static_cast<const double *>(A),
                           lda, w.LU, GR[1], GC[1], GP[1], GR[0], GC[0], GP[0], w.info, ctl);
    else
        hipLaunchKernelGGL(gj_step_kernel<float>, dim3(nt * nt), dim3(256), 0, s, N, Np, -1, static_cast<const float *>(A),
                           lda, w.LU, GR[1], GC[1], GP[1], GR[0], GC[0], GP[0], w.info, ctl);
    for (int k = 0; k < nt; ++k) {
        const int in = k & 1, out = in ^ 1;
        hipLaunchKernelGGL(gj_step_kernel<float>, dim3(nt * nt), dim3(256), 0, s, N, Np, k,
                           static_cast<const float *>(w.LU), int64_t(Np), w.LU, GR[in], GC[in], GP[in], GR[out],
                           GC[out], GP[out], w.info, ctl);
    }
    return hipGetLastError();
}
}  // namespace

int mixed_solve(int N, const void *d_A, int64_t lda, int a_prec, const double *d_beta, double *d_x, double tol,
                int max_iter, void *ws_base, double *hbuf, hipStream_t s, void **lookahead, SolveResult &res,
                std::string &msg)
{
    WS w = carve(ws_base, N);
    double *ctl = w.red + 40;
    auto fail = [&](int st, const char *m, hipError_t e) {
        msg = std::string(m) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
        return st;
    };
    // ||A||_inf for the backward error (one read of A) and the exact symmetry test
    const int ngrid = std::min(N, 1024);
    if (a_prec == 0) {
        launch_rowabs<double>(N, d_A, lda, w.red + 64, s);
        hipLaunchKernelGGL(asym_kernel<double>, dim3(ngrid), dim3(256), 0, s, N, static_cast<const double *>(d_A), lda, w.r);
    } else {
        launch_rowabs<float>(N, d_A, lda, w.red + 64, s);
        hipLaunchKernelGGL(asym_kernel<float>, dim3(ngrid), dim3(256), 0, s, N, static_cast<const float *>(d_A), lda, w.r);
    }
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, w.red + 64, ctl + CTL_NORMA);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, ngrid, w.r, ctl + CTL_ASYM);
    if (!hbuf) return fail(-1, "the solve needs a pinned host buffer", hipSuccess);
    hipError_t e;
    double normA = 0.0;
    bool na_known = false;
    // A symmetric matrix (the Galerkin matrix is) is first factored without
    // interchanges: stable for a positive definite matrix, the setting of the
    // method.  The FP64-refined solution is accepted only if the refinement
    // converges; a zero pivot or a refinement that stalls short of the target
    // means a refactorisation with partial pivoting, as for any other matrix.
    // Up to kGJMaxN the symmetry test is not waited for: the explicit inverse
    // starts at once and its kernels return at once for an asymmetric matrix,
    // whose first synchronisation then sends it to partial pivoting.
    bool pivot;
    if (N <= kGJMaxN) {
        pivot = false;
    } else {
        double na[2];
        if ((e = hipMemcpyAsync(na, ctl, sizeof na, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail(-5, "matrix norm", e);
        normA = na[1];
        na_known = true;
        pivot = !(na[0] == 0.0 && lu_without_pivoting_supported(N));
    }
    for (;;) {
        // Without interchanges and up to kGJMaxN the explicit inverse (one
        // matrix-vector product per refinement step); otherwise the LU factor.
        const bool gj = !pivot && N <= kGJMaxN;
        if (gj) {
            // Refinement in batches of up to four steps with the decisions on the
            // device (update_norms_kernel) and one synchronisation per batch,
            // whose last kernel writes the control block, the backward-error
            // norms of the final iterate and the zero-pivot flag to hbuf.
            const int Np = padded64(N);
            if ((e = gj_inverse(N, d_A, lda, a_prec, w, ctl, s)) != hipSuccess) return fail(-5, "Gauss-Jordan launch", e);
            hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(64), 0, s, ctl);
            hipLaunchKernelGGL(inv_apply_kernel, dim3((N + 3) / 4), dim3(256), 0, s, N, Np, w.LU, d_beta, w.v, ctl);
            hipLaunchKernelGGL(update_norms_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.v, d_beta, d_beta, 0, w.red,
                               static_cast<double *>(nullptr), w.info, tol);
            int launched = 0;
            volatile double *hb = hbuf;
            for (;;) {
                const int nb = std::min(4, max_iter - launched);
                for (int b = 0; b < nb; ++b) {
                    if (a_prec == 0) launch_residual<double>(N, d_A, lda, d_x, d_beta, w.r, s, ctl);
                    else launch_residual<float>(N, d_A, lda, d_x, d_beta, w.r, s, ctl);
                    hipLaunchKernelGGL(inv_apply_kernel, dim3((N + 3) / 4), dim3(256), 0, s, N, Np, w.LU, w.r, w.v, ctl);
                    hipLaunchKernelGGL(update_norms_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.v, w.r, d_beta, 1,
                                       w.red, ctl, w.info, tol);
                }
                launched += nb;
                if (a_prec == 0) launch_residual<double>(N, d_A, lda, d_x, d_beta, w.r, s);
                else launch_residual<float>(N, d_A, lda, d_x, d_beta, w.r, s);
                hipLaunchKernelGGL(final_norms_kernel, dim3(1), dim3(1024), 0, s, N, w.r, d_x, d_beta, ctl, w.info, hbuf);
                if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
                    return fail(-5, "refinement", e);
                if (hb[CTL_ASYM] != 0.0 || hb[CTL_STOP] != 0.0 || launched >= max_iter) break;
            }
            normA = hb[CTL_NORMA];
            na_known = true;
            if (hb[CTL_ASYM] != 0.0) {   // not symmetric: partial pivoting from the start
                pivot = true;
                continue;
            }
            const double stop = hb[CTL_STOP];
            res.pivoted = false;
            res.iters = int(hb[CTL_ITERS]);
            res.rel_update = hb[CTL_REL];
            res.backward_err = hb[CTL_BWD];
            // a zero pivot, a stalled or non-finite refinement, or no convergence
            // within max_iter steps: refactor with partial pivoting
            if (hb[CTL_SIZE + 3] != 0.0 || (stop != 1.0 && max_iter > 0)) {
                pivot = true;
                continue;
            }
            res.backward_err = hb[CTL_SIZE] / (normA * hb[CTL_SIZE + 1] + hb[CTL_SIZE + 2]);
            if (stop != 1.0) return fail(-4, "iterative refinement did not reach the tolerance", hipSuccess);
            return 0;
        }
        if (!na_known) {    // (every way here has read the norm; kept for safety)
            double na[2];
            if ((e = hipMemcpyAsync(na, ctl, sizeof na, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail(-5, "matrix norm", e);
            normA = na[1];
            na_known = true;
        }
        {
            // without interchanges A is exactly symmetric: a plain copy of its rows
            dim3 tg((N + 31) / 32, (N + 31) / 32), rg((N + 1023) / 1024, N);
            const bool vec = N % 4 == 0 && (a_prec == 0 ? rows_aligned16<double>(d_A, lda) : rows_aligned16<float>(d_A, lda));
            if (a_prec == 0) {
                const double *A64 = static_cast<const double *>(d_A);
                if (pivot) hipLaunchKernelGGL(to_colmajor_kernel<double>, tg, dim3(256), 0, s, N, A64, lda, w.LU);
                else if (vec) hipLaunchKernelGGL((copy_rows_kernel<double, true>), rg, dim3(256), 0, s, N, A64, lda, w.LU);
                else hipLaunchKernelGGL((copy_rows_kernel<double, false>), rg, dim3(256), 0, s, N, A64, lda, w.LU);
            } else {
                const float *A32 = static_cast<const float *>(d_A);
                if (pivot) hipLaunchKernelGGL(to_colmajor_kernel<float>, tg, dim3(256), 0, s, N, A32, lda, w.LU);
                else if (vec) hipLaunchKernelGGL((copy_rows_kernel<float, true>), rg, dim3(256), 0, s, N, A32, lda, w.LU);
                else hipLaunchKernelGGL((copy_rows_kernel<float, false>), rg, dim3(256), 0, s, N, A32, lda, w.LU);
            }
            if ((e = lu_factor_f32(N, w.LU, w.piv, w.info, w.DI, pivot, s, lookahead)) != hipSuccess)
                return fail(-5, "LU factorisation launch", e);
            // the triangular solves' inverted blocks: 1024-row super-blocks beyond
            // kGJMaxN, pairs of 64-row blocks below
            if (w.INV)
                blkinv_build(N, w.LU, w.DI, w.INV, s);
            else if ((N + 63) / 64 >= 2)     // at least one pair of diagonal blocks
                hipLaunchKernelGGL(pair_inverse_kernel, dim3(2 * ((N + 63) / 64 / 2)), dim3(256), 0, s, N, w.LU, w.DI, w.DI2);
        }
        // d = (LU)^-1 P rhs
        auto apply = [&](const double *rhs) {
            hipLaunchKernelGGL(permute_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, w.perm, rhs, w.v);
            if (w.INV) (void)lu_solve_blk(N, w.LU, w.INV, w.v, w.v2, s);
            else (void)lu_solve_f32(N, w.LU, w.DI, w.DI2, w.v, w.v2, s);
        };
        // the permutation from the interchange sequence (host, O(N)); none without
        // pivoting, and then no wait here either: the zero-pivot flag is read with
        // the first synchronisation the refinement makes anyway
        std::vector<int> piv(N), perm(N);
        int info = 0;
        bool info_read = false;
        if (pivot) {
            if ((e = hipMemcpyAsync(piv.data(), w.piv, N * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail(-5, "LU factorisation", e);
            if (info != 0) return fail(-3, "zero pivot in the FP32 LU factorisation", hipSuccess);
            info_read = true;
        }
        for (int i = 0; i < N; ++i) perm[i] = i;
        if (pivot)
            for (int j = 0; j < N; ++j) std::swap(perm[j], perm[piv[j]]);
        if ((e = hipMemcpyAsync(w.perm, perm.data(), N * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
            return fail(-5, "permutation upload", e);

        auto residual = [&]() {
            if (a_prec == 0) launch_residual<double>(N, d_A, lda, d_x, d_beta, w.r, s);
            else launch_residual<float>(N, d_A, lda, d_x, d_beta, w.r, s);
        };
        double red[4];
        // x0 = LU \ beta (or X beta)
        apply(d_beta);
        hipLaunchKernelGGL(update_norms_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.v, d_beta, d_beta, 0, w.red,
                           static_cast<double *>(nullptr), w.info, 0.0);
        res.iters = 0;
        res.rel_update = 1.0;
        res.backward_err = 1.0;
        res.pivoted = pivot;
        int status = -4;
        double prev = 1e300;
        // Refinement: stop when ||d|| <= tol ||x||, or when a correction does
        // not halve (||d_k|| > ||d_{k-1}|| / 2: the FP64 residual has reached the
        // cond(A) eps floor) with a backward error at the FP64 level.  Without
        // pivoting, above that level a correction that does not shrink at all,
        // or two in a row that do not halve, end the attempt (one slow step
        // alone is the ordinary scatter of a slowly contracting refinement).
        bool stalled = false, zero_pivot = false, slow = false;
        for (int it = 0; it < max_iter; ++it) {
            residual();
            apply(w.r);
            hipLaunchKernelGGL(update_norms_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.v, w.r, d_beta, 1, w.red,
                               static_cast<double *>(nullptr), w.info, 0.0);
            if ((e = hipMemcpyAsync(red, w.red, sizeof red, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (!info_read && (e = hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail(-5, "refinement step", e);
            if (!info_read) {
                info_read = true;
                if (info != 0) {      // zero pivot without interchanges: this attempt is void
                    zero_pivot = true;
                    break;
                }
            }
            res.iters = it + 1;
            // NaN in either norm stays NaN (and ends the loop below as no convergence)
            res.rel_update = red[0] == 0.0 ? 0.0 : red[0] / red[1];
            res.backward_err = red[2] / (normA * red[1] + red[3]);   // of the iterate before this step
            if (res.rel_update <= tol) {
                status = 0;
                break;
            }
            if (res.rel_update > 0.5 * prev) {
                if (res.backward_err <= 64 * 1.1102230246251565e-16) {
                    status = 0;
                    break;
                }
                if (!pivot && (res.rel_update >= prev || slow)) {
                    stalled = true;
                    break;
                }
                slow = true;
            } else {
                slow = false;
            }
            if (!(res.rel_update < 1e300)) {   // NaN or overflow: no convergence from here
                if (!pivot) stalled = true;
                break;
            }
            prev = res.rel_update;
        }
        if (!info_read) {             // no refinement step ran: read the flag now
            if ((e = hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail(-5, "LU factorisation", e);
            zero_pivot = info != 0;
        }
        if (zero_pivot || (status != 0 && !pivot && (stalled || max_iter > 0))) {
            pivot = true;
            continue;
        }
        // backward error of the returned x: ||beta - A x||_inf / (||A||_inf ||x||_inf + ||beta||_inf)
        residual();
        hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, w.r, w.red + 5);
        hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, d_x, w.red + 6);
        hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, s, N, d_beta, w.red + 7);
        double nr[3];
        if ((e = hipMemcpyAsync(nr, w.red + 5, sizeof nr, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail(-5, "backward error", e);
        res.backward_err = nr[0] / (normA * nr[1] + nr[2]);
        if (status != 0) return fail(-4, "iterative refinement did not reach the tolerance", hipSuccess);
        return 0;
    }
}

}  // namespace sgbem
