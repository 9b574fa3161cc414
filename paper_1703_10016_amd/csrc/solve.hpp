// Mixed-precision dense solve A x = beta: FP32 LU with partial pivoting,
// FP64 iterative refinement.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace sgbem {

struct SolveResult {
    int iters = 0;
    double rel_update = 0.0;
    double backward_err = 0.0;
    bool pivoted = true;     // false: factored without row interchanges
};

size_t solve_workspace_bytes(int N);

// Returns an sgbem_status value; synchronises `stream` before returning.
// hbuf: pinned host memory of kSolveHostDoubles doubles (hipHostMalloc), which
// the last kernel of each refinement batch writes.
constexpr int kSolveHostDoubles = 16;
// lookahead: the caller's slot for the factorisation's second stream and events
// (made on first use beyond N = 4096, released by lookahead_free); may be null.
int mixed_solve(int N, const void *d_A, int64_t lda, int a_prec, const double *d_beta, double *d_x, double tol,
                int max_iter, void *ws, double *hbuf, hipStream_t stream, void **lookahead, SolveResult &res,
                std::string &msg);
void lookahead_free(void *lookahead);

// Pieces, also used on their own by the tests and the serving loop.
// FP32 LU in place (column-major, ld = N), with partial pivoting or (pivot
// false, N within lu_without_pivoting_supported) with the diagonal as pivot;
// when diag_inv is given it receives the inverses of the 64 x 64 diagonal
// blocks of L and U.
bool lu_without_pivoting_supported(int N);
hipError_t lu_factor_f32(int N, float *LU, int *piv, int *info, void *diag_inv, bool pivot, hipStream_t s,
                         void **lookahead = nullptr);
// b := U^{-1} L^{-1} b for an already permuted b (tmp: N floats of scratch).
// pair_inv: the off-diagonal 64 x 64 blocks of the inverses of pairs of diagonal
// blocks (formed after the factorisation whenever N > 64).
hipError_t lu_solve_f32(int N, const float *LU, const float *diag_inv, const float *pair_inv, float *b, float *tmp,
                        hipStream_t s);

}  // namespace sgbem
