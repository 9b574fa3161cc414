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
};

size_t solve_workspace_bytes(int N);

// Returns an sgbem_status value; synchronises `stream` before returning.
int mixed_solve(int N, const void *d_A, int64_t lda, int a_prec, const double *d_beta, double *d_x, double tol,
                int max_iter, void *ws, hipStream_t stream, SolveResult &res, std::string &msg);

// Pieces, also used on their own by the tests and the serving loop.
hipError_t lu_factor_f32(int N, float *LU, int *piv, int *info, void *scratch, hipStream_t s);
hipError_t lu_solve_f32(int N, const float *LU, const int *piv, float *b, hipStream_t s);

}  // namespace sgbem
