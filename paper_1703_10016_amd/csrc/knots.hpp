// Fast-form assembly on non-uniform periodic knots: launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace sgbem {

// Device tables of rules on non-uniform knots (FP64):
//  W[N][Q], Bv[N][Q]: regular weights and B_i values on the support nodes 2R i + 1 + q (mod 2M);
//  Ws[2M][2M]: singular weights, row m the source eta_m;  eta[2M]: node parameters.
struct KnotArgs {
    int N, npts, P, Q;
    const double *X, *Y, *J;      // geometry at the nodes
    const double *eta;
    const double *W, *Bv, *Ws;
    double scale;                 // -1/(2 pi)
    double *out;
    int64_t lda;
};

// Upper-triangle tiles, mirrored (exactly symmetric output).  Returns
// hipErrorInvalidValue for a (p, P) without a compiled kernel.
hipError_t launch_assemble_knots(int p, const KnotArgs &a, hipStream_t s, const KernelEvents *ev);
bool assemble_knots_supported(int p, int P);

// beta_i = sum_q W[i][q] J[n] g[n], n = P i + 1 + q (mod npts).
hipError_t launch_rhs_knots(int N, int npts, int P, int Q, const double *W, const double *J, const double *g,
                            double *beta, hipStream_t s);

}  // namespace sgbem
