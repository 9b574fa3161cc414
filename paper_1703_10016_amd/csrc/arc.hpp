// Fast-form assembly on an open arc: launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace sgbem {

// Device tables of the open-arc rules (FP64), QM = 2R(p+1) - 1 + 2p:
//  W[N][QM], Bv[N][QM]: regular weights and B_i values on row i's support nodes
//  n0[i] + q, zero beyond its count; Ws[npts][npts]: singular weights, row m the
//  source eta_m; eta[npts]: node parameters.
struct ArcArgs {
    int N, npts, P;
    const double *X, *Y, *J;      // geometry at the nodes
    const double *eta;
    const double *W, *Bv, *Ws;
    const int32_t *n0;
    double scale;                 // -1/(2 pi)
    double *out;
    int64_t lda;
};

// Rows per tile of the open-arc kernel, and the node window of a tile: rows
// I0 .. I0+T-1 use the nodes n0[I0] .. n0[I0+T-1] + QM - 1, at most arc_window(p, P).
constexpr int kArcTile = 24;
constexpr int arc_qm(int p, int P) { return P * (p + 1) - 1 + 2 * p; }
constexpr int arc_window(int p, int P) { return P * (kArcTile - 1) + (p - 1) + arc_qm(p, P); }

// Every tile of the N x N matrix (no mirroring).  Returns hipErrorInvalidValue
// for a (p, P) without a compiled kernel.
hipError_t launch_assemble_arc(int p, const ArcArgs &a, hipStream_t s, const KernelEvents *ev);
bool assemble_arc_supported(int p, int P);

// beta_i = sum_{q < cnt_i} W[i][q] J[n] g[n], n = n0[i] + q.
hipError_t launch_rhs_arc(int N, int QM, const int32_t *n0, const int32_t *cnt, const double *W, const double *J,
                          const double *g, double *beta, hipStream_t s);

}  // namespace sgbem
