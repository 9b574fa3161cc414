// Collocation BEM with the weighted quadrature rules: launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sgbem {

bool colloc_supported(int p, int P);
// the N x N collocation matrix (FP64, row-major a.out / a.lda) from the fast form's
// node geometry and rule tables in `a` (a.scale = -1/(2 pi))
hipError_t launch_colloc(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev);
// b_i = g[(P i + c0) mod npts]: u_D at the collocation nodes
hipError_t launch_colloc_gather(int N, int npts, int P, int c0, const double *g, double *b, hipStream_t s);

}  // namespace sgbem
