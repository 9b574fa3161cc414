// Double-layer sweep of the direct formulation's right-hand side: launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sgbem {

struct GaussW {
    double w[8];          // composite Gauss weights w_q / N
};

// x, y, f1', f2' and coef = (w_q / N) u_D at the composite Gauss points of g (g.P <= 8).
hipError_t launch_dl_geometry(const CurveDev &c, const GridDesc &g, const GaussW &gw, const double *gval,
                              double *X, double *Y, double *DX, double *DY, double *coef, hipStream_t s);
// number of point chunks the sweep splits into (partials: nchunk x nn doubles)
int dl_chunks(int nn, int np);
hipError_t launch_dl_sweep(int nn, const double *X1, const double *Y1, int np, const double *X2, const double *Y2,
                           const double *DX2, const double *DY2, const double *coef, int nchunk, double *part,
                           hipStream_t s, const KernelEvents *ev);
hipError_t launch_dl_reduce(int nn, int nchunk, const double *part, const double *g, double *h, double *vout,
                            hipStream_t s);
// part[n] += the near Gauss points' terms evaluated without cancellation minus the
// sweep's values of them (nodes n / P1 per element, gu.w[q] the Gauss nodes on [0, 1]).
hipError_t launch_dl_near(const CurveDev &c, int N, int P1, int G, const GaussW &gu, int nn, const double *X1,
                          const double *Y1, const double *X2, const double *Y2, const double *DX2, const double *DY2,
                          const double *coef, double *part, hipStream_t s);

}  // namespace sgbem
