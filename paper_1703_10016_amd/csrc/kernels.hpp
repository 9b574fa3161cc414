// Launch interface of the HIP kernels (C++ linkage, used by the C ABI layer).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sgbem {

// Curve description in device memory.
struct CurveDev {
    int kind;        // 0 = periodic B-spline, 1 = polar, 2 = open B-spline (clamped knots)
    int degree;      // B-spline degree d
    int n_ctrl;      // B-spline control points
    int n_modes;     // polar Fourier modes
    double r0;       // polar base radius
    const double *ctrl;   // [n_ctrl][2]
    const double *knots;  // [n_ctrl + 1] breakpoints of one period (nonuniform), [n_ctrl + degree + 1] (open)
    const double *a;      // [n_modes]
    const double *phi;    // [n_modes]
    int nonuniform;       // B-spline: 0 = uniform knots k / n_ctrl, 1 = knots[]
    int inline_data;      // 1: ctrl / knots / a / phi live in inl[] below (no upload needed)
    double inl[200];      // B-spline: ctrl[64][2], knots (<= 72) from inl + 128; polar: a[64], phi[64]
};

// Point grid on [0, 1): n = e * P + q  ->  t = (e + off[q]) / N  (P <= 32),
// or t = n / npts when P == 0, or t = tpar[n] (device table) when tpar is set.
struct GridDesc {
    int N;
    int P;
    int npts;
    double off[32];
    const double *tpar;
};

hipError_t launch_geometry(const CurveDev &c, const GridDesc &g, double *X, double *Y, double *J, hipStream_t s);
hipError_t launch_points_xy(const double *X, const double *Y, int npts, double *xy, hipStream_t s);

// Sum-factorised tile assembly (upper-triangle tiles, mirrored output).
struct TileArgs {
    int N;                 // basis functions (matrix order)
    int npts;              // grid points = N * P
    const double *X, *Y, *J;
    const double *inv_s2;  // WQ: [npts] (pi/sin(pi d/npts))^2, entry 0 = 0
    const double *ws;      // WQ: [2][npts]
    const float *inv_s2f;  // WQ FP32 copies
    const float *wsf;
    double coefA[64];      // row weights on the support points (without J)
    double coefB[64];      // WQ: B_0 on the support points
    double scale;          // -1/(2 pi)
    void *out;
    int64_t lda;
};

// method 0 = WQ (P = 2 n_ref, Q = P (p+1) - 1, support starts at point 1),
// method 1 = EBE far part (P = G, Q = G (p+1), support starts at point 0).
// prec 0 = FP64, 1 = FP32.  Returns hipErrorInvalidValue when no kernel is
// compiled for (p, P).
// Optional timing of a launch: events recorded by the kernel's own dispatch
// (start and end of its execution), not by separate stream markers.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_assemble(int method, int prec, int p, int P, const TileArgs &a, hipStream_t s,
                           const KernelEvents *ev = nullptr);
bool assemble_supported(int method, int prec, int p, int P);

// EBE near pairs: L[(e*2 + type)][a][b], type 0 = coincident, 1 = (e, e+1).
struct NearArgs {
    int N, p;
    const double *X16, *Y16, *J16;   // geometry at the 16 Gauss points of every element
    const double *u16, *w16;         // Gauss nodes / weights on [0, 1]
    const double *mco, *madj;        // [16][16]
    const double *bv16;              // [p+1][16]: M_p(a + u_g)
    double *L;                       // [N][2][(p+1)^2]
};
hipError_t launch_near(const NearArgs &a, hipStream_t s);
// A[i][j] += scale * (near-pair corrections), band |i - j| <= p + 1 (cyclic).
hipError_t launch_band(int prec, int N, int p, const double *L, double scale, void *out, int64_t lda, hipStream_t s);

// beta_i = scale sum_q coef[q] J[n] g[n], n = (P i + s0 + q) mod npts.
hipError_t launch_rhs(int N, int npts, int P, int s0, int Q, const double *coef, double scale, const double *J,
                      const double *g, double *beta, hipStream_t s);

}  // namespace sgbem
