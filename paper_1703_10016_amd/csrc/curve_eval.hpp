// Curve geometry at one parameter value, shared by the single and batched
// geometry kernels and the host-side node points: f, f' and J = |f'| (eq. J).
//  polar:   f = r(theta) (cos theta, sin theta), theta = 2 pi t, closed-form derivative;
//  B-spline (periodic knots, Section 3): de Boor's algorithm on the span
//           containing t, and on the derivative curve with control points
//           d (Q_j - Q_{j-1}) / (tau_{j+d} - tau_j) at degree d-1 (uniform
//           knots tau_k = k / n_ctrl: n_ctrl (Q_j - Q_{j-1}));
//  open B-spline (clamped knot vector T of n_ctrl + d + 1 values, Section 3):
//           the same on the span T_l <= t < T_{l+1}, d <= l < n_ctrl (the
//           last span also holds t = T_{n_ctrl}).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace sgbem {

// sin and cos of pi x
__host__ __device__ inline void sincos_pi(double x, double *s, double *c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    sincospi(x, s, c);
#else
    // reduce to [-1/2, 1/2] so that the multiplication by pi stays accurate
    const double k = std::nearbyint(x);
    const double r = x - k;
    const double sg = (static_cast<long long>(k) & 1) ? -1.0 : 1.0;
    *s = sg * std::sin(3.14159265358979323846 * r);
    *c = sg * std::cos(3.14159265358979323846 * r);
#endif
}

__host__ __device__ inline void sin_cos(double x, double *s, double *c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    sincos(x, s, c);
#else
    *s = std::sin(x);
    *c = std::cos(x);
#endif
}

// Periodic B-spline on uniform knots at a compile-time degree D: the same
// arithmetic as the general branch below, with the de Boor arrays in registers
// (with a run-time degree they live in scratch).
template <int D>
__host__ __device__ __forceinline__ void eval_uniform_periodic(const CurveDev &c, const double *cq, double t, double &x,
                                                              double &y, double &dx, double &dy)
{
    const int nc = c.n_ctrl;
    const double u = t * nc;
    int l = int(std::floor(u));
    if (l >= nc) l = nc - 1;
    if (l < 0) l = 0;
    double px[D + 1], py[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) {
        int j = l - D + i;
        j = ((j % nc) + nc) % nc;
        px[i] = cq[2 * j];
        py[i] = cq[2 * j + 1];
    }
    double qx[D], qy[D];
#pragma unroll
    for (int i = 1; i <= D; ++i) {
        qx[i - 1] = nc * (px[i] - px[i - 1]);
        qy[i - 1] = nc * (py[i] - py[i - 1]);
    }
#pragma unroll
    for (int r = 1; r <= D; ++r) {
#pragma unroll
        for (int i = D; i >= r; --i) {
            const int j = l - D + i;
            const double al = (u - j) / double(D + 1 - r);
            px[i] = (1.0 - al) * px[i - 1] + al * px[i];
            py[i] = (1.0 - al) * py[i - 1] + al * py[i];
        }
    }
    x = px[D];
    y = py[D];
    constexpr int dd = D - 1;
#pragma unroll
    for (int r = 1; r <= dd; ++r) {
#pragma unroll
        for (int i = dd; i >= r; --i) {
            const int j = l - dd + i;
            const double al = (u - j) / double(dd + 1 - r);
            qx[i] = (1.0 - al) * qx[i - 1] + al * qx[i];
            qy[i] = (1.0 - al) * qy[i - 1] + al * qy[i];
        }
    }
    dx = qx[dd];
    dy = qy[dd];
}

// The clamped and non-uniform periodic branches at a compile-time degree D: the
// same arithmetic as the run-time-degree branch below, arrays in registers.
template <int D>
__host__ __device__ __forceinline__ void eval_knots_d(const CurveDev &c, const double *cq, double t, double &x, double &y,
                                                     double &dx, double &dy)
{
    const int nc = c.n_ctrl;
    const double *tk = c.inline_data ? c.inl + 128 : c.knots;
    double tau[2 * D + 1], px[D + 1], py[D + 1];   // knots l - D .. l + D and control points l - D .. l
    int lo, hi;
    if (c.kind == 2) {
        lo = D;
        hi = nc - 1;                  // the span l with T_l <= t < T_{l+1}
    } else {
        lo = 0;
        hi = nc - 1;                  // the span l with tau_l <= t < tau_{l+1}
    }
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tk[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const int l = lo;
    if (c.kind == 2) {
#pragma unroll
        for (int i = 0; i <= 2 * D; ++i) tau[i] = tk[l - D + i];
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            px[i] = cq[2 * (l - D + i)];
            py[i] = cq[2 * (l - D + i) + 1];
        }
    } else {
#pragma unroll
        for (int i = 0; i <= 2 * D; ++i) {
            const int k = l - D + i;
            const int kk = k < 0 ? k + nc : (k >= nc ? k - nc : k);
            tau[i] = tk[kk] + (k < 0 ? -1.0 : (k >= nc ? 1.0 : 0.0));
        }
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            int j = l - D + i;
            j = ((j % nc) + nc) % nc;
            px[i] = cq[2 * j];
            py[i] = cq[2 * j + 1];
        }
    }
    double qx[D], qy[D];
#pragma unroll
    for (int i = 1; i <= D; ++i) {
        const double s = D / (tau[i + D] - tau[i]);
        qx[i - 1] = s * (px[i] - px[i - 1]);
        qy[i - 1] = s * (py[i] - py[i - 1]);
    }
#pragma unroll
    for (int r = 1; r <= D; ++r) {
#pragma unroll
        for (int i = D; i >= r; --i) {
            const double al = (t - tau[i]) / (tau[i + D + 1 - r] - tau[i]);
            px[i] = (1.0 - al) * px[i - 1] + al * px[i];
            py[i] = (1.0 - al) * py[i - 1] + al * py[i];
        }
    }
    x = px[D];
    y = py[D];
    constexpr int dd = D - 1;
#pragma unroll
    for (int r = 1; r <= dd; ++r) {
#pragma unroll
        for (int i = dd; i >= r; --i) {
            const double al = (t - tau[i + 1]) / (tau[i + 1 + dd + 1 - r] - tau[i + 1]);
            qx[i] = (1.0 - al) * qx[i - 1] + al * qx[i];
            qy[i] = (1.0 - al) * qy[i - 1] + al * qy[i];
        }
    }
    dx = qx[dd];
    dy = qy[dd];
}

// f(t) and f'(t)
__host__ __device__ __forceinline__ void eval_curve_d(const CurveDev &c, double t, double &x, double &y, double &dx,
                                                      double &dy)
{
    const double *ca = c.inline_data ? c.inl : c.a;
    const double *cphi = c.inline_data ? c.inl + 64 : c.phi;
    const double *cq = c.inline_data ? c.inl : c.ctrl;
    if (c.kind == 1) {
        double sn, cs;
        sincos_pi(2.0 * t, &sn, &cs);
        const double th = 6.283185307179586476925286766559 * t;
        double r = 1.0, dr = 0.0;
        for (int k = 1; k <= c.n_modes; ++k) {
            double sk, ck;
            sin_cos(k * th + cphi[k - 1], &sk, &ck);
            r += ca[k - 1] * ck;
            dr -= k * ca[k - 1] * sk;
        }
        r *= c.r0;
        dr *= c.r0;
        x = r * cs;
        y = r * sn;
        dx = 6.283185307179586476925286766559 * (dr * cs - r * sn);
        dy = 6.283185307179586476925286766559 * (dr * sn + r * cs);
    } else if ((c.kind == 2 || c.nonuniform) && (c.degree == 2 || c.degree == 3)) {   // the workloads' arcs and graded curves
        if (c.degree == 2) eval_knots_d<2>(c, cq, t, x, y, dx, dy);
        else eval_knots_d<3>(c, cq, t, x, y, dx, dy);
    } else if (c.kind == 2 || c.nonuniform) {
        const int d = c.degree, nc = c.n_ctrl;
        const double *tk = c.inline_data ? c.inl + 128 : c.knots;
        // tau[i] = knot l - d + i, i = 0 .. 2d, and the control points l - d .. l of the span l
        double tau[16], px[8], py[8];
        if (c.kind == 2) {
            int lo = d, hi = nc - 1;      // the span l with T_l <= t < T_{l+1}
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tk[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            const int l = lo;
            for (int i = 0; i <= 2 * d; ++i) tau[i] = tk[l - d + i];
            for (int i = 0; i <= d; ++i) {
                px[i] = cq[2 * (l - d + i)];
                py[i] = cq[2 * (l - d + i) + 1];
            }
        } else {
            // breakpoints tau_0 = 0 < ... < tau_n = 1 of one period, tau_{k+n} = tau_k + 1;
            // B_j supported on [tau_j, tau_{j+d+1})
            int lo = 0, hi = nc - 1;      // the span l with tau_l <= t < tau_{l+1}
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (tk[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            const int l = lo;
            for (int i = 0; i <= 2 * d; ++i) {
                const int k = l - d + i;
                const int kk = k < 0 ? k + nc : (k >= nc ? k - nc : k);
                tau[i] = tk[kk] + (k < 0 ? -1.0 : (k >= nc ? 1.0 : 0.0));
            }
            for (int i = 0; i <= d; ++i) {
                int j = l - d + i;
                j = ((j % nc) + nc) % nc;
                px[i] = cq[2 * j];
                py[i] = cq[2 * j + 1];
            }
        }
        // derivative control points d (Q_j - Q_{j-1}) / (tau_{j+d} - tau_j), j = l-d+1 .. l
        double qx[8], qy[8];
        for (int i = 1; i <= d; ++i) {
            const double s = d / (tau[i + d] - tau[i]);
            qx[i - 1] = s * (px[i] - px[i - 1]);
            qy[i - 1] = s * (py[i] - py[i - 1]);
        }
        // de Boor, local index i <-> knot tau_{l-d+i} = tau[i]
        for (int r = 1; r <= d; ++r) {
            for (int i = d; i >= r; --i) {
                const double al = (t - tau[i]) / (tau[i + d + 1 - r] - tau[i]);
                px[i] = (1.0 - al) * px[i - 1] + al * px[i];
                py[i] = (1.0 - al) * py[i - 1] + al * py[i];
            }
        }
        x = px[d];
        y = py[d];
        // degree d-1 on the same knots: local index i <-> knot tau_{l-d+1+i} = tau[i + 1]
        const int dd = d - 1;
        for (int r = 1; r <= dd; ++r) {
            for (int i = dd; i >= r; --i) {
                const double al = (t - tau[i + 1]) / (tau[i + 1 + dd + 1 - r] - tau[i + 1]);
                qx[i] = (1.0 - al) * qx[i - 1] + al * qx[i];
                qy[i] = (1.0 - al) * qy[i - 1] + al * qy[i];
            }
        }
        dx = qx[dd];
        dy = qy[dd];
    } else if (c.degree == 3) {   // the cubic curves of the workloads
        eval_uniform_periodic<3>(c, cq, t, x, y, dx, dy);
    } else {
        const int d = c.degree, nc = c.n_ctrl;
        const double u = t * nc;
        int l = int(std::floor(u));
        if (l >= nc) l = nc - 1;
        if (l < 0) l = 0;
        double px[8], py[8];
        for (int i = 0; i <= d; ++i) {
            int j = l - d + i;
            j = ((j % nc) + nc) % nc;
            px[i] = cq[2 * j];
            py[i] = cq[2 * j + 1];
        }
        // derivative control points (degree d-1): n_ctrl (Q_j - Q_{j-1}), j = l-d+1 .. l
        double qx[8], qy[8];
        for (int i = 1; i <= d; ++i) {
            qx[i - 1] = nc * (px[i] - px[i - 1]);
            qy[i - 1] = nc * (py[i] - py[i - 1]);
        }
        // de Boor: B_j supported on [j, j + d + 1) in units of n_ctrl t
        for (int r = 1; r <= d; ++r) {
            for (int i = d; i >= r; --i) {
                const int j = l - d + i;
                const double al = (u - j) / double(d + 1 - r);
                px[i] = (1.0 - al) * px[i - 1] + al * px[i];
                py[i] = (1.0 - al) * py[i - 1] + al * py[i];
            }
        }
        x = px[d];
        y = py[d];
        const int dd = d - 1;
        for (int r = 1; r <= dd; ++r) {
            for (int i = dd; i >= r; --i) {
                const int j = l - dd + i;
                const double al = (u - j) / double(dd + 1 - r);
                qx[i] = (1.0 - al) * qx[i - 1] + al * qx[i];
                qy[i] = (1.0 - al) * qy[i - 1] + al * qy[i];
            }
        }
        dx = qx[dd];
        dy = qy[dd];
    }
}

// f(t) and J(t) = |f'(t)|
__host__ __device__ __forceinline__ void eval_curve(const CurveDev &c, double t, double &x, double &y, double &J)
{
    double dx, dy;
    eval_curve_d(c, t, x, y, dx, dy);
    J = std::sqrt(dx * dx + dy * dy);
}


}  // namespace sgbem
