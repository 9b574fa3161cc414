// Spline helpers of the host rule construction (Section 4.2): spans and
// Cox-de Boor values, the local monomial pieces of the B-splines on one
// element, and a banded SPD solver for the Gram matrix of Alg. 2's collocation.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "planner.hpp"

namespace sgbem {
namespace spline {

[[noreturn]] inline void fail(int status, const std::string &msg) { throw PlanError{status, msg}; }

// Periodic knots of one period, t[0] = 0 < ... < t[n] = 1, extended by t_{k+n} = t_k + 1.
struct PKnots {
    std::vector<double> t;
    int64_t n = 0;
    double operator()(int64_t k) const
    {
        int64_t q = k >= 0 ? k / n : -((-k + n - 1) / n);
        return t[size_t(k - q * n)] + double(q);
    }
    // span l in [0, n) with t_l <= x < t_{l+1} for x in [0, 1)
    int64_t span(double x) const
    {
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (t[size_t(mid)] <= x) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
};

// Clamped (open) knots on the breakpoints x_0 < ... < x_n: t_k = x_k for
// 0 <= k <= n, t_k = x_0 for k < 0 and x_n for k > n, so that every function
// k = -p .. n-1 has its knots t_k .. t_{k+p+1} and B_{-p}(x_0) = B_{n-1}(x_n) = 1.
struct OKnots {
    std::vector<double> x;
    int64_t n = 0;
    double operator()(int64_t k) const { return x[size_t(k < 0 ? 0 : (k > n ? n : k))]; }
};

// The p + 1 B-splines of degree p nonzero on span l at x (t_l <= x <= t_{l+1}):
// out[j] = B_{l-p+j}(x), by the triangular Cox-de Boor scheme.  K(k) is the
// extended knot t_k (periodic or clamped); no denominator vanishes on a span
// of positive length.
template <typename Knots>
inline void basis_funs(const Knots &K, int p, int64_t l, double x, double *out)
{
    double left[8], right[8];
    out[0] = 1.0;
    for (int r = 1; r <= p; ++r) {
        left[r] = x - K(l + 1 - r);
        right[r] = K(l + r) - x;
        double saved = 0.0;
        for (int j = 0; j < r; ++j) {
            const double tmp = out[j] / (right[j + 1] + left[r - j]);
            out[j] = saved + right[j + 1] * tmp;
            saved = left[r - j] * tmp;
        }
        out[r] = saved;
    }
}

// Monomial coefficients, in u = (x - t_e) / h_e on [0, 1], of the p + 1 B-splines
// nonzero on span e: coef[j * (p + 1) + a] for B_{e-p+j}; the Cox-de Boor
// recurrence carried out on polynomials of u.
template <typename Knots>
inline void local_pieces(const Knots &K, int p, int64_t e, double *coef)
{
    const int np = p + 1;
    const double a = K(e), h = K(e + 1) - K(e);
    // cur[m][deg] for B_{e-r+m, r}, m = 0..r
    std::vector<double> cur(np * np, 0.0), nxt(np * np, 0.0);
    cur[0] = 1.0;
    for (int r = 1; r <= p; ++r) {
        std::fill(nxt.begin(), nxt.end(), 0.0);
        for (int m = 0; m <= r; ++m) {
            const int64_t i = e - r + m;
            // (x - t_i)/(t_{i+r} - t_i) B_{i,r-1}: B_{i,r-1} is cur[m - 1] (function e - (r-1) + (m-1))
            if (m >= 1) {
                const double d = K(i + r) - K(i);
                const double c0 = (a - K(i)) / d, c1 = h / d;
                for (int q = 0; q < r; ++q) {
                    nxt[m * np + q] += c0 * cur[(m - 1) * np + q];
                    nxt[m * np + q + 1] += c1 * cur[(m - 1) * np + q];
                }
            }
            // (t_{i+r+1} - x)/(t_{i+r+1} - t_{i+1}) B_{i+1,r-1}: cur[m]
            if (m <= r - 1) {
                const double d = K(i + r + 1) - K(i + 1);
                const double c0 = (K(i + r + 1) - a) / d, c1 = -h / d;
                for (int q = 0; q < r; ++q) {
                    nxt[m * np + q] += c0 * cur[m * np + q];
                    nxt[m * np + q + 1] += c1 * cur[m * np + q];
                }
            }
        }
        cur.swap(nxt);
    }
    std::copy(cur.begin(), cur.end(), coef);
}

inline double horner(const double *c, int deg, double u)
{
    double v = 0.0;
    for (int a = deg; a >= 0; --a) v = v * u + c[a];
    return v;
}

// Symmetric positive definite cyclic banded matrix (half bandwidth hb, entries
// G(k, l) for cyclic |k - l| <= hb): bordered elimination, the first M - hb
// unknowns by banded Cholesky, the last hb through the dense Schur complement.
// A plain banded matrix is the case whose G returns 0 for the wrap couplings.
// Factored once; solve() is read-only and may run on several threads.
class CyclicBandSPD {
public:
    template <typename F>
    CyclicBandSPD(int64_t M, int hb, F G) : M_(M), hb_(hb), m1_(M - hb)
    {
        const int64_t m1 = m1_;
        Lb_.assign(size_t(m1) * (hb + 1), 0.0);
        for (int64_t k = 0; k < m1; ++k) {
            for (int64_t j = std::max<int64_t>(0, k - hb); j <= k; ++j) {
                double s = G(k, j);
                for (int64_t i = std::max<int64_t>(0, k - hb); i < j; ++i) s -= L(k, i) * L(j, i);
                if (j == k) {
                    if (!(s > 0.0)) fail(-3, "Gram matrix of the collocation is not positive definite");
                    Lb_[size_t(k) * (hb + 1) + hb] = std::sqrt(s);
                } else {
                    Lb_[size_t(k) * (hb + 1) + (j - k + hb)] = s / L(j, j);
                }
            }
        }
        // G12 rows (couplings of the first m1 unknowns to the last hb), X = G11^-1 G12
        G12_.assign(size_t(m1) * hb, 0.0);
        for (int64_t k = 0; k < m1; ++k)
            for (int c = 0; c < hb; ++c) {
                int64_t d = (m1 + c) - k;
                d = std::min(d, M - d);
                if (d <= hb) G12_[size_t(k) * hb + c] = G(k, m1 + c);
            }
        X_ = G12_;
        band_solve(X_.data(), hb);
        S_.assign(size_t(hb) * hb, 0.0);
        for (int a = 0; a < hb; ++a)
            for (int b = 0; b < hb; ++b) {
                double s = G(m1 + a, m1 + b);
                for (int64_t k = 0; k < m1; ++k) s -= G12_[size_t(k) * hb + a] * X_[size_t(k) * hb + b];
                S_[size_t(a) * hb + b] = s;
            }
        for (int a = 0; a < hb; ++a)
            for (int b = 0; b <= a; ++b) {
                double s = S_[size_t(a) * hb + b];
                for (int i = 0; i < b; ++i) s -= S_[size_t(a) * hb + i] * S_[size_t(b) * hb + i];
                if (a == b) {
                    if (!(s > 0.0)) fail(-3, "Schur complement of the Gram matrix is not positive definite");
                    S_[size_t(a) * hb + a] = std::sqrt(s);
                } else {
                    S_[size_t(a) * hb + b] = s / S_[size_t(b) * hb + b];
                }
            }
    }
    // x[k * nc + c] (M rows), in place
    void solve(double *x, int nc) const
    {
        const int64_t m1 = m1_;
        const int hb = hb_;
        band_solve(x, nc);
        std::vector<double> y2(size_t(hb) * nc);
        for (int a = 0; a < hb; ++a)
            for (int c = 0; c < nc; ++c) {
                double s = x[size_t(m1 + a) * nc + c];
                for (int64_t k = 0; k < m1; ++k) {
                    const double g = G12_[size_t(k) * hb + a];
                    if (g != 0.0) s -= g * x[size_t(k) * nc + c];
                }
                y2[size_t(a) * nc + c] = s;
            }
        for (int c = 0; c < nc; ++c) {
            for (int a = 0; a < hb; ++a) {
                double s = y2[size_t(a) * nc + c];
                for (int i = 0; i < a; ++i) s -= S_[size_t(a) * hb + i] * y2[size_t(i) * nc + c];
                y2[size_t(a) * nc + c] = s / S_[size_t(a) * hb + a];
            }
            for (int a = hb - 1; a >= 0; --a) {
                double s = y2[size_t(a) * nc + c];
                for (int i = a + 1; i < hb; ++i) s -= S_[size_t(i) * hb + a] * y2[size_t(i) * nc + c];
                y2[size_t(a) * nc + c] = s / S_[size_t(a) * hb + a];
            }
        }
        for (int64_t k = 0; k < m1; ++k)
            for (int c = 0; c < nc; ++c) {
                double s = x[size_t(k) * nc + c];
                for (int b = 0; b < hb; ++b) s -= X_[size_t(k) * hb + b] * y2[size_t(b) * nc + c];
                x[size_t(k) * nc + c] = s;
            }
        for (int a = 0; a < hb; ++a)
            for (int c = 0; c < nc; ++c) x[size_t(m1 + a) * nc + c] = y2[size_t(a) * nc + c];
    }

private:
    double L(int64_t k, int64_t j) const { return Lb_[size_t(k) * (hb_ + 1) + (j - k + hb_)]; }
    // G11^-1 x in place (forward and backward banded substitution), x[k * nc + c], k < m1;
    // values below 1e-290 flushed (the columns of G11^-1 G12 decay geometrically)
    void band_solve(double *x, int nc) const
    {
        const int64_t m1 = m1_;
        const int hb = hb_;
        auto flush = [](double v) { return std::fabs(v) < 1e-290 ? 0.0 : v; };
        for (int64_t k = 0; k < m1; ++k)
            for (int c = 0; c < nc; ++c) {
                double s = x[size_t(k) * nc + c];
                for (int64_t i = std::max<int64_t>(0, k - hb); i < k; ++i) s -= L(k, i) * x[size_t(i) * nc + c];
                x[size_t(k) * nc + c] = flush(s / L(k, k));
            }
        for (int64_t k = m1 - 1; k >= 0; --k)
            for (int c = 0; c < nc; ++c) {
                double s = x[size_t(k) * nc + c];
                for (int64_t i = k + 1; i <= std::min<int64_t>(m1 - 1, k + hb); ++i) s -= L(i, k) * x[size_t(i) * nc + c];
                x[size_t(k) * nc + c] = flush(s / L(k, k));
            }
    }
    int64_t M_;
    int hb_;
    int64_t m1_;
    std::vector<double> Lb_, G12_, X_, S_;
};

}  // namespace spline
}  // namespace sgbem
