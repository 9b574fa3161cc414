// Host FP64 construction of the quadrature rules of Section 4 (Alg. 1, Alg. 2,
// modified moments) and of the near-pair tables of the element-by-element
// rule (Section 5, Remark).  Everything here depends only on (p, N, n_ref) or
// on the Gauss orders, never on the curve; the result is uploaded once and
// kept on the device.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

namespace sgbem {

namespace {
constexpr double kPi = 3.14159265358979323846264338327950288;

[[noreturn]] void fail(int status, const std::string &msg) { throw PlanError{status, msg}; }
}  // namespace

// ------------------------------------------------------------------ Gauss rules
void gauss_legendre01(int n, double *x, double *w)
{
    // Newton iteration on P_n (three-term recurrence) from the Chebyshev-like
    // initial guesses; nodes are symmetric, so only half are iterated.
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        {   // final derivative at the converged node
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
        }
        const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        // ascending order on [0, 1]
        x[i] = 0.5 * (1.0 - z);
        x[n - 1 - i] = 0.5 * (1.0 + z);
        w[i] = w[n - 1 - i] = 0.5 * wt;
    }
}

void gauss_log01(int n, double *x, double *w)
{
    // Recurrence coefficients of the measure -ln(x) dx on [0, 1] by the modified
    // Chebyshev algorithm with monic shifted Legendre polynomials pi_k, whose
    // modified moments are int_0^1 pi_k (-ln x) dx = (-1)^k (k!)^2 / ((2k)! k (k+1)).
    const int m = 2 * n;
    std::vector<double> mom(m), a(m, 0.5), b(m, 0.0);
    double r = 1.0;   // (k!)^2 / (2k)!
    mom[0] = 1.0;
    for (int k = 1; k < m; ++k) {
        r *= double(k) / (2.0 * (2.0 * k - 1.0));
        mom[k] = ((k & 1) ? -1.0 : 1.0) * r / (double(k) * (k + 1.0));
        b[k] = double(k) * k / (4.0 * (4.0 * double(k) * k - 1.0));
    }
    std::vector<double> alpha(n), beta(n);
    std::vector<std::vector<double>> sig(n + 1, std::vector<double>(m + 1, 0.0));  // sig[k+1][l]
    for (int l = 0; l < m; ++l) sig[1][l] = mom[l];
    alpha[0] = a[0] + mom[1] / mom[0];
    beta[0] = mom[0];
    for (int k = 1; k < n; ++k) {
        for (int l = k; l < m - k; ++l) {
            sig[k + 1][l] = sig[k][l + 1] - (alpha[k - 1] - a[l]) * sig[k][l] - beta[k - 1] * sig[k - 1][l]
                            + b[l] * sig[k][l - 1];
        }
        alpha[k] = a[k] + sig[k + 1][k + 1] / sig[k + 1][k] - sig[k][k] / sig[k][k - 1];
        beta[k] = sig[k + 1][k] / sig[k][k - 1];
    }
    // Nodes: eigenvalues of the Jacobi matrix by bisection on Sturm counts.
    auto count_below = [&](double lam) {
        int c = 0;
        double q = alpha[0] - lam;
        if (q < 0) ++c;
        for (int i = 1; i < n; ++i) {
            if (q == 0.0) q = 1e-300;
            q = (alpha[i] - lam) - beta[i] / q;
            if (q < 0) ++c;
        }
        return c;
    };
    for (int i = 0; i < n; ++i) {
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (count_below(mid) > i) hi = mid; else lo = mid;
        }
        const double lam = 0.5 * (lo + hi);
        // Christoffel number from the orthonormal polynomials at lam.
        double pm = 0.0, pc = 1.0 / std::sqrt(beta[0]), s = pc * pc;
        for (int k = 0; k + 1 < n; ++k) {
            const double pn = ((lam - alpha[k]) * pc - (k > 0 ? std::sqrt(beta[k]) : 0.0) * pm) / std::sqrt(beta[k + 1]);
            pm = pc;
            pc = pn;
            s += pc * pc;
        }
        x[i] = lam;
        w[i] = 1.0 / s;
    }
}

namespace {
struct Rules16 {
    double gl_x[16], gl_w[16], lg_x[16], lg_w[16], gl32_x[32], gl32_w[32];
    Rules16()
    {
        gauss_legendre01(16, gl_x, gl_w);
        gauss_log01(16, lg_x, lg_w);
        gauss_legendre01(32, gl32_x, gl32_w);
    }
};
const Rules16 &rules16()
{
    static const Rules16 r;
    return r;
}
}  // namespace

// ------------------------------------------------------------------ B-spline pieces
std::vector<double> cardinal_pieces(int p)
{
    // Cox-de Boor recurrence carried out on polynomials: B_{k,r} on the unit
    // interval [c, c+1] as a polynomial in u = x - c.
    const int np = p + 1;
    // poly[k][c][a]
    std::vector<std::vector<std::vector<double>>> B(np, std::vector<std::vector<double>>(np, std::vector<double>(np, 0.0)));
    for (int k = 0; k < np; ++k) B[k][k][0] = 1.0;
    for (int r = 1; r <= p; ++r) {
        std::vector<std::vector<std::vector<double>>> Bn(np, std::vector<std::vector<double>>(np, std::vector<double>(np, 0.0)));
        for (int k = 0; k + r <= p; ++k) {
            for (int c = 0; c < np; ++c) {
                // (x - k)/r * B_{k,r-1} = ((c - k) + u)/r * B_{k,r-1}
                // (k + r + 1 - x)/r * B_{k+1,r-1} = ((k + r + 1 - c) - u)/r * B_{k+1,r-1}
                for (int a = 0; a < np; ++a) {
                    const double b0 = B[k][c][a], b1 = B[k + 1][c][a];
                    Bn[k][c][a] += ((c - k) * b0 + (k + r + 1 - c) * b1) / r;
                    if (a + 1 < np) Bn[k][c][a + 1] += (b0 - b1) / r;
                }
            }
        }
        B.swap(Bn);
    }
    std::vector<double> out(np * np);
    for (int c = 0; c < np; ++c)
        for (int a = 0; a < np; ++a) out[c * np + a] = B[0][c][a];
    return out;
}

double cardinal_eval(int p, const std::vector<double> &pieces, double x)
{
    if (!(x > 0.0) || !(x < p + 1.0)) return 0.0;
    int c = int(std::floor(x));
    if (c > p) c = p;
    const double u = x - c;
    double v = 0.0;
    for (int a = p; a >= 0; --a) v = v * u + pieces[c * (p + 1) + a];
    return v;
}

static inline double horner(const double *c, int deg, double u)
{
    double v = 0.0;
    for (int a = deg; a >= 0; --a) v = v * u + c[a];
    return v;
}

double int_poly_log(const double *c, int deg, double sigma)
{
    const Rules16 &R = rules16();
    if (std::fabs(sigma - 0.5) > 1.0) {
        double s = 0.0;
        for (int g = 0; g < 16; ++g) s += R.gl_w[g] * horner(c, deg, R.gl_x[g]) * std::log(std::fabs(R.gl_x[g] - sigma));
        return s;
    }
    // int_sigma^b P(u) ln|u - sigma| du = L int_0^1 P(sigma + L x) (ln|L| + ln x) dx, L = b - sigma,
    // with a Gauss-Legendre rule for the ln|L| part and the Gauss rule for -ln x for the other.
    auto F = [&](double b) {
        const double L = b - sigma;
        if (L == 0.0) return 0.0;
        double sg = 0.0, sl = 0.0;
        for (int g = 0; g < 16; ++g) {
            sg += R.gl_w[g] * horner(c, deg, sigma + L * R.gl_x[g]);
            sl += R.lg_w[g] * horner(c, deg, sigma + L * R.lg_x[g]);
        }
        return L * (std::log(std::fabs(L)) * sg - sl);
    };
    return F(1.0) - F(0.0);
}

// ------------------------------------------------------------------ small dense helpers
// Minimum-norm solution of A w = mu, A (m x n) row-major with m <= n, by the
// Householder QR factorisation of A^T.
std::vector<double> min_norm_solve(const std::vector<double> &A, int m, int n, const std::vector<double> &mu)
{
    std::vector<double> X(n * m);   // X = A^T, n rows x m cols, row-major
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) X[j * m + i] = A[i * n + j];
    std::vector<std::vector<double>> V(m);
    std::vector<double> tau(m, 0.0);
    double rmax = 0.0;
    for (int j = 0; j < m; ++j) {
        double nrm = 0.0;
        for (int i = j; i < n; ++i) nrm += X[i * m + j] * X[i * m + j];
        nrm = std::sqrt(nrm);
        std::vector<double> v(n - j);
        for (int i = j; i < n; ++i) v[i - j] = X[i * m + j];
        const double alpha = (v[0] > 0 ? -nrm : nrm);
        v[0] -= alpha;
        double vv = 0.0;
        for (double t : v) vv += t * t;
        tau[j] = (vv > 0 ? 2.0 / vv : 0.0);
        for (int c = j; c < m; ++c) {
            double d = 0.0;
            for (int i = j; i < n; ++i) d += v[i - j] * X[i * m + c];
            d *= tau[j];
            for (int i = j; i < n; ++i) X[i * m + c] -= d * v[i - j];
        }
        V[j] = std::move(v);
        rmax = std::max(rmax, std::fabs(X[j * m + j]));
    }
    for (int j = 0; j < m; ++j)
        if (std::fabs(X[j * m + j]) <= 1e-12 * rmax) fail(-3, "collocation matrix is rank deficient (Schoenberg-Whitney violated)");
    // R^T y = mu (R = upper triangle of X's first m rows)
    std::vector<double> z(n, 0.0);
    for (int j = 0; j < m; ++j) {
        double s = mu[j];
        for (int i = 0; i < j; ++i) s -= X[i * m + j] * z[i];
        z[j] = s / X[j * m + j];
    }
    // w = H_0 ... H_{m-1} [y; 0]
    for (int j = m - 1; j >= 0; --j) {
        double d = 0.0;
        for (int i = j; i < n; ++i) d += V[j][i - j] * z[i];
        d *= tau[j];
        for (int i = j; i < n; ++i) z[i] -= d * V[j][i - j];
    }
    return z;
}

namespace {

// Solve G y = rhs (nrhs columns, rhs[k*nrhs + r]) for the symmetric positive
// definite cyclic banded matrix G[k][l] = g[d], d = cyclic distance <= hb.
// Bordered elimination: the first M - hb unknowns form a plain band matrix
// (banded Cholesky); the last hb are eliminated through a dense Schur complement.
std::vector<double> cyclic_band_solve(const std::vector<double> &g, int hb, int64_t M, const std::vector<double> &rhs, int nrhs)
{
    const int64_t m1 = M - hb;
    auto Gent = [&](int64_t k, int64_t l) -> double {
        int64_t d = l - k;
        d = ((d % M) + M) % M;
        d = std::min(d, M - d);
        return d <= hb ? g[d] : 0.0;
    };
    // banded Cholesky of G11: Lb[k*(hb+1) + q] = L[k][k - hb + q]
    std::vector<double> Lb(m1 * (hb + 1), 0.0);
    for (int64_t k = 0; k < m1; ++k) {
        for (int64_t j = std::max<int64_t>(0, k - hb); j <= k; ++j) {
            double s = Gent(k, j);
            for (int64_t i = std::max<int64_t>(0, k - hb); i < j; ++i) {
                if (i < j - hb) continue;
                s -= Lb[k * (hb + 1) + (i - k + hb)] * Lb[j * (hb + 1) + (i - j + hb)];
            }
            if (j == k) {
                if (!(s > 0.0)) fail(-3, "Gram matrix of the collocation is not positive definite");
                Lb[k * (hb + 1) + hb] = std::sqrt(s);
            } else {
                Lb[k * (hb + 1) + (j - k + hb)] = s / Lb[j * (hb + 1) + hb];
            }
        }
    }
    // The columns of G11^{-1} G12 decay geometrically away from the wrap; values
    // below 1e-290 are flushed to zero so that the substitutions never run on
    // subnormal numbers (many times slower on the host, and far below rounding).
    auto flush = [](double v) { return std::fabs(v) < 1e-290 ? 0.0 : v; };
    auto band_solve = [&](std::vector<double> &x, int nc) {   // x[k*nc + c], in place
        for (int64_t k = 0; k < m1; ++k) {
            for (int c = 0; c < nc; ++c) {
                double s = x[k * nc + c];
                for (int64_t i = std::max<int64_t>(0, k - hb); i < k; ++i) s -= Lb[k * (hb + 1) + (i - k + hb)] * x[i * nc + c];
                x[k * nc + c] = flush(s / Lb[k * (hb + 1) + hb]);
            }
        }
        for (int64_t k = m1 - 1; k >= 0; --k) {
            for (int c = 0; c < nc; ++c) {
                double s = x[k * nc + c];
                for (int64_t i = k + 1; i <= std::min<int64_t>(m1 - 1, k + hb); ++i) s -= Lb[i * (hb + 1) + (k - i + hb)] * x[i * nc + c];
                x[k * nc + c] = flush(s / Lb[k * (hb + 1) + hb]);
            }
        }
    };
    // X = G11^{-1} G12, z = G11^{-1} rhs1
    // G12 couples the last hb unknowns only to rows within hb of the wrap:
    // k < 2 hb or k >= m1 - 2 hb (every other entry of G12 is zero).
    std::vector<int64_t> wrap_rows;
    for (int64_t k = 0; k < m1; ++k) {
        if (k == 2 * hb && m1 - 2 * hb > k) k = m1 - 2 * hb;
        wrap_rows.push_back(k);
    }
    std::vector<double> X(m1 * hb, 0.0);
    for (int64_t k : wrap_rows)
        for (int c = 0; c < hb; ++c) X[k * hb + c] = Gent(k, m1 + c);
    band_solve(X, hb);
    std::vector<double> z(m1 * nrhs);
    for (int64_t k = 0; k < m1; ++k)
        for (int r = 0; r < nrhs; ++r) z[k * nrhs + r] = rhs[k * nrhs + r];
    band_solve(z, nrhs);
    // Schur complement S = G22 - G12^T X, rhs2' = rhs2 - G12^T z
    std::vector<double> S(hb * hb), r2(hb * nrhs);
    for (int a = 0; a < hb; ++a) {
        for (int b = 0; b < hb; ++b) {
            double s = Gent(m1 + a, m1 + b);
            for (int64_t k : wrap_rows) {
                const double gk = Gent(k, m1 + a);
                if (gk != 0.0) s -= gk * X[k * hb + b];
            }
            S[a * hb + b] = s;
        }
        for (int r = 0; r < nrhs; ++r) {
            double s = rhs[(m1 + a) * nrhs + r];
            for (int64_t k : wrap_rows) {
                const double gk = Gent(k, m1 + a);
                if (gk != 0.0) s -= gk * z[k * nrhs + r];
            }
            r2[a * nrhs + r] = s;
        }
    }
    // dense Cholesky of S
    for (int a = 0; a < hb; ++a) {
        for (int b = 0; b <= a; ++b) {
            double s = S[a * hb + b];
            for (int i = 0; i < b; ++i) s -= S[a * hb + i] * S[b * hb + i];
            if (a == b) {
                if (!(s > 0.0)) fail(-3, "Schur complement of the Gram matrix is not positive definite");
                S[a * hb + a] = std::sqrt(s);
            } else {
                S[a * hb + b] = s / S[b * hb + b];
            }
        }
    }
    std::vector<double> y2(hb * nrhs);
    for (int r = 0; r < nrhs; ++r) {
        for (int a = 0; a < hb; ++a) {
            double s = r2[a * nrhs + r];
            for (int i = 0; i < a; ++i) s -= S[a * hb + i] * y2[i * nrhs + r];
            y2[a * nrhs + r] = s / S[a * hb + a];
        }
        for (int a = hb - 1; a >= 0; --a) {
            double s = y2[a * nrhs + r];
            for (int i = a + 1; i < hb; ++i) s -= S[i * hb + a] * y2[i * nrhs + r];
            y2[a * nrhs + r] = s / S[a * hb + a];
        }
    }
    std::vector<double> y(M * nrhs);
    for (int64_t k = 0; k < m1; ++k)
        for (int r = 0; r < nrhs; ++r) {
            double s = z[k * nrhs + r];
            for (int c = 0; c < hb; ++c) s -= X[k * hb + c] * y2[c * nrhs + r];
            y[k * nrhs + r] = s;
        }
    for (int a = 0; a < hb; ++a)
        for (int r = 0; r < nrhs; ++r) y[(m1 + a) * nrhs + r] = y2[a * nrhs + r];
    return y;
}

}  // namespace

// ------------------------------------------------------------------ rules of Section 4
WQRules build_wq_rules(int p, int N, int R)
{
    if (p < 1 || p > 6) fail(-1, "degree p must be in [1, 6]");
    if (R < 1 || R > 4) fail(-1, "n_ref must be in [1, 4]");
    if (N < 2 * (p + 1)) fail(-1, "N must be at least 2 (p + 1)");
    if (int64_t(2) * R * N > (int64_t(1) << 24)) fail(-1, "2 n_ref N exceeds 2^24 nodes");
    WQRules W;
    W.p = p;
    W.N = N;
    W.R = R;
    W.M = int64_t(R) * N;
    W.n_nodes = 2 * W.M;
    W.Q = 2 * R * (p + 1) - 1;
    const int Q = W.Q;
    const int64_t M = W.M;
    const std::vector<double> pc = cardinal_pieces(p);
    auto Mp = [&](double x) { return cardinal_eval(p, pc, x); };

    // ---- Alg. 1 for B_0 (every B_i is its translate by 2R nodes): exactness
    // functions Bbar_k, k = -p .. R(p+1)-1 (refined index relative to supp B_0),
    // nodes n = 1..Q; mu_k = int Bbar_k B_0 dt, exact by (p+1)-point Gauss per
    // refined element (integrand of degree 2p).
    const int Kc = R * (p + 1) + p;
    std::vector<double> Bl(Kc * Q), mu(Kc, 0.0);
    std::vector<double> gx(p + 1), gw(p + 1);
    gauss_legendre01(p + 1, gx.data(), gw.data());
    for (int kk = 0; kk < Kc; ++kk) {
        const int k = kk - p;
        for (int q = 0; q < Q; ++q) Bl[kk * Q + q] = Mp(0.5 * (q + 1) - k);
        double s = 0.0;
        for (int e = 0; e < R * (p + 1); ++e)
            for (int g = 0; g <= p; ++g) {
                const double u = e + gx[g];
                s += gw[g] * Mp(u - k) * Mp(u / R);
            }
        mu[kk] = s / double(M);
    }
    W.w0 = min_norm_solve(Bl, Kc, Q, mu);
    W.bvals.resize(Q);
    for (int q = 0; q < Q; ++q) W.bvals[q] = Mp((q + 1) / (2.0 * R));

    // ---- Alg. 2 for the two source classes s = 0 and s = 1/(2M).
    // modified moments mu_k(s) = int Bbar_k(t) ln|sin(pi (t - s)) / pi| dt, summed
    // over the p + 1 elements of supp Bbar_k.  On element e, in its local
    // coordinate u (t = (e + u) / M) with sigma the local coordinate of the image of
    // s nearest the element, the piece integrals
    //   I[e][c] = int_0^1 P_c(u) ln|sin(pi (u - sigma) / M) / pi| du,  c = 0..p,
    // are computed once per element:
    //  * |sigma - 1/2| <= 1 (s on the element or half an element away): split into
    //    ln|u - sigma| (int_poly_log) - ln M + ln sinc(pi (u - sigma) / M) (16-point Gauss);
    //  * otherwise the integrand is analytic on the element with its singularity at
    //    least one element away: one Gauss rule for the whole kernel, 12 points
    //    when the singularity is within 3 elements, 8 points beyond (both reach the
    //    rounding floor for polynomial pieces up to degree 6 at those distances).
    // The kernel values at the Gauss points are shared by all p + 1 pieces.
    const Rules16 &RR = rules16();
    std::vector<double> pint(p + 1, 0.0);
    for (int c = 0; c <= p; ++c)
        for (int a = 0; a <= p; ++a) pint[c] += pc[c * (p + 1) + a] / (a + 1.0);
    double gx12[12], gw12[12], gx8[8], gw8[8];
    gauss_legendre01(12, gx12, gw12);
    gauss_legendre01(8, gx8, gw8);
    // weighted piece values w_g P_c(u_g) for both far rules
    std::vector<double> wp12((p + 1) * 12), wp8((p + 1) * 8);
    for (int c = 0; c <= p; ++c) {
        for (int g = 0; g < 12; ++g) wp12[c * 12 + g] = gw12[g] * horner(&pc[c * (p + 1)], p, gx12[g]);
        for (int g = 0; g < 8; ++g) wp8[c * 8 + g] = gw8[g] * horner(&pc[c * (p + 1)], p, gx8[g]);
    }
    std::vector<double> mom(M * 2, 0.0);
    std::vector<double> I(size_t(M) * (p + 1));
    const double lnM = std::log(double(M));
    const double inv_pi = 1.0 / kPi;
    for (int par = 0; par < 2; ++par) {
        for (int64_t e = 0; e < M; ++e) {
            const double s0 = 0.5 * par - double(e);
            const double s1 = s0 + double(M);
            const double sigma = (std::fabs(s0 - 0.5) <= std::fabs(s1 - 0.5)) ? s0 : s1;
            double *Ie = &I[size_t(e) * (p + 1)];
            const double dist = std::fabs(sigma - 0.5) - 0.5;   // element lengths from s to the element
            if (dist <= 0.5) {
                for (int c = 0; c <= p; ++c) {
                    const double *cc = &pc[c * (p + 1)];
                    double sp = 0.0;
                    for (int g = 0; g < 16; ++g) {
                        const double x = (RR.gl_x[g] - sigma) / double(M);
                        const double px = kPi * x;
                        const double sinc = (px == 0.0) ? 1.0 : std::sin(px) / px;
                        sp += RR.gl_w[g] * horner(cc, p, RR.gl_x[g]) * std::log(sinc);
                    }
                    Ie[c] = int_poly_log(cc, p, sigma) - lnM * pint[c] + sp;
                }
                continue;
            }
            const bool close = dist < 3.0;
            const int ng = close ? 12 : 8;
            const double *gx = close ? gx12 : gx8;
            const double *wp = close ? wp12.data() : wp8.data();
            double kv[12];
            for (int g = 0; g < ng; ++g)
                kv[g] = std::log(std::fabs(std::sin(kPi * ((gx[g] - sigma) / double(M)))) * inv_pi);
            for (int c = 0; c <= p; ++c) {
                double s = 0.0;
                for (int g = 0; g < ng; ++g) s += wp[c * ng + g] * kv[g];
                Ie[c] = s;
            }
        }
        for (int64_t k = 0; k < M; ++k) {
            double acc = 0.0;
            for (int c = 0; c <= p; ++c) acc += I[size_t((k + c) % M) * (p + 1) + c];
            mom[k * 2 + par] = acc / double(M);
        }
    }
    // Gram matrix G = B B^T of the collocation matrix B[k][n] = Bbar_k(eta_n):
    // G[k][k+d] = sum over half-integers x of M_p(x) M_p(x - d).
    std::vector<double> g(p + 1, 0.0);
    for (int d = 0; d <= p; ++d)
        for (int n = 1; n <= 2 * p + 1; ++n) g[d] += Mp(0.5 * n) * Mp(0.5 * n - d);
    const std::vector<double> y = cyclic_band_solve(g, p, M, mom, 2);
    // w = B^T y (minimum-norm solution), then the translation-invariant tables.
    W.ws.assign(2 * W.n_nodes, 0.0);
    const int64_t n2 = W.n_nodes;
    // M_p at the half-integers x = j / 2, j = 0..2p+3 (zero outside (0, p+1))
    std::vector<double> mh(2 * p + 4);
    for (int j = 0; j < 2 * p + 4; ++j) mh[j] = Mp(0.5 * j);
    for (int par = 0; par < 2; ++par) {
        std::vector<double> wv(n2, 0.0);
        for (int64_t n = 0; n < n2; ++n) {
            const int64_t kh = n / 2;
            double s = 0.0;
            for (int64_t k = kh - p - 1; k <= kh; ++k) {
                const int64_t j = n - 2 * k;   // 2 (n/2 - k)
                const double b = (j > 0 && j < 2 * p + 4) ? mh[j] : 0.0;
                if (b != 0.0) s += b * y[(((k % M) + M) % M) * 2 + par];
            }
            wv[n] = s;
        }
        for (int64_t d = 0; d < n2; ++d) W.ws[par * n2 + d] = wv[(par + d) % n2];
    }
    // (pi / sin(pi d / 2M))^2 for the K1 ratio |f(s)-f(t)|^2 / (sin(pi (s-t)) / pi)^2
    W.inv_s2.assign(n2, 0.0);
    for (int64_t d = 1; d < n2; ++d) {
        const double x = double(std::min(d, n2 - d)) / double(n2);
        const double s = std::sin(kPi * x);
        W.inv_s2[d] = (kPi / s) * (kPi / s);
    }
    return W;
}

// ------------------------------------------------------------------ near-pair tables
namespace {
struct NearBuild {
    NearField nf;
    NearBuild()
    {
        const Rules16 &R = rules16();
        std::memcpy(nf.u, R.gl_x, sizeof nf.u);
        std::memcpy(nf.w, R.gl_w, sizeof nf.w);
        // barycentric weights of the Lagrange basis on the 16 Gauss nodes
        double lam[16];
        for (int a = 0; a < 16; ++a) {
            double pr = 1.0;
            for (int b = 0; b < 16; ++b)
                if (b != a) pr *= (nf.u[a] - nf.u[b]);
            lam[a] = 1.0 / pr;
        }
        auto lag = [&](double x, double *out) {
            for (int a = 0; a < 16; ++a)
                if (x == nf.u[a]) {
                    for (int b = 0; b < 16; ++b) out[b] = (a == b);
                    return;
                }
            double den = 0.0;
            for (int a = 0; a < 16; ++a) den += lam[a] / (x - nf.u[a]);
            for (int a = 0; a < 16; ++a) out[a] = lam[a] / (x - nf.u[a]) / den;
        };
        double la[16], lb[16];
        // coincident: int_0^1 ln w [S_ab(w) + S_ba(w)] dw, S_ab(w) = int_0^{1-w} l_a(u) l_b(u+w) du,
        // a polynomial of degree <= 31 in w: Gauss rule for -ln w with 16 nodes is exact.
        std::vector<double> S(256, 0.0);
        for (int i = 0; i < 16; ++i) {
            const double wv = R.lg_x[i];
            const double len = 1.0 - wv;
            for (int gq = 0; gq < 16; ++gq) {
                const double u = len * R.gl_x[gq];
                lag(u, la);
                lag(u + wv, lb);
                const double f = -R.lg_w[i] * len * R.gl_w[gq];
                for (int a = 0; a < 16; ++a)
                    for (int b = 0; b < 16; ++b) S[a * 16 + b] += f * la[a] * lb[b];
            }
        }
        for (int a = 0; a < 16; ++a)
            for (int b = 0; b < 16; ++b) nf.mco[a * 16 + b] = S[a * 16 + b] + S[b * 16 + a];
        // adjacent: int_0^2 T_ab(w) ln w dw with w = 1 + v - u,
        // T_ab(w) = int l_a(u) l_b(u + w - 1) du over u in [max(0,1-w), min(1,2-w)].
        for (int i = 0; i < 256; ++i) nf.madj[i] = 0.0;
        for (int i = 0; i < 16; ++i) {       // w in [0, 1]: u in [1-w, 1]
            const double wv = R.lg_x[i];
            for (int gq = 0; gq < 16; ++gq) {
                const double v = wv * R.gl_x[gq];
                lag(1.0 - wv + v, la);
                lag(v, lb);
                const double f = -R.lg_w[i] * wv * R.gl_w[gq];
                for (int a = 0; a < 16; ++a)
                    for (int b = 0; b < 16; ++b) nf.madj[a * 16 + b] += f * la[a] * lb[b];
            }
        }
        for (int i = 0; i < 32; ++i) {       // w in [1, 2]: u in [0, 2-w], smooth log
            const double wv = 1.0 + R.gl32_x[i];
            const double len = 2.0 - wv;
            for (int gq = 0; gq < 16; ++gq) {
                const double u = len * R.gl_x[gq];
                lag(u, la);
                lag(u + wv - 1.0, lb);
                const double f = R.gl32_w[i] * std::log(wv) * len * R.gl_w[gq];
                for (int a = 0; a < 16; ++a)
                    for (int b = 0; b < 16; ++b) nf.madj[a * 16 + b] += f * la[a] * lb[b];
            }
        }
    }
};
}  // namespace

const NearField &nearfield16()
{
    static const NearBuild b;
    return b.nf;
}

}  // namespace sgbem
