// Host FP64 construction of the quadrature rules of Section 4 on non-uniform
// periodic knots: Alg. 1 for every test function (the local systems are no
// longer shifts of one another) and Alg. 2 for every source (the full table of
// singular weights), with the modified moments of eq. mod_mom_gen in the local
// coordinate of each refined element.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "planner.hpp"

namespace sgbem {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

[[noreturn]] void fail(int status, const std::string &msg) { throw PlanError{status, msg}; }

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

// The p + 1 B-splines of degree p nonzero on span l at x (t_l <= x <= t_{l+1}):
// out[j] = B_{l-p+j}(x), by the triangular Cox-de Boor scheme.
void basis_funs(const PKnots &K, int p, int64_t l, double x, double *out)
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
void local_pieces(const PKnots &K, int p, int64_t e, double *coef)
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

double horner(const double *c, int deg, double u)
{
    double v = 0.0;
    for (int a = deg; a >= 0; --a) v = v * u + c[a];
    return v;
}

// Symmetric positive definite cyclic banded matrix (half bandwidth hb, entries
// G(k, l) for cyclic |k - l| <= hb): bordered elimination, the first M - hb
// unknowns by banded Cholesky, the last hb through the dense Schur complement.
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

}  // namespace

WQRulesKnots build_wq_rules_knots(int p, int N, int R, const double *tau)
{
    if (p < 1 || p > 6) fail(-1, "degree p must be in [1, 6]");
    if (R < 1 || R > 4) fail(-1, "n_ref must be in [1, 4]");
    if (N < 2 * (p + 1)) fail(-1, "N must be at least 2 (p + 1)");
    if (int64_t(2) * R * N > kMaxKnotNodes) fail(-6, "non-uniform knots: 2 n_ref N exceeds the limit of the full singular table");
    if (!tau) fail(-1, "knots is NULL");
    if (tau[0] != 0.0 || tau[N] != 1.0) fail(-1, "knots must run from 0 to 1 over one period");
    for (int k = 0; k < N; ++k)
        if (!(tau[k + 1] > tau[k])) fail(-1, "knots must be strictly increasing");
    WQRulesKnots W;
    W.p = p;
    W.N = N;
    W.R = R;
    W.M = int64_t(R) * N;
    W.n_nodes = 2 * W.M;
    W.Q = 2 * R * (p + 1) - 1;
    const int Q = W.Q, np = p + 1;
    const int64_t M = W.M, nn = W.n_nodes;

    PKnots C, F;     // coarse (approximation space) and refined (exactness space) knots
    C.n = N;
    C.t.assign(tau, tau + N + 1);
    F.n = M;
    F.t.resize(size_t(M) + 1);
    for (int e = 0; e < N; ++e)
        for (int r = 0; r < R; ++r) F.t[size_t(e) * R + r] = tau[e] + (tau[e + 1] - tau[e]) * r / R;
    F.t[size_t(M)] = 1.0;
    W.eta.resize(size_t(nn));
    for (int64_t k = 0; k < M; ++k) {
        W.eta[size_t(2 * k)] = F.t[size_t(k)];
        W.eta[size_t(2 * k + 1)] = 0.5 * (F.t[size_t(k)] + F.t[size_t(k + 1)]);
    }
    auto modM = [&](int64_t k) { return ((k % M) + M) % M; };
    auto modN = [&](int64_t k) { return ((k % N) + N) % N; };
    // refined functions at node n: span n / 2 (the element starting at or holding the node)
    auto node_vals = [&](int64_t n, double *v) {
        const int64_t nm = ((n % nn) + nn) % nn;
        basis_funs(F, p, nm / 2, W.eta[size_t(nm)], v);   // v[j] = Bbar_{nm/2 - p + j}
    };

    // ---- Alg. 1, every test function
    const int Kc = R * (p + 1) + p;
    std::vector<double> gx(np), gw(np);
    gauss_legendre01(np, gx.data(), gw.data());
    W.W.assign(size_t(N) * Q, 0.0);
    W.Bv.assign(size_t(N) * Q, 0.0);
    for (int i = 0; i < N; ++i) {
        const int64_t k0 = int64_t(R) * i - p;    // exactness set: k0 .. k0 + Kc - 1 (mod M)
        std::vector<double> Bl(size_t(Kc) * Q, 0.0), mu(Kc, 0.0);
        double v[8];
        for (int q = 0; q < Q; ++q) {
            const int64_t n = int64_t(2) * R * i + 1 + q;
            node_vals(n, v);
            const int64_t l = n / 2;            // unreduced span index (k relative ordering)
            for (int j = 0; j <= p; ++j) {
                const int64_t kk = l - p + j - k0;
                if (kk >= 0 && kk < Kc) Bl[size_t(kk) * Q + q] = v[j];
            }
            // B_i at the node: coarse span (l / R), function index relative i
            const int64_t nm = ((n % nn) + nn) % nn;
            const int64_t lc = (nm / 2) / R;
            basis_funs(C, p, lc, W.eta[size_t(nm)], v);
            for (int j = 0; j <= p; ++j)
                if (modN(lc - p + j) == i) W.Bv[size_t(i) * Q + q] = v[j];
        }
        // mu_k = int Bbar_k B_i over the R (p+1) refined elements of supp B_i, (p+1)-point Gauss each
        for (int c = 0; c < R * np; ++c) {
            const int64_t e = int64_t(R) * i + c;     // unreduced refined element
            const int64_t em = modM(e);
            const double a = F.t[size_t(em)], h = F.t[size_t(em) + 1] - a;
            const int64_t ec = em / R;                // coarse span
            for (int g = 0; g < np; ++g) {
                const double x = a + h * gx[g];
                double vf[8], vc[8];
                basis_funs(F, p, em, x, vf);
                basis_funs(C, p, ec, x, vc);
                double bi = 0.0;
                for (int j = 0; j <= p; ++j)
                    if (modN(ec - p + j) == i) bi = vc[j];
                for (int j = 0; j <= p; ++j) {
                    const int64_t kk = (e - p + j) - k0;
                    if (kk >= 0 && kk < Kc) mu[size_t(kk)] += h * gw[g] * vf[j] * bi;
                }
            }
        }
        const std::vector<double> w = min_norm_solve(Bl, Kc, Q, mu);
        std::copy(w.begin(), w.end(), W.W.begin() + size_t(i) * Q);
    }

    // ---- Alg. 2: Gram matrix G = B B^T of B[k][n] = Bbar_k(eta_n) (cyclic banded, hb = p)
    std::vector<double> Gb(size_t(M) * (2 * p + 1), 0.0);   // Gb[k][p + d] = G[k][k + d]
    {
        double v[8];
        for (int64_t n = 0; n < nn; ++n) {
            node_vals(n, v);
            const int64_t l = n / 2;
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p; ++b) Gb[size_t(modM(l - p + a)) * (2 * p + 1) + (b - a + p)] += v[a] * v[b];
        }
    }
    auto Gent = [&](int64_t k, int64_t l) -> double {
        int64_t d = l - k;
        if (d > M / 2) d -= M;
        if (d < -M / 2) d += M;
        return (d >= -p && d <= p) ? Gb[size_t(modM(k)) * (2 * p + 1) + (d + p)] : 0.0;
    };
    const CyclicBandSPD G(M, p, Gent);

    // per refined element: local pieces (near sources) and weighted piece values
    // at the far Gauss points (12 points within 3 element lengths, 8 beyond)
    double gx12[12], gw12[12], gx8[8], gw8[8], gx16[16], gw16[16];
    gauss_legendre01(12, gx12, gw12);
    gauss_legendre01(8, gx8, gw8);
    gauss_legendre01(16, gx16, gw16);
    std::vector<double> pieces(size_t(M) * np * np), wb12(size_t(M) * np * 12), wb8(size_t(M) * np * 8);
    std::vector<double> pint(size_t(M) * np);
    for (int64_t e = 0; e < M; ++e) {
        double *pc = &pieces[size_t(e) * np * np];
        local_pieces(F, p, e, pc);
        for (int j = 0; j <= p; ++j) {
            double s = 0.0;
            for (int a = 0; a <= p; ++a) s += pc[j * np + a] / (a + 1.0);
            pint[size_t(e) * np + j] = s;
            for (int g = 0; g < 12; ++g) wb12[(size_t(e) * np + j) * 12 + g] = gw12[g] * horner(pc + j * np, p, gx12[g]);
            for (int g = 0; g < 8; ++g) wb8[(size_t(e) * np + j) * 8 + g] = gw8[g] * horner(pc + j * np, p, gx8[g]);
        }
    }
    // moments of one source s into mu[k] (k < M):
    //   mu_k(s) = sum over the elements e of supp Bbar_k of h_e int_0^1 P(u) K2(s, t_e + h_e u) du,
    // K2(s, t) = ln|sin(pi (t - s)) / pi|.  Near (s within half an element length
    // of the element): ln|t - s*| + ln sinc, ln|t - s*| = ln h + ln|u - sigma| by
    // int_poly_log, the smooth sinc part by 16-point Gauss; far: one Gauss rule.
    auto moments = [&](double s, double *mu) {
        std::fill(mu, mu + M, 0.0);
        for (int64_t e = 0; e < M; ++e) {
            const double a = F.t[size_t(e)], h = F.t[size_t(e) + 1] - a;
            const double s_star = s + std::nearbyint((a + 0.5 * h) - s);
            const double sigma = (s_star - a) / h;
            const double dist = std::fabs(sigma - 0.5) - 0.5;
            const double *pc = &pieces[size_t(e) * np * np];
            double I[8];
            if (dist <= 0.5) {
                double ls[16];
                for (int g = 0; g < 16; ++g) {
                    const double x = h * (gx16[g] - sigma);
                    const double px = kPi * x;
                    ls[g] = std::log(px == 0.0 ? 1.0 : std::sin(px) / px);
                }
                const double lh = std::log(h);
                for (int j = 0; j <= p; ++j) {
                    double sp = 0.0;
                    for (int g = 0; g < 16; ++g) sp += gw16[g] * horner(pc + j * np, p, gx16[g]) * ls[g];
                    I[j] = h * (int_poly_log(pc + j * np, p, sigma) + lh * pint[size_t(e) * np + j] + sp);
                }
            } else {
                const bool close = dist < 3.0;
                const int ng = close ? 12 : 8;
                const double *gxx = close ? gx12 : gx8;
                const double *wb = close ? &wb12[size_t(e) * np * 12] : &wb8[size_t(e) * np * 8];
                double kv[12];
                for (int g = 0; g < ng; ++g) kv[g] = std::log(std::fabs(std::sin(kPi * (a + h * gxx[g] - s))) / kPi);
                for (int j = 0; j <= p; ++j) {
                    double acc = 0.0;
                    for (int g = 0; g < ng; ++g) acc += wb[j * ng + g] * kv[g];
                    I[j] = h * acc;
                }
            }
            for (int j = 0; j <= p; ++j) mu[size_t(modM(e - p + j))] += I[j];
        }
    };

    // sources in chunks over host threads: moments, the Gram solve, w = B^T y
    W.Ws.assign(size_t(nn) * nn, 0.0);
    const int64_t chunk = 64;
    const int64_t nchunks = (nn + chunk - 1) / chunk;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = unsigned(std::min<int64_t>(nth, nchunks));
    std::vector<std::thread> pool;
    std::vector<std::string> errs(nth);
    for (unsigned t = 0; t < nth; ++t) {
        pool.emplace_back([&, t]() {
            try {
                std::vector<double> rhs(size_t(M) * size_t(chunk));
                std::vector<double> mu(static_cast<size_t>(M));
                for (int64_t c = t; c < nchunks; c += nth) {
                    const int64_t m0 = c * chunk, nc = std::min(chunk, nn - m0);
                    for (int64_t r = 0; r < nc; ++r) {
                        moments(W.eta[size_t(m0 + r)], mu.data());
                        for (int64_t k = 0; k < M; ++k) rhs[size_t(k) * nc + r] = mu[size_t(k)];
                    }
                    G.solve(rhs.data(), int(nc));
                    double v[8];
                    for (int64_t n = 0; n < nn; ++n) {
                        node_vals(n, v);
                        const int64_t l = n / 2;
                        for (int64_t r = 0; r < nc; ++r) {
                            double s = 0.0;
                            for (int j = 0; j <= p; ++j) s += v[j] * rhs[size_t(modM(l - p + j)) * nc + r];
                            W.Ws[size_t(m0 + r) * nn + n] = s;
                        }
                    }
                }
            } catch (const PlanError &e) {
                errs[t] = e.msg;
            } catch (const std::exception &e) {
                errs[t] = e.what();
            }
        });
    }
    for (auto &th : pool) th.join();
    for (const std::string &e : errs)
        if (!e.empty()) fail(-3, e);
    return W;
}

}  // namespace sgbem
