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
#include "planner_spline.hpp"

namespace sgbem {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
using spline::basis_funs;
using spline::CyclicBandSPD;
using spline::fail;
using spline::horner;
using spline::local_pieces;
using spline::PKnots;

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
