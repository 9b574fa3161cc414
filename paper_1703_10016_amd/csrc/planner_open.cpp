// Host FP64 construction of the quadrature rules of Section 4 on an open arc:
// the approximation space of all N = n_el + p B-splines of the clamped knot
// vector (Section 3), the node vector with p + 2 points in the end elements,
// Alg. 1 per test function and Alg. 2 per source with K2(s, t) = ln|s - t| and
// minimum-norm solutions where the systems are underdetermined.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "planner.hpp"
#include "planner_spline.hpp"

namespace sgbem {

namespace {

using spline::basis_funs;
using spline::CyclicBandSPD;
using spline::fail;
using spline::horner;
using spline::local_pieces;
using spline::OKnots;

}  // namespace

WQRulesOpen build_wq_rules_open(int p, int n_el, int R, const double *x)
{
    if (p < 1 || p > 6) fail(-1, "degree p must be in [1, 6]");
    if (R < 1 || R > 4) fail(-1, "n_ref must be in [1, 4]");
    if (n_el < 1 || int64_t(R) * n_el < 2) fail(-1, "an open arc needs at least two refined elements");
    if (!x) fail(-1, "breaks is NULL");
    for (int k = 0; k < n_el; ++k)
        if (!(x[k + 1] > x[k]) || !std::isfinite(x[k]) || !std::isfinite(x[k + 1]))
            fail(-1, "breaks must be finite and strictly increasing");
    WQRulesOpen W;
    W.p = p;
    W.n_el = n_el;
    W.R = R;
    W.N = n_el + p;
    W.M = int64_t(R) * n_el;
    W.n_nodes = 2 * p + 2 * W.M - 1;
    if (W.n_nodes > kMaxKnotNodes) fail(-6, "open arc: 2p + 2 n_ref n_el - 1 exceeds the limit of the full singular table");
    const int np = p + 1, N = W.N;
    const int64_t M = W.M, nn = W.n_nodes, NE = M + p;

    OKnots C, F;     // coarse (approximation space) and refined (exactness space) breakpoints
    C.n = n_el;
    C.x.assign(x, x + n_el + 1);
    F.n = M;
    F.x.resize(size_t(M) + 1);
    for (int e = 0; e < n_el; ++e)
        for (int r = 0; r < R; ++r) F.x[size_t(e) * R + r] = x[e] + (x[e + 1] - x[e]) * r / R;
    F.x[size_t(M)] = x[n_el];

    // nodes: p + 2 points on refined element 0, midpoint + right breakpoint on
    // elements 1 .. M-2, p + 1 more points on element M-1; lb[e] = node index of
    // the breakpoint xbar_e, span[n] = the refined element holding node n
    W.eta.reserve(size_t(nn));
    std::vector<int64_t> lb(size_t(M) + 1), span;
    span.reserve(size_t(nn));
    {
        const double h0 = F.x[1] - F.x[0];
        for (int k = 0; k <= p; ++k) {
            W.eta.push_back(F.x[0] + h0 * k / (p + 1));
            span.push_back(0);
        }
        lb[0] = 0;
        for (int64_t e = 1; e <= M - 2; ++e) {
            lb[size_t(e)] = int64_t(W.eta.size());
            W.eta.push_back(F.x[size_t(e)]);
            span.push_back(e);
            W.eta.push_back(0.5 * (F.x[size_t(e)] + F.x[size_t(e) + 1]));
            span.push_back(e);
        }
        const double hl = F.x[size_t(M)] - F.x[size_t(M) - 1];
        lb[size_t(M) - 1] = int64_t(W.eta.size());
        W.eta.push_back(F.x[size_t(M) - 1]);
        span.push_back(M - 1);
        for (int k = 1; k <= p; ++k) {
            W.eta.push_back(F.x[size_t(M) - 1] + hl * k / (p + 1));
            span.push_back(M - 1);
        }
        lb[size_t(M)] = int64_t(W.eta.size());
        W.eta.push_back(F.x[size_t(M)]);
        span.push_back(M - 1);
        if (int64_t(W.eta.size()) != nn) fail(-1, "node vector construction (internal)");
    }

    // ---- Alg. 1, every test function (open index i: knots t_{i-p} .. t_{i+1})
    std::vector<double> gx(np), gw(np);
    gauss_legendre01(np, gx.data(), gw.data());
    W.n0.resize(size_t(N));
    W.cnt.resize(size_t(N));
    std::vector<std::vector<double>> rows;
    rows.resize(static_cast<size_t>(N));
    int QM = 0;
    for (int i = 0; i < N; ++i) {
        const int64_t c0 = std::max(i - p, 0), c1 = std::min(i + 1, n_el);   // coarse elements of supp B_i
        const int64_t e0 = R * c0, e1 = R * c1;                              // refined elements [e0, e1)
        const int64_t first = (i == 0) ? 0 : lb[size_t(e0)] + 1;
        const int64_t last = (i == N - 1) ? nn - 1 : lb[size_t(e1)] - 1;
        const int cnt = int(last - first + 1);
        const int Kc = int(e1 - e0) + p;                                      // refined functions e0 .. e1 - 1 + p
        if (cnt < Kc) fail(-3, "fewer support nodes than exactness conditions (internal)");
        W.n0[size_t(i)] = int32_t(first);
        W.cnt[size_t(i)] = cnt;
        QM = std::max(QM, cnt);
        std::vector<double> Bl(size_t(Kc) * cnt, 0.0), mu(size_t(Kc), 0.0);
        double v[8];
        for (int q = 0; q < cnt; ++q) {
            const int64_t n = first + q, l = span[size_t(n)];
            basis_funs(F, p, l, W.eta[size_t(n)], v);       // v[j]: refined function l + j
            for (int j = 0; j <= p; ++j) {
                const int64_t kk = l + j - e0;
                if (kk >= 0 && kk < Kc) Bl[size_t(kk) * cnt + q] = v[j];
            }
        }
        for (int64_t e = e0; e < e1; ++e) {
            const double a = F.x[size_t(e)], h = F.x[size_t(e) + 1] - a;
            const int64_t ec = e / R;
            for (int g = 0; g < np; ++g) {
                const double t = a + h * gx[g];
                double vf[8], vc[8];
                basis_funs(F, p, e, t, vf);
                basis_funs(C, p, ec, t, vc);
                const int64_t jc = i - ec;
                const double bi = (jc >= 0 && jc <= p) ? vc[jc] : 0.0;
                for (int j = 0; j <= p; ++j) mu[size_t(e + j - e0)] += h * gw[g] * vf[j] * bi;
            }
        }
        rows[size_t(i)] = min_norm_solve(Bl, Kc, cnt, mu);
    }
    W.QM = QM;
    W.W.assign(size_t(N) * QM, 0.0);
    W.Bv.assign(size_t(N) * QM, 0.0);
    for (int i = 0; i < N; ++i) {
        std::copy(rows[size_t(i)].begin(), rows[size_t(i)].end(), W.W.begin() + size_t(i) * QM);
        double v[8];
        for (int q = 0; q < W.cnt[size_t(i)]; ++q) {
            const int64_t n = W.n0[size_t(i)] + q;
            const int64_t lc = span[size_t(n)] / R;
            basis_funs(C, p, lc, W.eta[size_t(n)], v);
            const int64_t jc = i - lc;
            W.Bv[size_t(i) * QM + q] = (jc >= 0 && jc <= p) ? v[jc] : 0.0;
        }
    }

    // ---- Alg. 2: Gram matrix G = B B^T of B[k][n] = Bbar_k(eta_n), banded (hb = p), NE = M + p
    std::vector<double> Gb(size_t(NE) * (2 * p + 1), 0.0);   // Gb[k][p + d] = G[k][k + d]
    {
        double v[8];
        for (int64_t n = 0; n < nn; ++n) {
            const int64_t l = span[size_t(n)];
            basis_funs(F, p, l, W.eta[size_t(n)], v);
            for (int a = 0; a <= p; ++a)
                for (int b = 0; b <= p; ++b) Gb[size_t(l + a) * (2 * p + 1) + (b - a + p)] += v[a] * v[b];
        }
    }
    auto Gent = [&](int64_t k, int64_t l) -> double {
        const int64_t d = l - k;
        return (d >= -p && d <= p) ? Gb[size_t(k) * (2 * p + 1) + (d + p)] : 0.0;
    };
    const CyclicBandSPD G(NE, p, Gent);

    double gx12[12], gw12[12], gx8[8], gw8[8];
    gauss_legendre01(12, gx12, gw12);
    gauss_legendre01(8, gx8, gw8);
    std::vector<double> pieces(size_t(M) * np * np), wb12(size_t(M) * np * 12), wb8(size_t(M) * np * 8);
    std::vector<double> pint(size_t(M) * np);
    for (int64_t e = 0; e < M; ++e) {
        double *pc = &pieces[size_t(e) * np * np];
        local_pieces(F, p, e, pc);                      // piece j: refined function e + j
        for (int j = 0; j <= p; ++j) {
            double s = 0.0;
            for (int a = 0; a <= p; ++a) s += pc[j * np + a] / (a + 1.0);
            pint[size_t(e) * np + j] = s;
            for (int g = 0; g < 12; ++g) wb12[(size_t(e) * np + j) * 12 + g] = gw12[g] * horner(pc + j * np, p, gx12[g]);
            for (int g = 0; g < 8; ++g) wb8[(size_t(e) * np + j) * 8 + g] = gw8[g] * horner(pc + j * np, p, gx8[g]);
        }
    }
    // moments of one source s (eq. mod_mom_gen with K2 = ln|t - s|):
    //   mu_k(s) = sum over the elements e of supp Bbar_k of h_e int_0^1 P(u) ln|xbar_e + h_e u - s| du;
    // within half an element length: ln h + ln|u - sigma| by int_poly_log (closed form),
    // farther: Gauss (12 points within 3 element lengths, 8 beyond).
    auto moments = [&](double s, double *mu) {
        std::fill(mu, mu + NE, 0.0);
        for (int64_t e = 0; e < M; ++e) {
            const double a = F.x[size_t(e)], h = F.x[size_t(e) + 1] - a;
            const double sigma = (s - a) / h;
            const double dist = std::fabs(sigma - 0.5) - 0.5;
            const double *pc = &pieces[size_t(e) * np * np];
            double I[8];
            if (dist <= 0.5) {
                const double lh = std::log(h);
                for (int j = 0; j <= p; ++j) I[j] = h * (int_poly_log(pc + j * np, p, sigma) + lh * pint[size_t(e) * np + j]);
            } else {
                const bool close = dist < 3.0;
                const int ng = close ? 12 : 8;
                const double *gxx = close ? gx12 : gx8;
                const double *wb = close ? &wb12[size_t(e) * np * 12] : &wb8[size_t(e) * np * 8];
                double kv[12];
                for (int g = 0; g < ng; ++g) kv[g] = std::log(std::fabs(a + h * gxx[g] - s));
                for (int j = 0; j <= p; ++j) {
                    double acc = 0.0;
                    for (int g = 0; g < ng; ++g) acc += wb[j * ng + g] * kv[g];
                    I[j] = h * acc;
                }
            }
            for (int j = 0; j <= p; ++j) mu[size_t(e + j)] += I[j];
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
                std::vector<double> rhs(size_t(NE) * size_t(chunk));
                std::vector<double> mu(static_cast<size_t>(NE));
                for (int64_t c = t; c < nchunks; c += nth) {
                    const int64_t m0 = c * chunk, nc = std::min(chunk, nn - m0);
                    for (int64_t r = 0; r < nc; ++r) {
                        moments(W.eta[size_t(m0 + r)], mu.data());
                        for (int64_t k = 0; k < NE; ++k) rhs[size_t(k) * nc + r] = mu[size_t(k)];
                    }
                    G.solve(rhs.data(), int(nc));
                    double v[8];
                    for (int64_t n = 0; n < nn; ++n) {
                        const int64_t l = span[size_t(n)];
                        basis_funs(F, p, l, W.eta[size_t(n)], v);
                        for (int64_t r = 0; r < nc; ++r) {
                            double s = 0.0;
                            for (int j = 0; j <= p; ++j) s += v[j] * rhs[size_t(l + j) * nc + r];
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
