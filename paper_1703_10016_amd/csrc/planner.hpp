// Host FP64 construction of the quadrature rules (geometry independent).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sgbem {

struct PlanError {
    int status;
    std::string msg;
};

// Gauss-Legendre nodes / weights on [0, 1].
void gauss_legendre01(int n, double *x, double *w);
// Gauss rule for the weight -ln(x) on [0, 1] (exact for polynomials of degree <= 2n-1).
void gauss_log01(int n, double *x, double *w);

// Cardinal B-spline M_p on [0, p+1]: monomial coefficients of its pieces,
// coef[c*(p+1) + a] with M_p(c + u) = sum_a coef[c][a] u^a, u in [0, 1].
std::vector<double> cardinal_pieces(int p);
double cardinal_eval(int p, const std::vector<double> &pieces, double x);

// int_0^1 P(u) ln|u - sigma| du, P(u) = sum_a c[a] u^a of degree deg.
double int_poly_log(const double *c, int deg, double sigma);

struct WQRules {
    int p = 0, N = 0, R = 0;
    int64_t M = 0, n_nodes = 0;      // M = R N refined elements, 2M nodes
    int Q = 0;                       // nodes per support: 2R(p+1) - 1
    std::vector<double> w0;          // [Q]   regular weights of B_0 on nodes 1..Q
    std::vector<double> bvals;       // [Q]   B_0 at those nodes
    std::vector<double> ws;          // [2][2M] singular-weight tables
    std::vector<double> inv_s2;      // [2M]  (pi / sin(pi d / 2M))^2, entry 0 unused
};

// Build the rules; throws PlanError.
WQRules build_wq_rules(int p, int N, int R);

// Minimum-norm solution of A w = mu, A (m x n) row-major, m <= n (Householder
// QR of A^T); throws PlanError on a rank-deficient A.
std::vector<double> min_norm_solve(const std::vector<double> &A, int m, int n, const std::vector<double> &mu);

// Rules on non-uniform periodic knots (no translation invariance): the
// approximation space on the breakpoints tau[0] = 0 < ... < tau[N] = 1 of one
// period, the exactness space on the knots refined by splitting every element
// into R equal parts (M = R N), nodes eta at the refined breakpoints and
// midpoints.  Row i's Q = 2R(p+1) - 1 support nodes are 2R i + 1 + q (mod 2M),
// as for uniform knots.
struct WQRulesKnots {
    int p = 0, N = 0, R = 0;
    int64_t M = 0, n_nodes = 0;
    int Q = 0;
    std::vector<double> eta;   // [2M] node parameters
    std::vector<double> W;     // [N][Q] regular weights of B_i (Alg. 1)
    std::vector<double> Bv;    // [N][Q] B_i at its support nodes
    std::vector<double> Ws;    // [2M][2M] singular weights, row m: source eta_m (Alg. 2)
};
constexpr int64_t kMaxKnotNodes = 8192;   // 2M limit: the full singular table is (2M)^2 doubles

// Build them (host threads); throws PlanError.
WQRulesKnots build_wq_rules_knots(int p, int N, int R, const double *tau);

// Rules on an open arc (Section 3, all N = n_el + p B-splines of the clamped
// knot vector on the breakpoints x_0 < ... < x_{n_el}; Section 4, nodes with
// p + 2 equally spaced points in the first and the last refined element,
// midpoints and breakpoints elsewhere; K2 = ln|s - t|).  Row i's support nodes
// are n0[i] .. n0[i] + cnt[i] - 1 (the nodes where B_i is non-zero); its
// weights and B_i values are padded with zeros to QM = max cnt.
struct WQRulesOpen {
    int p = 0, n_el = 0, R = 0, N = 0;
    int64_t M = 0, n_nodes = 0;       // M = R n_el refined elements, 2p + 2M - 1 nodes
    int QM = 0;
    std::vector<double> eta;          // [n_nodes]
    std::vector<int32_t> n0, cnt;     // [N]
    std::vector<double> W, Bv;        // [N][QM]
    std::vector<double> Ws;           // [n_nodes][n_nodes], row m: source eta_m
};
WQRulesOpen build_wq_rules_open(int p, int n_el, int R, const double *breaks);

struct NearField {
    double u[16], w[16];
    double mco[256], madj[256];
};
const NearField &nearfield16();

}  // namespace sgbem
