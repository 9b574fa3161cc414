/*
 * sgbem.h -- C ABI of libsgbem: Galerkin assembly of the 2D Laplace
 * single-layer operator with periodic B-splines on a closed curve, by
 * B-spline weighted quadrature with row assembly and sum factorisation (the
 * fast form) or element by element with Gauss rules (the plain form), plus
 * the right-hand sides of the indirect and the direct formulation, a
 * mixed-precision dense solve, collocation with the same rules, one launch for
 * many curves and a continuous-batching server, on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Aimi, Calabro, Diligenti, Sampoli, Sangalli, Sestini, "Efficient
 * assembly based on B-spline tailored quadrature rules for the IgA-SGBEM".
 *
 * Problem (Section 2, eq. prima_BIE in indirect form on a closed curve):
 *   find phi_h = sum_j alpha_j B_j with
 *   A alpha = beta,  A_ij = -(1/2pi) int int B_i(s) J(s) ln|f(s)-f(t)| B_j(t) J(t) dt ds
 *   (eqs. Gmatrix, final_1),  beta_i = int B_i(s) J(s) g(f(s)) ds (eq. final_b1),
 * with B_i the cyclic B-splines of degree p on N elements of the parameter
 * interval [0, 1) (Section 3; uniform, or non-uniform periodic knots given to
 * sgbem_weights), f the curve and J = |f'| (eq. J).
 *
 * Conventions for every call:
 *  - every function returns an sgbem_status; no C++ exception crosses the ABI;
 *    on failure sgbem_last_error() returns a message (thread-local, never NULL);
 *  - "device" pointers are HIP device memory owned by the caller (e.g. a
 *    torch tensor's data_ptr); "host" pointers are ordinary host memory owned
 *    by the caller and only read during the call;
 *  - work is enqueued on the context's stream and is asynchronous unless
 *    stated otherwise; a context must be used from one host thread at a time
 *    (a server, sgbem_server_*, may be called from any thread);
 *  - matrices are row-major: entry (i, j) at ptr[i * lda + j], lda >= N;
 *  - basis index convention: B_i is supported on [tau_i, tau_{i+p+1}) mod 1
 *    (tau_k = k / N for uniform knots).
 */
#ifndef SGBEM_H
#define SGBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGBEM_OK = 0,
    SGBEM_E_INVAL = -1,        /* an argument is out of range or inconsistent          */
    SGBEM_E_NOMEM = -2,        /* device or host allocation failed / budget exceeded   */
    SGBEM_E_SINGULAR = -3,     /* zero pivot in the LU factorisation                   */
    SGBEM_E_NOCONV = -4,       /* iterative refinement did not reach the tolerance     */
    SGBEM_E_DEVICE = -5,       /* a HIP runtime call failed                            */
    SGBEM_E_UNSUPPORTED = -6   /* valid request with no kernel compiled for its shape    */
} sgbem_status;

typedef struct sgbem_ctx_s *sgbem_ctx;       /* one device + one HIP stream             */
typedef struct sgbem_rules_s *sgbem_rules;   /* device-resident quadrature rules (p,N,R) */
typedef struct sgbem_batch_s *sgbem_batch;   /* device-resident description of many curves */

typedef enum { SGBEM_CURVE_BSPLINE = 0, SGBEM_CURVE_POLAR = 1, SGBEM_CURVE_BSPLINE_OPEN = 2 } sgbem_curve_kind;
typedef enum { SGBEM_WQ = 0, SGBEM_EBE = 1 } sgbem_method;
typedef enum { SGBEM_FP64 = 0, SGBEM_FP32 = 1 } sgbem_precision;

/*
 * Closed curve f : [0, 1) -> R^2 (Section 3), or open arc f : [a, b] -> R^2
 * (Section 2, exterior problem; kind BSPLINE_OPEN).  Host memory, read during the
 * call: up to 64 control points (or any polar curve) travel inline in the
 * kernel arguments; larger control nets are copied to device memory owned by
 * the context.
 *  BSPLINE: f(t) = sum_j ctrl[j] B_j(t), the closed-curve representation of
 *           Section 3 (whose last d control points repeat the first ones; here
 *           they are not repeated) on the periodic extension of the knots of
 *           one period, tau_{k + n} = tau_k + 1, B_j of degree d supported on
 *           [tau_j, tau_{j+d+1}) mod 1:
 *           degree d in [1, 7], n_ctrl > d, ctrl_xy = [n_ctrl][2];
 *           knots = NULL for uniform knots tau_k = k / n_ctrl, else [n_ctrl + 1]
 *           breakpoints 0 = tau_0 < tau_1 < ... < tau_n = 1 (strictly
 *           increasing: simple knots, so the curve is C^(d-1)).
 *  BSPLINE_OPEN: f(t) = sum_j ctrl[j] B_j(t), t in [a, b], on the open
 *           (clamped) knot vector knots[n_ctrl + d + 1] (Section 3): the first
 *           d + 1 knots equal a, the last d + 1 equal b, the inner ones strictly
 *           increasing inside (a, b); degree d in [1, 7], n_ctrl > d,
 *           ctrl_xy = [n_ctrl][2].  Served only with rules of sgbem_weights_open
 *           on the same [a, b] (sgbem_assemble SGBEM_WQ FP64, sgbem_rhs and
 *           sgbem_rhs_points with SGBEM_WQ); up to 64 control points travel inline.
 *  POLAR:   f(t) = r(theta) (cos theta, sin theta), theta = 2 pi t,
 *           r(theta) = r0 (1 + sum_{k=1..n_modes} a[k-1] cos(k theta + phi[k-1])),
 *           r0 > 0, 0 <= n_modes <= 64, r must stay positive.
 * Unused fields are ignored.
 */
typedef struct {
    int32_t kind;
    int32_t degree;
    int32_t n_ctrl;
    const double *ctrl_xy;
    const double *knots;
    double r0;
    int32_t n_modes;
    const double *a;
    const double *phi;
} sgbem_curve;

typedef struct {
    int32_t iters;          /* refinement steps taken                                  */
    int32_t status;         /* same value as the call's return                          */
    double rel_update;      /* ||dx||_inf / ||x||_inf of the last refinement step       */
    double backward_err;    /* ||beta - A x||_inf / (||A||_inf ||x||_inf + ||beta||_inf) */
    int32_t pivoted;        /* 1: partial pivoting, 0: factored without row interchanges */
    int32_t reserved;
} sgbem_solve_info;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (NULL:
 * the null stream).  Allocates nothing on the device until first use; from
 * then on the device memory the context holds (rule tables of its
 * sgbem_weights handles, workspaces of the calls, batch descriptions) stays
 * within `hbm_budget_bytes` (0: no limit): a call whose allocation would
 * exceed it returns E_NOMEM before allocating or freeing anything, and the
 * context keeps what it held.  sgbem_memory_need gives the bytes each call
 * needs.  Errors: E_INVAL (bad device), E_DEVICE. */
sgbem_status sgbem_ctx_create(int32_t device, void *hip_stream, uint64_t hbm_budget_bytes, sgbem_ctx *out);

/* Device bytes the context holds now and its budget (0: no limit). */
sgbem_status sgbem_ctx_memory(sgbem_ctx ctx, int64_t *held_bytes, int64_t *budget_bytes);

/* Host-only: the device bytes a context allocates for one call of the kind
 * `what` (each buffer rounded up to 4096 bytes; the workspaces are grow-only
 * buffers of the context, reused by later calls of the same or smaller size):
 *  SGBEM_MEM_RULES:        one sgbem_weights handle of (p, N, n_ref): 72 M + O(1)
 *                          bytes, M = n_ref N;
 *  SGBEM_MEM_ASSEMBLE_WQ:  node geometry of sgbem_assemble (SGBEM_WQ), sgbem_rhs
 *                          (SGBEM_WQ) and sgbem_assemble_collocation: 48 M bytes;
 *  SGBEM_MEM_ASSEMBLE_EBE: sgbem_assemble with SGBEM_EBE and n_gauss points:
 *                          geometry on the Gauss and the 16-point near grids, the
 *                          near-pair matrices and the cached near-pair table;
 *  SGBEM_MEM_RHS_DIRECT:   sgbem_rhs_direct with n_gauss points: node geometry and
 *                          the double-layer sweep's workspace;
 *  SGBEM_MEM_SOLVE:        sgbem_solve of order N: 4 N_p^2 + about 1.8 N_p KB,
 *                          N_p = N rounded up to a multiple of 64, plus, for
 *                          N > 4096, 8 MiB per 1024 rows (the inverted
 *                          1024-row diagonal blocks of the triangular factors);
 *  SGBEM_MEM_RULES_OPEN:   one sgbem_weights_open handle (N = n_el elements):
 *                          16 N Q_M + 8 n_q^2 + 8 n_q + 8 N bytes, Q_M = 2 n_ref (p + 1)
 *                          - 1 + 2p, n_q = 2p + 2 n_ref n_el - 1 nodes, plus alignment;
 *  SGBEM_MEM_RULES_KNOTS:  one sgbem_weights handle on non-uniform knots:
 *                          32 M^2 + 16 N Q + 16 M bytes (the full singular table).
 * n_ctrl: control points of the B-spline curve of the call (0 for a polar
 * curve); beyond 64 they are copied to the device, 24 n_ctrl + 8 bytes more.
 * Errors: E_INVAL. */
typedef enum { SGBEM_MEM_RULES = 0, SGBEM_MEM_ASSEMBLE_WQ = 1, SGBEM_MEM_ASSEMBLE_EBE = 2,
               SGBEM_MEM_RHS_DIRECT = 3, SGBEM_MEM_SOLVE = 4, SGBEM_MEM_RULES_KNOTS = 5,
               SGBEM_MEM_RULES_OPEN = 6 } sgbem_memory_kind;
sgbem_status sgbem_memory_need(int32_t what, int32_t p, int32_t N, int32_t n_ref, int32_t n_gauss, int32_t n_ctrl,
                               int64_t *bytes);

/* Synchronise the stream, free every device buffer the context owns. */
sgbem_status sgbem_ctx_destroy(sgbem_ctx ctx);

/* Switch the stream used by later calls (the previous stream is synchronised). */
sgbem_status sgbem_ctx_set_stream(sgbem_ctx ctx, void *hip_stream);

/* Timing of the main kernel of every later assembly call: when `on`, the
 * tile kernel of each sgbem_assemble call (WQ: the fused sweep-and-contract
 * kernel; EBE: its far-pair kernel) and of each sgbem_batch_assemble call is
 * launched with a pair of HIP events that its own dispatch records at the start
 * and the end of its execution, on the context's stream.  Events are kept by
 * the context. */
sgbem_status sgbem_ctx_set_timing(sgbem_ctx ctx, int32_t on);

/* Wait for the recorded events and return the summed elapsed milliseconds and
 * the number of timed kernels since the last call (then forget them).
 * Errors: E_INVAL, E_DEVICE. */
sgbem_status sgbem_ctx_kernel_time(sgbem_ctx ctx, double *total_ms, int64_t *count);

/* Message of the last failing call on this host thread. */
const char *sgbem_last_error(void);

/* Library build string (architecture, build flags). */
const char *sgbem_version(void);

/* ---------------------------------------------------------------- rules */

/*
 * Build the quadrature rules of Section 4 for degree p, N elements and
 * refinement n_ref (the exactness space: B-splines of degree p on the knots
 * refined by splitting every element into n_ref equal parts, M = n_ref N
 * elements), and upload them to the device.  Synchronous.
 *  - knots: NULL for uniform periodic knots tau_k = k / N, else the N + 1
 *    breakpoints 0 = tau_0 < tau_1 < ... < tau_N = 1 of one period (host,
 *    read during the call), extended periodically (Section 3);
 *  - nodes (Section 4): all breakpoints and midpoints of the refined mesh,
 *    2M nodes (eta_n = n / (2M) for uniform knots);
 *  - regular rules (Alg. 1, eq. reg_exactness): minimum-norm weights on the
 *    2 n_ref (p+1) - 1 nodes inside supp B_i, exact for every refined
 *    Bbar_k meeting it;
 *  - singular rules (Alg. 2, eqs. sing_exactness, mod_mom_gen): for each source
 *    eta_m, minimum-norm weights on all nodes exact for int Bbar_k(t) K2(eta_m,t) dt,
 *    K2(s,t) = ln|sin(pi (s-t)) / pi| (the kernel split of Section 3.1 made
 *    periodic), modified moments from the closed forms of Section 4.2.
 *    With uniform periodic knots the weights depend only on (m mod 2, n - m mod 2M),
 *    so two tables of length 2M are kept; on non-uniform knots every test
 *    function has its own regular rule and the singular weights form a full
 *    2M x 2M table (32 M^2 bytes), built by host threads.
 * Limits: p in [1, 6], n_ref in [1, 4], N >= 2 (p + 1), 2 n_ref N <= 2^24;
 * non-uniform knots: 2 n_ref N <= 8192 (else E_UNSUPPORTED), and the rules
 * serve the FP64 fast form (sgbem_assemble with SGBEM_WQ, n_ref in {1, 2}),
 * sgbem_rhs with SGBEM_WQ and sgbem_rhs_points with SGBEM_WQ only (the other
 * entry points return E_UNSUPPORTED for them).
 * Errors: E_INVAL, E_NOMEM, E_DEVICE, E_SINGULAR (rank-deficient collocation),
 * E_UNSUPPORTED.  The handle is freed with sgbem_rules_free (or with its context).
 */
sgbem_status sgbem_weights(sgbem_ctx ctx, int32_t p, int32_t N, int32_t n_ref, const double *knots,
                           sgbem_rules *out);

sgbem_status sgbem_rules_free(sgbem_ctx ctx, sgbem_rules rules);

/* Host-only view of the same rules, without any device (for inspection):
 *  w0[Q]       regular weights of B_0 on nodes n = 1..Q, Q = 2 n_ref (p+1) - 1
 *              (B_i uses the same weights on nodes 2 n_ref i + 1 + q);
 *  bvals[Q]    B_0(eta_n) on the same nodes;
 *  ws[2][2M]   singular weights: w_n^(eta_m) = ws[m mod 2][(n - m) mod 2M].
 * Any output pointer may be NULL.  Errors: E_INVAL, E_NOMEM, E_SINGULAR. */
sgbem_status sgbem_weights_host(int32_t p, int32_t N, int32_t n_ref,
                                double *w0, double *bvals, double *ws);

/* Host-only view of the rules on non-uniform knots (same arguments as
 * sgbem_weights with knots): W[N][Q] regular weights of B_i on the nodes
 * 2 n_ref i + 1 + q (mod 2M), Bv[N][Q] B_i at those nodes, Ws[2M][2M] singular
 * weights (row m: source eta_m), eta[2M] node parameters.  Any output may be
 * NULL.  Errors: E_INVAL, E_NOMEM, E_SINGULAR, E_UNSUPPORTED. */
sgbem_status sgbem_weights_host_knots(int32_t p, int32_t N, int32_t n_ref, const double *knots,
                                      double *W, double *Bv, double *Ws, double *eta);

/*
 * Quadrature rules of Section 4 on an open arc (Section 2, exterior problem
 * in the indirect form eq. prima_BIE), uploaded to the device.  Synchronous.
 *  - approximation space (Section 3, eq. lift): all N = n_el + p B-splines of
 *    degree p on the clamped knot vector over the breakpoints
 *    breaks[0] = a < breaks[1] < ... < breaks[n_el] = b (host, read during the
 *    call); B_0(a) = B_{N-1}(b) = 1, B_i supported on [T_i, T_{i+p+1}];
 *  - exactness space: the same on the mesh refined by splitting every element
 *    into n_ref equal parts (M = n_ref n_el elements, M + p functions);
 *  - nodes (Section 4): p + 2 equally spaced points in the first and in the last
 *    refined element, breakpoints and midpoints elsewhere: n_q = 2p + 2M - 1;
 *  - regular rules (Alg. 1): for each B_i, minimum-norm weights on the nodes
 *    where B_i is non-zero (underdetermined where an end element is involved);
 *  - singular rules (Alg. 2): for each node as source s, minimum-norm weights on
 *    all nodes exact for int Bbar_k(t) ln|t - s| dt (K2 = ln|s - t| as printed in
 *    Section 3.1), modified moments in closed form (Section 4.2).
 * The matrix of sgbem_assemble with these rules keeps every entry of eq.
 * IK1e2_bis (it is not mirrored, so it is not exactly symmetric): each row
 * integrates the whole spline space, which a mirrored row would not.
 * Limits: p in [1, 6], n_ref in [1, 4], n_ref n_el >= 2, n_q <= 8192 (else
 * E_UNSUPPORTED); assembly kernels exist for n_ref in {1, 2}.
 * Errors: E_INVAL, E_NOMEM, E_DEVICE, E_SINGULAR, E_UNSUPPORTED.
 */
sgbem_status sgbem_weights_open(sgbem_ctx ctx, int32_t p, int32_t n_el, int32_t n_ref, const double *breaks,
                                sgbem_rules *out);

/* Host-only view of the open-arc rules (same arguments as sgbem_weights_open):
 * *q_max = Q_M, the row length 2 n_ref (p + 1) - 1 + 2p of W and Bv;
 * n0[N], cnt[N]: row i's support nodes n0[i] .. n0[i] + cnt[i] - 1;
 * W[N][Q_M] regular weights of B_i on them (zeros beyond cnt[i]), Bv[N][Q_M] B_i
 * there, Ws[n_q][n_q] singular weights (row m: source eta_m), eta[n_q] node
 * parameters.  Any output may be NULL (a first call with only q_max gives the
 * sizes).  Errors: E_INVAL, E_NOMEM, E_SINGULAR, E_UNSUPPORTED. */
sgbem_status sgbem_weights_host_open(int32_t p, int32_t n_el, int32_t n_ref, const double *breaks, int32_t *q_max,
                                     int32_t *n0, int32_t *cnt, double *W, double *Bv, double *Ws, double *eta);

/* Host-only reference matrices of the element-by-element near-pair rule
 * (Section 5, Remark): on unit elements with the 16 Gauss-Legendre points u_a
 * and Lagrange polynomials l_a, mco[a][b] = int_0^1 int_0^1 l_a(u) l_b(v) ln|u - v|,
 * madj[a][b] = int int l_a(u) l_b(v) ln(1 + v - u) (u left, v right element).
 * Outputs are [16][16] (or NULL); u16, w16 are the Gauss nodes / weights. */
sgbem_status sgbem_nearfield_host(double *u16, double *w16, double *mco, double *madj);

/* ---------------------------------------------------------------- assembly */

/*
 * Points where the Dirichlet datum g must be sampled for sgbem_rhs, written
 * to device memory d_xy as [count][2] FP64 (x, y):
 *   WQ:  f(eta_n), n = 0..2M-1                                   (count = 2M;
 *        open-arc rules: the n_q nodes of sgbem_weights_open)
 *   EBE: f((e + u_g) / N), e = 0..N-1, g = 0..n_gauss-1 (G-point Gauss-Legendre
 *        nodes on [0, 1])                                         (count = N n_gauss)
 * `cap` is the capacity of d_xy in points; *count receives the count (also
 * when cap is too small, then E_INVAL).  Asynchronous.
 */
sgbem_status sgbem_rhs_points(sgbem_ctx ctx, const sgbem_curve *curve, sgbem_rules rules,
                              int32_t method, int32_t n_gauss,
                              double *d_xy, int64_t cap, int64_t *count);

/*
 * Host-only: the fast form's node points f(eta_n), eta_n = n / (2 n_ref N),
 * n = 0 .. 2 n_ref N - 1 (Section 5), written to xy as [2 n_ref N][2] FP64, by
 * the same curve evaluation as the device's (last-bit differences in the
 * trigonometric functions are possible).  For clients that sample g on the host
 * (sgbem_rhs with SGBEM_WQ, sgbem_server_submit).  Errors: E_INVAL.
 */
sgbem_status sgbem_node_points_host(const sgbem_curve *curve, int32_t N, int32_t n_ref, double *xy);

/*
 * Assemble the N x N Galerkin matrix into device memory d_A (row-major, lda,
 * FP64 `double` or FP32 `float` as `precision` says).  Asynchronous.
 *  WQ (fast form): eqs. IK1e2 and IK1e2_bis by row assembly and sum
 *      factorisation (Alg. 3), the singular rule used for every pair as the paper
 *      does; K1 on the node grid with K1(s, s) = ln J(s) (eq. F1_lim).  The row of
 *      eq. IK1e2_bis is not exactly symmetric: rows i <= j are computed and
 *      mirrored, so d_A is exactly symmetric.  Open arcs (rules of
 *      sgbem_weights_open, a BSPLINE_OPEN curve on the same [a, b]): order
 *      N = n_el + p, K1(s, t) = ln(|f(s) - f(t)| / |s - t|), every entry of eq.
 *      IK1e2_bis computed (d_A not symmetric); FP64 only.
 *  EBE (plain form): eq. elbyelint; far element pairs by n_gauss x n_gauss
 *      Gauss-Legendre, coincident / adjacent pairs (the wrap pair included) by the
 *      kernel split: regular part with 16 x 16 Gauss, ln|s - t| part integrated
 *      exactly after interpolating B J at 16 Gauss points per element.
 * FP32: kernel values, products and sums in FP32 (node coordinates are
 *      differenced in FP64); the rule tables stay FP64 until rounded once.
 * Limits: n_gauss in [1, 8] for EBE (ignored by WQ).
 * Errors: E_INVAL (also: an open arc with closed-curve rules or the reverse, or
 *      an arc whose parameter interval is not the rules' [a, b]), E_UNSUPPORTED
 *      (a (p, n_ref) or (p, n_gauss) pair without a compiled kernel), E_NOMEM,
 *      E_DEVICE.
 */
sgbem_status sgbem_assemble(sgbem_ctx ctx, const sgbem_curve *curve, sgbem_rules rules,
                            int32_t method, int32_t n_gauss, int32_t precision,
                            void *d_A, int64_t lda);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fast
 * form of sgbem_assemble (method SGBEM_WQ, same kernels, same results) with
 * no allocation of any kind.  The node geometry (f and J on the 2 n_ref N
 * nodes), which sgbem_assemble keeps in a buffer of the context, goes to a
 * fixed device array of the library instead: SGBEM_NOALLOC_MAX_NODES nodes
 * (3 doubles each, 1.5 MiB), one array per device, held until the process
 * ends; its address is looked up when the first context on the device is
 * created.  Every call on one device shares that array: calls that overlap
 * on one device (two streams, or two host threads) race, and the caller
 * must order them.  Nothing in it needs clearing between calls (every node
 * is written before it is read).  The curve must travel inline (polar, or
 * B-spline with at most 64 control points).  Kernel timing
 * (sgbem_ctx_set_timing) does not apply.  Asynchronous, launches only.
 * Errors: E_INVAL (2 n_ref N > SGBEM_NOALLOC_MAX_NODES, or the arguments of
 *      sgbem_assemble), E_UNSUPPORTED (a curve that does not travel inline, a
 *      (p, n_ref) without a compiled kernel), E_DEVICE.
 */
#define SGBEM_NOALLOC_MAX_NODES 65536
sgbem_status sgbem_assemble_noalloc(sgbem_ctx ctx, const sgbem_curve *curve, sgbem_rules rules,
                                    int32_t precision, void *d_A, int64_t lda);

/*
 * Right-hand side beta_i = int B_i J g(f) ds (eq. final_b1), FP64:
 *  WQ:  sum_n w_n^(i) J(eta_n) g_n (Section 5);   EBE: G-point Gauss per element.
 *  Open arcs: the WQ form with the rules of sgbem_weights_open (the right-hand
 *  side int B_i J u_D of the indirect form on the arc), d_beta [n_el + p].
 * d_g: device [count] FP64 samples of g at the sgbem_rhs_points of the same
 * method / n_gauss; d_beta: device [N] FP64.  Asynchronous.  Errors: E_INVAL.
 */
sgbem_status sgbem_rhs(sgbem_ctx ctx, const sgbem_curve *curve, sgbem_rules rules,
                       int32_t method, int32_t n_gauss, const double *d_g, double *d_beta);

/*
 * Right-hand side of the direct formulation (Section 2, eq. seconda_BIE in the
 * weak form eq. weakpb), whose solution with the sgbem_assemble matrix is the
 * outward flux q = du/dn:  F_i = b1_i / 2 - b2_i / (2 pi), FP64, with b1 of
 * eq. final_b1 and b2 of eq. final_b2,
 *   b2_i = int B_i(s) J(s) int Kbar(s, t) u_D(t) dt ds,
 *   Kbar(s, t) = [(f1(t) - f1(s)) f2'(t) - (f2(t) - f2(s)) f1'(t)] / |f(s) - f(t)|^2
 * (the normal derivative of ln|x - y| for the outward normal of a
 * counter-clockwise curve, times J(t); the expression printed in Section 3.2
 * has the opposite sign, that of a clockwise parametrisation), by the rule of
 * Section 5: the regular weighted rule of `rules` outside, composite
 * Gauss-Legendre with n_gauss points per element inside.
 *  d_g_nodes: device [2 n_ref N] FP64, u_D at sgbem_rhs_points(SGBEM_WQ);
 *  d_g_gauss: device [N n_gauss] FP64, u_D at sgbem_rhs_points(SGBEM_EBE, n_gauss);
 *  d_F: device [N] FP64 (output); d_b2: device [N] FP64 or NULL (b2 alone).
 * n_gauss in {2, 4, 6, 8} (even, so that no Gauss point falls on a node).
 * Needs a curve with continuous curvature (Section 3.2); workspace of
 * (5 N n_gauss + (chunks + 2) 2 n_ref N) doubles is kept by the context.
 * Asynchronous.  Errors: E_INVAL, E_NOMEM, E_DEVICE.
 */
sgbem_status sgbem_rhs_direct(sgbem_ctx ctx, const sgbem_curve *curve, sgbem_rules rules, int32_t n_gauss,
                              const double *d_g_nodes, const double *d_g_gauss, double *d_F, double *d_b2);

/*
 * Collocation BEM with the same rules (Conclusions: the outer collocation node
 * fixed, the new rules for the inner integral): the N x N matrix, FP64,
 * row-major in d_A with lda,
 *   A_ij = -1/(2 pi) [ sum_n w_n^(j) K1(x_i, eta_n) J(eta_n)          (Alg. 1 rule of B_j)
 *                      + sum_n w_n^(x_i) J(eta_n) B_j(eta_n) ]        (Alg. 2 rule at x_i),
 * the single-layer equation V phi = u_D collocated at the Greville abscissae
 * x_i = (i + (p+1)/2) / N, which are the nodes 2 n_ref i + n_ref (p+1) of
 * sgbem_rhs_points(SGBEM_WQ).  Not symmetric.  n_ref in {1, 2}.  Asynchronous.
 * Errors: E_INVAL, E_UNSUPPORTED, E_NOMEM, E_DEVICE.
 */
sgbem_status sgbem_assemble_collocation(sgbem_ctx ctx, const sgbem_curve *curve, sgbem_rules rules,
                                        double *d_A, int64_t lda);

/* Right-hand side of the collocation system: d_b[i] = u_D(x_i) picked from
 * d_g_nodes (device [2 n_ref N] FP64, u_D at sgbem_rhs_points(SGBEM_WQ));
 * d_b: device [N] FP64.  Asynchronous.  Errors: E_INVAL. */
sgbem_status sgbem_collocation_rhs(sgbem_ctx ctx, sgbem_rules rules, const double *d_g_nodes, double *d_b);

/* ---------------------------------------------------------------- batches */

/*
 * Describe a batch of n curves for the fast form (eqs. IK1e2, IK1e2_bis,
 * Alg. 3), each with its own rules (n_ref = 1, p in {2, 3, 4}, any N) and its
 * own output matrix d_A[b] (device, row-major, lda[b], FP64 or FP32 as
 * `precision`).  Everything the launch needs (curve descriptions, rule
 * pointers, support coefficients, the tile index space) is uploaded once to
 * device memory owned by the batch, so sgbem_batch_assemble enqueues kernel
 * launches only and can be captured in a HIP graph.  The rules handles and the
 * output buffers must outlive the batch.  Curves: polar, or B-spline with at
 * most 64 control points.  Synchronous.
 * Errors: E_INVAL, E_UNSUPPORTED, E_NOMEM, E_DEVICE.
 */
sgbem_status sgbem_batch_create(sgbem_ctx ctx, int32_t n, const sgbem_curve *curves, const sgbem_rules *rules,
                                int32_t precision, void *const *d_A, const int64_t *lda, sgbem_batch *out);

/* Assemble every matrix of the batch: one geometry launch for all curves and
 * one persistent launch that strides over the upper-triangle tiles of all
 * matrices (curves of different degree and size in the same launch), with the
 * tile shape chosen by sgbem_batch_tune (default: 32 x 32 tiles, 8-column
 * strips).  Asynchronous; same results as sgbem_assemble per curve. */
sgbem_status sgbem_batch_assemble(sgbem_ctx ctx, sgbem_batch batch);

/* Autotuner: time every compiled tile shape (32x32 / 16x16 tiles, strips of
 * 4 to 16 columns, grid sized from the kernel's occupancy) on this batch, reps
 * launches each, keep the fastest for the batch and as the context's default
 * for later batches of the same precision.  Synchronous; writes the outputs. */
sgbem_status sgbem_batch_tune(sgbem_ctx ctx, sgbem_batch batch, int32_t reps, int32_t *best_cfg, double *best_ms);

sgbem_status sgbem_batch_free(sgbem_ctx ctx, sgbem_batch batch);

/* ---------------------------------------------------------------- solve */

/*
 * Solve A x = beta (eq. sistlin) for one N x N matrix on the device.
 * A is LU-factorised in FP32; x is then refined in FP64: r = beta - A x with
 * A as stored (FP64 or FP32 widened), d = LU \ r in FP32, x += d, until
 * ||d||_inf <= tol ||x||_inf or max_iter steps (or a correction does not
 * halve with the backward error at the FP64 rounding level).
 * Factorisation: an exactly symmetric A with N <= 16384 (the Galerkin matrix,
 * positive definite in the paper's setting, eq. sistlin) is first factored
 * without row interchanges, which is stable for a positive definite matrix;
 * that attempt is kept only if the refinement converges.  A zero pivot or a
 * stalled refinement (above the FP64 level a correction that does not shrink,
 * or two in a row that do not halve; possible when the curve's logarithmic
 * capacity is near or above 1 and A is nearly singular or indefinite) means a
 * refactorisation with partial pivoting, which every other matrix gets from
 * the start.  info->pivoted says which was used.
 *  d_A:     device, row-major, lda, FP64 or FP32 per a_prec; not modified.
 *  d_beta:  device [N] FP64.    d_x: device [N] FP64 (output).
 *  info:    host, may be NULL; written before return (the call synchronises).
 * Workspace (4 N^2 + O(N) bytes, sgbem_memory_need) is allocated in the
 * context and kept, as is a small pinned host buffer the kernels write the
 * refinement's results to.
 * Errors: E_INVAL, E_NOMEM, E_SINGULAR (zero pivot), E_NOCONV (x holds the
 *      last iterate), E_DEVICE.
 */
sgbem_status sgbem_solve(sgbem_ctx ctx, int32_t N, const void *d_A, int64_t lda, int32_t a_prec,
                         const double *d_beta, double *d_x, double tol, int32_t max_iter,
                         sgbem_solve_info *info);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous-batching server: a stream of independent problems (curve, p, N,
 * Dirichlet data), each assembled by the fast form in the configured precision
 * (eqs. IK1e2, IK1e2_bis, Alg. 3), its right-hand side formed (eq. final_b1)
 * and the system (eq. sistlin) solved like sgbem_solve.  Threads of the library
 * do the work: a dispatcher releases each request at its arrival time and
 * admits it, first in first out, when one of `workers` slots is free and its
 * device footprint fits into the free space of a device arena of
 * `budget_bytes` (allocated once at creation; nothing is allocated per
 * request).  Each slot is a host thread with its own HIP stream, so the kernels
 * of admitted requests overlap on the device.  Quadrature rules are built on
 * first use of a (p, N) by the slot that needs them and kept in a device cache
 * of `max_rules` entries (least recently used evicted when unused).
 * Per-request results are the same as running the request alone.
 */
typedef struct sgbem_server_s *sgbem_server;

typedef struct {
    int32_t device;
    int32_t workers;        /* concurrent requests, 1 .. 64                        */
    int64_t budget_bytes;   /* device arena for admitted requests                 */
    int32_t precision;      /* storage of the assembled matrix (SGBEM_FP64 / FP32) */
    int32_t max_N;          /* largest N accepted                                 */
    int32_t max_rules;      /* rule-cache entries, at least 2 workers + 1         */
    int32_t max_iter;       /* refinement limit of each solve                     */
    double tol;             /* refinement tolerance of each solve                 */
} sgbem_server_config;

typedef struct {
    sgbem_curve curve;      /* copied by submit (arrays included)                 */
    int32_t p;              /* spline degree, 1 .. 6                              */
    int32_t N;              /* elements, 2 (p + 1) .. max_N                       */
    const double *g;        /* host [2N]: g(f(n / 2N)), see sgbem_node_points_host; copied */
    double *x;              /* host [N]: alpha, written before the completion is posted */
    double arrival_s;       /* release time on the server clock (sgbem_server_clock) */
    uint64_t tag;           /* returned with the completion                       */
} sgbem_request;

typedef struct {
    uint64_t tag;
    int32_t status;         /* sgbem_status of the request                        */
    int32_t iters;          /* refinement steps                                   */
    double t_arrival;       /* server clock, seconds: release ...                 */
    double t_admit;         /*   ... admission (memory and slot granted) ...      */
    double t_done;          /*   ... result in x                                  */
    double backward_err;
    int64_t footprint;      /* device bytes the request held                      */
    char message[96];       /* error text when status != SGBEM_OK                 */
} sgbem_completion;

typedef struct {
    int64_t submitted, rejected, completed, failed;
    int32_t waiting;        /* submitted, not admitted (released or not)          */
    int32_t in_flight;      /* admitted, not completed                            */
    int32_t peak_in_flight;
    int32_t rules_cached;
    int64_t arena_bytes;    /* budget_bytes                                       */
    int64_t peak_bytes;     /* high-water mark of the admitted footprints         */
    int64_t rules_hits, rules_misses;
} sgbem_server_info;

/* Device bytes one request of size N holds while admitted (host-only):
 * A (N^2 in the matrix precision) + the solve workspace (4 N^2 + O(N)) + g,
 * beta and x, each part 256-byte aligned.  Errors: E_INVAL. */
sgbem_status sgbem_server_footprint(int32_t N, int32_t precision, int64_t *bytes);

/* Create the server (allocates the arenas, starts the threads).
 * Errors: E_INVAL (a field out of range), E_NOMEM, E_DEVICE. */
sgbem_status sgbem_server_create(const sgbem_server_config *config, sgbem_server *out);

/* Queue a request.  Rejected with E_NOMEM when its footprint exceeds the
 * arena (it could never be admitted), E_INVAL / E_UNSUPPORTED for bad
 * arguments (E_UNSUPPORTED: a B-spline curve of more than 64 control points,
 * which would need device memory of its own); a rejected request produces no
 * completion. */
sgbem_status sgbem_server_submit(sgbem_server s, const sgbem_request *req);

/* Move up to cap completions into out (oldest first), waiting up to
 * timeout_s seconds for the first one.  *n receives the number moved. */
sgbem_status sgbem_server_poll(sgbem_server s, sgbem_completion *out, int32_t cap, double timeout_s, int32_t *n);

/* Seconds since the server was created (the clock of arrival_s and t_*). */
sgbem_status sgbem_server_clock(sgbem_server s, double *now_s);

sgbem_status sgbem_server_stats(sgbem_server s, sgbem_server_info *out);

/* Stop: requests not yet admitted are dropped (no completion), admitted ones
 * finish; then the threads end and the arenas are freed. */
sgbem_status sgbem_server_destroy(sgbem_server s);

#ifdef __cplusplus
}
#endif

#endif /* SGBEM_H */
