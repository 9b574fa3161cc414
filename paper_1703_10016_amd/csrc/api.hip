// C ABI of libsgbem (declared in include/sgbem.h): contexts, rule handles,
// argument validation and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sgbem.h"
#include "ctx.hpp"
#include "kernels.hpp"
#include "planner.hpp"
#include "solve.hpp"
#include "batch.hpp"
#include "curve_eval.hpp"
#include "dlayer.hpp"
#include "colloc.hpp"
#include "knots.hpp"
#include "arc.hpp"

namespace sgbem {
hipError_t launch_wq_f64(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev);
hipError_t launch_wq_f32(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev);
hipError_t launch_ebe_f64(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev);
hipError_t launch_ebe_f32(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev);

hipError_t launch_assemble(int method, int prec, int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev)
{
    if (method == 0) return prec == 0 ? launch_wq_f64(p, P, a, s, ev) : launch_wq_f32(p, P, a, s, ev);
    return prec == 0 ? launch_ebe_f64(p, P, a, s, ev) : launch_ebe_f32(p, P, a, s, ev);
}
bool assemble_supported(int method, int, int p, int P)
{
    if (p < 1 || p > 6) return false;
    if (method == 0) return P == 2 || P == 4 || P == 6 || P == 8;
    return P >= 1 && P <= 8;
}
}  // namespace sgbem

using namespace sgbem;

// Node geometry of sgbem_assemble_noalloc (X, Y, J of up to
// SGBEM_NOALLOC_MAX_NODES nodes): a fixed array, one copy per device, held
// until the process ends.  Host code never uses this name as an address: it
// passes the device address that scratch_address() looked up.
static __device__ __align__(256) double scratch[3 * SGBEM_NOALLOC_MAX_NODES];

namespace {
thread_local std::string g_err;

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_addr;   // device address of `scratch`, per device (nullptr: not looked up)
}  // namespace

namespace sgbem {

sgbem_status set_err(sgbem_status st, const std::string &m)
{
    g_err = m;
    return st;
}

size_t buf_bytes(size_t bytes)
{
    const size_t nb = bytes < 4096 ? 4096 : bytes;
    return (nb + 4095) & ~size_t(4095);
}

sgbem_status budget_check(sgbem_ctx c, size_t bytes, size_t releasing)
{
    if (c->budget == 0) return SGBEM_OK;
    const uint64_t after = c->held - releasing + bytes;
    if (after <= c->budget) return SGBEM_OK;
    char m[200];
    std::snprintf(m, sizeof m, "context HBM budget: %llu bytes needed, %llu held of %llu",
                  (unsigned long long)bytes, (unsigned long long)c->held, (unsigned long long)c->budget);
    return set_err(SGBEM_E_NOMEM, m);
}

sgbem_status ctx_malloc(sgbem_ctx c, void **p, size_t bytes)
{
    *p = nullptr;
    sgbem_status st = budget_check(c, bytes, 0);
    if (st) return st;
    HIPCHK(hipMalloc(p, bytes));
    c->held += bytes;
    return SGBEM_OK;
}

void ctx_free(sgbem_ctx c, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    c->held -= bytes;
}

sgbem_status ensure_hbuf(sgbem_ctx c)
{
    if (c->hbuf) return SGBEM_OK;
    void *p = nullptr;
    HIPCHK(hipHostMalloc(&p, kSolveHostDoubles * sizeof(double), hipHostMallocCoherent));
    c->hbuf = static_cast<double *>(p);
    return SGBEM_OK;
}

sgbem_status ensure(sgbem_ctx c, DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes) return SGBEM_OK;
    const size_t nb = buf_bytes(bytes);
    sgbem_status st = budget_check(c, nb, b.bytes);
    if (st) return st;
    if (b.ptr) {
        HIPCHK(hipStreamSynchronize(c->stream));
        ctx_free(c, b.ptr, b.bytes);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    void *q = nullptr;
    if ((st = ctx_malloc(c, &q, nb))) return st;
    b.ptr = q;
    b.bytes = nb;
    return SGBEM_OK;
}

namespace {
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

size_t rules_block_bytes(int64_t npts)
{
    const size_t n = size_t(npts);
    return align256(n * 8) + align256(2 * n * 8) + align256(64 * 8) + align256(n * 4) + align256(2 * n * 4);
}

size_t knot_rules_block_bytes(int N, int R, int p)
{
    const size_t Q = size_t(2 * R * (p + 1) - 1), nn = size_t(2) * R * N;
    return 2 * align256(size_t(N) * Q * 8) + align256(nn * nn * 8) + align256(nn * 8);
}

size_t open_rules_block_bytes(int n_el, int R, int p)
{
    const size_t N = size_t(n_el) + size_t(p), QM = size_t(arc_qm(p, 2 * R));
    const size_t nn = size_t(2 * p) + size_t(2) * R * size_t(n_el) - 1;
    return 2 * align256(N * QM * 8) + align256(nn * nn * 8) + align256(nn * 8) + 2 * align256(N * 4);
}

void free_rules(sgbem_rules r)
{
    if (!r) return;
    if (r->owned) (void)hipFree(r->block);
    delete r;
}

sgbem_status make_rules(int p, int N, int R, void *block, hipStream_t stream, sgbem_rules &out)
{
    out = nullptr;
    WQRules W;
    try {
        W = build_wq_rules(p, N, R);
    } catch (const PlanError &e) {
        return set_err(sgbem_status(e.status), e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    auto *r = new (std::nothrow) sgbem_rules_s;
    if (!r) return set_err(SGBEM_E_NOMEM, "host allocation failed");
    r->p = p;
    r->N = N;
    r->R = R;
    r->Q = W.Q;
    r->M = W.M;
    r->npts = W.n_nodes;
    r->w0 = W.w0;
    r->bvals = W.bvals;
    const size_t n = size_t(W.n_nodes);
    std::vector<float> f_inv(n), f_ws(2 * n);
    for (size_t i = 0; i < n; ++i) f_inv[i] = float(W.inv_s2[i]);
    for (size_t i = 0; i < 2 * n; ++i) f_ws[i] = float(W.ws[i]);
    hipError_t e = hipSuccess;
    if (block) {
        r->block = block;
    } else {
        e = hipMalloc(&r->block, rules_block_bytes(W.n_nodes));
        r->owned = e == hipSuccess;
    }
    if (e == hipSuccess) {
        char *b = static_cast<char *>(r->block);
        r->d_inv_s2 = reinterpret_cast<double *>(b);
        b += align256(n * 8);
        r->d_ws = reinterpret_cast<double *>(b);
        b += align256(2 * n * 8);
        r->d_w0 = reinterpret_cast<double *>(b);
        b += align256(64 * 8);
        r->d_inv_s2f = reinterpret_cast<float *>(b);
        b += align256(n * 4);
        r->d_wsf = reinterpret_cast<float *>(b);
    }
    // pageable sources: each copy has completed when hipMemcpyAsync returns or at the final synchronisation
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_inv_s2, W.inv_s2.data(), n * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_ws, W.ws.data(), 2 * n * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_w0, W.w0.data(), W.w0.size() * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_inv_s2f, f_inv.data(), n * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_wsf, f_ws.data(), 2 * n * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        free_rules(r);
        return set_err(e == hipErrorOutOfMemory ? SGBEM_E_NOMEM : SGBEM_E_DEVICE,
                       std::string("uploading rules: ") + hipGetErrorString(e));
    }
    out = r;
    return SGBEM_OK;
}

bool valid_rules(sgbem_ctx c, sgbem_rules r)
{
    if (r && r->shared) return true;
    for (auto *x : c->rules)
        if (x == r) return true;
    return false;
}

}  // namespace sgbem

namespace {

}  // namespace

namespace sgbem {
sgbem_status check_curve(const sgbem_curve *c, bool open)
{
    if (!c) return set_err(SGBEM_E_INVAL, "curve is NULL");
    if (open && c->kind != SGBEM_CURVE_BSPLINE_OPEN)
        return set_err(SGBEM_E_INVAL, "rules of sgbem_weights_open need an open arc (SGBEM_CURVE_BSPLINE_OPEN)");
    if (c->kind == SGBEM_CURVE_BSPLINE_OPEN) {
        if (!open)
            return set_err(SGBEM_E_INVAL, "an open arc needs the rules of sgbem_weights_open and the fast form");
        const int d = c->degree, n = c->n_ctrl;
        if (d < 1 || d > 7) return set_err(SGBEM_E_INVAL, "B-spline curve degree must be in [1, 7]");
        if (n <= d) return set_err(SGBEM_E_INVAL, "B-spline curve needs n_ctrl > degree");
        if (!c->ctrl_xy || !c->knots) return set_err(SGBEM_E_INVAL, "open arc without control points or knots");
        const double *k = c->knots;
        const double a = k[0], b = k[n + d];
        if (!std::isfinite(a) || !std::isfinite(b) || !(b > a)) return set_err(SGBEM_E_INVAL, "open arc: knots[0] < knots[n_ctrl + d] needed");
        for (int i = 0; i <= d; ++i)
            if (k[i] != a || k[n + i] != b)
                return set_err(SGBEM_E_INVAL, "open arc: the first and the last d + 1 knots must be equal (clamped)");
        for (int i = d; i < n; ++i)
            if (!(k[i + 1] > k[i])) return set_err(SGBEM_E_INVAL, "open arc: inner knots must be strictly increasing");
    } else if (c->kind == SGBEM_CURVE_BSPLINE) {
        if (c->degree < 1 || c->degree > 7) return set_err(SGBEM_E_INVAL, "B-spline curve degree must be in [1, 7]");
        if (c->n_ctrl <= c->degree) return set_err(SGBEM_E_INVAL, "B-spline curve needs n_ctrl > degree");
        if (!c->ctrl_xy) return set_err(SGBEM_E_INVAL, "B-spline curve without control points");
        if (c->knots) {
            const double *k = c->knots;
            if (k[0] != 0.0 || k[c->n_ctrl] != 1.0)
                return set_err(SGBEM_E_INVAL, "B-spline knots must run from 0 to 1 over one period");
            for (int i = 0; i < c->n_ctrl; ++i)
                if (!(k[i + 1] > k[i])) return set_err(SGBEM_E_INVAL, "B-spline knots must be strictly increasing");
        }
    } else if (c->kind == SGBEM_CURVE_POLAR) {
        if (!(c->r0 > 0.0)) return set_err(SGBEM_E_INVAL, "polar curve needs r0 > 0");
        if (c->n_modes < 0 || c->n_modes > 64) return set_err(SGBEM_E_INVAL, "polar curve n_modes must be in [0, 64]");
        if (c->n_modes > 0 && (!c->a || !c->phi)) return set_err(SGBEM_E_INVAL, "polar curve modes missing");
        double amp = 0.0;
        for (int k = 0; k < c->n_modes; ++k) amp += std::fabs(c->a[k]);
        if (!(amp < 1.0)) return set_err(SGBEM_E_INVAL, "polar curve: sum |a_k| must be < 1 so that r > 0");
    } else {
        return set_err(SGBEM_E_INVAL, "unknown curve kind");
    }
    return SGBEM_OK;
}

}  // namespace sgbem

namespace {

// Device description of a curve whose arrays fit the inline storage.
sgbem_status inline_curve(const sgbem_curve *cv, CurveDev &d, bool open = false)
{
    sgbem_status st = check_curve(cv, open);
    if (st) return st;
    std::memset(&d, 0, sizeof d);
    d.kind = cv->kind;
    d.inline_data = 1;
    if (cv->kind == SGBEM_CURVE_BSPLINE_OPEN) {
        if (cv->n_ctrl > 64) return set_err(SGBEM_E_UNSUPPORTED, "a curve that travels inline has at most 64 control points");
        d.degree = cv->degree;
        d.n_ctrl = cv->n_ctrl;
        std::memcpy(d.inl, cv->ctrl_xy, size_t(cv->n_ctrl) * 2 * sizeof(double));
        std::memcpy(d.inl + 128, cv->knots, size_t(cv->n_ctrl + cv->degree + 1) * sizeof(double));
    } else if (cv->kind == SGBEM_CURVE_BSPLINE) {
        if (cv->n_ctrl > 64) return set_err(SGBEM_E_UNSUPPORTED, "a curve that travels inline has at most 64 control points");
        d.degree = cv->degree;
        d.n_ctrl = cv->n_ctrl;
        std::memcpy(d.inl, cv->ctrl_xy, size_t(cv->n_ctrl) * 2 * sizeof(double));
        if (cv->knots) {
            d.nonuniform = 1;
            std::memcpy(d.inl + 128, cv->knots, size_t(cv->n_ctrl + 1) * sizeof(double));
        }
    } else {
        d.r0 = cv->r0;
        d.n_modes = cv->n_modes;
        if (cv->n_modes > 0) {
            std::memcpy(d.inl, cv->a, size_t(cv->n_modes) * sizeof(double));
            std::memcpy(d.inl + 64, cv->phi, size_t(cv->n_modes) * sizeof(double));
        }
    }
    return SGBEM_OK;
}

int batch_grid(sgbem_ctx c, int cfg, int prec, int total)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1) cus = 256;
    const int g = batch_blocks_per_cu(cfg, prec) * cus;
    return total < g ? (total > 0 ? total : 1) : g;
}

bool valid_batch(sgbem_ctx c, sgbem_batch b)
{
    for (auto *x : c->batches)
        if (x == b) return true;
    return false;
}

// With `device` current: the device address of that device's copy of
// `scratch`, looked up once per device and kept.
sgbem_status scratch_address(int device, double *&out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    try {
        if (int(g_scratch_addr.size()) <= device) g_scratch_addr.resize(size_t(device) + 1, nullptr);
    } catch (...) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_err(SGBEM_E_DEVICE, "hipGetSymbolAddress returned no address for the fixed geometry array");
        g_scratch_addr[device] = static_cast<double *>(p);
    }
    out = g_scratch_addr[device];
    return SGBEM_OK;
}

// Upload the curve's arrays and return the device description.
sgbem_status upload_curve(sgbem_ctx c, const sgbem_curve *cv, CurveDev &d, bool open = false)
{
    sgbem_status st = check_curve(cv, open);
    if (st) return st;
    std::memset(&d, 0, sizeof d);
    d.kind = cv->kind;
    if ((cv->kind == SGBEM_CURVE_BSPLINE || cv->kind == SGBEM_CURVE_BSPLINE_OPEN) && cv->n_ctrl <= 64)
        return inline_curve(cv, d, open);
    if (cv->kind == SGBEM_CURVE_POLAR) {
        d.r0 = cv->r0;
        d.n_modes = cv->n_modes;
        d.inline_data = 1;
        if (cv->n_modes > 0) {
            std::memcpy(d.inl, cv->a, size_t(cv->n_modes) * sizeof(double));
            std::memcpy(d.inl + 64, cv->phi, size_t(cv->n_modes) * sizeof(double));
        }
        return SGBEM_OK;
    }
    {
        // control points, then the knots of a non-uniform curve or of an open arc
        d.degree = cv->degree;
        d.n_ctrl = cv->n_ctrl;
        const bool arc = cv->kind == SGBEM_CURVE_BSPLINE_OPEN;
        const size_t bc = size_t(cv->n_ctrl) * 2 * sizeof(double);
        const size_t bk = cv->knots ? size_t(cv->n_ctrl + 1 + (arc ? cv->degree : 0)) * sizeof(double) : 0;
        if ((st = ensure(c, c->params, bc + bk))) return st;
        HIPCHK(hipMemcpyAsync(c->params.ptr, cv->ctrl_xy, bc, hipMemcpyHostToDevice, c->stream));
        d.ctrl = static_cast<const double *>(c->params.ptr);
        if (cv->knots) {
            double *kd = static_cast<double *>(c->params.ptr) + 2 * size_t(cv->n_ctrl);
            HIPCHK(hipMemcpyAsync(kd, cv->knots, bk, hipMemcpyHostToDevice, c->stream));
            d.knots = kd;
            d.nonuniform = arc ? 0 : 1;
        }
    }
    return SGBEM_OK;
}

sgbem_status geometry(sgbem_ctx c, const CurveDev &cd, const GridDesc &g, DevBuf &buf, double *&X, double *&Y, double *&J)
{
    sgbem_status st = ensure(c, buf, size_t(g.npts) * 3 * sizeof(double));
    if (st) return st;
    X = static_cast<double *>(buf.ptr);
    Y = X + g.npts;
    J = Y + g.npts;
    HIPCHK(launch_geometry(cd, g, X, Y, J, c->stream));
    return SGBEM_OK;
}

GridDesc wq_grid(sgbem_rules r)
{
    GridDesc g{};
    g.N = r->N;
    g.P = 0;
    g.npts = int(r->npts);
    g.tpar = (r->knots || r->open) ? r->d_eta : nullptr;   // non-uniform knots, open arcs: the node parameters
    return g;
}

// Tile-kernel arguments of the fast form: node geometry X, Y, J on the grid of
// r, the rule tables and the support coefficients (output fields left to the caller).
void wq_tile_args(sgbem_rules r, const double *X, const double *Y, const double *J, TileArgs &ta)
{
    ta.npts = int(r->npts);
    ta.X = X;
    ta.Y = Y;
    ta.J = J;
    ta.inv_s2 = r->d_inv_s2;
    ta.ws = r->d_ws;
    ta.inv_s2f = r->d_inv_s2f;
    ta.wsf = r->d_wsf;
    for (int q = 0; q < r->Q; ++q) {
        ta.coefA[q] = r->w0[q];
        ta.coefB[q] = r->bvals[q];
    }
}

GridDesc gauss_grid(int N, int G)
{
    GridDesc g{};
    g.N = N;
    g.P = G;
    g.npts = N * G;
    double w[32];
    gauss_legendre01(G, g.off, w);
    return g;
}

// Device copy of a host table, made once per key and kept by the context
// (a synchronous upload the first time a key is used).
sgbem_status cached_table(sgbem_ctx c, int key, const std::vector<double> &host, const double *&dev)
{
    auto it = c->tables.find(key);
    if (it != c->tables.end()) {
        dev = it->second;
        return SGBEM_OK;
    }
    void *dv = nullptr;
    const size_t nb = buf_bytes(host.size() * sizeof(double));
    sgbem_status st = ctx_malloc(c, &dv, nb);
    if (st) return st;
    double *d = static_cast<double *>(dv);
    hipError_t e = hipMemcpy(d, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx_free(c, d, nb);
        return set_err(SGBEM_E_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
    }
    c->tables[key] = d;
    dev = d;
    return SGBEM_OK;
}

std::vector<double> near_table(int p)
{
    const std::vector<double> pcs = cardinal_pieces(p);
    const NearField &nf = nearfield16();
    std::vector<double> tab(544 + size_t(p + 1) * 16);
    std::memcpy(&tab[0], nf.u, 16 * sizeof(double));
    std::memcpy(&tab[16], nf.w, 16 * sizeof(double));
    std::memcpy(&tab[32], nf.mco, 256 * sizeof(double));
    std::memcpy(&tab[288], nf.madj, 256 * sizeof(double));
    for (int a = 0; a <= p; ++a)
        for (int q = 0; q < 16; ++q) tab[544 + a * 16 + q] = cardinal_eval(p, pcs, a + nf.u[q]);
    return tab;
}

// w_g M_p(a + u_g) for a = 0..p, g = 0..G-1 (index a G + g).
std::vector<double> gauss_basis_coef(int p, int G)
{
    const std::vector<double> pcs = cardinal_pieces(p);
    double gx[32], gw[32];
    gauss_legendre01(G, gx, gw);
    std::vector<double> coef(size_t(G) * (p + 1));
    for (int a = 0; a <= p; ++a)
        for (int q = 0; q < G; ++q) coef[a * G + q] = gw[q] * cardinal_eval(p, pcs, a + gx[q]);
    return coef;
}

// When timing is on: the next pair of the context's events, to be recorded by
// the main kernel's own dispatch (execution start and end); kev stays NULL
// when timing is off.
sgbem_status timing_events(sgbem_ctx c, KernelEvents &ke, const KernelEvents *&kev)
{
    kev = nullptr;
    if (!c->timing) return SGBEM_OK;
    while (c->ev.size() < c->ev_used + 2) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->ev.push_back(e);
    }
    ke.start = c->ev[c->ev_used++];
    ke.stop = c->ev[c->ev_used++];
    kev = &ke;
    return SGBEM_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *sgbem_last_error(void) { return g_err.c_str(); }

const char *sgbem_version(void)
{
    return "libsgbem 1.0 (gfx950)";
}

sgbem_status sgbem_ctx_create(int32_t device, void *hip_stream, uint64_t hbm_budget_bytes, sgbem_ctx *out)
{
    if (!out) return set_err(SGBEM_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return set_err(SGBEM_E_INVAL, "no such HIP device");
    double *scr = nullptr;
    {
        DeviceGuard g(device);
        sgbem_status st = scratch_address(device, scr);
        if (st) return st;
    }
    auto *c = new (std::nothrow) sgbem_ctx_s;
    if (!c) return set_err(SGBEM_E_NOMEM, "host allocation failed");
    c->device = device;
    c->noalloc_scratch = scr;
    c->budget = hbm_budget_bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    return SGBEM_OK;
}

sgbem_status sgbem_ctx_memory(sgbem_ctx c, int64_t *held_bytes, int64_t *budget_bytes)
{
    if (!c) return set_err(SGBEM_E_INVAL, "ctx is NULL");
    if (held_bytes) *held_bytes = int64_t(c->held);
    if (budget_bytes) *budget_bytes = int64_t(c->budget);
    return SGBEM_OK;
}

sgbem_status sgbem_memory_need(int32_t what, int32_t p, int32_t N, int32_t n_ref, int32_t n_gauss, int32_t n_ctrl,
                               int64_t *bytes)
{
    if (!bytes) return set_err(SGBEM_E_INVAL, "bytes is NULL");
    *bytes = 0;
    if (N < 1 || N > (1 << 24) || n_ctrl < 0) return set_err(SGBEM_E_INVAL, "bad N or n_ctrl");
    const bool need_rules = what == SGBEM_MEM_RULES || what == SGBEM_MEM_ASSEMBLE_WQ || what == SGBEM_MEM_RHS_DIRECT ||
                            what == SGBEM_MEM_RULES_KNOTS || what == SGBEM_MEM_RULES_OPEN;
    if (need_rules && (n_ref < 1 || n_ref > 4)) return set_err(SGBEM_E_INVAL, "n_ref must be in [1, 4]");
    if (what != SGBEM_MEM_SOLVE && (p < 1 || p > 6)) return set_err(SGBEM_E_INVAL, "p must be in [1, 6]");
    const size_t n = size_t(N), M = size_t(n_ref) * n;
    // control points beyond the inline storage (and the knots of a non-uniform curve)
    const size_t params = n_ctrl > 64 ? buf_bytes(size_t(3 * n_ctrl + 1) * sizeof(double)) : 0;
    size_t b = 0;
    switch (what) {
    case SGBEM_MEM_RULES:
        b = buf_bytes(rules_block_bytes(int64_t(2 * M)));
        break;
    case SGBEM_MEM_ASSEMBLE_WQ:
        b = buf_bytes(3 * 2 * M * sizeof(double)) + params;
        break;
    case SGBEM_MEM_ASSEMBLE_EBE: {
        if (n_gauss < 1 || n_gauss > 8) return set_err(SGBEM_E_INVAL, "n_gauss must be in [1, 8]");
        const size_t G = size_t(n_gauss), q = size_t(p + 1);
        b = buf_bytes(3 * n * G * sizeof(double)) + buf_bytes(3 * n * 16 * sizeof(double)) +
            buf_bytes(n * 2 * q * q * sizeof(double)) + buf_bytes((544 + q * 16) * sizeof(double)) +
            buf_bytes(G * q * sizeof(double)) + params;
        break;
    }
    case SGBEM_MEM_RHS_DIRECT: {
        if (n_gauss < 2 || n_gauss > 8 || (n_gauss & 1)) return set_err(SGBEM_E_INVAL, "n_gauss must be 2, 4, 6 or 8");
        const int nn = int(2 * M), np = int(n) * n_gauss;
        const size_t nchunk = size_t(dl_chunks(nn, np));
        b = buf_bytes(3 * size_t(nn) * sizeof(double)) +
            buf_bytes(sizeof(double) * (5 * size_t(np) + nchunk * size_t(nn) + 2 * size_t(nn))) + params;
        break;
    }
    case SGBEM_MEM_SOLVE:
        b = buf_bytes(solve_workspace_bytes(N));
        break;
    case SGBEM_MEM_RULES_KNOTS:
        b = buf_bytes(knot_rules_block_bytes(N, n_ref, p));
        break;
    case SGBEM_MEM_RULES_OPEN:
        b = buf_bytes(open_rules_block_bytes(N, n_ref, p));
        break;
    default:
        return set_err(SGBEM_E_INVAL, "unknown memory kind");
    }
    *bytes = int64_t(b);
    return SGBEM_OK;
}

sgbem_status sgbem_ctx_set_stream(sgbem_ctx c, void *hip_stream)
{
    if (!c) return set_err(SGBEM_E_INVAL, "ctx is NULL");
    DeviceGuard g(c->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stream = static_cast<hipStream_t>(hip_stream);
    return SGBEM_OK;
}

sgbem_status sgbem_ctx_destroy(sgbem_ctx c)
{
    if (!c) return SGBEM_OK;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf *b : {&c->geo, &c->geo16, &c->nearL, &c->params, &c->solve_ws, &c->dl})
        if (b->ptr) (void)hipFree(b->ptr);
    for (auto &kv : c->tables) (void)hipFree(kv.second);   // (the context goes: no accounting)
    for (auto *r : c->rules) free_rules(r);
    for (auto *b : c->batches) {
        (void)hipFree(b->mem);
        delete b;
    }
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    lookahead_free(c->lookahead);
    delete c;
    return SGBEM_OK;
}

sgbem_status sgbem_ctx_set_timing(sgbem_ctx c, int32_t on)
{
    if (!c) return set_err(SGBEM_E_INVAL, "ctx is NULL");
    c->timing = on ? 1 : 0;
    c->ev_used = 0;
    return SGBEM_OK;
}

sgbem_status sgbem_ctx_kernel_time(sgbem_ctx c, double *total_ms, int64_t *count)
{
    if (!c || !total_ms || !count) return set_err(SGBEM_E_INVAL, "NULL argument");
    DeviceGuard g(c->device);
    double tot = 0.0;
    int64_t n = 0;
    if (c->ev_used >= 2) HIPCHK(hipEventSynchronize(c->ev[c->ev_used - 1]));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        tot += ms;
        ++n;
    }
    c->ev_used = 0;
    *total_ms = tot;
    *count = n;
    return SGBEM_OK;
}

sgbem_status sgbem_weights_host(int32_t p, int32_t N, int32_t n_ref, double *w0, double *bvals, double *ws)
{
    try {
        WQRules W = build_wq_rules(p, N, n_ref);
        if (w0) std::memcpy(w0, W.w0.data(), W.w0.size() * sizeof(double));
        if (bvals) std::memcpy(bvals, W.bvals.data(), W.bvals.size() * sizeof(double));
        if (ws) std::memcpy(ws, W.ws.data(), W.ws.size() * sizeof(double));
    } catch (const PlanError &e) {
        return set_err(sgbem_status(e.status), e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    return SGBEM_OK;
}

sgbem_status sgbem_nearfield_host(double *u16, double *w16, double *mco, double *madj)
{
    const NearField &nf = nearfield16();
    if (u16) std::memcpy(u16, nf.u, sizeof nf.u);
    if (w16) std::memcpy(w16, nf.w, sizeof nf.w);
    if (mco) std::memcpy(mco, nf.mco, sizeof nf.mco);
    if (madj) std::memcpy(madj, nf.madj, sizeof nf.madj);
    return SGBEM_OK;
}

sgbem_status sgbem_node_points_host(const sgbem_curve *curve, int32_t N, int32_t n_ref, double *xy)
{
    if (!xy) return set_err(SGBEM_E_INVAL, "xy is NULL");
    if (N < 1 || n_ref < 1 || n_ref > 4) return set_err(SGBEM_E_INVAL, "bad N or n_ref");
    sgbem_status st = check_curve(curve);
    if (st) return st;
    CurveDev d;
    std::memset(&d, 0, sizeof d);
    d.kind = curve->kind;
    d.degree = curve->degree;
    d.n_ctrl = curve->n_ctrl;
    d.n_modes = curve->n_modes;
    d.r0 = curve->r0;
    d.ctrl = curve->ctrl_xy;
    d.knots = curve->knots;
    d.nonuniform = curve->kind == SGBEM_CURVE_BSPLINE && curve->knots ? 1 : 0;
    d.a = curve->a;
    d.phi = curve->phi;
    const int64_t npts = int64_t(2) * n_ref * N;
    for (int64_t n = 0; n < npts; ++n) {
        double x, y, J;
        eval_curve(d, double(n) / double(npts), x, y, J);
        xy[2 * n] = x;
        xy[2 * n + 1] = y;
    }
    return SGBEM_OK;
}

namespace {
// Rules on non-uniform knots: built on the host, uploaded into one block of
// the context (within its budget).
sgbem_status make_knot_rules(sgbem_ctx c, int p, int N, int R, const double *knots, sgbem_rules &out)
{
    out = nullptr;
    WQRulesKnots K;
    try {
        K = build_wq_rules_knots(p, N, R, knots);
    } catch (const PlanError &e) {
        return set_err(sgbem_status(e.status), e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    const size_t nb = buf_bytes(knot_rules_block_bytes(N, R, p));
    void *block = nullptr;
    sgbem_status st = ctx_malloc(c, &block, nb);
    if (st) return st;
    auto *r = new (std::nothrow) sgbem_rules_s;
    if (!r) {
        ctx_free(c, block, nb);
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    r->p = p;
    r->N = N;
    r->R = R;
    r->Q = K.Q;
    r->M = K.M;
    r->npts = K.n_nodes;
    r->knots = true;
    r->block = block;
    r->block_bytes = nb;
    r->owned = true;
    const size_t NQ = size_t(N) * K.Q, nn = size_t(K.n_nodes);
    char *b = static_cast<char *>(block);
    r->d_W = reinterpret_cast<double *>(b);
    b += align256(NQ * 8);
    r->d_Bv = reinterpret_cast<double *>(b);
    b += align256(NQ * 8);
    r->d_Wsg = reinterpret_cast<double *>(b);
    b += align256(nn * nn * 8);
    r->d_eta = reinterpret_cast<double *>(b);
    hipError_t e = hipMemcpy(r->d_W, K.W.data(), NQ * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_Bv, K.Bv.data(), NQ * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_Wsg, K.Ws.data(), nn * nn * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_eta, K.eta.data(), nn * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx_free(c, block, nb);
        delete r;
        return set_err(SGBEM_E_DEVICE, std::string("rules upload: ") + hipGetErrorString(e));
    }
    out = r;
    return SGBEM_OK;
}
}  // namespace

namespace {
// Rules on an open arc: built on the host, uploaded into one block of the
// context (within its budget); the tile windows of the assembly are checked here.
sgbem_status make_open_rules(sgbem_ctx c, int p, int n_el, int R, const double *breaks, sgbem_rules &out)
{
    out = nullptr;
    WQRulesOpen K;
    try {
        K = build_wq_rules_open(p, n_el, R, breaks);
    } catch (const PlanError &e) {
        return set_err(sgbem_status(e.status), e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    const int N = K.N, P = 2 * R, QM = arc_qm(p, P);
    if (K.QM > QM) return set_err(SGBEM_E_SINGULAR, "open-arc rules: a support longer than its bound (internal)");
    for (int I0 = 0; I0 < N; I0 += kArcTile)
        if (K.n0[size_t(std::min(I0 + kArcTile - 1, N - 1))] - K.n0[size_t(I0)] + QM > arc_window(p, P))
            return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: a tile's node window exceeds the kernel's (internal)");
    const size_t nb = buf_bytes(open_rules_block_bytes(n_el, R, p));
    void *block = nullptr;
    sgbem_status st = ctx_malloc(c, &block, nb);
    if (st) return st;
    auto *r = new (std::nothrow) sgbem_rules_s;
    if (!r) {
        ctx_free(c, block, nb);
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    r->p = p;
    r->N = N;
    r->R = R;
    r->Q = QM;
    r->QM = QM;
    r->M = K.M;
    r->npts = K.n_nodes;
    r->open = true;
    r->n_el = n_el;
    r->a = breaks[0];
    r->b = breaks[n_el];
    r->block = block;
    r->block_bytes = nb;
    r->owned = true;
    const size_t NQ = size_t(N) * QM, nn = size_t(K.n_nodes);
    std::vector<double> Wp(NQ, 0.0), Bp(NQ, 0.0);    // rows padded from K.QM to the kernel's QM
    for (int i = 0; i < N; ++i)
        for (int q = 0; q < K.QM; ++q) {
            Wp[size_t(i) * QM + q] = K.W[size_t(i) * K.QM + q];
            Bp[size_t(i) * QM + q] = K.Bv[size_t(i) * K.QM + q];
        }
    char *b = static_cast<char *>(block);
    r->d_W = reinterpret_cast<double *>(b);
    b += align256(NQ * 8);
    r->d_Bv = reinterpret_cast<double *>(b);
    b += align256(NQ * 8);
    r->d_Wsg = reinterpret_cast<double *>(b);
    b += align256(nn * nn * 8);
    r->d_eta = reinterpret_cast<double *>(b);
    b += align256(nn * 8);
    r->d_n0 = reinterpret_cast<int32_t *>(b);
    b += align256(size_t(N) * 4);
    r->d_cnt = reinterpret_cast<int32_t *>(b);
    try {
        r->n0 = K.n0;
    } catch (...) {
        ctx_free(c, block, nb);
        delete r;
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    hipError_t e = hipMemcpy(r->d_W, Wp.data(), NQ * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_Bv, Bp.data(), NQ * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_Wsg, K.Ws.data(), nn * nn * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_eta, K.eta.data(), nn * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_n0, K.n0.data(), size_t(N) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(r->d_cnt, K.cnt.data(), size_t(N) * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ctx_free(c, block, nb);
        delete r;
        return set_err(SGBEM_E_DEVICE, std::string("rules upload: ") + hipGetErrorString(e));
    }
    out = r;
    return SGBEM_OK;
}
}  // namespace

sgbem_status sgbem_weights_open(sgbem_ctx c, int32_t p, int32_t n_el, int32_t n_ref, const double *breaks,
                                sgbem_rules *out)
{
    if (!c || !out || !breaks) return set_err(SGBEM_E_INVAL, "ctx, breaks or out is NULL");
    *out = nullptr;
    if (p < 1 || p > 6 || n_ref < 1 || n_ref > 4 || n_el < 1 || int64_t(n_ref) * n_el < 2)
        return set_err(SGBEM_E_INVAL, "need p in [1, 6], n_ref in [1, 4], n_ref n_el >= 2");
    if (int64_t(2) * p + int64_t(2) * n_ref * n_el - 1 > kMaxKnotNodes)
        return set_err(SGBEM_E_UNSUPPORTED, "open arc: 2p + 2 n_ref n_el - 1 exceeds the limit of the full singular table");
    DeviceGuard g(c->device);
    sgbem_rules r = nullptr;
    sgbem_status st = make_open_rules(c, p, n_el, n_ref, breaks, r);
    if (st) return st;
    try {
        c->rules.push_back(r);
    } catch (...) {
        ctx_free(c, r->block, r->block_bytes);
        r->owned = false;
        free_rules(r);
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    *out = r;
    return SGBEM_OK;
}

sgbem_status sgbem_weights_host_open(int32_t p, int32_t n_el, int32_t n_ref, const double *breaks, int32_t *q_max,
                                     int32_t *n0, int32_t *cnt, double *W, double *Bv, double *Ws, double *eta)
{
    if (!breaks) return set_err(SGBEM_E_INVAL, "breaks is NULL");
    if (p < 1 || p > 6 || n_ref < 1 || n_ref > 4 || n_el < 1 || int64_t(n_ref) * n_el < 2)
        return set_err(SGBEM_E_INVAL, "need p in [1, 6], n_ref in [1, 4], n_ref n_el >= 2");
    const int QM = arc_qm(p, 2 * n_ref);
    if (q_max) *q_max = QM;
    if (!n0 && !cnt && !W && !Bv && !Ws && !eta) return SGBEM_OK;
    try {
        const WQRulesOpen K = build_wq_rules_open(p, n_el, n_ref, breaks);
        if (K.QM > QM) return set_err(SGBEM_E_SINGULAR, "open-arc rules: a support longer than its bound (internal)");
        if (n0) std::memcpy(n0, K.n0.data(), K.n0.size() * sizeof(int32_t));
        if (cnt) std::memcpy(cnt, K.cnt.data(), K.cnt.size() * sizeof(int32_t));
        for (int i = 0; i < K.N; ++i)
            for (int q = 0; q < QM; ++q) {
                const bool in = q < K.QM;
                if (W) W[size_t(i) * QM + q] = in ? K.W[size_t(i) * K.QM + q] : 0.0;
                if (Bv) Bv[size_t(i) * QM + q] = in ? K.Bv[size_t(i) * K.QM + q] : 0.0;
            }
        if (Ws) std::memcpy(Ws, K.Ws.data(), K.Ws.size() * sizeof(double));
        if (eta) std::memcpy(eta, K.eta.data(), K.eta.size() * sizeof(double));
    } catch (const PlanError &e) {
        return set_err(sgbem_status(e.status), e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    return SGBEM_OK;
}

sgbem_status sgbem_weights(sgbem_ctx c, int32_t p, int32_t N, int32_t n_ref, const double *knots, sgbem_rules *out)
{
    if (!c || !out) return set_err(SGBEM_E_INVAL, "ctx or out is NULL");
    *out = nullptr;
    if (p < 1 || p > 6 || n_ref < 1 || n_ref > 4 || N < 2 * (p + 1) || int64_t(2) * n_ref * N > (int64_t(1) << 24))
        return set_err(SGBEM_E_INVAL, "need p in [1, 6], n_ref in [1, 4], N >= 2 (p + 1), 2 n_ref N <= 2^24");
    DeviceGuard g(c->device);
    sgbem_rules r = nullptr;
    sgbem_status st;
    if (knots) {
        if ((st = make_knot_rules(c, p, N, n_ref, knots, r))) return st;
    } else {
        // the block within the context's budget, before the host work
        const size_t nb = buf_bytes(rules_block_bytes(int64_t(2) * n_ref * N));
        void *block = nullptr;
        if ((st = ctx_malloc(c, &block, nb))) return st;
        if ((st = make_rules(p, N, n_ref, block, c->stream, r))) {
            ctx_free(c, block, nb);
            return st;
        }
        r->owned = true;
        r->block_bytes = nb;
    }
    try {
        c->rules.push_back(r);
    } catch (...) {
        ctx_free(c, r->block, r->block_bytes);
        r->owned = false;
        free_rules(r);
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    *out = r;
    return SGBEM_OK;
}

sgbem_status sgbem_weights_host_knots(int32_t p, int32_t N, int32_t n_ref, const double *knots, double *W, double *Bv,
                                      double *Ws, double *eta)
{
    if (!knots) return set_err(SGBEM_E_INVAL, "knots is NULL");
    try {
        const WQRulesKnots K = build_wq_rules_knots(p, N, n_ref, knots);
        if (W) std::memcpy(W, K.W.data(), K.W.size() * sizeof(double));
        if (Bv) std::memcpy(Bv, K.Bv.data(), K.Bv.size() * sizeof(double));
        if (Ws) std::memcpy(Ws, K.Ws.data(), K.Ws.size() * sizeof(double));
        if (eta) std::memcpy(eta, K.eta.data(), K.eta.size() * sizeof(double));
    } catch (const PlanError &e) {
        return set_err(sgbem_status(e.status), e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    return SGBEM_OK;
}

sgbem_status sgbem_rules_free(sgbem_ctx c, sgbem_rules r)
{
    if (!c) return set_err(SGBEM_E_INVAL, "ctx is NULL");
    if (!r) return SGBEM_OK;
    if (r->shared || !valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    DeviceGuard g(c->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->rules.size(); ++i)
        if (c->rules[i] == r) {
            c->rules.erase(c->rules.begin() + i);
            break;
        }
    if (r->owned) c->held -= r->block_bytes;
    free_rules(r);
    return SGBEM_OK;
}

namespace {
// An open arc served by open-arc rules must have the rules' parameter interval.
sgbem_status check_arc_interval(const sgbem_curve *curve, sgbem_rules r)
{
    if (!r->open || !curve || curve->kind != SGBEM_CURVE_BSPLINE_OPEN || !curve->knots) return SGBEM_OK;
    const double a = curve->knots[0], b = curve->knots[curve->n_ctrl + curve->degree];
    if (a != r->a || b != r->b)
        return set_err(SGBEM_E_INVAL, "open arc: the curve's parameter interval differs from the rules' [a, b]");
    return SGBEM_OK;
}
}  // namespace

sgbem_status sgbem_rhs_points(sgbem_ctx c, const sgbem_curve *curve, sgbem_rules r, int32_t method, int32_t n_gauss,
                              double *d_xy, int64_t cap, int64_t *count)
{
    if (!c || !r || !count) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (method != SGBEM_WQ && method != SGBEM_EBE) return set_err(SGBEM_E_INVAL, "unknown method");
    if (r->knots && method != SGBEM_WQ) return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: fast-form assembly and its right-hand side only");
    if (r->open && method != SGBEM_WQ) return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: fast-form assembly (FP64), its right-hand side and node points only");
    if (method == SGBEM_EBE && (n_gauss < 1 || n_gauss > 8)) return set_err(SGBEM_E_INVAL, "n_gauss must be in [1, 8]");
    DeviceGuard g(c->device);
    const GridDesc grid = method == SGBEM_WQ ? wq_grid(r) : gauss_grid(r->N, n_gauss);
    *count = grid.npts;
    if (cap < grid.npts || !d_xy) return set_err(SGBEM_E_INVAL, "output capacity too small");
    CurveDev cd;
    sgbem_status st = check_arc_interval(curve, r);
    if (st) return st;
    st = upload_curve(c, curve, cd, r->open);
    if (st) return st;
    double *X, *Y, *J;
    if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
    HIPCHK(launch_points_xy(X, Y, grid.npts, d_xy, c->stream));
    return SGBEM_OK;
}

sgbem_status sgbem_assemble(sgbem_ctx c, const sgbem_curve *curve, sgbem_rules r, int32_t method, int32_t n_gauss,
                            int32_t precision, void *d_A, int64_t lda)
{
    if (!c || !r || !d_A) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (method != SGBEM_WQ && method != SGBEM_EBE) return set_err(SGBEM_E_INVAL, "unknown method");
    if (precision != SGBEM_FP64 && precision != SGBEM_FP32) return set_err(SGBEM_E_INVAL, "unknown precision");
    if (lda < r->N) return set_err(SGBEM_E_INVAL, "lda < N");
    if (method == SGBEM_EBE && (n_gauss < 1 || n_gauss > 8)) return set_err(SGBEM_E_INVAL, "n_gauss must be in [1, 8]");
    const int p = r->p, N = r->N;
    const int P = method == SGBEM_WQ ? 2 * r->R : n_gauss;
    if (r->open) {
        // open arc: ragged per-row rules, the full singular table, every entry of eq. IK1e2_bis
        if (method != SGBEM_WQ || precision != SGBEM_FP64 || !assemble_arc_supported(p, P))
            return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: FP64 fast form with n_ref in {1, 2} only");
        sgbem_status st = check_arc_interval(curve, r);
        if (st) return st;
        DeviceGuard g(c->device);
        CurveDev cd;
        if ((st = upload_curve(c, curve, cd, true))) return st;
        const GridDesc grid = wq_grid(r);
        double *X, *Y, *J;
        if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
        ArcArgs aa;
        aa.N = N;
        aa.npts = grid.npts;
        aa.P = P;
        aa.X = X;
        aa.Y = Y;
        aa.J = J;
        aa.eta = r->d_eta;
        aa.W = r->d_W;
        aa.Bv = r->d_Bv;
        aa.Ws = r->d_Wsg;
        aa.n0 = r->d_n0;
        aa.scale = -1.0 / (2.0 * kPi);
        aa.out = static_cast<double *>(d_A);
        aa.lda = lda;
        KernelEvents ke;
        const KernelEvents *kev;
        if ((st = timing_events(c, ke, kev))) return st;
        HIPCHK(launch_assemble_arc(p, aa, c->stream, kev));
        return SGBEM_OK;
    }
    if (r->knots) {
        // non-uniform knots: per-row rules and the full singular table (FP64 fast form)
        if (method != SGBEM_WQ || precision != SGBEM_FP64 || !assemble_knots_supported(p, P))
            return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: FP64 fast form with n_ref in {1, 2} only");
        DeviceGuard g(c->device);
        CurveDev cd;
        sgbem_status st = upload_curve(c, curve, cd);
        if (st) return st;
        const GridDesc grid = wq_grid(r);
        double *X, *Y, *J;
        if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
        KnotArgs ka;
        ka.N = N;
        ka.npts = grid.npts;
        ka.P = P;
        ka.Q = r->Q;
        ka.X = X;
        ka.Y = Y;
        ka.J = J;
        ka.eta = r->d_eta;
        ka.W = r->d_W;
        ka.Bv = r->d_Bv;
        ka.Ws = r->d_Wsg;
        ka.scale = -1.0 / (2.0 * kPi);
        ka.out = static_cast<double *>(d_A);
        ka.lda = lda;
        KernelEvents ke;
        const KernelEvents *kev;
        if ((st = timing_events(c, ke, kev))) return st;
        HIPCHK(launch_assemble_knots(p, ka, c->stream, kev));
        return SGBEM_OK;
    }
    if (!assemble_supported(method, precision, p, P)) return set_err(SGBEM_E_UNSUPPORTED, "no kernel compiled for this (p, P)");
    DeviceGuard g(c->device);
    CurveDev cd;
    sgbem_status st = upload_curve(c, curve, cd);
    if (st) return st;

    TileArgs ta;
    std::memset(&ta, 0, sizeof ta);
    ta.N = N;
    ta.scale = -1.0 / (2.0 * kPi);
    ta.out = d_A;
    ta.lda = lda;
    if (method == SGBEM_WQ) {
        const GridDesc grid = wq_grid(r);
        double *X, *Y, *J;
        if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
        wq_tile_args(r, X, Y, J, ta);
        KernelEvents ke;
        const KernelEvents *kev;
        if ((st = timing_events(c, ke, kev))) return st;
        HIPCHK(launch_assemble(0, precision, p, P, ta, c->stream, kev));
        return SGBEM_OK;
    }
    // ---- element by element: far part by the tile kernel, near pairs by their own rule
    const int G = n_gauss;
    const GridDesc grid = gauss_grid(N, G);
    double *X, *Y, *J;
    if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
    const GridDesc g16 = gauss_grid(N, 16);
    double *X16, *Y16, *J16;
    if ((st = geometry(c, cd, g16, c->geo16, X16, Y16, J16))) return st;
    const double *dt = nullptr;
    if ((st = cached_table(c, p, near_table(p), dt))) return st;
    if ((st = ensure(c, c->nearL, size_t(N) * 2 * (p + 1) * (p + 1) * sizeof(double)))) return st;
    NearArgs na;
    na.N = N;
    na.p = p;
    na.X16 = X16;
    na.Y16 = Y16;
    na.J16 = J16;
    na.u16 = dt;
    na.w16 = dt + 16;
    na.mco = dt + 32;
    na.madj = dt + 288;
    na.bv16 = dt + 544;
    na.L = static_cast<double *>(c->nearL.ptr);
    HIPCHK(launch_near(na, c->stream));

    ta.npts = grid.npts;
    ta.X = X;
    ta.Y = Y;
    ta.J = J;
    const std::vector<double> gc = gauss_basis_coef(p, G);
    for (size_t q = 0; q < gc.size(); ++q) ta.coefA[q] = gc[q] / N;      // h w_g M_p(a + u_g)
    KernelEvents ke;
    const KernelEvents *kev;
    if ((st = timing_events(c, ke, kev))) return st;
    HIPCHK(launch_assemble(1, precision, p, P, ta, c->stream, kev));
    HIPCHK(launch_band(precision, N, p, na.L, ta.scale, d_A, lda, c->stream));
    return SGBEM_OK;
}

sgbem_status sgbem_assemble_noalloc(sgbem_ctx c, const sgbem_curve *curve, sgbem_rules r, int32_t precision,
                                    void *d_A, int64_t lda)
{
    if (!c || !r || !d_A) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (precision != SGBEM_FP64 && precision != SGBEM_FP32) return set_err(SGBEM_E_INVAL, "unknown precision");
    if (lda < r->N) return set_err(SGBEM_E_INVAL, "lda < N");
    if (r->npts > SGBEM_NOALLOC_MAX_NODES)
        return set_err(SGBEM_E_INVAL, "2 n_ref N exceeds SGBEM_NOALLOC_MAX_NODES (the fixed geometry array)");
    if (r->knots) return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: fast-form assembly and its right-hand side only");
    if (r->open) return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: fast-form assembly (FP64), its right-hand side and node points only");
    const int p = r->p, P = 2 * r->R;
    if (!assemble_supported(SGBEM_WQ, precision, p, P))
        return set_err(SGBEM_E_UNSUPPORTED, "no kernel compiled for this (p, n_ref)");
    if (!c->noalloc_scratch) return set_err(SGBEM_E_DEVICE, "the fixed geometry array has no device address");
    CurveDev cd;
    sgbem_status st = inline_curve(curve, cd);
    if (st) return st;
    DeviceGuard g(c->device);
    const GridDesc grid = wq_grid(r);
    double *X = c->noalloc_scratch, *Y = X + grid.npts, *J = Y + grid.npts;
    HIPCHK(launch_geometry(cd, grid, X, Y, J, c->stream));
    TileArgs ta;
    std::memset(&ta, 0, sizeof ta);
    ta.N = r->N;
    ta.scale = -1.0 / (2.0 * kPi);
    ta.out = d_A;
    ta.lda = lda;
    wq_tile_args(r, X, Y, J, ta);
    HIPCHK(launch_assemble(0, precision, p, P, ta, c->stream, nullptr));
    return SGBEM_OK;
}

sgbem_status sgbem_rhs(sgbem_ctx c, const sgbem_curve *curve, sgbem_rules r, int32_t method, int32_t n_gauss,
                       const double *d_g, double *d_beta)
{
    if (!c || !r || !d_g || !d_beta) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (method != SGBEM_WQ && method != SGBEM_EBE) return set_err(SGBEM_E_INVAL, "unknown method");
    if (method == SGBEM_EBE && (n_gauss < 1 || n_gauss > 8)) return set_err(SGBEM_E_INVAL, "n_gauss must be in [1, 8]");
    if (r->open && method != SGBEM_WQ) return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: fast-form assembly (FP64), its right-hand side and node points only");
    sgbem_status st = check_arc_interval(curve, r);
    if (st) return st;
    DeviceGuard g(c->device);
    CurveDev cd;
    if ((st = upload_curve(c, curve, cd, r->open))) return st;
    const int p = r->p, N = r->N;
    if (method == SGBEM_WQ) {
        const GridDesc grid = wq_grid(r);
        double *X, *Y, *J;
        if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
        if (r->open) HIPCHK(launch_rhs_arc(N, r->QM, r->d_n0, r->d_cnt, r->d_W, J, d_g, d_beta, c->stream));
        else if (r->knots) HIPCHK(launch_rhs_knots(N, grid.npts, 2 * r->R, r->Q, r->d_W, J, d_g, d_beta, c->stream));
        else HIPCHK(launch_rhs(N, grid.npts, 2 * r->R, 1, r->Q, r->d_w0, 1.0, J, d_g, d_beta, c->stream));
        return SGBEM_OK;
    }
    if (r->knots) return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: fast-form assembly and its right-hand side only");
    const int G = n_gauss;
    const GridDesc grid = gauss_grid(N, G);
    double *X, *Y, *J;
    if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
    const double *dcoef = nullptr;
    if ((st = cached_table(c, 1000 + 64 * p + G, gauss_basis_coef(p, G), dcoef))) return st;
    HIPCHK(launch_rhs(N, grid.npts, G, 0, G * (p + 1), dcoef, 1.0 / N, J, d_g, d_beta, c->stream));
    return SGBEM_OK;
}

sgbem_status sgbem_rhs_direct(sgbem_ctx c, const sgbem_curve *curve, sgbem_rules r, int32_t n_gauss,
                              const double *d_g_nodes, const double *d_g_gauss, double *d_F, double *d_b2)
{
    if (!c || !r || !d_g_nodes || !d_g_gauss || !d_F) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (n_gauss < 2 || n_gauss > 8 || (n_gauss & 1))
        return set_err(SGBEM_E_INVAL, "n_gauss must be 2, 4, 6 or 8 (even: no Gauss point on a node)");
    if (r->knots) return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: fast-form assembly and its right-hand side only");
    if (r->open) return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: fast-form assembly (FP64), its right-hand side and node points only");
    DeviceGuard g(c->device);
    CurveDev cd;
    sgbem_status st = upload_curve(c, curve, cd);
    if (st) return st;
    const int N = r->N, G = n_gauss;
    const GridDesc nodes = wq_grid(r);
    double *X1, *Y1, *J1;
    if ((st = geometry(c, cd, nodes, c->geo, X1, Y1, J1))) return st;
    const GridDesc gg = gauss_grid(N, G);
    GaussW gw, gu;   // composite weights w_q / N, and the nodes u_q on [0, 1]
    {
        double gx[32], gwt[32];
        gauss_legendre01(G, gx, gwt);
        for (int q = 0; q < 8; ++q) {
            gw.w[q] = q < G ? gwt[q] / N : 0.0;
            gu.w[q] = q < G ? gx[q] : 0.0;
        }
    }
    const int nn = nodes.npts, np = gg.npts;
    const int nchunk = dl_chunks(nn, np);
    const size_t bytes = sizeof(double) * (size_t(5) * np + size_t(nchunk) * nn + 2 * size_t(nn));
    if ((st = ensure(c, c->dl, bytes))) return st;
    double *X2 = static_cast<double *>(c->dl.ptr), *Y2 = X2 + np, *DX2 = Y2 + np, *DY2 = DX2 + np, *coef = DY2 + np;
    double *part = coef + np, *h = part + size_t(nchunk) * nn, *v = h + nn;
    HIPCHK(launch_dl_geometry(cd, gg, gw, d_g_gauss, X2, Y2, DX2, DY2, coef, c->stream));
    KernelEvents ke;
    const KernelEvents *kev;
    if ((st = timing_events(c, ke, kev))) return st;
    HIPCHK(launch_dl_sweep(nn, X1, Y1, np, X2, Y2, DX2, DY2, coef, nchunk, part, c->stream, kev));
    HIPCHK(launch_dl_near(cd, N, 2 * r->R, G, gu, nn, X1, Y1, X2, Y2, DX2, DY2, coef, part, c->stream));
    HIPCHK(launch_dl_reduce(nn, nchunk, part, d_g_nodes, h, d_b2 ? v : nullptr, c->stream));
    HIPCHK(launch_rhs(N, nn, 2 * r->R, 1, r->Q, r->d_w0, 1.0, J1, h, d_F, c->stream));
    if (d_b2) HIPCHK(launch_rhs(N, nn, 2 * r->R, 1, r->Q, r->d_w0, 1.0, J1, v, d_b2, c->stream));
    return SGBEM_OK;
}

sgbem_status sgbem_assemble_collocation(sgbem_ctx c, const sgbem_curve *curve, sgbem_rules r, double *d_A, int64_t lda)
{
    if (!c || !r || !d_A) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (lda < r->N) return set_err(SGBEM_E_INVAL, "lda < N");
    if (r->knots) return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: fast-form assembly and its right-hand side only");
    if (r->open) return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: fast-form assembly (FP64), its right-hand side and node points only");
    const int p = r->p, P = 2 * r->R;
    if (!colloc_supported(p, P)) return set_err(SGBEM_E_UNSUPPORTED, "collocation: n_ref in {1, 2} only");
    DeviceGuard g(c->device);
    CurveDev cd;
    sgbem_status st = upload_curve(c, curve, cd);
    if (st) return st;
    const GridDesc grid = wq_grid(r);
    double *X, *Y, *J;
    if ((st = geometry(c, cd, grid, c->geo, X, Y, J))) return st;
    TileArgs ta;
    std::memset(&ta, 0, sizeof ta);
    ta.N = r->N;
    ta.npts = grid.npts;
    ta.X = X;
    ta.Y = Y;
    ta.J = J;
    ta.inv_s2 = r->d_inv_s2;
    ta.ws = r->d_ws;
    for (int q = 0; q < r->Q; ++q) {
        ta.coefA[q] = r->w0[q];
        ta.coefB[q] = r->bvals[q];
    }
    ta.scale = -1.0 / (2.0 * kPi);
    ta.out = d_A;
    ta.lda = lda;
    KernelEvents ke;
    const KernelEvents *kev;
    if ((st = timing_events(c, ke, kev))) return st;
    HIPCHK(launch_colloc(p, P, ta, c->stream, kev));
    return SGBEM_OK;
}

sgbem_status sgbem_collocation_rhs(sgbem_ctx c, sgbem_rules r, const double *d_g_nodes, double *d_b)
{
    if (!c || !r || !d_g_nodes || !d_b) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (!valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "rules handle does not belong to this context");
    if (r->knots) return set_err(SGBEM_E_UNSUPPORTED, "rules on non-uniform knots: fast-form assembly and its right-hand side only");
    if (r->open) return set_err(SGBEM_E_UNSUPPORTED, "open-arc rules: fast-form assembly (FP64), its right-hand side and node points only");
    DeviceGuard g(c->device);
    HIPCHK(launch_colloc_gather(r->N, int(r->npts), 2 * r->R, r->R * (r->p + 1), d_g_nodes, d_b, c->stream));
    return SGBEM_OK;
}

sgbem_status sgbem_batch_create(sgbem_ctx c, int32_t n, const sgbem_curve *curves, const sgbem_rules *rules,
                                int32_t precision, void *const *d_A, const int64_t *lda, sgbem_batch *out)
{
    if (!c || !curves || !rules || !d_A || !lda || !out || n < 1) return set_err(SGBEM_E_INVAL, "NULL argument or n < 1");
    if (precision != SGBEM_FP64 && precision != SGBEM_FP32) return set_err(SGBEM_E_INVAL, "unknown precision");
    *out = nullptr;
    DeviceGuard g(c->device);
    std::vector<CurveDev> cd(n);
    std::vector<int> npts(n), deg(n);
    std::vector<std::vector<int>> pre(kNumBatchConfigs, std::vector<int>(n + 1, 0));
    std::vector<int64_t> goff(n);
    std::vector<TileArgs> args(n);
    std::vector<TileArgsF> argsf(n);
    int64_t gsum = 0;
    int max_npts = 0;
    for (int b = 0; b < n; ++b) {
        sgbem_rules r = rules[b];
        if (!r || !valid_rules(c, r)) return set_err(SGBEM_E_INVAL, "batch: rules handle does not belong to this context");
        if (r->knots) return set_err(SGBEM_E_UNSUPPORTED, "batch: rules on non-uniform knots are not batched");
        if (r->open) return set_err(SGBEM_E_UNSUPPORTED, "batch: open-arc rules are not batched");
        if (r->R != 1 || r->p < 2 || r->p > 4)
            return set_err(SGBEM_E_UNSUPPORTED, "batch: n_ref = 1 and p in {2, 3, 4} only");
        if (!d_A[b] || lda[b] < r->N) return set_err(SGBEM_E_INVAL, "batch: NULL matrix or lda < N");
        sgbem_status st = inline_curve(&curves[b], cd[b]);
        if (st) return st;
        npts[b] = int(r->npts);
        deg[b] = r->p;
        goff[b] = gsum;
        gsum += r->npts;
        if (npts[b] > max_npts) max_npts = npts[b];
        for (int k = 0; k < kNumBatchConfigs; ++k) {
            const int64_t T = kBatchConfigs[k].T, nb = (r->N + T - 1) / T;
            const int64_t tiles = nb * (nb + 1) / 2;
            if (int64_t(pre[k][b]) + tiles > (int64_t(1) << 31) - 1) return set_err(SGBEM_E_INVAL, "batch: too many tiles");
            pre[k][b + 1] = pre[k][b] + int(tiles);
        }
        TileArgs &ta = args[b];
        std::memset(&ta, 0, sizeof ta);
        ta.N = r->N;
        ta.npts = int(r->npts);
        ta.inv_s2 = r->d_inv_s2;
        ta.ws = r->d_ws;
        ta.inv_s2f = r->d_inv_s2f;
        ta.wsf = r->d_wsf;
        for (int q = 0; q < r->Q; ++q) {
            ta.coefA[q] = r->w0[q];
            ta.coefB[q] = r->bvals[q];
            argsf[b].coefA[q] = float(r->w0[q]);
            argsf[b].coefB[q] = float(r->bvals[q]);
        }
        ta.scale = -1.0 / (2.0 * kPi);
        ta.out = d_A[b];
        ta.lda = lda[b];
    }
    // one allocation: curves | npts | goff | args | argsf | deg | prefix per tile configuration | geometry
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_curves = 0;
    const size_t o_npts = o_curves + al(sizeof(CurveDev) * n);
    const size_t o_goff = o_npts + al(sizeof(int) * n);
    const size_t o_args = o_goff + al(sizeof(int64_t) * n);
    const size_t o_argsf = o_args + al(sizeof(TileArgs) * n);
    const size_t o_deg = o_argsf + al(sizeof(TileArgsF) * n);
    const size_t o_pre = o_deg + al(sizeof(int) * n);
    const size_t o_geo = o_pre + kNumBatchConfigs * al(sizeof(int) * (n + 1));
    const size_t total_bytes = o_geo + al(sizeof(double) * 3 * size_t(gsum));
    auto *bt = new (std::nothrow) sgbem_batch_s;
    if (!bt) return set_err(SGBEM_E_NOMEM, "host allocation failed");
    const size_t mem_bytes = buf_bytes(total_bytes);
    {
        const sgbem_status sa = ctx_malloc(c, &bt->mem, mem_bytes);
        if (sa) {
            delete bt;
            return sa;
        }
    }
    bt->mem_bytes = mem_bytes;
    hipError_t e = hipSuccess;
    char *base = static_cast<char *>(bt->mem);
    bt->d.curves = reinterpret_cast<CurveDev *>(base + o_curves);
    bt->d.npts = reinterpret_cast<int *>(base + o_npts);
    bt->d.goff = reinterpret_cast<int64_t *>(base + o_goff);
    bt->d.args = reinterpret_cast<TileArgs *>(base + o_args);
    bt->d.argsf = reinterpret_cast<TileArgsF *>(base + o_argsf);
    bt->d.deg = reinterpret_cast<int *>(base + o_deg);
    for (int k = 0; k < kNumBatchConfigs; ++k)
        bt->d.prefix[k] = reinterpret_cast<int *>(base + o_pre + k * al(sizeof(int) * (n + 1)));
    bt->d.geo = reinterpret_cast<double *>(base + o_geo);
    for (int b = 0; b < n; ++b) {
        args[b].X = bt->d.geo + 3 * goff[b];
        args[b].Y = args[b].X + npts[b];
        args[b].J = args[b].Y + npts[b];
    }
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    };
    std::vector<Up> ups = {{bt->d.curves, cd.data(), sizeof(CurveDev) * n}, {bt->d.npts, npts.data(), sizeof(int) * n},
                           {bt->d.goff, goff.data(), sizeof(int64_t) * n}, {bt->d.args, args.data(), sizeof(TileArgs) * n},
                           {bt->d.argsf, argsf.data(), sizeof(TileArgsF) * n}, {bt->d.deg, deg.data(), sizeof(int) * n}};
    for (int k = 0; k < kNumBatchConfigs; ++k) ups.push_back({bt->d.prefix[k], pre[k].data(), sizeof(int) * (n + 1)});
    for (const Up &u : ups) {
        if ((e = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice)) != hipSuccess) {
            ctx_free(c, bt->mem, bt->mem_bytes);
            delete bt;
            return set_err(SGBEM_E_DEVICE, std::string("batch upload: ") + hipGetErrorString(e));
        }
    }
    bt->n = n;
    bt->prec = precision;
    bt->max_npts = max_npts;
    for (int k = 0; k < kNumBatchConfigs; ++k) bt->total[k] = pre[k][n];
    bt->cfg = c->batch_cfg[precision] >= 0 ? c->batch_cfg[precision] : 0;
    bt->grid = batch_grid(c, bt->cfg, precision, bt->total[bt->cfg]);
    c->batches.push_back(bt);
    *out = bt;
    return SGBEM_OK;
}

sgbem_status sgbem_batch_assemble(sgbem_ctx c, sgbem_batch b)
{
    if (!c || !b || !valid_batch(c, b)) return set_err(SGBEM_E_INVAL, "batch handle does not belong to this context");
    DeviceGuard g(c->device);
    HIPCHK(launch_batch_geometry(b->d, b->n, b->max_npts, c->stream));
    const int tot = b->total[b->cfg];
    sgbem_status st;
    KernelEvents ke;
    const KernelEvents *kev;
    if ((st = timing_events(c, ke, kev))) return st;
    HIPCHK(launch_batch_tiles(b->cfg, b->prec, b->d, b->n, tot, b->grid, c->stream, kev));
    return SGBEM_OK;
}

sgbem_status sgbem_batch_tune(sgbem_ctx c, sgbem_batch b, int32_t reps, int32_t *best_cfg, double *best_ms)
{
    if (!c || !b || !valid_batch(c, b)) return set_err(SGBEM_E_INVAL, "batch handle does not belong to this context");
    if (reps < 1) reps = 3;
    DeviceGuard g(c->device);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best = 1e300;
    int bestc = 0;
    HIPCHK(launch_batch_geometry(b->d, b->n, b->max_npts, c->stream));
    for (int cfg = 0; cfg < kNumBatchConfigs; ++cfg) {
        const int tot = b->total[cfg];
        const int grid = batch_grid(c, cfg, b->prec, tot);
        HIPCHK(launch_batch_tiles(cfg, b->prec, b->d, b->n, tot, grid, c->stream));   // warm
        HIPCHK(hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) HIPCHK(launch_batch_tiles(cfg, b->prec, b->d, b->n, tot, grid, c->stream));
        HIPCHK(hipEventRecord(e1, c->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms / reps < best) {
            best = ms / reps;
            bestc = cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->cfg = bestc;
    b->grid = batch_grid(c, bestc, b->prec, b->total[bestc]);
    c->batch_cfg[b->prec] = bestc;
    if (best_cfg) *best_cfg = bestc;
    if (best_ms) *best_ms = best;
    return SGBEM_OK;
}

sgbem_status sgbem_batch_free(sgbem_ctx c, sgbem_batch b)
{
    if (!c) return set_err(SGBEM_E_INVAL, "ctx is NULL");
    if (!b) return SGBEM_OK;
    if (!valid_batch(c, b)) return set_err(SGBEM_E_INVAL, "batch handle does not belong to this context");
    DeviceGuard g(c->device);
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->batches.size(); ++i)
        if (c->batches[i] == b) {
            c->batches.erase(c->batches.begin() + i);
            break;
        }
    ctx_free(c, b->mem, b->mem_bytes);
    delete b;
    return SGBEM_OK;
}

sgbem_status sgbem_solve(sgbem_ctx c, int32_t N, const void *d_A, int64_t lda, int32_t a_prec, const double *d_beta,
                         double *d_x, double tol, int32_t max_iter, sgbem_solve_info *info)
{
    if (!c || !d_A || !d_beta || !d_x) return set_err(SGBEM_E_INVAL, "NULL argument");
    if (N < 1 || lda < N) return set_err(SGBEM_E_INVAL, "bad N or lda");
    if (a_prec != SGBEM_FP64 && a_prec != SGBEM_FP32) return set_err(SGBEM_E_INVAL, "unknown precision");
    if (max_iter < 0 || !(tol >= 0.0)) return set_err(SGBEM_E_INVAL, "bad tol or max_iter");
    DeviceGuard g(c->device);
    const size_t bytes = solve_workspace_bytes(N);
    sgbem_status st = ensure(c, c->solve_ws, bytes);
    if (st) return st;
    if ((st = ensure_hbuf(c))) return st;
    SolveResult res;
    std::string msg;
    const int rc = mixed_solve(N, d_A, lda, a_prec, d_beta, d_x, tol, max_iter, c->solve_ws.ptr, c->hbuf, c->stream,
                               &c->lookahead,
                               res, msg);
    if (info) {
        info->iters = res.iters;
        info->status = rc;
        info->rel_update = res.rel_update;
        info->backward_err = res.backward_err;
        info->pivoted = res.pivoted ? 1 : 0;
        info->reserved = 0;
    }
    if (rc != SGBEM_OK) return set_err(sgbem_status(rc), msg);
    return SGBEM_OK;
}

}  // extern "C"
