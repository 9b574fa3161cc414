// Internal state behind the opaque handles of the C ABI (contexts, rule
// handles, batches) and the helpers shared by the entry points and the
// serving loop.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/sgbem.h"
#include "batch.hpp"

namespace sgbem {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Records the calling thread's error message and passes the status through.
sgbem_status set_err(sgbem_status st, const std::string &m);

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::sgbem::set_err(e_ == hipErrorOutOfMemory ? SGBEM_E_NOMEM : SGBEM_E_DEVICE, \
                                    std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// Grow-only device buffer owned by a context (bytes: its allocated size).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace sgbem

// Device tables of one rule set live in one block:
//   inv_s2 [npts] f64 | ws [2][npts] f64 | w0 [64] f64 | inv_s2f [npts] f32 | wsf [2][npts] f32
// (each part 256-byte aligned).  `owned`: the block was allocated for the
// handle and is freed with it; otherwise it belongs to a caller's arena.
// `shared`: the handle may be used with any context on its device.
struct sgbem_rules_s {
    int p = 0, N = 0, R = 0, Q = 0;
    int64_t M = 0, npts = 0;
    std::vector<double> w0, bvals;
    double *d_inv_s2 = nullptr, *d_ws = nullptr, *d_w0 = nullptr;
    float *d_inv_s2f = nullptr, *d_wsf = nullptr;
    void *block = nullptr;
    size_t block_bytes = 0;   // allocated size of an owned block
    bool owned = false;
    bool shared = false;
    // rules on non-uniform knots (no translation invariance; FP64 fast form only):
    // W[N][Q], Bv[N][Q], Ws[2M][2M], eta[2M] in the block
    bool knots = false;
    double *d_W = nullptr, *d_Bv = nullptr, *d_Wsg = nullptr, *d_eta = nullptr;
    // rules on an open arc (sgbem_weights_open): N = n_el + p, npts = 2p + 2M - 1,
    // W[N][QM], Bv[N][QM], Ws[npts][npts], eta[npts], n0[N], cnt[N] in the block
    // (d_W, d_Bv, d_Wsg, d_eta as above); [a, b] the parameter interval
    bool open = false;
    int QM = 0, n_el = 0;
    double a = 0.0, b = 0.0;
    int32_t *d_n0 = nullptr, *d_cnt = nullptr;
    std::vector<int32_t> n0;      // host copy of n0 (tile windows are checked at launch)
};

struct sgbem_batch_s {
    int n = 0, prec = 0, max_npts = 0;
    int total[sgbem::kNumBatchConfigs] = {};
    int cfg = 0, grid = 0;
    sgbem::BatchDev d{};
    void *mem = nullptr;     // one device allocation holding the whole description
    size_t mem_bytes = 0;
};

struct sgbem_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    // device address of the fixed geometry array of sgbem_assemble_noalloc on this device
    double *noalloc_scratch = nullptr;
    // device bytes held by the context (buffers, tables, owned rule blocks,
    // batches) and the limit set at creation (0: none)
    uint64_t held = 0, budget = 0;
    // pinned host buffer the solve's kernels write their results to (made on first use)
    double *hbuf = nullptr;
    // the solve's second stream and events beyond N = 4096 (made on first use)
    void *lookahead = nullptr;
    sgbem::DevBuf geo, geo16, nearL, params, solve_ws, dl;
    std::vector<sgbem_rules_s *> rules;
    std::vector<sgbem_batch_s *> batches;
    // geometry-independent element-by-element tables, uploaded once per key:
    // key p      -> u16, w16, mco, madj, M_p(a + u16)       (near pairs)
    // key 1000 + 64p + G -> RHS coefficients w_g M_p(a + u_g) without h
    std::map<int, double *> tables;
    // autotuned batched tile configuration per precision (-1: not tuned yet)
    int batch_cfg[2] = {-1, -1};
    // optional HIP-event timing of the main kernel of each call
    int timing = 0;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
};

namespace sgbem {

// Grow b to at least `bytes` (synchronises the context's stream before a
// reallocation).  Sizes are rounded up to 4096 bytes; E_NOMEM, with b and
// everything else the context holds unchanged, when the grown buffer would
// exceed the context's budget.
sgbem_status ensure(sgbem_ctx c, DevBuf &b, size_t bytes);

// The context's pinned host buffer for the solve (hipHostMalloc on first use).
sgbem_status ensure_hbuf(sgbem_ctx c);

// Allocation size of a context buffer of `bytes` (at least 4096, a multiple of 4096).
size_t buf_bytes(size_t bytes);

// E_NOMEM when allocating `bytes` while releasing `releasing` would take the
// context beyond its budget.
sgbem_status budget_check(sgbem_ctx c, size_t bytes, size_t releasing);

// hipMalloc / hipFree with the context's accounting (ctx_malloc checks the budget first).
sgbem_status ctx_malloc(sgbem_ctx c, void **p, size_t bytes);
void ctx_free(sgbem_ctx c, void *p, size_t bytes);

// Bytes of the device block of a rule set with npts nodes.
size_t rules_block_bytes(int64_t npts);

// Bytes of the device block of rules on non-uniform knots.
size_t knot_rules_block_bytes(int N, int R, int p);
size_t open_rules_block_bytes(int n_el, int R, int p);

// Build the rules of (p, N, R) on the host and upload them on `stream`
// (synchronised before return).  block: device memory of rules_block_bytes
// bytes to hold the tables, or nullptr to allocate it.
sgbem_status make_rules(int p, int N, int R, void *block, hipStream_t stream, sgbem_rules &out);
void free_rules(sgbem_rules r);

// Rules handles the given context can use (its own, or shared ones).
bool valid_rules(sgbem_ctx c, sgbem_rules r);

// Argument check of a curve description.
sgbem_status check_curve(const sgbem_curve *c, bool open = false);

}  // namespace sgbem
