// Continuous-batching server over the fast-form assembly and the
// mixed-precision solve (declared in include/sgbem.h).
//
// Threads: one dispatcher that releases requests at their arrival times and
// admits them, and `workers` slots, each a host thread with its own HIP stream
// and context, that run assemble -> right-hand side -> solve for one admitted
// request at a time.  Admission is first in first out and needs a free slot
// and a free range of the request arena big enough for the request's
// footprint; a request that does not fit waits (and so do the ones behind it)
// until completions return memory.  Device memory is allocated only at
// creation: the request arena, the rule arena that backs the rule cache, and
// each slot's node-geometry buffer sized for the largest N; served curves
// travel inline in the kernel arguments (polar, or at most 64 control points),
// so a request allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sgbem.h"
#include "ctx.hpp"
#include "solve.hpp"

namespace sgbem {
namespace {

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// First-fit allocator over [0, size): free ranges by offset, merged with their
// neighbours on release.
class Arena {
public:
    void reset(int64_t size)
    {
        free_.clear();
        if (size > 0) free_[0] = size;
        used_ = 0;
    }
    int64_t alloc(int64_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }

private:
    std::map<int64_t, int64_t> free_;
    int64_t used_ = 0;
};

// Device layout of one admitted request (offsets from its arena range).
struct Layout {
    size_t A = 0, ws = 0, g = 0, beta = 0, x = 0, total = 0;
};

Layout layout(int N, int prec)
{
    Layout l;
    const size_t n = size_t(N);
    l.A = al256(n * n * (prec == SGBEM_FP64 ? 8 : 4));
    l.ws = al256(solve_workspace_bytes(N));
    l.g = al256(2 * n * 8);
    l.beta = al256(n * 8);
    l.x = al256(n * 8);
    l.total = l.A + l.ws + l.g + l.beta + l.x;
    return l;
}

struct Req {
    sgbem_request r{};
    std::vector<double> ctrl, knots, a, phi, g;
    Layout lay;
    int64_t off = -1;
    double t_admit = 0.0;
};

struct RuleEntry {
    sgbem_rules r = nullptr;
    int refs = 0;
    bool ready = false;
    sgbem_status st = SGBEM_OK;
    std::string msg;
    uint64_t last = 0;
    int64_t off = -1, bytes = 0;
};

struct Worker {
    hipStream_t stream = nullptr;
    sgbem_ctx ctx = nullptr;
};

}  // namespace
}  // namespace sgbem

using namespace sgbem;

struct sgbem_server_s {
    sgbem_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    void *arena_mem = nullptr;
    Arena arena;
    void *rules_mem = nullptr;
    Arena rules_arena;
    std::mutex mu;
    std::condition_variable cv_disp, cv_work, cv_done, cv_rules;
    std::multimap<double, Req *> future;     // submitted, not yet released (equal times keep submission order)
    std::deque<Req *> waiting;                // released, not admitted
    std::deque<Req *> ready;                  // admitted, not yet taken by a slot
    std::deque<sgbem_completion> done;
    std::map<int64_t, RuleEntry> rules;       // key p << 32 | N
    uint64_t tick = 0;
    int in_flight = 0;
    bool stop = false, stop_workers = false;
    sgbem_server_info st{};
    std::vector<Worker> workers;
    std::thread dispatcher;
    std::vector<std::thread> threads;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

// Under s->mu: admit released requests while a slot and memory are free.
void admit(sgbem_server s)
{
    while (!s->stop && !s->waiting.empty() && s->in_flight < s->cfg.workers) {
        Req *q = s->waiting.front();
        const int64_t off = s->arena.alloc(int64_t(q->lay.total));
        if (off < 0) break;
        s->waiting.pop_front();
        q->off = off;
        q->t_admit = s->now();
        ++s->in_flight;
        s->st.peak_in_flight = std::max(s->st.peak_in_flight, s->in_flight);
        s->st.peak_bytes = std::max(s->st.peak_bytes, s->arena.used());
        s->ready.push_back(q);
        s->cv_work.notify_one();
    }
}

void dispatcher_loop(sgbem_server s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        const double t = s->now();
        while (!s->future.empty() && s->future.begin()->first <= t) {
            s->waiting.push_back(s->future.begin()->second);
            s->future.erase(s->future.begin());
        }
        admit(s);
        if (s->future.empty()) {
            s->cv_disp.wait(lk);
        } else {
            const auto when = s->t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                          std::chrono::duration<double>(s->future.begin()->first));
            s->cv_disp.wait_until(lk, when);
        }
    }
}

int64_t rule_key(int p, int N) { return (int64_t(p) << 32) | int64_t(N); }

// Take a reference to the rules of (p, N), building them into the rule arena
// on a miss (outside the lock, on the slot's stream).
sgbem_status acquire_rules(sgbem_server s, Worker &w, int p, int N, sgbem_rules &out, std::string &msg)
{
    const int64_t key = rule_key(p, N);
    const int64_t bytes = int64_t(rules_block_bytes(int64_t(2) * N));
    std::unique_lock<std::mutex> lk(s->mu);
    int64_t off = -1;
    for (;;) {
        auto it = s->rules.find(key);
        if (it != s->rules.end()) {   // cached, or being built by another slot
            RuleEntry &e = it->second;
            ++e.refs;
            e.last = ++s->tick;
            ++s->st.rules_hits;
            s->cv_rules.wait(lk, [&] { return e.ready; });
            if (e.st != SGBEM_OK) {
                msg = e.msg;
                const sgbem_status st = e.st;
                if (--e.refs == 0) {
                    s->rules_arena.release(e.off, e.bytes);
                    s->rules.erase(key);
                }
                return st;
            }
            out = e.r;
            return SGBEM_OK;
        }
        if (int(s->rules.size()) < s->cfg.max_rules) {
            off = s->rules_arena.alloc(bytes);
            if (off >= 0) break;
        }
        // evict the least recently used entry nobody holds
        auto victim = s->rules.end();
        for (auto jt = s->rules.begin(); jt != s->rules.end(); ++jt)
            if (jt->second.refs == 0 && jt->second.ready &&
                (victim == s->rules.end() || jt->second.last < victim->second.last))
                victim = jt;
        if (victim != s->rules.end()) {
            s->rules_arena.release(victim->second.off, victim->second.bytes);
            free_rules(victim->second.r);
            s->rules.erase(victim);
            continue;
        }
        s->cv_rules.wait(lk);   // every entry is held by a running request; one will be released
    }
    ++s->st.rules_misses;
    RuleEntry &e = s->rules[key];
    e.refs = 1;
    e.last = ++s->tick;
    e.off = off;
    e.bytes = bytes;
    lk.unlock();
    sgbem_rules r = nullptr;
    const sgbem_status st = make_rules(p, N, 1, static_cast<char *>(s->rules_mem) + off, w.stream, r);
    const std::string m = st ? std::string(sgbem_last_error()) : std::string();
    lk.lock();
    e.ready = true;
    e.st = st;
    e.msg = m;
    if (st == SGBEM_OK) {
        r->shared = true;
        e.r = r;
        out = r;
    } else {
        msg = m;
        if (--e.refs == 0) {
            s->rules_arena.release(e.off, e.bytes);
            s->rules.erase(key);
        }
    }
    s->cv_rules.notify_all();
    return st;
}

void release_rules(sgbem_server s, int p, int N)
{
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->rules.find(rule_key(p, N));
    if (it != s->rules.end()) --it->second.refs;
    s->cv_rules.notify_all();
}

// assemble -> right-hand side -> solve -> copy alpha to the host, on the slot's stream
sgbem_completion run(sgbem_server s, Worker &w, Req *q)
{
    sgbem_completion c;
    std::memset(&c, 0, sizeof c);
    c.tag = q->r.tag;
    c.t_arrival = q->r.arrival_s;
    c.t_admit = q->t_admit;
    c.footprint = int64_t(q->lay.total);
    const int N = q->r.N, p = q->r.p, prec = s->cfg.precision;
    char *base = static_cast<char *>(s->arena_mem) + q->off;
    void *dA = base;
    void *dws = base + q->lay.A;
    double *dg = reinterpret_cast<double *>(base + q->lay.A + q->lay.ws);
    double *dbeta = reinterpret_cast<double *>(base + q->lay.A + q->lay.ws + q->lay.g);
    double *dx = reinterpret_cast<double *>(base + q->lay.A + q->lay.ws + q->lay.g + q->lay.beta);
    std::string msg;
    sgbem_rules rules = nullptr;
    sgbem_status st = acquire_rules(s, w, p, N, rules, msg);
    const bool held = st == SGBEM_OK;
    if (held) {
        st = sgbem_assemble(w.ctx, &q->r.curve, rules, SGBEM_WQ, 0, prec, dA, N);
        if (st == SGBEM_OK) {
            const hipError_t e = hipMemcpyAsync(dg, q->g.data(), size_t(2) * N * 8, hipMemcpyHostToDevice, w.stream);
            if (e != hipSuccess) {
                st = SGBEM_E_DEVICE;
                msg = std::string("upload of g: ") + hipGetErrorString(e);
            }
        } else {
            msg = sgbem_last_error();
        }
        if (st == SGBEM_OK) {
            st = sgbem_rhs(w.ctx, &q->r.curve, rules, SGBEM_WQ, 0, dg, dbeta);
            if (st) msg = sgbem_last_error();
        }
        if (st == SGBEM_OK) {
            SolveResult res;
            st = sgbem_status(mixed_solve(N, dA, N, prec, dbeta, dx, s->cfg.tol, s->cfg.max_iter, dws, w.ctx->hbuf,
                                          w.stream, &w.ctx->lookahead, res, msg));
            c.iters = res.iters;
            c.backward_err = res.backward_err;
            if (st == SGBEM_OK || st == SGBEM_E_NOCONV) {
                hipError_t e = hipMemcpyAsync(q->r.x, dx, size_t(N) * 8, hipMemcpyDeviceToHost, w.stream);
                if (e == hipSuccess) e = hipStreamSynchronize(w.stream);
                if (e != hipSuccess) {
                    st = SGBEM_E_DEVICE;
                    msg = std::string("copy of alpha: ") + hipGetErrorString(e);
                }
            }
        }
    }
    // the request's memory and its rules are given back only after its last kernel
    (void)hipStreamSynchronize(w.stream);
    if (held) release_rules(s, p, N);
    c.status = st;
    if (st != SGBEM_OK) std::snprintf(c.message, sizeof c.message, "%s", msg.c_str());
    c.t_done = s->now();
    return c;
}

void worker_loop(sgbem_server s, int id)
{
    Worker &w = s->workers[id];
    (void)hipSetDevice(s->cfg.device);
    for (;;) {
        Req *q = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop_workers || !s->ready.empty(); });
            if (s->ready.empty()) return;
            q = s->ready.front();
            s->ready.pop_front();
        }
        sgbem_completion c;
        try {
            c = run(s, w, q);
        } catch (...) {
            std::memset(&c, 0, sizeof c);
            c.tag = q->r.tag;
            c.status = SGBEM_E_NOMEM;
            std::snprintf(c.message, sizeof c.message, "host allocation failed");
            c.t_arrival = q->r.arrival_s;
            c.t_admit = q->t_admit;
            c.t_done = s->now();
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->arena.release(q->off, int64_t(q->lay.total));
            --s->in_flight;
            ++s->st.completed;
            if (c.status != SGBEM_OK) ++s->st.failed;
            s->done.push_back(c);
            admit(s);
        }
        s->cv_done.notify_all();
        delete q;
    }
}

void teardown(sgbem_server s)
{
    for (Worker &w : s->workers) {
        if (w.ctx) (void)sgbem_ctx_destroy(w.ctx);
        if (w.stream) (void)hipStreamDestroy(w.stream);
    }
    for (auto &kv : s->rules) free_rules(kv.second.r);
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->rules_mem) (void)hipFree(s->rules_mem);
    delete s;
}

}  // namespace

extern "C" {

sgbem_status sgbem_server_footprint(int32_t N, int32_t precision, int64_t *bytes)
{
    if (!bytes) return set_err(SGBEM_E_INVAL, "bytes is NULL");
    if (N < 1 || N > 65536) return set_err(SGBEM_E_INVAL, "N must be in [1, 65536]");
    if (precision != SGBEM_FP64 && precision != SGBEM_FP32) return set_err(SGBEM_E_INVAL, "unknown precision");
    *bytes = int64_t(layout(N, precision).total);
    return SGBEM_OK;
}

sgbem_status sgbem_server_create(const sgbem_server_config *cfg, sgbem_server *out)
{
    if (!cfg || !out) return set_err(SGBEM_E_INVAL, "NULL argument");
    *out = nullptr;
    if (cfg->workers < 1 || cfg->workers > 64) return set_err(SGBEM_E_INVAL, "workers must be in [1, 64]");
    if (cfg->budget_bytes < 4096) return set_err(SGBEM_E_INVAL, "budget_bytes too small");
    if (cfg->precision != SGBEM_FP64 && cfg->precision != SGBEM_FP32) return set_err(SGBEM_E_INVAL, "unknown precision");
    if (cfg->max_N < 4 || cfg->max_N > 65536) return set_err(SGBEM_E_INVAL, "max_N must be in [4, 65536]");
    if (cfg->max_rules < 2 * cfg->workers + 1) return set_err(SGBEM_E_INVAL, "max_rules must be at least 2 workers + 1");
    if (cfg->max_iter < 0 || !(cfg->tol >= 0.0)) return set_err(SGBEM_E_INVAL, "bad tol or max_iter");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return set_err(SGBEM_E_INVAL, "no such HIP device");
    DeviceGuard g(cfg->device);
    auto *s = new (std::nothrow) sgbem_server_s;
    if (!s) return set_err(SGBEM_E_NOMEM, "host allocation failed");
    s->cfg = *cfg;
    s->st.arena_bytes = cfg->budget_bytes;
    hipError_t e = hipMalloc(&s->arena_mem, size_t(cfg->budget_bytes));
    const size_t rbytes = size_t(cfg->max_rules) * rules_block_bytes(int64_t(2) * cfg->max_N);
    if (e == hipSuccess) e = hipMalloc(&s->rules_mem, rbytes);
    if (e != hipSuccess) {
        const std::string m = std::string("server arenas: ") + hipGetErrorString(e);
        teardown(s);
        return set_err(e == hipErrorOutOfMemory ? SGBEM_E_NOMEM : SGBEM_E_DEVICE, m);
    }
    s->arena.reset(cfg->budget_bytes);
    s->rules_arena.reset(int64_t(rbytes));
    s->workers.resize(cfg->workers);
    for (Worker &w : s->workers) {
        sgbem_status st = SGBEM_OK;
        e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            w.stream = nullptr;
            st = SGBEM_E_DEVICE;
            set_err(st, std::string("stream: ") + hipGetErrorString(e));
        }
        if (st == SGBEM_OK) st = sgbem_ctx_create(cfg->device, w.stream, 0, &w.ctx);
        // geometry buffer for the largest request, so that no slot reallocates while serving,
        // and the solve's pinned host buffer
        if (st == SGBEM_OK) st = ensure(w.ctx, w.ctx->geo, size_t(cfg->max_N) * 2 * 3 * sizeof(double));
        if (st == SGBEM_OK) st = ensure_hbuf(w.ctx);
        if (st != SGBEM_OK) {
            const std::string m = sgbem_last_error();
            teardown(s);
            return set_err(st, m);
        }
    }
    s->t0 = std::chrono::steady_clock::now();
    try {
        s->dispatcher = std::thread(dispatcher_loop, s);
        for (int i = 0; i < cfg->workers; ++i) s->threads.emplace_back(worker_loop, s, i);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = s->stop_workers = true;
        }
        s->cv_disp.notify_all();
        s->cv_work.notify_all();
        if (s->dispatcher.joinable()) s->dispatcher.join();
        for (auto &t : s->threads) t.join();
        teardown(s);
        return set_err(SGBEM_E_NOMEM, "thread creation failed");
    }
    *out = s;
    return SGBEM_OK;
}

sgbem_status sgbem_server_submit(sgbem_server s, const sgbem_request *req)
{
    if (!s || !req) return set_err(SGBEM_E_INVAL, "NULL argument");
    const int p = req->p, N = req->N;
    if (p < 1 || p > 6) return set_err(SGBEM_E_UNSUPPORTED, "p must be in [1, 6]");
    if (N < 2 * (p + 1) || N > s->cfg.max_N) return set_err(SGBEM_E_INVAL, "N out of [2 (p + 1), max_N]");
    if (!req->g || !req->x) return set_err(SGBEM_E_INVAL, "g or x is NULL");
    if (!(req->arrival_s == req->arrival_s)) return set_err(SGBEM_E_INVAL, "arrival_s is NaN");
    sgbem_status st = check_curve(&req->curve);
    if (st) return st;
    if (req->curve.kind == SGBEM_CURVE_BSPLINE && req->curve.n_ctrl > 64)
        return set_err(SGBEM_E_UNSUPPORTED, "served curves travel inline: at most 64 control points");
    const Layout lay = layout(N, s->cfg.precision);
    if (int64_t(lay.total) > s->cfg.budget_bytes) {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->st.rejected;
        return set_err(SGBEM_E_NOMEM, "request footprint exceeds the server budget");
    }
    Req *q = new (std::nothrow) Req;
    if (!q) return set_err(SGBEM_E_NOMEM, "host allocation failed");
    try {
        q->r = *req;
        q->lay = lay;
        const sgbem_curve &cv = req->curve;
        if (cv.kind == SGBEM_CURVE_BSPLINE) {
            q->ctrl.assign(cv.ctrl_xy, cv.ctrl_xy + size_t(cv.n_ctrl) * 2);
            q->r.curve.ctrl_xy = q->ctrl.data();
            if (cv.knots) {
                q->knots.assign(cv.knots, cv.knots + size_t(cv.n_ctrl) + 1);
                q->r.curve.knots = q->knots.data();
            }
        } else if (cv.n_modes > 0) {
            q->a.assign(cv.a, cv.a + cv.n_modes);
            q->phi.assign(cv.phi, cv.phi + cv.n_modes);
            q->r.curve.a = q->a.data();
            q->r.curve.phi = q->phi.data();
        }
        q->g.assign(req->g, req->g + size_t(2) * N);
        q->r.g = q->g.data();
    } catch (...) {
        delete q;
        return set_err(SGBEM_E_NOMEM, "host allocation failed");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete q;
            return set_err(SGBEM_E_INVAL, "server is stopping");
        }
        s->future.emplace(req->arrival_s, q);
        ++s->st.submitted;
    }
    s->cv_disp.notify_one();
    return SGBEM_OK;
}

sgbem_status sgbem_server_poll(sgbem_server s, sgbem_completion *out, int32_t cap, double timeout_s, int32_t *n)
{
    if (!s || !n || (cap > 0 && !out)) return set_err(SGBEM_E_INVAL, "NULL argument");
    *n = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_s > 0.0)
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !s->done.empty(); });
    int32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return SGBEM_OK;
}

sgbem_status sgbem_server_clock(sgbem_server s, double *now_s)
{
    if (!s || !now_s) return set_err(SGBEM_E_INVAL, "NULL argument");
    *now_s = s->now();
    return SGBEM_OK;
}

sgbem_status sgbem_server_stats(sgbem_server s, sgbem_server_info *out)
{
    if (!s || !out) return set_err(SGBEM_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->waiting = int32_t(s->future.size() + s->waiting.size());
    out->in_flight = s->in_flight;
    out->rules_cached = int32_t(s->rules.size());
    return SGBEM_OK;
}

sgbem_status sgbem_server_destroy(sgbem_server s)
{
    if (!s) return SGBEM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &kv : s->future) delete kv.second;
        s->future.clear();
        for (Req *q : s->waiting) delete q;
        s->waiting.clear();
    }
    s->cv_disp.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_workers = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->threads) t.join();
    DeviceGuard g(s->cfg.device);
    teardown(s);
    return SGBEM_OK;
}

}  // extern "C"
