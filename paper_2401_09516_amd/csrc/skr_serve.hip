// Serving runtime of libskr (skr_serve_start .. skr_serve_stop): systems submitted one at a time
// join the nearest chain of their shape (the greedy nearest-neighbour rule of Alg. 1 applied
// online; chains as the independent slices of App. E), and host worker threads drive the chains,
// each on its own HIP stream with its own workspace and device-resident recycle space.
//
// Determinism: the chain a system joins and its position there are decided at submission, under
// one lock, in submission order, from exact distances; a chain solves its systems strictly in that
// order with fixed-order reductions. So every result depends only on the chain's history, not on
// how the workers interleave the chains. (A deferred admission is the exception: it is decided
// when capacity frees, which depends on timing; that can only happen when the arena or max_chains
// is exhausted.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "skr_host.hpp"

namespace skr {
void launch_dd_dist(hipStream_t s, const double* a, const double* const* bs, int K, long p, double* part,
                    double* out);
long dd_slices(long p);

namespace {

enum { JOB_WAITING = 0, JOB_QUEUED = 1, JOB_RUNNING = 2, JOB_DONE = 3 };

struct Job {
    skr_op op{};
    const double* b = nullptr;
    double* x = nullptr;
    skr_opts opts{};
    int64_t p = 0;
    double pnorm2 = 0.0;          // ||params||^2 (host, for the split rule)
    double* params = nullptr;     // device copy, kept while admission is deferred
    int chain = -1;
    int64_t pos = -1;
    int state = JOB_WAITING;
    int rc = SKR_OK;
    std::string err;
    skr_result res{};
};

struct Chain {
    int id = 0;
    int n = 0, m = 0, k = 0;
    uint32_t mixed = 0;
    int64_t p = 0;
    hipStream_t stream = nullptr;
    skr_ctx* ctx = nullptr;       // own stream, workspace and recycle space
    double* tail = nullptr;       // params of the most recently admitted system (device)
    int kin = 0;                  // recycled vectors held for the next system
    std::deque<uint64_t> queue;   // admitted, not yet started
    bool busy = false;
    int64_t admitted = 0;
    size_t bytes = 0;
    uint64_t last_use = 0;
    skr_ctx* owner = nullptr;     // the serving context (its allocator holds tail)
};

}  // namespace

struct Server {
    skr_ctx* owner = nullptr;
    skr_serve_opts o{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<std::thread> workers;
    std::map<int, Chain*> chains;            // by id (ordered: ties go to the lower id)
    std::unordered_map<uint64_t, Job> jobs;
    std::deque<uint64_t> deferred;
    uint64_t next_ticket = 1;
    int next_chain = 0;
    uint64_t clock = 0;
    size_t bytes_in_use = 0;
    bool stopping = false;
    skr_serve_stats st{};
    // distance scratch on the owner's stream
    double* dpart = nullptr;
    size_t dpart_cap = 0;
    double* dout = nullptr;
    double* hout = nullptr;       // pinned
    const double** dptrs = nullptr;   // device array of the candidates' tail pointers
    const double** hptrs = nullptr;   // pinned staging of that array
    int dout_cap = 0;
    double* zero = nullptr;       // zeros, for ||params||^2 with the same exact arithmetic
    size_t zero_cap = 0;
};

namespace {

size_t chain_bytes(int n, int m, int k, int64_t p) {
    return work_bytes(n, m, k) + round256((size_t)p * sizeof(double));
}

bool same_shape(const Chain* c, const Job& j) {
    return c->n == j.op.n && c->p == j.p && c->m == j.opts.m && c->k == j.opts.k &&
           c->mixed == (j.opts.flags & SKR_FLAG_MIXED);
}

void free_chain(Chain* c) {
    if (c->ctx) {
        (void)hipStreamSynchronize(c->stream);
        skr_ctx_destroy(c->ctx);
    }
    if (c->tail) dev_free(c->owner, c->tail);
    c->tail = nullptr;
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// d2 from params to the tail of every chain in cand, in that order (owner stream; lock held).
int distances(Server* S, const double* params, int64_t p, const std::vector<Chain*>& cand, std::vector<double>& d2) {
    d2.assign(cand.size(), NAN);
    if (cand.empty()) return SKR_OK;
    const size_t need = 2 * (size_t)dd_slices((long)p) * cand.size();
    if (S->dpart_cap < need) {
        if (S->dpart) (void)hipFree(S->dpart);
        S->dpart = nullptr;
        S->dpart_cap = 0;
        HIPCHK(hipMalloc((void**)&S->dpart, need * sizeof(double)));
        S->dpart_cap = need;
    }
    if (S->dout_cap < (int)cand.size()) {
        if (S->dout) (void)hipFree(S->dout);
        if (S->hout) (void)hipHostFree(S->hout);
        if (S->dptrs) (void)hipFree(S->dptrs);
        if (S->hptrs) (void)hipHostFree(S->hptrs);
        S->dout = nullptr;
        S->hout = nullptr;
        S->dptrs = nullptr;
        S->hptrs = nullptr;
        S->dout_cap = 0;
        HIPCHK(hipMalloc((void**)&S->dout, cand.size() * sizeof(double)));
        HIPCHK(hipHostMalloc((void**)&S->hout, cand.size() * sizeof(double), hipHostMallocDefault));
        HIPCHK(hipMalloc((void**)&S->dptrs, cand.size() * sizeof(double*)));
        HIPCHK(hipHostMalloc((void**)&S->hptrs, cand.size() * sizeof(double*), hipHostMallocDefault));
        S->dout_cap = (int)cand.size();
    }
    hipStream_t s = S->owner->stream;
    for (size_t c = 0; c < cand.size(); ++c) S->hptrs[c] = cand[c]->tail;
    HIPCHK(hipMemcpyAsync(S->dptrs, S->hptrs, cand.size() * sizeof(double*), hipMemcpyHostToDevice, s));
    launch_dd_dist(s, params, S->dptrs, (int)cand.size(), (long)p, S->dpart, S->dout);
    HIPLAUNCHCHK();
    HIPCHK(hipMemcpyAsync(S->hout, S->dout, cand.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t c = 0; c < cand.size(); ++c) d2[c] = S->hout[c];
    return SKR_OK;
}

// Room for one more chain of `bytes` (its workspace block of `wbytes` and its parameter tail): under
// the chain count and the byte budget of the serving options, and, on a context with a caller arena,
// both blocks must fit the arena's free blocks now.
bool can_add(Server* S, size_t bytes, size_t wbytes) {
    if ((int)S->chains.size() >= S->o.max_chains) return false;
    if (S->o.arena_bytes != 0 && S->bytes_in_use + bytes > S->o.arena_bytes) return false;
    if (S->owner->arena) {
        const size_t sz[2] = {wbytes, bytes - wbytes};
        if (!S->owner->arena->can_fit(sz, 2)) return false;
    }
    return true;
}

// Retire idle chains, least recently used first, until a chain of `bytes` can be added.
void make_room(Server* S, size_t bytes, size_t wbytes) {
    while (!can_add(S, bytes, wbytes)) {
        Chain* victim = nullptr;
        for (auto& kv : S->chains) {
            Chain* c = kv.second;
            if (c->busy || !c->queue.empty()) continue;
            if (!victim || c->last_use < victim->last_use) victim = c;
        }
        if (!victim) return;
        S->chains.erase(victim->id);
        S->bytes_in_use -= victim->bytes;
        S->st.chains_retired++;
        free_chain(victim);
    }
}

int new_chain(Server* S, const Job& j, Chain** out) {
    *out = nullptr;
    Chain* c = new Chain();
    c->id = S->next_chain++;
    c->n = j.op.n;
    c->m = j.opts.m;
    c->k = j.opts.k;
    c->mixed = j.opts.flags & SKR_FLAG_MIXED;
    c->p = j.p;
    c->bytes = chain_bytes(c->n, c->m, c->k, c->p);
    c->owner = S->owner;
    int rc = SKR_OK;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        rc = fail(SKR_EHIP, "chain stream creation failed");
    } else if ((rc = ctx_make(S->owner->device, c->stream, &c->ctx, S->owner->arena)) == SKR_OK) {
        if ((rc = prepare_solve(c->ctx, c->n, j.opts)) == SKR_OK &&
            dev_alloc(S->owner, (void**)&c->tail, (size_t)c->p * sizeof(double)) != hipSuccess)
            rc = fail(SKR_ENOMEM, "chain parameter buffer (%lld doubles)", (long long)c->p);
    }
    if (rc) {
        free_chain(c);
        return rc;
    }
    S->chains[c->id] = c;
    S->bytes_in_use += c->bytes;
    S->st.chains_created++;
    *out = c;
    return SKR_OK;
}

// Assign job t (params on the device at `params`) to a chain, or leave it deferred (*assigned
// false). Lock held.
int assign(Server* S, uint64_t t, const double* params, bool& assigned) {
    assigned = false;
    Job& j = S->jobs[t];
    // candidates: the chains of the job's shape that are not full (all of them when every one is
    // full and no chain can be added, so the job still joins the nearest)
    const size_t bytes = chain_bytes(j.op.n, j.opts.m, j.opts.k, j.p);
    const size_t wbytes = work_bytes(j.op.n, j.opts.m, j.opts.k);
    const int cap = S->o.max_chain_systems;
    std::vector<Chain*> cand, full;
    for (auto& kv : S->chains)
        if (same_shape(kv.second, j)) (cap > 0 && kv.second->admitted >= cap ? full : cand).push_back(kv.second);
    bool all_full = cand.empty() && !full.empty();
    if (all_full && !can_add(S, bytes, wbytes)) {
        cand.swap(full);
        all_full = false;
    }
    std::vector<double> d2;
    int rc = distances(S, params, j.p, cand, d2);
    if (rc) return rc;
    Chain* best = nullptr;
    double bd = INFINITY;
    for (size_t c = 0; c < cand.size(); ++c)      // strict <: ties to the lower id, NaN never chosen
        if (d2[c] < bd) {
            bd = d2[c];
            best = cand[c];
        }
    if (!best && !cand.empty()) best = cand[0];       // no finite distance: the lowest chain id
    // A shape without a chain gets one, retiring idle chains if needed, or waits (deferred). A shape
    // with chains splits off a new one only when there is room without retiring anything: which
    // chains are idle depends on timing, and the choice must not. So does a shape whose chains are
    // all full.
    Chain* target = best;
    if (all_full) {
        if ((rc = new_chain(S, j, &target))) return rc;
    } else if (!best) {
        make_room(S, bytes, wbytes);
        if (!can_add(S, bytes, wbytes)) return SKR_OK;       // deferred
        if ((rc = new_chain(S, j, &target))) return rc;
    } else if (bd > S->o.split_d2_rel * j.pnorm2 && can_add(S, bytes, wbytes)) {
        if ((rc = new_chain(S, j, &target))) return rc;
    }
    HIPCHK(hipMemcpyAsync(target->tail, params, (size_t)j.p * sizeof(double), hipMemcpyDeviceToDevice,
                          S->owner->stream));
    HIPCHK(hipStreamSynchronize(S->owner->stream));
    j.chain = target->id;
    j.pos = target->admitted++;
    j.state = JOB_QUEUED;
    target->queue.push_back(t);
    assigned = true;
    return SKR_OK;
}

// Admit deferred jobs in submission order while there is room (lock held).
void admit_deferred(Server* S) {
    while (!S->deferred.empty()) {
        const uint64_t t = S->deferred.front();
        Job& j = S->jobs[t];
        bool ok = false;
        const int rc = assign(S, t, j.params, ok);
        if (rc) {
            j.rc = rc;
            j.err = last_error();
            j.state = JOB_DONE;
        } else if (!ok) {
            return;
        }
        if (j.params) (void)hipFree(j.params);
        j.params = nullptr;
        S->deferred.pop_front();
    }
}

void worker_main(Server* S) {
    (void)hipSetDevice(S->owner->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // the idle chain whose next system was submitted first
        Chain* pick = nullptr;
        for (auto& kv : S->chains) {
            Chain* c = kv.second;
            if (c->busy || c->queue.empty()) continue;
            if (!pick || c->queue.front() < pick->queue.front()) pick = c;
        }
        if (!pick) {
            bool any_running = false;
            for (auto& kv : S->chains) any_running = any_running || kv.second->busy;
            if (!any_running && !S->deferred.empty()) {
                const size_t before = S->deferred.size();
                admit_deferred(S);       // everything is idle, so there is room now
                if (S->deferred.size() != before) {
                    S->cv_done.notify_all();
                    continue;
                }
            }
            if (S->stopping && S->deferred.empty() && !any_running) return;
            S->cv_work.wait(lk);
            continue;
        }
        const uint64_t t = pick->queue.front();
        pick->queue.pop_front();
        pick->busy = true;
        Job& j = S->jobs[t];
        j.state = JOB_RUNNING;
        const skr_op op = j.op;
        const double* b = j.b;
        double* x = j.x;
        const skr_opts o = j.opts;
        lk.unlock();
        skr_result res;
        std::memset(&res, 0, sizeof res);
        int rc = prepare_solve(pick->ctx, pick->n, o);
        if (rc == SKR_OK) rc = solve_system(pick->ctx, op, b, x, o, pick->kin, res);
        const std::string err = rc ? last_error() : std::string();
        lk.lock();
        Job& jd = S->jobs[t];
        jd.rc = rc;
        jd.err = err;
        jd.res = res;
        jd.state = JOB_DONE;
        if (rc) pick->kin = 0;           // the recycle space may be incomplete after a failure
        pick->busy = false;
        pick->last_use = ++S->clock;
        S->st.completed++;
        if (!S->deferred.empty()) admit_deferred(S);
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

int collect(Server* S, uint64_t t, skr_result* out) {
    auto it = S->jobs.find(t);
    if (it == S->jobs.end()) return fail(SKR_EINVAL, "unknown or already collected ticket %llu", (unsigned long long)t);
    Job& j = it->second;
    if (j.state != JOB_DONE) return SKR_PENDING;
    *out = j.res;
    const int rc = j.rc;
    if (rc) fail(rc, "%s", j.err.c_str());
    S->jobs.erase(it);
    return rc;
}

}  // namespace

void serve_free(skr_ctx* ctx) {
    if (ctx && ctx->server) skr_serve_stop(ctx);
}

}  // namespace skr

using namespace skr;

extern "C" {

int skr_serve_start(skr_ctx* ctx, const skr_serve_opts* opts) {
    if (!ctx || !opts) return fail(SKR_EINVAL, "NULL argument");
    if (ctx->server) return fail(SKR_EINVAL, "serving already started on this context");
    if (opts->max_chains < 1 || opts->workers < 1 || opts->workers > 64)
        return fail(SKR_EINVAL, "need max_chains >= 1 and 1 <= workers <= 64");
    if (!(opts->split_d2_rel >= 0.0)) return fail(SKR_EINVAL, "split_d2_rel must be >= 0 (INFINITY: never split)");
    if (opts->max_chain_systems < 0) return fail(SKR_EINVAL, "max_chain_systems must be >= 0 (0: no limit)");
    HIPCHK(hipSetDevice(ctx->device));
    Server* S = new Server();
    S->owner = ctx;
    S->o = *opts;
    ctx->server = S;
    for (int q = 0; q < opts->workers; ++q) S->workers.emplace_back(worker_main, S);
    return SKR_OK;
}

int skr_submit(skr_ctx* ctx, const skr_op* op, const double* params_dev, int64_t p, const double* b_dev,
               double* x_dev, const skr_opts* opts, uint64_t* ticket) {
    if (!ctx || !ctx->server) return fail(SKR_EINVAL, "serving is not started on this context");
    if (!op || !params_dev || p < 1 || !b_dev || !x_dev || !ticket) return fail(SKR_EINVAL, "bad argument");
    int rc = check_opts(opts);
    if (rc) return rc;
    DevOp d;
    int64_t nv;
    if ((rc = to_devop(*op, d, nv))) return rc;
    Server* S = ctx->server;
    const size_t bytes = chain_bytes(op->n, opts->m, opts->k, p);
    if (S->o.arena_bytes && bytes > S->o.arena_bytes)
        return fail(SKR_ENOMEM, "a chain of this shape needs %zu bytes, more than the arena (%llu)", bytes,
                    (unsigned long long)S->o.arena_bytes);
    if (ctx->arena && bytes > ctx->arena->size)
        return fail(SKR_ENOMEM, "a chain of this shape needs %zu bytes, more than the context's arena (%zu)",
                    bytes, ctx->arena->size);
    HIPCHK(hipSetDevice(ctx->device));
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->stopping) return fail(SKR_EINVAL, "serving is stopping");
    // ||params||^2 for the split rule (same exact distance, to a zero vector)
    double pn2 = 0.0;
    if (S->o.split_d2_rel < INFINITY) {
        if (S->zero_cap < (size_t)p) {
            if (S->zero) (void)hipFree(S->zero);
            S->zero = nullptr;
            S->zero_cap = 0;
            HIPCHK(hipMalloc((void**)&S->zero, (size_t)p * sizeof(double)));
            HIPCHK(hipMemsetAsync(S->zero, 0, (size_t)p * sizeof(double), ctx->stream));
            S->zero_cap = (size_t)p;
        }
        Chain tmp;
        tmp.tail = S->zero;
        std::vector<Chain*> one{&tmp};
        std::vector<double> v;
        rc = distances(S, params_dev, p, one, v);
        tmp.tail = nullptr;
        if (rc) return rc;
        pn2 = v[0];
    }
    const uint64_t t = S->next_ticket++;
    Job& j = S->jobs[t];
    j.op = *op;
    j.b = b_dev;
    j.x = x_dev;
    j.opts = *opts;
    j.p = p;
    j.pnorm2 = pn2;
    S->st.submitted++;
    bool ok = false;
    if (S->deferred.empty()) {
        rc = assign(S, t, params_dev, ok);
        if (rc) {
            S->jobs.erase(t);
            S->st.submitted--;
            return rc;
        }
    }
    if (!ok) {
        // deferred: keep a copy of the parameters until a chain can take the system
        if (hipMalloc((void**)&j.params, (size_t)p * sizeof(double)) != hipSuccess) {
            S->jobs.erase(t);
            S->st.submitted--;
            return fail(SKR_ENOMEM, "deferred parameter copy");
        }
        HIPCHK(hipMemcpyAsync(j.params, params_dev, (size_t)p * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        S->deferred.push_back(t);
    }
    *ticket = t;
    S->cv_work.notify_all();
    return SKR_OK;
}

int skr_poll(skr_ctx* ctx, uint64_t ticket, skr_result* out) {
    if (!ctx || !ctx->server || !out) return fail(SKR_EINVAL, "serving is not started, or NULL result");
    Server* S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    return collect(S, ticket, out);
}

int skr_wait(skr_ctx* ctx, uint64_t ticket, skr_result* out) {
    if (!ctx || !ctx->server || !out) return fail(SKR_EINVAL, "serving is not started, or NULL result");
    Server* S = ctx->server;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        const int rc = collect(S, ticket, out);
        if (rc != SKR_PENDING) return rc;
        S->cv_done.wait(lk);
    }
}

int skr_ticket_chain(skr_ctx* ctx, uint64_t ticket, int32_t* chain, int64_t* position) {
    if (!ctx || !ctx->server || !chain || !position) return fail(SKR_EINVAL, "serving is not started, or NULL out");
    Server* S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(SKR_EINVAL, "unknown or already collected ticket");
    *chain = it->second.chain;
    *position = it->second.pos;
    return SKR_OK;
}

int skr_serve_stats_get(skr_ctx* ctx, skr_serve_stats* out) {
    if (!ctx || !ctx->server || !out) return fail(SKR_EINVAL, "serving is not started, or NULL out");
    Server* S = ctx->server;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->chains_live = (int32_t)S->chains.size();
    out->deferred = (int32_t)S->deferred.size();
    out->bytes_in_use = S->bytes_in_use;
    return SKR_OK;
}

int skr_serve_stop(skr_ctx* ctx) {
    if (!ctx || !ctx->server) return SKR_OK;
    Server* S = ctx->server;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto& th : S->workers) th.join();
    (void)hipSetDevice(ctx->device);
    for (auto& kv : S->chains) free_chain(kv.second);
    for (auto& kv : S->jobs)
        if (kv.second.params) (void)hipFree(kv.second.params);
    if (S->dpart) (void)hipFree(S->dpart);
    if (S->dout) (void)hipFree(S->dout);
    if (S->hout) (void)hipHostFree(S->hout);
    if (S->zero) (void)hipFree(S->zero);
    if (S->dptrs) (void)hipFree(S->dptrs);
    if (S->hptrs) (void)hipHostFree(S->hptrs);
    delete S;
    ctx->server = nullptr;
    return SKR_OK;
}

}  // extern "C"
