// Several sorted chains in one launch (skr_solve_chains): the sorted order cut into contiguous
// chains, one per worker (App. E), advanced in lockstep on one stream. Every kernel launch covers
// all chains that take part in that phase (chain = grid row), so one launch advances, say, Arnoldi
// step j of every live chain; a chain whose cycle stopped early is skipped by its stop flag, as in
// the single-chain path. Each chain has its own workspace and recycle space, and runs exactly the
// kernel bodies and launch shapes of skr_solve_sequence, so its results equal that chain solved
// alone, bit for bit. The host mirrors the per-system control of skr_solve_sequence for every chain.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "skr_host.hpp"

namespace skr {
void blaunch_gather(const Batch&, CtrlHost*, int*);
void blaunch_clear_nonfinite(const Batch&);
void blaunch_init(const Batch&, double);
void blaunch_check_finite(const Batch&, long);
void blaunch_to_f32(const Batch&, long);
void blaunch_check_sym(const Batch&);
void blaunch_zero(const Batch&);
void blaunch_true_residual(const Batch&);
void blaunch_spmm(const Batch&);
void blaunch_startup_gram(const Batch&, int);
void blaunch_chol(const Batch&, int);
void blaunch_startup_apply(const Batch&, int, int);
void blaunch_startup_project(const Batch&, int, int);
void blaunch_apply_c(const Batch&, int, int);
void blaunch_step(const Batch&, int, int, int, hipEvent_t*);
void blaunch_close_basis(const Batch&, int, int, int);
void blaunch_cycle_gram(const Batch&, int, int);
void blaunch_cycle_dense(const Batch&, int);
void blaunch_cycle_update(const Batch&, int);
}  // namespace skr

using namespace skr;

namespace skr {
// What skr_solve_chains keeps on a context between calls: one context per chain (its workspace,
// the recycle space it carries, the launch-length prediction) and the device and pinned tables.
struct ChainSet {
    std::vector<skr_ctx*> sub;
    ChainDesc* tab = nullptr;     // device, cap entries
    CtrlHost* gath_d = nullptr;   // device, cap entries
    int* keff_d = nullptr;
    CtrlHost* gath_h = nullptr;   // pinned
    int* keff_h = nullptr;
    int cap = 0;
};
void chains_free(skr_ctx* ctx) {
    ChainSet* S = ctx->chains;
    if (!S) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (skr_ctx* c : S->sub) skr_ctx_destroy(c);
    dev_free(ctx, S->tab);
    dev_free(ctx, S->gath_d);
    dev_free(ctx, S->keff_d);
    if (S->gath_h) (void)hipHostFree(S->gath_h);
    if (S->keff_h) (void)hipHostFree(S->keff_h);
    delete S;
    ctx->chains = nullptr;
}
}  // namespace skr

namespace {

// Host state of one chain during the solve of its current system (the locals of the single-chain
// solve, one set per chain).
struct CState {
    skr_ctx* sub = nullptr;       // owns the chain's workspace; enqueues on the batch stream
    int64_t first = 0, len = 0;   // its systems: order[first .. first + len)
    int kin = 0;                  // recycled columns carried to the next system
    // current system
    int64_t idx = -1;
    bool live = false;            // still being solved
    bool cycling = false;         // takes part in the cycle loop
    int status = -1;
    int64_t iters = 0, spmv = 0;
    int cycles = 0, kc = 0;
    bool r_fresh = true, z_valid = false, input_nf = false;
    int prev_jd = 0, prev_scyc = 0, scyc = 0;
    int64_t nv = 0;               // stored operator values (CSR), for the profile's byte counts
    double prev_rate = 0.0, est = 0.0, bnorm = 0.0, tol_abs = 0.0;
    skr_result res{};
    std::chrono::steady_clock::time_point t0;
};

size_t elem(const Work& w) { return w.mixed ? sizeof(float) : sizeof(double); }
const void* bcol(const Work& w, int c) { return (const char*)w.basis + (size_t)c * w.ld * elem(w); }

}  // namespace

extern "C" int skr_solve_chains(skr_ctx* ctx, int32_t C, const int64_t* chain_start, const skr_op* ops,
                                const double* const* b_dev, double* const* x_dev, int64_t N, const int64_t* order,
                                const skr_opts* opts, skr_result* results_host) {
    if (!ctx || !opts) return fail(SKR_EINVAL, "NULL context or options");
    if (C < 1 || !chain_start) return fail(SKR_EINVAL, "need C >= 1 and chain_start");
    if (N < 0) return fail(SKR_EINVAL, "N must be >= 0");
    if (chain_start[0] != 0 || chain_start[C] != N) return fail(SKR_EINVAL, "chain_start must run from 0 to N");
    for (int c = 0; c < C; ++c)
        if (chain_start[c + 1] < chain_start[c]) return fail(SKR_EINVAL, "chain_start must not decrease");
    if (N == 0) return SKR_OK;
    if (!ops || !b_dev || !x_dev || !results_host) return fail(SKR_EINVAL, "NULL array argument");
    int rc = check_opts(opts);
    if (rc) return rc;
    const int n = ops[0].n;
    std::vector<char> seen((size_t)N, 0);
    for (int64_t q = 0; q < N; ++q) {
        const int64_t idx = order ? order[q] : q;
        if (idx < 0 || idx >= N || seen[(size_t)idx]) return fail(SKR_EINVAL, "order is not a permutation of 0..N-1");
        seen[(size_t)idx] = 1;
        if (ops[idx].n != n) return fail(SKR_EINVAL, "all operators must have the same n");
        if (ops[idx].kind != ops[0].kind) return fail(SKR_EINVAL, "all operators must be of one kind");
        if (!b_dev[idx] || !x_dev[idx]) return fail(SKR_EINVAL, "NULL b or x pointer for system %lld", (long long)idx);
        DevOp d;
        int64_t nv;
        if ((rc = to_devop(ops[idx], d, nv))) return rc;
    }
    const int mixed_flag = (opts->flags & SKR_FLAG_MIXED) ? 1 : 0;
    const bool cont = (opts->flags & SKR_FLAG_CONTINUE) != 0;
    if (cont) {
        ChainSet* S = ctx->chains;
        bool ok = S && (int)S->sub.size() == C;
        for (int c = 0; ok && c < C; ++c) {
            const skr_ctx* q = S->sub[c];
            ok = q->carry_valid && q->carry_n == n && q->carry_m == opts->m && q->carry_kmax == opts->k &&
                 q->carry_mixed == mixed_flag;
        }
        if (!ok)
            return fail(SKR_EINVAL, "SKR_FLAG_CONTINUE: the context carries no %d chains for n = %d, m = %d, k = %d "
                        "and this precision", C, n, opts->m, opts->k);
    }
    HIPCHK(hipSetDevice(ctx->device));
    const int m = opts->m, k = opts->k, kind = ops[0].kind;
    const double rtol = opts->rtol;
    const int64_t maxit = opts->maxit;
    hipStream_t s = ctx->stream;

    // chain contexts (own workspaces on the caller's stream and arena), kept for the next call
    if (!ctx->chains) ctx->chains = new ChainSet();
    ChainSet& S = *ctx->chains;
    while ((int)S.sub.size() > C) {
        HIPCHK(hipStreamSynchronize(s));
        skr_ctx_destroy(S.sub.back());
        S.sub.pop_back();
    }
    while ((int)S.sub.size() < C) {
        skr_ctx* q = nullptr;
        if ((rc = ctx_make(ctx->device, s, &q, ctx->arena))) return rc;
        S.sub.push_back(q);
    }
    if (S.cap < C) {
        HIPCHK(hipStreamSynchronize(s));
        dev_free(ctx, S.tab);
        dev_free(ctx, S.gath_d);
        dev_free(ctx, S.keff_d);
        if (S.gath_h) (void)hipHostFree(S.gath_h);
        if (S.keff_h) (void)hipHostFree(S.keff_h);
        S.tab = nullptr;
        S.gath_d = nullptr;
        S.keff_d = nullptr;
        S.gath_h = nullptr;
        S.keff_h = nullptr;
        S.cap = 0;
        if (dev_alloc(ctx, (void**)&S.tab, sizeof(ChainDesc) * C) != hipSuccess ||
            dev_alloc(ctx, (void**)&S.gath_d, sizeof(CtrlHost) * C) != hipSuccess ||
            dev_alloc(ctx, (void**)&S.keff_d, sizeof(int) * C) != hipSuccess)
            return fail(SKR_ENOMEM, "chain tables for %d chains", C);
        HIPCHK(hipHostMalloc((void**)&S.gath_h, sizeof(CtrlHost) * C, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&S.keff_h, sizeof(int) * C, hipHostMallocDefault));
        S.cap = C;
    }
    std::vector<CState> cs((size_t)C);
    std::vector<ChainDesc> hd((size_t)C);
    ChainDesc* dd = S.tab;
    CtrlHost* hg = S.gath_h;
    CtrlHost* dg = S.gath_d;
    int* hk = S.keff_h;
    int* dk = S.keff_d;
    for (int c = 0; c < C; ++c) {
        cs[c].sub = S.sub[c];
        cs[c].first = chain_start[c];
        cs[c].len = chain_start[c + 1] - chain_start[c];
        cs[c].kin = cont ? S.sub[c]->carry_k : 0;
        S.sub[c]->carry_valid = false;
        if ((rc = prepare_solve(cs[c].sub, n, *opts))) return rc;
    }
    const Work& w0 = cs[0].sub->w;
    Batch B{s, dd, C, w0};
    const bool mixed = w0.mixed != 0;
    const bool profile = (opts->flags & SKR_FLAG_PROFILE) && ctx->ev_ok;

    auto upload = [&]() -> int {
        // the kernels of the previous phase read the table: finish them before it changes
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipMemcpy(dd, hd.data(), sizeof(ChainDesc) * C, hipMemcpyHostToDevice));
        return SKR_OK;
    };
    auto gather = [&]() -> int {
        blaunch_gather(B, dg, dk);
        HIPLAUNCHCHK();
        HIPCHK(hipMemcpyAsync(hg, dg, sizeof(CtrlHost) * C, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hk, dk, sizeof(int) * C, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return SKR_OK;
    };
    auto mask = [&](auto pred) {
        bool any = false;
        for (int c = 0; c < C; ++c) {
            hd[c].on = pred(c) ? 1 : 0;
            any = any || hd[c].on;
        }
        return any;
    };
    auto finish = [&](int c, int status) {
        CState& q = cs[c];
        q.status = status;
        q.live = false;
        q.cycling = false;
    };
    // x += U C^T r, r -= C C^T r for the chains in `sel`, grouped by kc (uniform per launch)
    auto project = [&](auto sel) -> int {
        std::vector<int> ks;
        for (int c = 0; c < C; ++c)
            if (sel(c) && cs[c].kc > 0) ks.push_back(cs[c].kc);
        std::sort(ks.begin(), ks.end());
        ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
        for (int g : ks) {
            mask([&](int c) { return sel(c) && cs[c].kc == g; });
            for (int c = 0; c < C; ++c) {
                hd[c].kc = cs[c].kc;
                hd[c].Lp = {{bcol(cs[c].sub->w, 0), nullptr, nullptr, nullptr}, {g, 0, 0, 0}};
            }
            int r2;
            if ((r2 = upload())) return r2;
            blaunch_startup_project(B, g, 1);
            HIPLAUNCHCHK();
        }
        return SKR_OK;
    };

    int64_t maxlen = 0;
    for (auto& q : cs) maxlen = std::max(maxlen, q.len);
    bool any_maxit = false;
    for (int64_t t = 0; t < maxlen; ++t) {
        // ---- set-up of system t of every chain that has one
        long cmax[3] = {0, 0, 0};
        for (int c = 0; c < C; ++c) {
            CState& q = cs[c];
            q = CState{q.sub, q.first, q.len, q.kin};
            ChainDesc& h = hd[c];
            std::memset(&h, 0, sizeof h);
            h.w = q.sub->w;
            if (t >= q.len) continue;
            const int64_t pos = q.first + t;
            q.idx = order ? order[pos] : pos;
            q.live = true;
            q.t0 = std::chrono::steady_clock::now();
            int64_t nv = 0;
            to_devop(ops[q.idx], h.op, nv);
            q.nv = nv;
            h.b = b_dev[q.idx];
            h.x = x_dev[q.idx];
            if (h.op.kind == SKR_OP_CSR) {
                h.cnt[0] = (long)nv;
                h.arr[0] = h.op.val;
            } else {
                const long nzl = h.op.kind == SKR_OP_STENCIL7 ? (long)h.op.nz : 1L;
                h.cnt[0] = nzl * h.op.ny * (h.op.nx + 1);
                h.cnt[1] = nzl * (h.op.ny + 1) * h.op.nx;
                h.arr[0] = h.op.ax;
                h.arr[1] = h.op.ay;
                if (h.op.kind == SKR_OP_STENCIL7) {
                    h.cnt[2] = (nzl + 1) * h.op.ny * h.op.nx;
                    h.arr[2] = h.op.az;
                }
            }
            for (int p = 0; p < 3; ++p) cmax[p] = std::max(cmax[p], h.cnt[p]);
            if (mixed) {
                skr_ctx* sub = q.sub;
                const size_t need = (size_t)(h.cnt[0] + h.cnt[1] + h.cnt[2]);
                if (sub->op32_cap < need) {
                    dev_free(sub, sub->op32);
                    sub->op32 = nullptr;
                    sub->op32_cap = 0;
                    if (dev_alloc(sub, (void**)&sub->op32, need * sizeof(float)) != hipSuccess)
                        return fail(SKR_ENOMEM, "FP32 operator copy (%zu bytes)", need * sizeof(float));
                    sub->op32_cap = need;
                }
                h.arr32[0] = sub->op32;
                h.arr32[1] = sub->op32 + h.cnt[0];
                h.arr32[2] = sub->op32 + h.cnt[0] + h.cnt[1];
                if (h.op.kind == SKR_OP_CSR) {
                    h.op.val32 = h.arr32[0];
                } else {
                    h.op.ax32 = h.arr32[0];
                    h.op.ay32 = h.arr32[1];
                    h.op.az32 = h.cnt[2] ? h.arr32[2] : nullptr;
                }
            }
        }
        // ---- init, input checks (Alg. 2 inputs), the FP32 operator copy
        mask([&](int c) { return cs[c].live; });
        for (int p = 0; p < 3; ++p) {
            if (p > 0 && cmax[p] == 0) continue;
            for (int c = 0; c < C; ++c) hd[c].part = p;
            if ((rc = upload())) return rc;
            if (p == 0) {
                blaunch_clear_nonfinite(B);
                blaunch_init(B, rtol);
                blaunch_check_sym(B);
            }
            blaunch_check_finite(B, cmax[p]);
            HIPLAUNCHCHK();
        }
        if ((rc = gather())) return rc;
        std::vector<char> zx((size_t)C, 0);     // x = 0 for these chains (non-finite input or iterate)
        auto zero_x = [&]() -> int {
            if (!mask([&](int c) { return zx[c] != 0; })) return SKR_OK;
            int r2;
            if ((r2 = upload())) return r2;
            blaunch_zero(B);
            HIPLAUNCHCHK();
            std::fill(zx.begin(), zx.end(), 0);
            return SKR_OK;
        };
        for (int c = 0; c < C; ++c) {
            CState& q = cs[c];
            if (!q.live) continue;
            const CtrlHost& h = hg[c];
            if (h.nonfinite || !std::isfinite(h.bnorm)) {
                // the carried recycle space is passed on untouched
                finish(c, SKR_NONFINITE);
                q.input_nf = true;
                zx[c] = 1;
            } else if (h.bnorm == 0.0) {
                finish(c, SKR_CONVERGED);
            } else {
                q.bnorm = h.bnorm;
                q.tol_abs = h.tol_abs;
            }
        }
        if ((rc = zero_x())) return rc;
        if (mixed && mask([&](int c) { return cs[c].live; })) {
            for (int p = 0; p < 3; ++p) {
                if (cmax[p] == 0) continue;
                for (int c = 0; c < C; ++c) hd[c].part = p;
                if ((rc = upload())) return rc;
                blaunch_to_f32(B, cmax[p]);
                HIPLAUNCHCHK();
            }
        }
        // ---- start-up with the carried recycle space (App. B.1), grouped by the carried columns
        {
            std::vector<int> ks;
            for (int c = 0; c < C; ++c)
                if (cs[c].live && k > 0 && cs[c].kin > 0) ks.push_back(cs[c].kin);
            std::sort(ks.begin(), ks.end());
            ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
            bool any_start = false;
            for (int g : ks) {
                auto inS = [&](int c) { return cs[c].live && k > 0 && cs[c].kin == g; };
                mask(inS);
                for (int c = 0; c < C; ++c) {
                    hd[c].kin = cs[c].kin;
                    hd[c].Ls = {{bcol(cs[c].sub->w, 0), nullptr, nullptr, nullptr}, {g, 0, 0, 0}};
                }
                if ((rc = upload())) return rc;
                blaunch_spmm(B);
                blaunch_startup_gram(B, g);
                blaunch_chol(B, 1);
                blaunch_startup_apply(B, 1, 0);
                HIPLAUNCHCHK();
                if ((rc = gather())) return rc;
                for (int c = 0; c < C; ++c)
                    if (inS(c)) {
                        cs[c].spmv += g;
                        cs[c].res.rank_dropped = g - hk[c];
                        hd[c].ke = hk[c];
                    }
                any_start = true;
            }
            if (any_start) {
                // second CholQR pass and projection, grouped by the kept columns
                std::vector<int> kes;
                for (int c = 0; c < C; ++c)
                    if (cs[c].live && k > 0 && cs[c].kin > 0 && hd[c].ke > 0) kes.push_back(hd[c].ke);
                std::sort(kes.begin(), kes.end());
                kes.erase(std::unique(kes.begin(), kes.end()), kes.end());
                for (int g : kes) {
                    mask([&](int c) { return cs[c].live && k > 0 && cs[c].kin > 0 && hd[c].ke == g; });
                    for (int c = 0; c < C; ++c) {
                        hd[c].kc = g;
                        hd[c].Ls = {{bcol(cs[c].sub->w, 0), nullptr, nullptr, nullptr}, {g, 0, 0, 0}};
                        hd[c].Lp = hd[c].Ls;
                    }
                    if ((rc = upload())) return rc;
                    blaunch_startup_gram(B, g);
                    blaunch_chol(B, 0);
                    blaunch_startup_apply(B, 0, 1);
                    blaunch_startup_project(B, g, 0);
                    HIPLAUNCHCHK();
                }
                if ((rc = gather())) return rc;
                for (int c = 0; c < C; ++c)
                    if (cs[c].live && k > 0 && cs[c].kin > 0) {
                        cs[c].kc = hg[c].kc;
                        cs[c].res.k_start = cs[c].kc;
                    }
            }
        }
        for (int c = 0; c < C; ++c) {
            CState& q = cs[c];
            if (!q.live) continue;
            q.est = hg[c].beta;
            q.r_fresh = q.kc == 0 || !mixed;
            q.cycling = true;
        }
        // ---- the projection alone may meet the tolerance: true residual
        auto exit_test = [&](auto sel, bool from_cycle) -> int {
            if (!mask(sel)) return SKR_OK;
            int r2;
            if ((r2 = upload())) return r2;
            blaunch_true_residual(B);
            HIPLAUNCHCHK();
            std::vector<char> brk((size_t)C, 0), was((size_t)C, 0);
            for (int c = 0; c < C; ++c) {
                was[c] = hd[c].on;
                brk[c] = from_cycle ? hg[c].breakdown : 0;
            }
            if ((r2 = gather())) return r2;
            std::vector<char> restart((size_t)C, 0);
            for (int c = 0; c < C; ++c) {
                if (!was[c]) continue;
                CState& q = cs[c];
                q.spmv += 1;
                if (std::sqrt(hg[c].res2) <= q.tol_abs) {
                    q.res.relres_true = std::sqrt(hg[c].res2) / q.bnorm;
                    finish(c, brk[c] ? SKR_BREAKDOWN : SKR_CONVERGED);
                } else {
                    q.r_fresh = true;
                    restart[c] = q.kc > 0;
                }
            }
            if ((r2 = project([&](int c) { return restart[c] != 0; }))) return r2;
            return SKR_OK;
        };
        if ((rc = exit_test([&](int c) { return cs[c].cycling && hg[c].beta <= cs[c].tol_abs; }, false))) return rc;
        // ---- Arnoldi cycles (Alg. 2)
        for (;;) {
            for (int c = 0; c < C; ++c) {
                CState& q = cs[c];
                if (q.cycling && q.iters >= maxit) {
                    q.status = SKR_MAXIT;
                    q.cycling = false;
                }
            }
            if (!mask([&](int c) { return cs[c].cycling; })) break;
            // refinement (mixed) and the projection at the cycle start
            if (mixed && mask([&](int c) { return cs[c].cycling && !cs[c].r_fresh; })) {
                if ((rc = upload())) return rc;
                blaunch_true_residual(B);
                HIPLAUNCHCHK();
                for (int c = 0; c < C; ++c)
                    if (hd[c].on) cs[c].spmv += 1;
            }
            std::vector<char> proj((size_t)C, 0);
            for (int c = 0; c < C; ++c) proj[c] = cs[c].cycling && !cs[c].r_fresh;
            if ((rc = project([&](int c) { return proj[c] != 0; }))) return rc;
            for (int c = 0; c < C; ++c)
                if (cs[c].cycling) cs[c].r_fresh = false;
            // Z = A C where the merged step needs it
            if (w0.merged) {
                std::vector<int> ks;
                for (int c = 0; c < C; ++c)
                    if (cs[c].cycling && cs[c].kc > 0 && !cs[c].z_valid) ks.push_back(cs[c].kc);
                std::sort(ks.begin(), ks.end());
                ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
                for (int g : ks) {
                    mask([&](int c) { return cs[c].cycling && cs[c].kc == g && !cs[c].z_valid; });
                    for (int c = 0; c < C; ++c) hd[c].kc = cs[c].kc;
                    if ((rc = upload())) return rc;
                    blaunch_apply_c(B, kind, g);
                    HIPLAUNCHCHK();
                }
                for (int c = 0; c < C; ++c)
                    if (cs[c].cycling && cs[c].kc > 0) cs[c].z_valid = true;
            }
            // step samples of this cycle (profile): kernel times of one step of a group of chains
            struct Samp {
                int j, kc;
                std::vector<char> in;
            };
            std::vector<Samp> samps;
            // cycle length per chain and the groups of equal (kc, cycle length)
            std::vector<std::pair<int, int>> groups;
            for (int c = 0; c < C; ++c) {
                CState& q = cs[c];
                if (!q.cycling) continue;
                int sc = (q.kc == 0) ? m : m - q.kc;
                sc = (int)std::min<int64_t>(sc, maxit - q.iters);
                q.scyc = sc;
                groups.push_back({q.kc, sc});
            }
            std::sort(groups.begin(), groups.end());
            groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
            for (const auto& grp : groups) {
                const int gk = grp.first, gs = grp.second;
                auto inG = [&](int c) { return cs[c].cycling && cs[c].kc == gk && cs[c].scyc == gs; };
                mask(inG);
                // launch length: the longest prediction of the group (see the single-chain solve)
                int nfirst = 0;
                for (int c = 0; c < C; ++c) {
                    if (!inG(c)) continue;
                    CState& q = cs[c];
                    int pred = 0;
                    if (q.cycles == 0) pred = q.sub->pred_first;
                    else if (q.prev_jd < q.prev_scyc) pred = q.prev_jd;
                    else if (q.prev_rate > 0.0 && q.prev_rate < 1.0 && q.est > q.tol_abs) {
                        const double st = std::ceil(std::log(q.tol_abs / q.est) / std::log(q.prev_rate));
                        if (st < gs) pred = std::max(1, (int)st);
                    }
                    const int nf = pred > 0 ? std::min(gs, pred + std::max(2, pred / 4)) : gs;
                    nfirst = std::max(nfirst, nf);
                }
                for (int c = 0; c < C; ++c) {
                    hd[c].kc = cs[c].kc;
                    hd[c].scyc = cs[c].scyc;
                }
                if ((rc = upload())) return rc;
                auto launch_j = [&](int j) {
                    hipEvent_t* ev = nullptr;
                    if (profile && (ctx->step_counter++ % PROF_PERIOD) == PROF_PERIOD / 2 &&
                        (int)samps.size() < PROF_MAXSAMP) {
                        ev = ctx->ev + 6 * samps.size();
                        Samp sp{j, gk, std::vector<char>((size_t)C, 0)};
                        for (int c = 0; c < C; ++c) sp.in[c] = inG(c) ? 1 : 0;
                        samps.push_back(std::move(sp));
                    }
                    blaunch_step(B, kind, gk, j, ev);
                };
                for (int j = 0; j < nfirst; ++j) launch_j(j);
                HIPLAUNCHCHK();
                if (nfirst < gs) {
                    if ((rc = gather())) return rc;
                    bool any_running = false;
                    for (int c = 0; c < C; ++c)
                        if (inG(c) && !hg[c].stop) any_running = true;
                    if (any_running)
                        for (int j = nfirst; j < gs; ++j) launch_j(j);
                }
                blaunch_close_basis(B, kind, gk, gs);
                if (gk > 0) {
                    for (int c = 0; c < C; ++c) {
                        const Work& wc = cs[c].sub->w;
                        hd[c].Lg = {{bcol(wc, 0), bcol(wc, wc.k), wc.U, nullptr}, {gk, gs + 1, gk, 0}};
                        if (!mixed) hd[c].Rg = {{wc.U, wc.r, nullptr, nullptr}, {gk, 1, 0, 0}};
                        else hd[c].Rg = {{wc.U, nullptr, nullptr, nullptr}, {gk, 0, 0, 0}};
                    }
                    if ((rc = upload())) return rc;
                    blaunch_cycle_gram(B, gk, gs);
                }
                HIPLAUNCHCHK();
            }
            // cycle end of every cycling chain: the dense stages, then the update by bucket
            mask([&](int c) { return cs[c].cycling; });
            if ((rc = upload())) return rc;
            blaunch_cycle_dense(B, k);
            HIPLAUNCHCHK();
            const int kb_full = k <= 8 ? 8 : k <= 16 ? 16 : k <= 20 ? 20 : k <= 24 ? 24 : 32;
            for (int form = 0; form < 2; ++form) {
                auto inU = [&](int c) {
                    const bool forms = k > 0 && (cs[c].kc > 0 || cs[c].scyc > k);
                    return cs[c].cycling && forms == (form == 1);
                };
                if (!mask(inU)) continue;
                if ((rc = upload())) return rc;
                blaunch_cycle_update(B, form ? kb_full : 0);
                HIPLAUNCHCHK();
            }
            if ((rc = gather())) return rc;
            if (profile) {
                // the sampled steps: kernel times of the launch, algorithmic bytes of the chains it
                // advanced (those still running at that step)
                skr_profile& pr = ctx->prof;
                for (size_t q = 0; q < samps.size(); ++q) {
                    const Samp& sp = samps[q];
                    float tm[3] = {0.f, 0.f, 0.f};
                    const int nk = w0.merged ? 2 : 3;
                    for (int e = 0; e < nk; ++e)
                        HIPCHK(hipEventElapsedTime(&tm[e], ctx->ev[6 * q + 2 * e], ctx->ev[6 * q + 2 * e + 1]));
                    double ba = 0.0, bb = 0.0, bc = 0.0;
                    for (int c = 0; c < C; ++c) {
                        if (!sp.in[c] || sp.j >= hg[c].j_done) continue;
                        double a1, b1, c1;
                        step_bytes(hd[c].op, cs[c].nv, sp.kc, sp.j, mixed, w0.merged != 0, a1, b1, c1);
                        ba += a1;
                        bb += b1;
                        bc += c1;
                    }
                    if (ba == 0.0) continue;      // every chain of the launch had stopped
                    pr.step_a.launches++; pr.step_a.ms += tm[0]; pr.step_a.bytes += ba;
                    pr.step_b.launches++; pr.step_b.ms += tm[1]; pr.step_b.bytes += bb;
                    if (nk == 3) { pr.step_c.launches++; pr.step_c.ms += tm[2]; pr.step_c.bytes += bc; }
                }
                for (int c = 0; c < C; ++c) {
                    if (!cs[c].cycling) continue;
                    for (int j = 0; j < hg[c].j_done; ++j) {
                        double a1, b1, c1;
                        step_bytes(hd[c].op, cs[c].nv, cs[c].kc, j, mixed, w0.merged != 0, a1, b1, c1);
                        pr.step_bytes += a1 + b1 + c1;
                    }
                    pr.steps += hg[c].j_done;
                    pr.cycles += 1;
                }
            }
            std::vector<char> need_exit((size_t)C, 0);
            for (int c = 0; c < C; ++c) {
                CState& q = cs[c];
                if (!q.cycling) continue;
                const CtrlHost& h = hg[c];
                const int jd = h.j_done;
                if (jd < 1 || jd > q.scyc) return fail(SKR_EHIP, "internal: Arnoldi cycle reported %d steps", jd);
                if (h.route == 1) ctx->prof.eig_symmetric++;
                else if (h.route == 2) ctx->prof.eig_general++;
                if (q.cycles == 0) q.sub->pred_first = jd < q.scyc ? jd : 0;
                q.prev_jd = jd;
                q.prev_scyc = q.scyc;
                q.prev_rate = (h.beta > 0.0 && h.est > 0.0) ? std::pow(h.est / h.beta, 1.0 / jd) : 0.0;
                q.iters += jd;
                q.spmv += jd;
                q.cycles += 1;
                q.est = h.est;
                if (h.k_new > 0) q.z_valid = false;
                q.kc = h.k_new;
                if (!std::isfinite(q.est)) {
                    q.kc = 0;
                    finish(c, SKR_NONFINITE);
                    zx[c] = 1;
                    continue;
                }
                if (q.est <= q.tol_abs || h.breakdown) need_exit[c] = 1;
            }
            if ((rc = zero_x())) return rc;
            if ((rc = exit_test([&](int c) { return need_exit[c] != 0; }, true))) return rc;
        }
        // ---- systems that stopped at maxit: their true residual
        if (mask([&](int c) { return cs[c].live && cs[c].status == SKR_MAXIT; })) {
            if ((rc = upload())) return rc;
            blaunch_true_residual(B);
            HIPLAUNCHCHK();
            std::vector<char> was((size_t)C, 0);
            for (int c = 0; c < C; ++c) was[c] = hd[c].on;
            if ((rc = gather())) return rc;
            for (int c = 0; c < C; ++c)
                if (was[c]) {
                    cs[c].spmv += 1;
                    cs[c].res.relres_true = std::sqrt(hg[c].res2) / cs[c].bnorm;
                    cs[c].live = false;
                }
        }
        // ---- results
        HIPCHK(hipStreamSynchronize(s));
        const auto tend = std::chrono::steady_clock::now();
        for (int c = 0; c < C; ++c) {
            CState& q = cs[c];
            if (t >= q.len) continue;
            skr_result& r = q.res;
            r.status = q.status;
            r.cycles = q.cycles;
            r.iters = q.iters;
            r.spmv = q.spmv;
            if (q.input_nf) {
                r.relres_true = NAN;
                r.relres_est = NAN;
            } else if (q.bnorm > 0.0) {
                // solved: the recycle space it leaves goes to the next system of the chain
                if (q.status == SKR_NONFINITE) r.relres_true = NAN;
                r.relres_est = q.est / q.bnorm;
                q.kin = (k > 0) ? q.kc : 0;
            }
            r.seconds = std::chrono::duration<double>(tend - q.t0).count();
            results_host[q.idx] = r;
            any_maxit = any_maxit || r.status == SKR_MAXIT;
        }
    }
    // each chain context carries its chain's recycle space to a later call with SKR_FLAG_CONTINUE
    for (int c = 0; c < C; ++c) {
        skr_ctx* q = cs[c].sub;
        q->carry_valid = true;
        q->carry_k = cs[c].kin;
        q->carry_n = n;
        q->carry_m = m;
        q->carry_kmax = k;
        q->carry_mixed = mixed_flag;
    }
    return any_maxit ? SKR_WARN_NOTCONVERGED : SKR_OK;
}
