// C ABI of libskr (include/skr.h): context, device workspace and the host-side control of the
// sorted-sequence GCRO-DR solve. All arithmetic runs in the kernels of skr_solver.hip,
// skr_dense.hip and skr_sort.hip; the host only sequences launches and reads a small control
// block once per Arnoldi cycle.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "skr_host.hpp"

namespace skr {
struct ColList;
void launch_init(hipStream_t, const Work&, const double*, double*, double);
void launch_clear_nonfinite(hipStream_t, const Work&);
void launch_check_finite(hipStream_t, const Work&, const double*, long);
void launch_check_sym(hipStream_t, const Work&, const DevOp&);
void launch_to_f32(hipStream_t, const double*, float*, long);
void launch_zero(hipStream_t, double*, int);
void launch_copy_u(hipStream_t, const Work&, double*, long, int, int);
void launch_step(hipStream_t, const Work&, const DevOp&, int, int, int, hipEvent_t* ev);
void launch_close_basis(hipStream_t, const Work&, const DevOp&, int, int);
void launch_apply_c(hipStream_t, const Work&, const DevOp&, int);
void launch_cycle_gram(hipStream_t, const Work&, int, int);
void launch_cycle_dense(hipStream_t, const Work&, int, int, int);
void launch_cycle_update(hipStream_t, const Work&, double*, int, int, int spec_kc);
void launch_true_residual(hipStream_t, const Work&, const DevOp&, const double*, const double*,
                          const int* gate = nullptr);
const int* spec_gate(const Work&);
void launch_spmm(hipStream_t, const Work&, const DevOp&, int);
void launch_startup_gram(hipStream_t, const Work&, int);
void launch_chol(hipStream_t, const Work&, int, int);
void launch_startup_apply(hipStream_t, const Work&, int, int);
void launch_startup_project(hipStream_t, const Work&, double*, int, int, const int* gate = nullptr);
void launch_spmv(hipStream_t, const DevOp&, const double*, double*);
void launch_spmv_repeat(hipStream_t, const DevOp&, const double*, double*, int);
void launch_sort(hipStream_t, const double*, long, long, long, double*, double*, long long*, double*);
hipError_t noalloc_setup(int);
long sort_nmax();
long sort_part_doubles(long, long);
}  // namespace skr

using namespace skr;

static thread_local std::string g_err;

namespace skr {
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
const std::string& last_error() { return g_err; }
}  // namespace skr

// Algorithmic bytes of the three step kernels at step j with ncol = kc + j + 1 basis columns.
// Bytes of one product with the operator: its values (FP64, or FP32 for the inner products of the
// mixed mode) with the CSR column indices and row pointers, the FP64 operand and result.
static double op_bytes(const DevOp& op, int64_t nvals, bool fp32_values) {
    const double n = op.n, vb = fp32_values ? 4.0 : 8.0;
    if (op.kind == SKR_OP_CSR) return (vb + 4.0) * (double)nvals + 4.0 * (n + 1) + 16.0 * n;
    if (op.kind == SKR_OP_STENCIL7)
        return vb * (double)op.nz * ((double)op.ny * (op.nx + 1) + (double)(op.ny + 1) * op.nx) +
               vb * (double)(op.nz + 1) * op.ny * op.nx + 16.0 * n;
    return vb * ((double)op.ny * (op.nx + 1) + (double)(op.ny + 1) * op.nx) + 16.0 * n;
}
// Algorithmic bytes of the kernels of Arnoldi step j. es: bytes per stored basis element (8, or 4
// with an FP32 basis, whose mode also takes the operator values in FP32); w stays FP64. A step is
// passes A, B and C, or with two kernels (merged) pass A at step 0, the merged kernel after it,
// which also reads the kc columns of Z = A C (FP32), and pass B; there is no pass C (c = 0).
void skr::step_bytes(const DevOp& op, int64_t nvals, int kc, int j, bool mixed, bool merged, double& a, double& b,
                     double& c) {
    const double n = op.n;
    const int ncol = kc + j + 1;
    const double es = mixed ? 4.0 : 8.0;
    // pass A: the product (operand and result counted in op_bytes), v_j stored, the other columns
    a = op_bytes(op, nvals, mixed) + es * n /* v_j */ + es * n * (ncol - 1);
    b = es * n * ncol + 16.0 * n;
    if (!merged) {
        c = es * n * ncol + 16.0 * n;
    } else {
        if (j > 0) a += 4.0 * n * kc;
        c = 0.0;
    }
}

// ---------------------------------------------------------------------------------------------
// Device memory: the caller's arena or hipMalloc
// ---------------------------------------------------------------------------------------------
skr::Arena::Arena(void* b, size_t n) : base((char*)b), size(n / 256 * 256) {
    // the first block starts at the first 256-byte boundary of the buffer
    const size_t skew = (256 - ((uintptr_t)base & 255)) & 255;
    if (size > skew) {
        base += skew;
        size = (n - skew) / 256 * 256;
        if (size) free_blocks[0] = size;
    } else {
        size = 0;
    }
}
void* skr::Arena::alloc(size_t bytes) {
    const size_t need = round256(std::max<size_t>(bytes, 1));
    std::lock_guard<std::mutex> lk(mu);
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
        if (it->second < need) continue;
        const size_t off = it->first, len = it->second;
        free_blocks.erase(it);
        if (len > need) free_blocks[off + need] = len - need;
        live[off] = need;
        in_use += need;
        return base + off;
    }
    return nullptr;
}
void skr::Arena::release(void* p) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = live.find((size_t)((char*)p - base));
    if (it == live.end()) return;
    size_t off = it->first, len = it->second;
    live.erase(it);
    in_use -= len;
    auto nx = free_blocks.lower_bound(off);
    if (nx != free_blocks.end() && nx->first == off + len) {
        len += nx->second;
        free_blocks.erase(nx);
    }
    auto pv = free_blocks.lower_bound(off);
    if (pv != free_blocks.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            off = pv->first;
            len += pv->second;
            free_blocks.erase(pv);
        }
    }
    free_blocks[off] = len;
}
bool skr::Arena::can_fit(const size_t* sizes, int count) {
    std::lock_guard<std::mutex> lk(mu);
    std::map<size_t, size_t> fb = free_blocks;
    for (int q = 0; q < count; ++q) {
        const size_t need = round256(std::max<size_t>(sizes[q], 1));
        auto it = fb.begin();
        while (it != fb.end() && it->second < need) ++it;
        if (it == fb.end()) return false;
        const size_t off = it->first, len = it->second;
        fb.erase(it);
        if (len > need) fb[off + need] = len - need;
    }
    return true;
}
hipError_t skr::dev_alloc(skr_ctx* ctx, void** p, size_t bytes) {
    if (!ctx->arena) return hipMalloc(p, std::max<size_t>(bytes, 1));
    *p = ctx->arena->alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
void skr::dev_free(skr_ctx* ctx, void* p) {
    if (!p) return;
    if (ctx->arena) ctx->arena->release(p);
    else (void)hipFree(p);
}

// Places every workspace buffer for (w.n, w.m, w.k) in one block at base, each on a 256-byte
// boundary (base == nullptr: measures only); returns the block's bytes.
static size_t layout_work(Work& w, char* base) {
    const size_t ld = (size_t)w.ld;
    size_t off = 0;
    auto take = [&](auto*& ptr, size_t count) {
        using T = std::remove_reference_t<decltype(*ptr)>;
        off = round256(off);
        ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
    };
    take(w.basis, (size_t)(w.k + w.m + 1) * ld);
    take(w.U, (size_t)std::max(w.k, 1) * ld);
    take(w.Z, (size_t)std::max(w.k, 1) * ld);
    take(w.W[0], ld);
    take(w.W[1], ld);
    take(w.r, ld);
    take(w.part_a, (size_t)w.nblk * NC);
    take(w.part_b, (size_t)w.nblk * NC);
    take(w.part_n, (size_t)w.nblk);
    take(w.part, (size_t)w.nblk * NC);
    take(w.gpart, (size_t)w.ngblk * w.gram_max);
    take(w.gram, w.gram_max);
    take(w.fold_a, (size_t)NFOLD * NC);
    take(w.fold_b, (size_t)NFOLD * NC);
    take(w.fold_n, (size_t)NFOLD);
    take(w.red1, NC);
    take(w.red2, NC);
    take(w.gcorr, 2 * NC);
    take(w.H, (size_t)LDH * MMAX);
    take(w.Bm, (size_t)KMAX * MMAX);
    take(w.ctrl, 1);
    take(w.coef, 1);
    take(w.dense, 1);
    take(w.counters, 8);
    return round256(off);
}

static void set_shape(Work& w, int n, int m, int k) {
    w.n = n;
    w.m = m;
    w.k = k;
    w.ld = (n + 63) / 64 * 64;
    w.nblk = (n + ROWS - 1) / ROWS;
    w.ngblk = std::min(256, std::max(1, (n + 255) / 256));
    w.gram_max = (size_t)gram_cols_max(m, k);
}

static void free_work(skr_ctx* ctx) {
    dev_free(ctx, ctx->w.block);
    ctx->w = Work();
}

static int ensure_work(skr_ctx* ctx, int n, int m, int k) {
    Work& w = ctx->w;
    if (w.block && w.n == n && w.m == m && w.k == k) return SKR_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->carry_valid = false;      // the carried recycle space goes with the old workspace
    free_work(ctx);
    set_shape(w, n, m, k);
    const size_t bytes = layout_work(w, nullptr);
    void* blk = nullptr;
    const hipError_t ea = dev_alloc(ctx, &blk, bytes);
    if (ea != hipSuccess) {
        w = Work();
        if (ctx->arena)
            return fail(SKR_ENOMEM, "the workspace for n = %d, m = %d, k = %d needs %zu bytes of the arena "
                        "(%zu of %zu bytes in use)", n, m, k, bytes, ctx->arena->in_use, ctx->arena->size);
        return fail(SKR_ENOMEM, "device workspace allocation of %zu bytes failed: %s", bytes, hipGetErrorString(ea));
    }
    w.block = blk;
    layout_work(w, (char*)blk);
    const size_t ld = (size_t)w.ld;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    // zero everything once so that unused basis columns never hold NaN bit patterns
    chk(hipMemsetAsync(w.basis, 0, (size_t)(k + m + 1) * ld * sizeof(double), ctx->stream));
    chk(hipMemsetAsync(w.U, 0, (size_t)std::max(k, 1) * ld * sizeof(double), ctx->stream));
    chk(hipMemsetAsync(w.W[0], 0, ld * sizeof(double), ctx->stream));
    chk(hipMemsetAsync(w.W[1], 0, ld * sizeof(double), ctx->stream));
    chk(hipMemsetAsync(w.H, 0, (size_t)LDH * MMAX * sizeof(double), ctx->stream));
    chk(hipMemsetAsync(w.Bm, 0, (size_t)KMAX * MMAX * sizeof(double), ctx->stream));
    chk(hipMemsetAsync(w.ctrl, 0, sizeof(Ctrl), ctx->stream));
    chk(hipMemsetAsync(w.coef, 0, sizeof(Coef), ctx->stream));
    chk(hipMemsetAsync(w.dense, 0, sizeof(DenseWork), ctx->stream));
    chk(hipMemsetAsync(w.counters, 0, 8 * sizeof(unsigned), ctx->stream));
    if (e != hipSuccess) return fail(SKR_EHIP, "workspace initialisation failed: %s", hipGetErrorString(e));
    return SKR_OK;
}

size_t skr::work_bytes(int n, int m, int k) {
    Work w;
    set_shape(w, n, m, k);
    return layout_work(w, nullptr);
}

static int read_ctrl(skr_ctx* ctx) {
    HIPCHK(hipMemcpyAsync(ctx->hctrl, ctx->w.ctrl, sizeof(CtrlHost), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SKR_OK;
}

int skr::to_devop(const skr_op& o, DevOp& d, int64_t& nvals) {
    d = DevOp();
    d.kind = o.kind;
    d.n = o.n;
    if (o.n <= 0) return fail(SKR_EINVAL, "operator n must be positive (got %d)", o.n);
    if (o.kind == SKR_OP_CSR) {
        if (!o.rowptr || !o.colind || !o.values || o.nnz < 0)
            return fail(SKR_EINVAL, "CSR operator needs rowptr, colind, values and nnz >= 0");
        d.rowptr = o.rowptr;
        d.colind = o.colind;
        d.val = o.values;
        nvals = o.nnz;
    } else if (o.kind == SKR_OP_STENCIL5) {
        if (!o.ax || !o.ay || o.nx <= 0 || o.ny <= 0 || (int64_t)o.nx * o.ny != o.n)
            return fail(SKR_EINVAL, "stencil operator needs ax, ay and nx * ny == n");
        d.nx = o.nx;
        d.ny = o.ny;
        d.inv_h2 = o.inv_h2;
        d.ax = o.ax;
        d.ay = o.ay;
        nvals = 0;
    } else if (o.kind == SKR_OP_STENCIL7) {
        if (!o.ax || !o.ay || !o.az || o.nx <= 0 || o.ny <= 0 || o.nz <= 0 ||
            (int64_t)o.nx * o.ny * o.nz != o.n)
            return fail(SKR_EINVAL, "7-point stencil operator needs ax, ay, az and nx * ny * nz == n");
        d.nx = o.nx;
        d.ny = o.ny;
        d.nz = o.nz;
        d.inv_h2 = o.inv_h2;
        d.ax = o.ax;
        d.ay = o.ay;
        d.az = o.az;
        nvals = 0;
    } else {
        return fail(SKR_EINVAL, "unknown operator kind %d", o.kind);
    }
    return SKR_OK;
}

// Solves one system A x = b on the context's stream (Alg. 2), starting from the recycle space the
// context holds (kin columns of U, left by the system solved before on this context) and leaving
// the next one there (kin updated). The workspace must be sized for (n, m, k), with the fold and
// storage modes set (prepare_solve). Returns SKR_OK with the outcome in res, or an error code.
static int solve_system_body(skr_ctx* ctx, const skr_op& opin, const double* b, double* x, const skr_opts& opts, int& kin,
                 skr_result& res) {
    Work& w = ctx->w;
    hipStream_t s = ctx->stream;
    CtrlHost& hc = *ctx->hctrl;
    const int n = w.n, m = opts.m, k = opts.k;
    const double rtol = opts.rtol;
    const int64_t maxit = opts.maxit;
    const bool profile = (opts.flags & SKR_FLAG_PROFILE) && ctx->ev_ok;
    int samp_j[PROF_MAXSAMP];
    int rc;
    DevOp op;
    int64_t nvals;
    to_devop(opin, op, nvals);
    std::memset(&res, 0, sizeof res);

    launch_clear_nonfinite(s, w);
    launch_init(s, w, b, x, rtol);
    if (op.kind == SKR_OP_CSR) {
        launch_check_finite(s, w, op.val, (long)nvals);
        launch_check_sym(s, w, op);
    } else {
        const long nzl = op.kind == SKR_OP_STENCIL7 ? (long)op.nz : 1L;
        launch_check_finite(s, w, op.ax, nzl * op.ny * (op.nx + 1));
        launch_check_finite(s, w, op.ay, nzl * (op.ny + 1) * op.nx);
        if (op.kind == SKR_OP_STENCIL7) launch_check_finite(s, w, op.az, (nzl + 1) * op.ny * op.nx);
    }
    HIPLAUNCHCHK();
    if ((rc = read_ctrl(ctx))) return rc;
    if (hc.nonfinite || !std::isfinite(hc.bnorm)) {
        launch_zero(s, x, n);
        res.status = SKR_NONFINITE;
        res.relres_true = NAN;
        res.relres_est = NAN;
        return SKR_OK;   // the carried recycle space is passed on untouched
    }
    if (hc.bnorm == 0.0) {
        res.status = SKR_CONVERGED;
        return SKR_OK;
    }
    if (w.mixed) {
        // the inner cycle's operator: its values (CSR) or faces (stencils) rounded to FP32; true
        // residuals keep the FP64 operator
        long cnt[3] = {0, 0, 0};
        const double* srcs[3] = {nullptr, nullptr, nullptr};
        if (op.kind == SKR_OP_CSR) {
            cnt[0] = (long)nvals;
            srcs[0] = op.val;
        } else {
            const long nzl = op.kind == SKR_OP_STENCIL7 ? (long)op.nz : 1L;
            cnt[0] = nzl * op.ny * (op.nx + 1);
            cnt[1] = nzl * (op.ny + 1) * op.nx;
            srcs[0] = op.ax;
            srcs[1] = op.ay;
            if (op.kind == SKR_OP_STENCIL7) {
                cnt[2] = (nzl + 1) * op.ny * op.nx;
                srcs[2] = op.az;
            }
        }
        const size_t need = (size_t)(cnt[0] + cnt[1] + cnt[2]);
        if (ctx->op32_cap < need) {
            dev_free(ctx, ctx->op32);
            ctx->op32 = nullptr;
            ctx->op32_cap = 0;
            if (dev_alloc(ctx, (void**)&ctx->op32, need * sizeof(float)) != hipSuccess)
                return fail(SKR_ENOMEM, "FP32 operator copy (%zu bytes)", need * sizeof(float));
            ctx->op32_cap = need;
        }
        float* dst32 = ctx->op32;
        const float* parts[3] = {dst32, dst32 + cnt[0], dst32 + cnt[0] + cnt[1]};
        for (int q = 0; q < 3; ++q) launch_to_f32(s, srcs[q], (float*)parts[q], cnt[q]);
        HIPLAUNCHCHK();
        if (op.kind == SKR_OP_CSR) {
            op.val32 = parts[0];
        } else {
            op.ax32 = parts[0];
            op.ay32 = parts[1];
            op.az32 = cnt[2] ? parts[2] : nullptr;
        }
    }
    const double bnorm = hc.bnorm, tol_abs = hc.tol_abs;
    int64_t iters = 0, spmv = 0;
    int cycles = 0;
    int kc = 0;
    // ---- start-up with the carried recycle space (App. B.1)
    if (k > 0 && kin > 0) {
        launch_spmm(s, w, op, kin);
        launch_startup_gram(s, w, kin);
        launch_chol(s, w, kin, 1);
        launch_startup_apply(s, w, 1, 0);
        HIPLAUNCHCHK();
        HIPCHK(hipMemcpyAsync(ctx->hkeff, &w.coef->k_eff, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const int ke = *ctx->hkeff;
        spmv += kin;
        res.rank_dropped = kin - ke;
        if (ke > 0) {
            launch_startup_gram(s, w, ke);
            launch_chol(s, w, ke, 0);
            launch_startup_apply(s, w, 0, 1);
            launch_startup_project(s, w, x, ke, 0);
            HIPLAUNCHCHK();
        }
        if ((rc = read_ctrl(ctx))) return rc;
        kc = hc.kc;
        res.k_start = kc;
    }
    bool z_valid = false;      // Z = A C holds for the current C (two-kernel steps only)
    int status = -1;
    double est = hc.beta;
    // r is fresh: b - A x computed directly (at x = 0), or just projected onto range(C)'s
    // complement. With FP32-stored C and U the first cycle still refines from the true residual
    // (A U equals C only to FP32 rounding).
    bool r_fresh = kc == 0 || !w.mixed;
    int prev_jd = 0, prev_scyc = 0;     // launch-length prediction (see the cycle loop)
    double prev_rate = 0.0;
    bool ahead = false;                 // this cycle's opening was launched before the last read
    // A failed exit test goes on from the true residual, projected onto range(C) as at a system
    // start (App. B.1): the next cycle's v_0 must be orthogonal to C, which the cycle-end
    // eigenproblem's block structure of W^T V assumes.
    auto restart_from_true = [&]() -> int {
        r_fresh = true;
        if (kc > 0) {
            launch_startup_project(s, w, x, kc, 1);
            HIPLAUNCHCHK();
            return read_ctrl(ctx);
        }
        return SKR_OK;
    };
    if (hc.beta <= tol_abs) {
        launch_true_residual(s, w, op, b, x);
        HIPLAUNCHCHK();
        if ((rc = read_ctrl(ctx))) return rc;
        spmv += 1;
        if (std::sqrt(hc.res2) <= tol_abs) status = SKR_CONVERGED;
        else if ((rc = restart_from_true())) return rc;
    }
    // ---- Arnoldi cycles (Alg. 2)
    while (status < 0) {
        if (iters >= maxit) { status = SKR_MAXIT; break; }
        // The opening of a cycle: the refinement residual (FP32 basis), the projection and Z = A C.
        // After a cycle end that did not finish the solve, these were launched before the host read
        // that cycle end (see below), so only the count is kept here.
        const bool opened = ahead;
        ahead = false;
        if (!r_fresh) {
            if (w.mixed) {
                // refinement step: true FP64 residual, projected onto range(C) as at a system start
                if (!opened) launch_true_residual(s, w, op, b, x);
                spmv += 1;
            }
            // x += U C^T r, r -= C C^T r (App. B.1's projection): zero in exact arithmetic; it
            // removes the rounding-level component along C that a cycle leaves in r, which would
            // otherwise persist at a fixed absolute size and, relative to the shrinking residual,
            // tilt v_0 = r/||r|| and the next C out of orthogonality
            if (kc > 0 && !opened) launch_startup_project(s, w, x, kc, 1);
            HIPLAUNCHCHK();
        }
        r_fresh = false;
        if (w.merged && kc > 0 && !z_valid) {
            if (!opened) launch_apply_c(s, w, op, kc);
            HIPLAUNCHCHK();
            z_valid = true;
        }
        int scyc = (kc == 0) ? m : m - kc;
        scyc = (int)std::min<int64_t>(scyc, maxit - iters);
        // Launch length. A step launched after the cycle has stopped exits at once, but still costs a
        // launch, so when this cycle is predicted to stop early (the previous cycle stopped early, or
        // the previous cycle's contraction per step reaches the tolerance) only the predicted steps
        // plus a margin are launched, the control block is read, and the rest follow only if the
        // cycle has not stopped. The kernels and their order are the same either way.
        int pred = 0;
        if (cycles == 0) {
            pred = ctx->pred_first;
        } else if (prev_jd < prev_scyc) {
            pred = prev_jd;
        } else if (prev_rate > 0.0 && prev_rate < 1.0 && est > tol_abs) {
            const double steps = std::ceil(std::log(tol_abs / est) / std::log(prev_rate));
            if (steps < scyc) pred = std::max(1, (int)steps);
        }
        const int nfirst = pred > 0 ? std::min(scyc, pred + std::max(2, pred / 4)) : scyc;
        int nsamp = 0;
        auto launch_steps = [&](int j0, int j1) {
            for (int j = j0; j < j1; ++j) {
                hipEvent_t* ev = nullptr;
                if (profile && (ctx->step_counter++ % PROF_PERIOD) == PROF_PERIOD / 2 && nsamp < PROF_MAXSAMP) {
                    ev = ctx->ev + 6 * nsamp;
                    samp_j[nsamp++] = j;
                }
                launch_step(s, w, op, kc, j, scyc, ev);
            }
        };
        launch_steps(0, nfirst);
        if (nfirst < scyc) {
            HIPLAUNCHCHK();
            if ((rc = read_ctrl(ctx))) return rc;
            if (!hc.stop) launch_steps(nfirst, scyc);
        }
        launch_close_basis(s, w, op, kc, scyc);
        if (kc > 0) launch_cycle_gram(s, w, kc, scyc);
        launch_cycle_dense(s, w, kc, scyc, k);
        // the new recycle size is at most k (0 when no recycle space is formed this cycle)
        const bool forms = k > 0 && (kc > 0 || scyc > k);
        // Look-ahead: unless the solve might end here, the next cycle's opening (for the usual k new
        // columns) is launched behind the read of this cycle end, so that the GPU has work while the
        // host waits for the read. The cycle-end kernel decides on the device, with the same test
        // the host applies below, whether the next cycle starts as assumed; when it does not (the
        // estimate met the tolerance, a breakdown, a non-finite value, fewer new columns), the
        // opening's kernels that write x, r or the control block return at once, and the host
        // continues as if they had not been launched (the others fill scratch that is recomputed
        // before its next use).
        const int kspec = forms ? k : 0;
        const bool look = (kspec > 0 || w.mixed) && iters + scyc < maxit;
        launch_cycle_update(s, w, x, kc, forms ? (k <= 8 ? 8 : k <= 16 ? 16 : k <= 20 ? 20 : k <= 24 ? 24 : 32) : 0,
                            look ? kspec : -1);
        HIPLAUNCHCHK();
        HIPCHK(hipMemcpyAsync(ctx->hctrl, w.ctrl, sizeof(CtrlHost), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ctx->ev_ctrl, s));
        if (look) {
            const int* gate = spec_gate(w);
            if (w.mixed) launch_true_residual(s, w, op, b, x, gate);
            if (kspec > 0) launch_startup_project(s, w, x, kspec, 1, gate);
            if (kspec > 0) launch_apply_c(s, w, op, kspec);
            HIPLAUNCHCHK();
        }
        HIPCHK(hipEventSynchronize(ctx->ev_ctrl));
        ahead = look && !hc.spec_skip;
        const int jd = hc.j_done;
        if (jd < 1 || jd > scyc) return fail(SKR_EHIP, "internal: Arnoldi cycle reported %d steps", jd);
        if (hc.route == 1) ctx->prof.eig_symmetric++;
        else if (hc.route == 2) ctx->prof.eig_general++;
        if (profile) {
            skr_profile& pr = ctx->prof;
            for (int q = 0; q < nsamp; ++q) {
                if (samp_j[q] >= jd) continue;   // steps after the stop are skipped launches
                float t[3] = {0.f, 0.f, 0.f};
                const int nk = w.merged ? 2 : 3;    // kernels per step
                for (int e = 0; e < nk; ++e)
                    HIPCHK(hipEventElapsedTime(&t[e], ctx->ev[6 * q + 2 * e], ctx->ev[6 * q + 2 * e + 1]));
                double ba, bb, bc;
                step_bytes(op, nvals, kc, samp_j[q], w.mixed != 0, w.merged != 0, ba, bb, bc);
                pr.step_a.launches++; pr.step_a.ms += t[0]; pr.step_a.bytes += ba;
                pr.step_b.launches++; pr.step_b.ms += t[1]; pr.step_b.bytes += bb;
                if (nk == 3) { pr.step_c.launches++; pr.step_c.ms += t[2]; pr.step_c.bytes += bc; }
            }
            for (int j = 0; j < jd; ++j) {
                double ba, bb, bc;
                step_bytes(op, nvals, kc, j, w.mixed != 0, w.merged != 0, ba, bb, bc);
                pr.step_bytes += ba + bb + bc;
            }
            pr.steps += jd;
            pr.cycles += 1;
        }
        if (cycles == 0) ctx->pred_first = jd < scyc ? jd : 0;
        prev_jd = jd;
        prev_scyc = scyc;
        prev_rate = (hc.beta > 0.0 && hc.est > 0.0) ? std::pow(hc.est / hc.beta, 1.0 / jd) : 0.0;
        iters += jd;
        spmv += jd;
        cycles += 1;
        est = hc.est;
        if (hc.k_new > 0) z_valid = false;     // the cycle end rewrote C
        kc = hc.k_new;
        if (!std::isfinite(est)) {
            launch_zero(s, x, n);
            status = SKR_NONFINITE;
            kc = 0;
            break;
        }
        if (est <= tol_abs || hc.breakdown) {
            const int brk = hc.breakdown;
            launch_true_residual(s, w, op, b, x);
            HIPLAUNCHCHK();
            if ((rc = read_ctrl(ctx))) return rc;
            spmv += 1;
            if (std::sqrt(hc.res2) <= tol_abs) {
                status = brk ? SKR_BREAKDOWN : SKR_CONVERGED;
                break;
            }
            if ((rc = restart_from_true())) return rc;
        }
    }
    if (status == SKR_MAXIT) {
        launch_true_residual(s, w, op, b, x);
        HIPLAUNCHCHK();
        if ((rc = read_ctrl(ctx))) return rc;
        spmv += 1;
    }
    res.status = status;
    res.cycles = cycles;
    res.iters = iters;
    res.spmv = spmv;
    res.relres_true = status == SKR_NONFINITE ? NAN : std::sqrt(hc.res2) / bnorm;
    res.relres_est = est / bnorm;
    kin = (k > 0) ? kc : 0;
    return SKR_OK;
}

// One system of a chain (solve_system_body) with its host wall-clock time in res.seconds.
int skr::solve_system(skr_ctx* ctx, const skr_op& opin, const double* b, double* x, const skr_opts& opts, int& kin,
                 skr_result& res) {
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = solve_system_body(ctx, opin, b, x, opts, kin, res);
    res.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

// Checks m, k, rtol and maxit (Alg. 2 inputs).
int skr::check_opts(const skr_opts* opts) {
    if (!opts) return fail(SKR_EINVAL, "NULL options");
    const int m = opts->m, k = opts->k;
    if (m < 1 || m > MMAX) return fail(SKR_EINVAL, "m must be in [1, %d] (got %d)", MMAX, m);
    if (k < 0 || k > KMAX || k >= m) return fail(SKR_EINVAL, "k must satisfy 0 <= k < m and k <= %d (got %d)", KMAX, k);
    if (!(opts->rtol > 0.0)) return fail(SKR_EINVAL, "rtol must be > 0");
    if (opts->maxit < 0) return fail(SKR_EINVAL, "maxit must be >= 0");
    return SKR_OK;
}

// Sizes the context's workspace for (n, m, k) and sets the per-solve modes.
int skr::prepare_solve(skr_ctx* ctx, int n, const skr_opts& opts) {
    HIPCHK(hipSetDevice(ctx->device));
    int rc = ensure_work(ctx, n, opts.m, opts.k);
    if (rc) return rc;
    Work& w = ctx->w;
    w.fold = (w.nblk > FOLD_MIN || (opts.flags & SKR_FLAG_FOLD)) ? 1 : 0;
    w.mixed = (opts.flags & SKR_FLAG_MIXED) ? 1 : 0;
    // Two kernels per Arnoldi step where the step is bound by latency (at most 256 workgroups, no
    // folding) and the basis is FP64. With an FP32 basis the product must be taken on the stored
    // (rounded) vector, and on folded (HBM-streaming) grids the three-kernel step keeps more waves.
    w.merged = (!w.mixed && !w.fold) ? 1 : 0;
    return SKR_OK;
}

int skr::ctx_make(int device, hipStream_t stream, skr_ctx** out, Arena* arena) {
    HIPCHK(hipSetDevice(device));
    skr_ctx* c = new skr_ctx();
    c->device = device;
    c->stream = stream;
    c->arena = arena;
    if (hipHostMalloc((void**)&c->hctrl, sizeof(CtrlHost), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->hkeff, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(SKR_EHIP, "pinned host allocation failed");
    }
    if (hipEventCreateWithFlags(&c->ev_ctrl, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(c->hctrl);
        (void)hipHostFree(c->hkeff);
        delete c;
        return fail(SKR_EHIP, "event creation failed");
    }
    c->ev_ok = true;
    for (int q = 0; q < PROF_MAXSAMP * 6; ++q)
        if (hipEventCreate(&c->ev[q]) != hipSuccess) c->ev_ok = false;
    *out = c;
    g_err.clear();
    return SKR_OK;
}

extern "C" {

const char* skr_version(void) { return "skr-gfx950 0.1"; }

const char* skr_last_error(void) { return g_err.c_str(); }

int skr_ctx_create(int device, void* hip_stream, void* arena_dev, size_t arena_bytes, skr_ctx** out) {
    if (!out) return fail(SKR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!arena_dev != !arena_bytes) return fail(SKR_EINVAL, "arena_dev and arena_bytes must be both set or both 0");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(SKR_EINVAL, "device %d out of range (%d devices)", device, ndev);
    Arena* ar = arena_dev ? new Arena(arena_dev, arena_bytes) : nullptr;
    const int rc = ctx_make(device, (hipStream_t)hip_stream, out, ar);
    if (rc != SKR_OK) {
        delete ar;
        return rc;
    }
    (*out)->owns_arena = ar != nullptr;
    // locate this device's copy of skr_sort_noalloc's scratch array once, with the device current; a
    // failure is reported by that entry point, not here
    if (rc == SKR_OK) (void)noalloc_setup(device);
    return rc;
}


int skr_ctx_destroy(skr_ctx* ctx) {
    if (!ctx) return SKR_OK;
    serve_free(ctx);
    chains_free(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    free_work(ctx);
    dev_free(ctx, ctx->sortD);
    dev_free(ctx, ctx->sortP);
    dev_free(ctx, ctx->order_d);
    dev_free(ctx, ctx->dist_d);
    dev_free(ctx, ctx->op32);
    if (ctx->hctrl) (void)hipHostFree(ctx->hctrl);
    if (ctx->hkeff) (void)hipHostFree(ctx->hkeff);
    for (int q = 0; q < PROF_MAXSAMP * 6; ++q)
        if (ctx->ev[q]) (void)hipEventDestroy(ctx->ev[q]);
    if (ctx->ev_ctrl) (void)hipEventDestroy(ctx->ev_ctrl);
    if (ctx->owns_arena) delete ctx->arena;
    delete ctx;
    return SKR_OK;
}

int skr_spmv(skr_ctx* ctx, const skr_op* op, const double* x_dev, double* y_dev) {
    if (!ctx || !op || !x_dev || !y_dev) return fail(SKR_EINVAL, "NULL argument");
    HIPCHK(hipSetDevice(ctx->device));
    DevOp d;
    int64_t nv;
    int rc = to_devop(*op, d, nv);
    if (rc) return rc;
    launch_spmv(ctx->stream, d, x_dev, y_dev);
    HIPLAUNCHCHK();
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SKR_OK;
}

int skr_spmv_repeat(skr_ctx* ctx, const skr_op* op, const double* x_dev, double* y_dev, int32_t repeats,
                    double* ms_per_launch) {
    if (!ctx || !op || !x_dev || !y_dev || !ms_per_launch || repeats < 1) return fail(SKR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(ctx->device));
    DevOp d;
    int64_t nv;
    int rc = to_devop(*op, d, nv);
    if (rc) return rc;
    if (!ctx->ev_ok) return fail(SKR_EHIP, "events unavailable");
    HIPCHK(hipEventRecord(ctx->ev[0], ctx->stream));
    launch_spmv_repeat(ctx->stream, d, x_dev, y_dev, repeats);
    HIPLAUNCHCHK();
    HIPCHK(hipEventRecord(ctx->ev[1], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    *ms_per_launch = (double)ms / repeats;
    return SKR_OK;
}

int skr_profile_get(skr_ctx* ctx, skr_profile* out) {
    if (!ctx || !out) return fail(SKR_EINVAL, "NULL argument");
    *out = ctx->prof;
    return SKR_OK;
}

int skr_profile_reset(skr_ctx* ctx) {
    if (!ctx) return fail(SKR_EINVAL, "NULL argument");
    std::memset(&ctx->prof, 0, sizeof ctx->prof);
    return SKR_OK;
}

int skr_sort(skr_ctx* ctx, const double* params_dev, int64_t N, int64_t p, int64_t start, int64_t* order_host,
             double* step_d2_host) {
    if (!ctx) return fail(SKR_EINVAL, "NULL context");
    if (N < 0) return fail(SKR_EINVAL, "N must be >= 0");
    if (N == 0) return SKR_OK;
    if (!order_host) return fail(SKR_EINVAL, "order_host is NULL");
    if (p < 1 || !params_dev) return fail(SKR_EINVAL, "need p >= 1 and params_dev");
    if (start < 0 || start >= N) return fail(SKR_EINVAL, "start %lld out of range", (long long)start);
    if (N > sort_nmax()) return fail(SKR_EINVAL, "N > %ld is not supported", sort_nmax());
    HIPCHK(hipSetDevice(ctx->device));
    const size_t need = (size_t)N * (size_t)N;
    if (ctx->sortD_cap < need) {
        dev_free(ctx, ctx->sortD);
        ctx->sortD = nullptr;
        ctx->sortD_cap = 0;
        if (dev_alloc(ctx, (void**)&ctx->sortD, need * sizeof(double)) != hipSuccess)
            return fail(SKR_ENOMEM, "sort distance matrix (%zu bytes)", need * sizeof(double));
        ctx->sortD_cap = need;
    }
    if (ctx->sortN_cap < (size_t)N) {
        dev_free(ctx, ctx->order_d);
        dev_free(ctx, ctx->dist_d);
        ctx->order_d = nullptr;
        ctx->dist_d = nullptr;
        ctx->sortN_cap = 0;
        if (dev_alloc(ctx, (void**)&ctx->order_d, N * sizeof(long long)) != hipSuccess ||
            dev_alloc(ctx, (void**)&ctx->dist_d, N * sizeof(double)) != hipSuccess)
            return fail(SKR_ENOMEM, "sort output buffers");
        ctx->sortN_cap = (size_t)N;
    }
    const size_t needp = (size_t)sort_part_doubles((long)N, (long)p);
    if (ctx->sortP_cap < needp) {
        dev_free(ctx, ctx->sortP);
        ctx->sortP = nullptr;
        ctx->sortP_cap = 0;
        if (dev_alloc(ctx, (void**)&ctx->sortP, needp * sizeof(double)) != hipSuccess)
            return fail(SKR_ENOMEM, "sort slice partials (%zu bytes)", needp * sizeof(double));
        ctx->sortP_cap = needp;
    }
    launch_sort(ctx->stream, params_dev, (long)N, (long)p, (long)start, ctx->sortD, ctx->sortP, ctx->order_d,
                ctx->dist_d);
    HIPLAUNCHCHK();
    HIPCHK(hipMemcpyAsync(order_host, ctx->order_d, N * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    if (step_d2_host)
        HIPCHK(hipMemcpyAsync(step_d2_host, ctx->dist_d, N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SKR_OK;
}

int skr_solve_sequence(skr_ctx* ctx, const skr_op* ops, const double* const* b_dev, double* const* x_dev, int64_t N,
                       const int64_t* order, const skr_opts* opts, skr_result* results_host) {
    if (!ctx || !opts) return fail(SKR_EINVAL, "NULL context or options");
    if (N < 0) return fail(SKR_EINVAL, "N must be >= 0");
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
        if (!b_dev[idx] || !x_dev[idx]) return fail(SKR_EINVAL, "NULL b or x pointer for system %lld", (long long)idx);
        DevOp d;
        int64_t nv;
        rc = to_devop(ops[idx], d, nv);
        if (rc) return rc;
    }
    const int mixed = (opts->flags & SKR_FLAG_MIXED) ? 1 : 0;
    const bool cont = (opts->flags & SKR_FLAG_CONTINUE) != 0;
    if (cont && !(ctx->carry_valid && ctx->carry_n == n && ctx->carry_m == opts->m &&
                  ctx->carry_kmax == opts->k && ctx->carry_mixed == mixed))
        return fail(SKR_EINVAL, "SKR_FLAG_CONTINUE: the context carries no recycle space for n = %d, m = %d, "
                    "k = %d and this precision", n, opts->m, opts->k);
    if ((rc = prepare_solve(ctx, n, *opts))) return rc;
    // recycled vectors carried from the previous system (held in w.U)
    int kin = cont ? ctx->carry_k : 0;
    ctx->carry_valid = false;
    bool any_maxit = false;
    for (int64_t q = 0; q < N; ++q) {
        const int64_t idx = order ? order[q] : q;
        skr_result res;
        if ((rc = solve_system(ctx, ops[idx], b_dev[idx], x_dev[idx], *opts, kin, res))) return rc;
        results_host[idx] = res;
        any_maxit = any_maxit || res.status == SKR_MAXIT;
    }
    ctx->carry_valid = true;
    ctx->carry_k = kin;
    ctx->carry_n = n;
    ctx->carry_m = opts->m;
    ctx->carry_kmax = opts->k;
    ctx->carry_mixed = mixed;
    return any_maxit ? SKR_WARN_NOTCONVERGED : SKR_OK;
}

size_t skr_workspace_bytes(int64_t n, int32_t m, int32_t k, uint32_t flags) {
    (void)flags;
    if (n < 1 || n > INT32_MAX || m < 1 || m > MMAX || k < 0 || k >= m || k > KMAX) return 0;
    return work_bytes((int)n, m, k);
}

int skr_recycle_get(skr_ctx* ctx, int32_t* k_out, double* U_dev, int64_t ld) {
    if (!ctx || !k_out) return fail(SKR_EINVAL, "NULL context or k_out");
    if (!ctx->carry_valid) return fail(SKR_EINVAL, "the context carries no recycle space (no completed solve)");
    *k_out = ctx->carry_k;
    if (!U_dev || ctx->carry_k == 0) return SKR_OK;
    if (ld < ctx->carry_n) return fail(SKR_EINVAL, "ld (%lld) < n (%d)", (long long)ld, ctx->carry_n);
    HIPCHK(hipSetDevice(ctx->device));
    launch_copy_u(ctx->stream, ctx->w, U_dev, (long)ld, ctx->carry_k, 0);
    HIPLAUNCHCHK();
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return SKR_OK;
}

int skr_recycle_set(skr_ctx* ctx, const skr_opts* opts, int64_t n, int32_t kcols, const double* U_dev, int64_t ld) {
    if (!ctx || !opts) return fail(SKR_EINVAL, "NULL context or options");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (n < 1 || n > INT32_MAX) return fail(SKR_EINVAL, "n must be in [1, 2^31)");
    if (kcols < 0 || kcols > opts->k) return fail(SKR_EINVAL, "kcols must be in [0, k] (got %d, k = %d)", kcols, opts->k);
    if (kcols > 0 && (!U_dev || ld < n)) return fail(SKR_EINVAL, "need U_dev and ld >= n");
    if ((rc = prepare_solve(ctx, (int)n, *opts))) return rc;
    launch_copy_u(ctx->stream, ctx->w, const_cast<double*>(U_dev), (long)ld, kcols, 1);
    HIPLAUNCHCHK();
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->carry_valid = true;
    ctx->carry_k = kcols;
    ctx->carry_n = (int)n;
    ctx->carry_m = opts->m;
    ctx->carry_kmax = opts->k;
    ctx->carry_mixed = (opts->flags & SKR_FLAG_MIXED) ? 1 : 0;
    return SKR_OK;
}

}  // extern "C"
