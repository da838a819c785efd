// Row-parallel kernels of the GCRO-DR solve (Alg. 2, App. B.2) for gfx950.
//
// Every kernel here maps one matrix row to one thread and ROWS rows to a workgroup, with the
// same logical-block mapping, so a given row stays on the same XCD (and in its L2) from kernel
// to kernel. Grid-wide sums use per-workgroup partials and a fixed-order final sum done by the
// last workgroup to arrive, so every result is bitwise reproducible.
//
// One Arnoldi step with the operator (I - C C^T) A (Eq. 6) and classical Gram-Schmidt with one
// re-orthogonalisation (CGS2) against Q = [C, V_0..V_j] is three kernels:
//   A: v_j = w_prev * inv_h (stored), w = A v_j, partial Q^T w and ||w||^2
//   B: w -= Q h1, partial Q^T w            (the basis row is loaded once and used twice)
//   C: w -= Q h2, partial ||w||^2; the last workgroup assembles column j of B and H,
//      advances the progressive Givens QR of H and decides whether the cycle stops.
#include "skr_internal.hpp"

namespace skr {

// Column c of Q = [C (kc columns), V (j+1 columns)] inside the basis buffer.
__device__ __forceinline__ const double* qcol(const double* basis, int ld, int kc, int vbase, int c) {
    return c < kc ? basis + (size_t)c * ld : basis + (size_t)(vbase + c - kc) * ld;
}

// ---------------------------------------------------------------------------------------------
// Solve set-up: x = 0, r = b, ||b||, finiteness of b.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_init(const double* __restrict__ b, double* __restrict__ x,
                                               double* __restrict__ r, int n, int nblk, double rtol,
                                               double* part1, unsigned* counter, Ctrl* ctrl) {
    __shared__ double sh[NWAVE * NC];
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        v = bi * bi;
    }
    double tot;
    if (grid_sum1(v, part1, counter, nblk, lb, sh, &tot)) {
        if (threadIdx.x == 0) {
            const double bn = sqrt(tot);
            ctrl->stop = 0;
            ctrl->j_done = 0;
            ctrl->breakdown = 0;
            ctrl->kc = 0;
            ctrl->k_new = 0;
            ctrl->eig_fail = 0;
            ctrl->nonfinite = (isfinite(bn) ? 0 : 1) | ctrl->nonfinite;
            ctrl->bnorm = bn;
            ctrl->tol_abs = rtol * bn;
            ctrl->beta = bn;
            ctrl->inv_h = bn > 0.0 ? 1.0 / bn : 0.0;
            ctrl->est = bn;
            ctrl->res2 = tot;
            ctrl->g[0] = bn;
        }
    }
}

__global__ void k_clear_nonfinite(Ctrl* ctrl) { ctrl->nonfinite = 0; }

__global__ __launch_bounds__(ROWS) void k_check_finite(const double* __restrict__ v, long count, Ctrl* ctrl) {
    int bad = 0;
    for (long e = blockIdx.x * (long)ROWS + threadIdx.x; e < count; e += (long)gridDim.x * ROWS)
        bad |= !isfinite(v[e]);
    if (__any(bad) && lane_id() == 0) atomicOr(&ctrl->nonfinite, 1);
}

__global__ __launch_bounds__(ROWS) void k_zero(double* __restrict__ x, int n) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// ---------------------------------------------------------------------------------------------
// Arnoldi step, pass A
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_step_a(DevOp op, const double* __restrict__ src,
                                                 double* __restrict__ dst, double* __restrict__ basis,
                                                 int ld, int kc, int vbase, int j, int nblk,
                                                 double* part, unsigned* counter, double* red_out,
                                                 const Ctrl* ctrl) {
    if (ctrl->stop) return;
    __shared__ double sh[NWAVE * NC];
    const int n = op.n;
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const double scale = ctrl->inv_h;
    double vj = 0.0, w = 0.0;
    if (valid) {
        vj = src[i] * scale;
        basis[(size_t)(vbase + j) * ld + i] = vj;
        w = op_row(op, src, i, scale);
        dst[i] = w;
    }
    const int ncol = kc + j + 1;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double q = 0.0;
        if (valid && c < ncol) q = (c == ncol - 1) ? vj : qcol(basis, ld, kc, vbase, c)[i];
        acc[c] = q * w;
    }
    acc[NORM_COL] = w * w;
    const double s = wave_reduce_scatter64(acc);
    sh[wave_id() * NC + lane_id()] = s;
    __syncthreads();
    if (threadIdx.x < NC) {
        double t = sh[threadIdx.x];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q) t += sh[q * NC + threadIdx.x];
        part[lb * NC + threadIdx.x] = t;
    }
    if (last_block_arrive(counter, (unsigned)nblk)) final_reduce64(part, nblk, sh, red_out);
}

// ---------------------------------------------------------------------------------------------
// Arnoldi step, pass B: w -= Q h1, partial Q^T w
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_step_b(double* __restrict__ w_io, const double* __restrict__ basis,
                                                 int n, int ld, int kc, int vbase, int j, int nblk,
                                                 const double* __restrict__ h1, double* part,
                                                 unsigned* counter, double* red_out, const Ctrl* ctrl) {
    if (ctrl->stop) return;
    __shared__ double sh[NWAVE * NC];
    __shared__ double hs[NC];
    if (threadIdx.x < NC) hs[threadIdx.x] = h1[threadIdx.x];
    __syncthreads();
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const int ncol = kc + j + 1;
    double q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = (valid && c < ncol) ? qcol(basis, ld, kc, vbase, c)[i] : 0.0;
    double w = valid ? w_io[i] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < ncol) w = fma(-q[c], hs[c], w);
    if (valid) w_io[i] = w;
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] *= w;
    const double s = wave_reduce_scatter64(q);
    sh[wave_id() * NC + lane_id()] = s;
    __syncthreads();
    if (threadIdx.x < NC) {
        double t = sh[threadIdx.x];
#pragma unroll
        for (int qq = 1; qq < NWAVE; ++qq) t += sh[qq * NC + threadIdx.x];
        part[lb * NC + threadIdx.x] = t;
    }
    if (last_block_arrive(counter, (unsigned)nblk)) final_reduce64(part, nblk, sh, red_out);
}

// ---------------------------------------------------------------------------------------------
// Arnoldi step, pass C: w -= Q h2, ||w||; the last workgroup closes the step.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_step_c(double* __restrict__ w_io, const double* __restrict__ basis,
                                                 int n, int ld, int kc, int vbase, int j, int s_cycle,
                                                 int nblk, const double* __restrict__ h1,
                                                 const double* __restrict__ h2, double* part1,
                                                 unsigned* counter, double* H, double* Bm, Ctrl* ctrl) {
    if (ctrl->stop) return;
    __shared__ double sh[NWAVE * NC];
    __shared__ double hs[NC];
    if (threadIdx.x < NC) hs[threadIdx.x] = h2[threadIdx.x];
    __syncthreads();
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const int ncol = kc + j + 1;
    double w = valid ? w_io[i] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (valid && c < ncol) w = fma(-qcol(basis, ld, kc, vbase, c)[i], hs[c], w);
    if (valid) w_io[i] = w;
    double tot;
    if (!grid_sum1(w * w, part1, counter, nblk, lb, sh, &tot)) return;
    if (threadIdx.x >= 64) return;
    // Wave 0 closes the step; lane t handles row t of the new column (j + 2 <= 64 rows).
    const int t = threadIdx.x;
    const double hnorm = sqrt(tot);
    const double anorm = sqrt(h1[NORM_COL]);
    const int brk = (hnorm <= 1e-14 * anorm) ? 1 : 0;
    const double hlast = brk ? 0.0 : hnorm;
    // Column j of B (rows of C) and of Hbar (rows of V): sums of both CGS passes (Eq. 6).
    if (t < kc) Bm[t + j * KMAX] = h1[t] + h2[t];
    double colt = 0.0;
    if (t <= j) {
        colt = h1[kc + t] + h2[kc + t];
        H[t + j * LDH] = colt;
    }
    if (t == 0) H[j + 1 + j * LDH] = hlast;
    // Progressive Givens QR of Hbar. Only the running entry is needed: after rotation q it is
    // a_{q+1} = -sn_q a_q + cs_q col[q+1]; lane q holds (cs_q, sn_q, col[q+1]).
    const double up = __shfl(colt, (t + 1) & 63, 64);
    const double cnext = (t < j) ? up : (t == j ? hlast : 0.0);
    const double cs_t = (t < j) ? ctrl->cs[t] : 0.0;
    const double sn_t = (t < j) ? ctrl->sn[t] : 0.0;
    double a = __shfl(colt, 0, 64);
    for (int q = 0; q < j; ++q) {
        const double mq = __shfl(sn_t, q, 64), cq = __shfl(cs_t, q, 64), bq = __shfl(cnext, q, 64);
        a = fma(-mq, a, cq * bq);
    }
    if (t != 0) return;
    const double rho = hypot(a, hlast);
    const double cs = rho > 0.0 ? a / rho : 1.0, sn = rho > 0.0 ? hlast / rho : 0.0;
    ctrl->cs[j] = cs;
    ctrl->sn[j] = sn;
    const double gj = ctrl->g[j];
    ctrl->g[j] = cs * gj;
    ctrl->g[j + 1] = -sn * gj;
    const double est = fabs(sn * gj);
    ctrl->est = est;
    ctrl->inv_h = brk ? 0.0 : 1.0 / hnorm;
    if (brk || !(est > ctrl->tol_abs) || j + 1 >= s_cycle) {
        ctrl->stop = 1;
        ctrl->j_done = j + 1;
        ctrl->breakdown = brk;
    }
}

// v_{j_done} = w_last / h (zero after a breakdown), closing the basis of the cycle.
__global__ __launch_bounds__(ROWS) void k_close_basis(const double* __restrict__ w0, const double* __restrict__ w1,
                                                      double* __restrict__ basis, int n, int ld, int vbase,
                                                      const Ctrl* ctrl) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i >= n) return;
    const int jd = ctrl->j_done;
    const double* wl = ((jd - 1) & 1) ? w1 : w0;
    basis[(size_t)(vbase + jd) * ld + i] = ctrl->breakdown ? 0.0 : wl[i] * ctrl->inv_h;
}

// ---------------------------------------------------------------------------------------------
// Tall-skinny Gram products out = L^T R over all rows (L, R: lists of columns), used for
// [C V]^T U, C^T r, U^T U at a cycle end and for the start-up CholQR.
// ---------------------------------------------------------------------------------------------
struct ColList {
    const double* seg[4];
    int cnt[4];
};
constexpr int GCHUNK = 32;               // rows staged per LDS chunk
constexpr int GL_MAX = 2 * KMAX + MMAX + 2;   // max columns on the left
constexpr int GR_MAX = KMAX + 1;              // max columns on the right
constexpr int GQ = (GL_MAX * GR_MAX + ROWS - 1) / ROWS;

__device__ __forceinline__ const double* col_of(const ColList& L, int a, int ld) {
    int base = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (a < base + L.cnt[s]) return L.seg[s] + (size_t)(a - base) * ld;
        base += L.cnt[s];
    }
    return nullptr;
}

__global__ __launch_bounds__(ROWS) void k_gram_partial(ColList L, int nl, ColList R, int nr, int n, int ld,
                                                       int rows_per_block, double* __restrict__ gpart) {
    __shared__ double Ls[GL_MAX * (GCHUNK + 1)];
    __shared__ double Rs[GR_MAX * (GCHUNK + 1)];
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    const int E = nl * nr;
    double acc[GQ];
#pragma unroll
    for (int q = 0; q < GQ; ++q) acc[q] = 0.0;
    for (int c0 = r0; c0 < r1; c0 += GCHUNK) {
        const int rows = min(GCHUNK, r1 - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < nl * GCHUNK; e += ROWS) {
            const int a = e / GCHUNK, rr = e - a * GCHUNK;
            Ls[a * (GCHUNK + 1) + rr] = rr < rows ? col_of(L, a, ld)[c0 + rr] : 0.0;
        }
        for (int e = threadIdx.x; e < nr * GCHUNK; e += ROWS) {
            const int a = e / GCHUNK, rr = e - a * GCHUNK;
            Rs[a * (GCHUNK + 1) + rr] = rr < rows ? col_of(R, a, ld)[c0 + rr] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
            const int e = threadIdx.x + q * ROWS;
            if (e < E) {
                const int a = e / nr, b = e - a * nr;
                const double* lp = Ls + a * (GCHUNK + 1);
                const double* rp = Rs + b * (GCHUNK + 1);
                double s = acc[q];
                for (int rr = 0; rr < GCHUNK; ++rr) s = fma(lp[rr], rp[rr], s);
                acc[q] = s;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < GQ; ++q) {
        const int e = threadIdx.x + q * ROWS;
        if (e < E) gpart[(size_t)blockIdx.x * E + e] = acc[q];
    }
}

__global__ __launch_bounds__(ROWS) void k_gram_reduce(const double* __restrict__ gpart, int nb, int E,
                                                      double* __restrict__ out) {
    const int e = blockIdx.x * ROWS + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += gpart[(size_t)b * E + e];
    out[e] = s;
}

// ---------------------------------------------------------------------------------------------
// Cycle end: x += [U V] y, r -= [C V] (G y), C <- [C V] Qc, U <- [U V] Qu (in place, row-wise),
// then ||r|| for the next cycle (Alg. 2: x_i, r_i and the recycle-space update).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_cycle_update(double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ basis, double* __restrict__ U,
                                                       int n, int ld, int vbase, int nblk, const Coef* coef,
                                                       double* part1, unsigned* counter, Ctrl* ctrl) {
    __shared__ double sQc[LDQC * KMAX];
    __shared__ double sQu[LDQU * KMAX];
    __shared__ double sy[KMAX + MMAX + 1];
    __shared__ double sr[KMAX + MMAX + 2];
    __shared__ double sh[NWAVE * NC];
    const int kc = ctrl->kc, jd = ctrl->j_done, brk = ctrl->breakdown, kn = ctrl->k_new;
    const int nv = jd + (brk ? 0 : 1);     // V columns of W-hat that enter (v_{jd} is zero after a breakdown)
    for (int e = threadIdx.x; e < LDQC * kn; e += ROWS) sQc[e] = coef->Qc[e];
    for (int e = threadIdx.x; e < LDQU * kn; e += ROWS) sQu[e] = coef->Qu[e];
    for (int e = threadIdx.x; e < kc; e += ROWS) {
        sy[e] = coef->yU[e];
        sr[e] = coef->rC[e];
    }
    for (int e = threadIdx.x; e < jd; e += ROWS) sy[kc + e] = coef->yV[e];
    for (int e = threadIdx.x; e < nv; e += ROWS) sr[kc + e] = coef->rV[e];
    __syncthreads();
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double rn2 = 0.0;
    if (i < n) {
        double xi = x[i], ri = r[i];
        double cn[KMAX], un[KMAX];
#pragma unroll
        for (int o = 0; o < KMAX; ++o) { cn[o] = 0.0; un[o] = 0.0; }
        for (int c = 0; c < kc; ++c) {
            const double cv = basis[(size_t)c * ld + i];
            ri = fma(-cv, sr[c], ri);
#pragma unroll
            for (int o = 0; o < KMAX; ++o)
                if (o < kn) cn[o] = fma(cv, sQc[c + o * LDQC], cn[o]);
        }
        for (int c = 0; c < kc; ++c) {
            const double uv = U[(size_t)c * ld + i];
            xi = fma(uv, sy[c], xi);
#pragma unroll
            for (int o = 0; o < KMAX; ++o)
                if (o < kn) un[o] = fma(uv, sQu[c + o * LDQU], un[o]);
        }
        for (int t = 0; t < nv; ++t) {
            const double vv = basis[(size_t)(vbase + t) * ld + i];
            ri = fma(-vv, sr[kc + t], ri);
#pragma unroll
            for (int o = 0; o < KMAX; ++o)
                if (o < kn) cn[o] = fma(vv, sQc[kc + t + o * LDQC], cn[o]);
            if (t < jd) {
                xi = fma(vv, sy[kc + t], xi);
#pragma unroll
                for (int o = 0; o < KMAX; ++o)
                    if (o < kn) un[o] = fma(vv, sQu[kc + t + o * LDQU], un[o]);
            }
        }
        x[i] = xi;
        r[i] = ri;
#pragma unroll
        for (int o = 0; o < KMAX; ++o)
            if (o < kn) {
                basis[(size_t)o * ld + i] = cn[o];
                U[(size_t)o * ld + i] = un[o];
            }
        rn2 = ri * ri;
    }
    double tot;
    if (grid_sum1(rn2, part1, counter, nblk, lb, sh, &tot) && threadIdx.x == 0) {
        const double bt = sqrt(tot);
        ctrl->beta = bt;
        ctrl->inv_h = bt > 0.0 ? 1.0 / bt : 0.0;
        ctrl->g[0] = bt;
        ctrl->stop = 0;
        ctrl->kc = kn;
    }
}

// ---------------------------------------------------------------------------------------------
// True residual r = b - A x (overwrites r) and ||r||^2.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_true_residual(DevOp op, const double* __restrict__ b,
                                                        const double* __restrict__ x, double* __restrict__ r,
                                                        int nblk, double* part1, unsigned* counter, Ctrl* ctrl) {
    __shared__ double sh[NWAVE * NC];
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double v = 0.0;
    if (i < op.n) {
        const double ri = b[i] - op_row(op, x, i, 1.0);
        r[i] = ri;
        v = ri * ri;
    }
    double tot;
    if (grid_sum1(v, part1, counter, nblk, lb, sh, &tot) && threadIdx.x == 0) {
        const double bt = sqrt(tot);
        ctrl->res2 = tot;
        ctrl->beta = bt;
        ctrl->inv_h = bt > 0.0 ? 1.0 / bt : 0.0;
        ctrl->g[0] = bt;
        ctrl->stop = 0;
    }
}

// ---------------------------------------------------------------------------------------------
// Start-up with a carried recycle space (App. B.1): Z = A Y, CholQR2 of Z with column drops,
// C = Q, U = Y R^{-1}, x1 = U C^T r0, r1 = r0 - C C^T r0.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_spmm(DevOp op, const double* __restrict__ Y, double* __restrict__ Z,
                                               int ld, int kin) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i >= op.n) return;
    for (int c = 0; c < kin; ++c) Z[(size_t)c * ld + i] = op_row(op, Y + (size_t)c * ld, i, 1.0);
}

// Row-wise triangular solves z <- z R^{-1} (R upper, k x k, ld KMAX) on Z (kept columns gathered
// through keep[]) and on U, compacting both to the first k_eff columns.
__global__ __launch_bounds__(ROWS) void k_startup_apply(double* __restrict__ Z, double* __restrict__ U, int n,
                                                        int ld, const Coef* coef, int use_keep, int second) {
    __shared__ double Rs[KMAX * KMAX];
    __shared__ int ks[KMAX];
    const int ke = coef->k_eff;
    const double* Rsrc = second ? coef->R2 : coef->R;
    for (int e = threadIdx.x; e < KMAX * KMAX; e += ROWS) Rs[e] = Rsrc[e];
    for (int e = threadIdx.x; e < KMAX; e += ROWS) ks[e] = use_keep ? coef->keep[e] : e;
    __syncthreads();
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i >= n) return;
    double z[KMAX], u[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        z[c] = c < ke ? Z[(size_t)ks[c] * ld + i] : 0.0;
        u[c] = c < ke ? U[(size_t)ks[c] * ld + i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < KMAX; ++c) {
        if (c < ke) {
            double sz = z[c], su = u[c];
#pragma unroll
            for (int t = 0; t < c; ++t) {
                sz = fma(-z[t], Rs[t + c * KMAX], sz);
                su = fma(-u[t], Rs[t + c * KMAX], su);
            }
            const double d = Rs[c + c * KMAX];
            z[c] = sz / d;
            u[c] = su / d;
        }
    }
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
        if (c < ke) {
            Z[(size_t)c * ld + i] = z[c];
            U[(size_t)c * ld + i] = u[c];
        }
}

// cvec = C^T r0 (partials + last-workgroup reduction into red_out[0..k_eff)).
__global__ __launch_bounds__(ROWS) void k_ctr(const double* __restrict__ C, const double* __restrict__ r, int n,
                                              int ld, int nblk, const Coef* coef, double* part, unsigned* counter,
                                              double* red_out) {
    __shared__ double sh[NWAVE * NC];
    const int ke = coef->k_eff;
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const double ri = valid ? r[i] : 0.0;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = (valid && c < ke) ? C[(size_t)c * ld + i] * ri : 0.0;
    const double s = wave_reduce_scatter64(acc);
    sh[wave_id() * NC + lane_id()] = s;
    __syncthreads();
    if (threadIdx.x < NC) {
        double t = sh[threadIdx.x];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q) t += sh[q * NC + threadIdx.x];
        part[lb * NC + threadIdx.x] = t;
    }
    if (last_block_arrive(counter, (unsigned)nblk)) final_reduce64(part, nblk, sh, red_out);
}

// x1 = U c, r1 = r0 - C c, ||r1|| -> control block (next cycle starts from r1).
__global__ __launch_bounds__(ROWS) void k_startup_project(double* __restrict__ x, double* __restrict__ r,
                                                          const double* __restrict__ C, const double* __restrict__ U,
                                                          int n, int ld, int nblk, const Coef* coef,
                                                          const double* __restrict__ cvec, double* part1,
                                                          unsigned* counter, Ctrl* ctrl) {
    __shared__ double sh[NWAVE * NC];
    __shared__ double cs[KMAX];
    const int ke = coef->k_eff;
    if (threadIdx.x < KMAX) cs[threadIdx.x] = threadIdx.x < ke ? cvec[threadIdx.x] : 0.0;
    __syncthreads();
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        double xi = 0.0, ri = r[i];
        for (int c = 0; c < ke; ++c) {
            xi = fma(U[(size_t)c * ld + i], cs[c], xi);
            ri = fma(-C[(size_t)c * ld + i], cs[c], ri);
        }
        x[i] = xi;
        r[i] = ri;
        v = ri * ri;
    }
    double tot;
    if (grid_sum1(v, part1, counter, nblk, lb, sh, &tot) && threadIdx.x == 0) {
        const double bt = sqrt(tot);
        ctrl->beta = bt;
        ctrl->inv_h = bt > 0.0 ? 1.0 / bt : 0.0;
        ctrl->g[0] = bt;
        ctrl->est = bt;
        ctrl->stop = 0;
        ctrl->kc = ke;
    }
}

// ---------------------------------------------------------------------------------------------
// Plain y = A x (the sparse product alone, for the SpMV entry point).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(ROWS) void k_spmv(DevOp op, const double* __restrict__ x, double* __restrict__ y) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i < op.n) y[i] = op_row(op, x, i, 1.0);
}

// ---------------------------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------------------------
static inline int blocks_for(long n) { return (int)((n + ROWS - 1) / ROWS); }

void launch_init(hipStream_t s, const Work& w, const double* b, double* x, double rtol) {
    hipLaunchKernelGGL(k_init, dim3(w.nblk), dim3(ROWS), 0, s, b, x, w.r, w.n, w.nblk, rtol, w.part1,
                       w.counters + 0, w.ctrl);
}
void launch_clear_nonfinite(hipStream_t s, const Work& w) {
    hipLaunchKernelGGL(k_clear_nonfinite, dim3(1), dim3(1), 0, s, w.ctrl);
}
void launch_check_finite(hipStream_t s, const Work& w, const double* v, long count) {
    if (count <= 0) return;
    const int g = (int)std::min<long>(1024, (count + ROWS - 1) / ROWS);
    hipLaunchKernelGGL(k_check_finite, dim3(g), dim3(ROWS), 0, s, v, count, w.ctrl);
}
void launch_zero(hipStream_t s, double* x, int n) {
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n)), dim3(ROWS), 0, s, x, n);
}
void launch_step(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, int s_cycle) {
    const int vbase = w.k;
    const double* src = (j == 0) ? w.r : w.W[(j - 1) & 1];
    double* dst = w.W[j & 1];
    hipLaunchKernelGGL(k_step_a, dim3(w.nblk), dim3(ROWS), 0, s, op, src, dst, w.basis, w.ld, kc, vbase, j,
                       w.nblk, w.part, w.counters + 1, w.red1, w.ctrl);
    hipLaunchKernelGGL(k_step_b, dim3(w.nblk), dim3(ROWS), 0, s, dst, (const double*)w.basis, w.n, w.ld, kc,
                       vbase, j, w.nblk, (const double*)w.red1, w.part, w.counters + 2, w.red2,
                       (const Ctrl*)w.ctrl);
    hipLaunchKernelGGL(k_step_c, dim3(w.nblk), dim3(ROWS), 0, s, dst, (const double*)w.basis, w.n, w.ld, kc,
                       vbase, j, s_cycle, w.nblk, (const double*)w.red1, (const double*)w.red2, w.part1,
                       w.counters + 3, w.H, w.Bm, w.ctrl);
}
void launch_close_basis(hipStream_t s, const Work& w) {
    hipLaunchKernelGGL(k_close_basis, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, (const double*)w.W[0],
                       (const double*)w.W[1], w.basis, w.n, w.ld, w.k, (const Ctrl*)w.ctrl);
}
void launch_gram(hipStream_t s, const Work& w, const ColList& L, int nl, const ColList& R, int nr, double* out) {
    const int E = nl * nr;
    const int rpb = ((w.n + w.ngblk - 1) / w.ngblk + GCHUNK - 1) / GCHUNK * GCHUNK;
    const int nb = (w.n + rpb - 1) / rpb;
    hipLaunchKernelGGL(k_gram_partial, dim3(nb), dim3(ROWS), 0, s, L, nl, R, nr, w.n, w.ld, rpb, w.gpart);
    hipLaunchKernelGGL(k_gram_reduce, dim3(blocks_for(E)), dim3(ROWS), 0, s, (const double*)w.gpart, nb, E, out);
}
void launch_cycle_gram(hipStream_t s, const Work& w, int kc, int jd_max) {
    // L = [C (kc), V_0..V_jd (jd+1), U (kc)], R = [U (kc), r]; jd is bounded on the host by the
    // cycle length, the columns past j_done only add products that nobody reads.
    ColList L = {{w.basis, w.basis + (size_t)w.k * w.ld, w.U, nullptr}, {kc, jd_max + 1, kc, 0}};
    ColList R = {{w.U, w.r, nullptr, nullptr}, {kc, 1, 0, 0}};
    launch_gram(s, w, L, 2 * kc + jd_max + 1, R, kc + 1, w.gram);
}
void launch_cycle_update(hipStream_t s, const Work& w, double* x) {
    hipLaunchKernelGGL(k_cycle_update, dim3(w.nblk), dim3(ROWS), 0, s, x, w.r, w.basis, w.U, w.n, w.ld, w.k,
                       w.nblk, (const Coef*)w.coef, w.part1, w.counters + 4, w.ctrl);
}
void launch_true_residual(hipStream_t s, const Work& w, const DevOp& op, const double* b, const double* x) {
    hipLaunchKernelGGL(k_true_residual, dim3(w.nblk), dim3(ROWS), 0, s, op, b, x, w.r, w.nblk, w.part1,
                       w.counters + 5, w.ctrl);
}
void launch_spmm(hipStream_t s, const Work& w, const DevOp& op, int kin) {
    hipLaunchKernelGGL(k_spmm, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, op, (const double*)w.U, w.basis, w.ld, kin);
}
void launch_startup_gram(hipStream_t s, const Work& w, int kcols) {
    ColList L = {{w.basis, nullptr, nullptr, nullptr}, {kcols, 0, 0, 0}};
    launch_gram(s, w, L, kcols, L, kcols, w.gram);
}
void launch_startup_apply(hipStream_t s, const Work& w, int use_keep, int second) {
    hipLaunchKernelGGL(k_startup_apply, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, w.basis, w.U, w.n, w.ld,
                       (const Coef*)w.coef, use_keep, second);
}
void launch_startup_project(hipStream_t s, const Work& w, double* x) {
    hipLaunchKernelGGL(k_ctr, dim3(w.nblk), dim3(ROWS), 0, s, (const double*)w.basis, (const double*)w.r, w.n,
                       w.ld, w.nblk, (const Coef*)w.coef, w.part, w.counters + 6, w.red1);
    hipLaunchKernelGGL(k_startup_project, dim3(w.nblk), dim3(ROWS), 0, s, x, w.r, (const double*)w.basis,
                       (const double*)w.U, w.n, w.ld, w.nblk, (const Coef*)w.coef, (const double*)w.red1,
                       w.part1, w.counters + 7, w.ctrl);
}
void launch_spmv(hipStream_t s, const DevOp& op, const double* x, double* y) {
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(op.n)), dim3(ROWS), 0, s, op, x, y);
}

int gram_cols_max(int m, int k) { return (2 * k + m + 2) * (k + 1); }

}  // namespace skr
