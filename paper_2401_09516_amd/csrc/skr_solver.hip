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
#include <hip/hip_ext.h>

#include "skr_internal.hpp"

namespace skr {

// Column c of Q = [C (kc columns), V (j+1 columns)] inside the basis buffer.
__device__ __forceinline__ const double* qcol(const double* basis, int ld, int kc, int vbase, int c) {
    return c < kc ? basis + (size_t)c * ld : basis + (size_t)(vbase + c - kc) * ld;
}

// ---------------------------------------------------------------------------------------------
// Solve set-up: x = 0, r = b, partials of ||b||^2 (closed by k_norm_finish).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void k_init_body(const double* __restrict__ b, double* __restrict__ x,
                                               double* __restrict__ r, int n, int nblk, double* part_n) {
    __shared__ double sh[NWAVE];
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        v = bi * bi;
    }
    block_partial1(v, part_n, lb, sh);
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_init(const double* __restrict__ b, double* __restrict__ x,
                                               double* __restrict__ r, int n, int nblk, double* part_n) {
    k_init_body(b, x, r, n, nblk, part_n);
}
#endif


// Close of a squared-norm reduction whose per-workgroup partials (folded or not) the previous
// kernel left: one workgroup sums them in the fixed order every Arnoldi pass A uses for the same
// partials, so the host and the next cycle see bitwise the same value, and sets the control-block
// fields that follow from it. No fences or atomics: the kernel boundary orders it after the writer.
enum { FIN_INIT = 0, FIN_TRUE_RES = 1, FIN_PROJECT = 2 };
__device__ __forceinline__ void k_norm_finish_body(const double* __restrict__ pn, int npn, int mode, double rtol,
                                                      int ke, Ctrl* ctrl) {
    __shared__ double sh[NWAVE * NC];
    const double tot = sum_partials1(pn, npn, sh);
    if (threadIdx.x != 0) return;
    const double bt = sqrt(tot);
    ctrl->beta = bt;
    ctrl->inv_h = bt > 0.0 ? 1.0 / bt : 0.0;
    ctrl->g[0] = bt;
    ctrl->stop = 0;
    if (mode == FIN_INIT) {
        ctrl->j_done = 0;
        ctrl->breakdown = 0;
        ctrl->kc = 0;
        ctrl->k_new = 0;
        ctrl->eig_fail = 0;
        ctrl->nonfinite = (isfinite(bt) ? 0 : 1) | ctrl->nonfinite;
        ctrl->bnorm = bt;
        ctrl->tol_abs = rtol * bt;
        ctrl->est = bt;
        ctrl->res2 = tot;
    } else if (mode == FIN_TRUE_RES) {
        ctrl->res2 = tot;
    } else {
        ctrl->est = bt;
        ctrl->kc = ke;
    }
}
#ifndef SKR_CHAINS_UNIT
// gate (when given): the control block's spec_skip; a kernel launched ahead of the host's read of a
// cycle end returns at once when that cycle end cleared the way for none (every thread reads the
// same value, so the whole grid returns)
__global__ __launch_bounds__(ROWS) void k_norm_finish(const double* __restrict__ pn, int npn, int mode, double rtol,
                                                      int ke, Ctrl* ctrl, const int* __restrict__ gate) {
    if (gate && *gate) return;
    k_norm_finish_body(pn, npn, mode, rtol, ke, ctrl);
}
#endif


__device__ __forceinline__ void k_clear_nonfinite_body(Ctrl* ctrl) {
    ctrl->nonfinite = 0;
    ctrl->nonsym = 0;
}
#ifndef SKR_CHAINS_UNIT
__global__  void k_clear_nonfinite(Ctrl* ctrl) {
    k_clear_nonfinite_body(ctrl);
}
#endif


// Exact symmetry of a CSR operator: entry (i, c, v) with c != i needs an entry (c, i) of the same
// value (duplicates are summed, as in the product). One row per thread; row c is scanned for
// column i (rows need not be sorted). Any mismatch sets ctrl->nonsym.
__device__ __forceinline__ void k_check_sym_csr_body(DevOp op, Ctrl* ctrl) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    int bad = 0;
    if (i < op.n) {
        const int e1 = op.rowptr[i + 1];
        for (int e = op.rowptr[i]; e < e1 && !bad; ++e) {
            const int c = op.colind[e];
            if (c == i) continue;
            if (c < 0 || c >= op.n) { bad = 1; break; }
            double vij = 0.0, vji = 0.0;
            for (int f = op.rowptr[i]; f < e1; ++f) vij += (op.colind[f] == c) ? op.val[f] : 0.0;
            const int f1 = op.rowptr[c + 1];
            for (int f = op.rowptr[c]; f < f1; ++f) vji += (op.colind[f] == i) ? op.val[f] : 0.0;
            bad = (vij == vji) ? 0 : 1;
        }
    }
    if (__any(bad) && lane_id() == 0) atomicOr(&ctrl->nonsym, 1);
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_check_sym_csr(DevOp op, Ctrl* ctrl) {
    k_check_sym_csr_body(op, ctrl);
}
#endif


__device__ __forceinline__ void k_check_finite_body(const double* __restrict__ v, long count, Ctrl* ctrl) {
    int bad = 0;
    for (long e = blockIdx.x * (long)ROWS + threadIdx.x; e < count; e += (long)gridDim.x * ROWS)
        bad |= !isfinite(v[e]);
    if (__any(bad) && lane_id() == 0) atomicOr(&ctrl->nonfinite, 1);
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_check_finite(const double* __restrict__ v, long count, Ctrl* ctrl) {
    k_check_finite_body(v, count, ctrl);
}
#endif


__device__ __forceinline__ void k_zero_body(double* __restrict__ x, int n) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i < n) x[i] = 0.0;
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_zero(double* __restrict__ x, int n) {
    k_zero_body(x, n);
}
#endif


// ---------------------------------------------------------------------------------------------
// Arnoldi step kernels. NL (a multiple of 8, >= the columns used) is the number of basis loads per
// row, fixed at compile time so that all loads of a row are unconditional and in flight together:
// columns past the last one used re-read the last column (same address, a cache hit) and get a zero
// coefficient. Rows past n re-read row n-1 and contribute zero. NR is the reduction width.
// ---------------------------------------------------------------------------------------------
// NR covers columns 0..63, NR2 the columns from 64 on (NL > 64): a lane of the reduce-scatter then
// holds one column of each group.
template <int NL>
struct Width {
    static constexpr int NR = NL <= 16 ? 16 : (NL <= 32 ? 32 : 64);
    static constexpr int NR2 = NL <= 64 ? 0 : (NL <= 80 ? 16 : 32);
};

__device__ __forceinline__ size_t qoff(int c, int kc, int vbase, int ld) {
    return (size_t)(c < kc ? c : vbase + c - kc) * (size_t)ld;
}

// Block-combine NR column values (one reduce-scattered value per lane) into the per-workgroup
// partial part[lb * NC + OFF + c], c < NR; columns past cmax are written as zero (so a caller can
// leave products of no meaning in them instead of selecting zero per lane and column). sh:
// NWAVE * NR doubles of its own.
template <int NR, int OFF = 0>
__device__ __forceinline__ void block_partials(double s, double* sh, double* part, int lb, int cmax = NC + 64) {
    if (lane_id() < NR) sh[wave_id() * NR + lane_id()] = s;
    __syncthreads();
    if (threadIdx.x < NR) {
        double t = sh[threadIdx.x];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q) t += sh[q * NR + threadIdx.x];
        part[lb * NC + OFF + threadIdx.x] = (OFF + (int)threadIdx.x <= cmax) ? t : 0.0;
    }
}

// Close step jj of the current cycle once tot = ||w||^2 is known (Eq. 6): column jj of B (rows of
// C) and of Hbar (rows of V) are the sums of the two CGS passes h1 + h2, h_{jj+1,jj} = ||w|| (zero
// at a happy breakdown, h <= 1e-14 ||A v_jj||), and the progressive Givens QR of Hbar gives the
// least-squares residual estimate |g_{jj+1}|; g3, when given, is subtracted from the column (the
// correction of the merged kernel below). Run by wave 0 of every calling workgroup on identical
// inputs, so all get identical results; only the writer workgroup stores the column, the new
// rotation and g_{jj+1}. Only the running entry of the rotated column is needed: after rotation q
// it is a_{q+1} = -sn_q a_q + cs_q col[q+1], run by lane 0 from LDS copies (shc, 3 x 128 doubles;
// lane t handles the column entries t and t + 64).
// The global inputs of close_step for lane t of the closing wave: h1 at the rows of the column and
// of B (e = t, t + 64), ||A v||^2 = h1[ncol], the rotations stored by the earlier closings and g_jj.
// Every one was written by an earlier kernel, so the caller loads them with its first loads, ahead
// of the partial sums (clamped indices, unneeded entries zero).
struct CloseIn {
    double h1c[2], h1b[2], cs[2], sn[2], anorm2, gj;
    __device__ __forceinline__ void load(int jj, int kc, const double* __restrict__ h1, const Ctrl* ctrl) {
        const int t = threadIdx.x;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int e = t + 64 * half;
            const double a = h1[kc + min(e, jj)], b = h1[min(e, max(kc - 1, 0))];
            const double c = ctrl->cs[min(e, max(jj - 1, 0))], d = ctrl->sn[min(e, max(jj - 1, 0))];
            h1c[half] = e <= jj ? a : 0.0;
            h1b[half] = e < kc ? b : 0.0;
            cs[half] = e < jj ? c : 0.0;
            sn[half] = e < jj ? d : 0.0;
        }
        anorm2 = h1[kc + jj + 1];
        gj = ctrl->g[jj];
    }
};
// h2 at the same rows (e = t, t + 64: the column's rows kc + e and B's rows e), from global memory
// (loaded early like CloseIn) or from LDS.
__device__ __forceinline__ void load_h2(int jj, int kc, const double* __restrict__ h2, double h2c[2], double h2b[2]) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int e = threadIdx.x + 64 * half;
        const double a = h2[kc + min(e, jj)], b = h2[min(e, max(kc - 1, 0))];
        h2c[half] = e <= jj ? a : 0.0;
        h2b[half] = e < kc ? b : 0.0;
    }
}
__device__ __forceinline__ double close_step(int jj, int kc, double tot, const CloseIn& ci, const double h2c[2],
                                             const double h2b[2], double* H, double* Bm, Ctrl* ctrl,
                                             bool writer, int& brk_out, double& hnorm_out, double* shc,
                                             const double* __restrict__ g3 = nullptr) {
    const int t = threadIdx.x;
    const double hnorm = sqrt(tot);
    const double anorm = sqrt(ci.anorm2);
    const int brk = (hnorm <= 1e-14 * anorm) ? 1 : 0;
    const double hlast = brk ? 0.0 : hnorm;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int e = t + 64 * half;
        double colt = 0.0;
        if (e <= jj) colt = ci.h1c[half] + h2c[half] - (g3 ? g3[kc + e] : 0.0);
        if (writer) {
            if (e < kc) Bm[e + jj * KMAX] = ci.h1b[half] + h2b[half] - (g3 ? g3[e] : 0.0);
            if (e <= jj) H[e + jj * LDH] = colt;
        }
        shc[e] = colt;
        shc[128 + e] = ci.cs[half];
        shc[256 + e] = ci.sn[half];
    }
    if (writer && t == 0) H[jj + 1 + jj * LDH] = hlast;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    double a = 0.0;
    if (t == 0) {
        a = shc[0];
        for (int q = 0; q < jj; ++q) a = fma(-shc[256 + q], a, shc[128 + q] * shc[q + 1]);
    }
    a = first_lane(a);
    const double rho = hypot(a, hlast);
    const double cs = rho > 0.0 ? a / rho : 1.0, sn = rho > 0.0 ? hlast / rho : 0.0;
    const double gj = ci.gj;
    const double est = fabs(sn * gj);
    if (writer && t == 0) {
        ctrl->cs[jj] = cs;
        ctrl->sn[jj] = sn;
        ctrl->g[jj + 1] = -sn * gj;
        ctrl->est = est;
    }
    brk_out = brk;
    hnorm_out = hnorm;
    return est;
}

// Pass A of step j: first closes step j-1 from the partials of ||w||^2 left by pass C (for j = 0,
// the partials of ||r||^2 left by the kernel that prepared r give beta), stopping the cycle when
// the estimate meets the tolerance or the step broke down; then v_j = w * inv_h (stored as a basis
// column), w = A v_j, and partials of Q^T w (Q = [C, V_0..V_j], ncol = kc + j + 1 columns) and of
// ||w||^2 (reduction column ncol).
template <int NL, int KIND, typename BT>
__device__ __forceinline__ void k_step_a_body(DevOp op, const double* __restrict__ src,
                                                 double* __restrict__ dst, BT* __restrict__ basis,
                                                 int ld, int kc, int vbase, int j, int nblk, int npn,
                                                 const double* __restrict__ part_n, double* __restrict__ part_a,
                                                 const double* __restrict__ red1, const double* __restrict__ red2,
                                                 double* H, double* Bm, Ctrl* ctrl) {
    constexpr int NR = Width<NL>::NR, NR2 = Width<NL>::NR2;
    __shared__ double sh[NWAVE * NC];
    __shared__ double s_scale;
    __shared__ int s_stop;
    const bool writer = blockIdx.x == 0;
    const int n = op.n;
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    const int ncol = kc + j + 1;
    const int nst = ncol - 1;                 // stored columns (v_j itself is formed here)
    // Every global load of the kernel is issued before the first decision that waits on one: the
    // stop flag, the basis rows, the product with the unscaled previous vector (A is linear, so the
    // scale is applied afterwards) and the partials of ||w||^2. With an FP32 basis the product is
    // taken on the stored (rounded) vector, which needs the scale: it follows the closing instead.
    constexpr bool MIX = sizeof(BT) == 4;
    const int stopped = ctrl->stop;
    double q[NL];
    if (nst > 0) {
#pragma unroll
        for (int c = 0; c < NL; ++c) q[c] = (double)basis[qoff(c < nst ? c : nst - 1, kc, vbase, ld) + ii];
    } else {
#pragma unroll
        for (int c = 0; c < NL; ++c) q[c] = 0.0;
    }
    double pn[4] = {0.0, 0.0, 0.0, 0.0};
    const bool few = npn <= 4 * 64;
    if (few && threadIdx.x < 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = threadIdx.x + 64 * u;
            pn[u] = (b < npn) ? part_n[b] : 0.0;
        }
    }
    const double xi = src[ii];
    double wraw = 0.0;
    if constexpr (!MIX) wraw = op_row_k<KIND>(op, src, ii, 1.0);
    CloseIn ci;
    double h2c[2], h2b[2];
    if (j > 0 && threadIdx.x < 64) {
        ci.load(j - 1, kc, red1, ctrl);
        load_h2(j - 1, kc, red2, h2c, h2b);
    }
    if (stopped) return;
    double tot;
    if (few) {
        // same order as sum_partials1: lane-strided sums, then the wave butterfly
        if (threadIdx.x < 64) {
            const double ws = wave_sum(((pn[0] + pn[1]) + pn[2]) + pn[3]);
            if (threadIdx.x == 0) sh[0] = ws;
        }
        __syncthreads();
        tot = sh[0];
        __syncthreads();
    } else {
        tot = sum_partials1(part_n, npn, sh);
    }
    if (j == 0) {
        if (threadIdx.x == 0) {
            const double bt = sqrt(tot);
            s_scale = bt > 0.0 ? 1.0 / bt : 0.0;
            s_stop = 0;
            if (writer) {
                ctrl->beta = bt;
                ctrl->g[0] = bt;
                ctrl->inv_h = s_scale;
            }
        }
    } else if (threadIdx.x < 64) {
        int brk;
        double hn;
        const double est = close_step(j - 1, kc, tot, ci, h2c, h2b, H, Bm, ctrl, writer, brk, hn, sh + 64);
        if (threadIdx.x == 0) {
            const int stop = (brk || !(est > ctrl->tol_abs)) ? 1 : 0;
            s_stop = stop;
            s_scale = brk ? 0.0 : 1.0 / hn;
            if (writer) {
                ctrl->inv_h = s_scale;
                if (stop) {
                    ctrl->j_done = j;
                    ctrl->breakdown = brk;
                    ctrl->stop = 1;
                }
            }
        }
    }
    __syncthreads();
    if (s_stop) return;
    const double scale = s_scale;
    double vj, w;
    if constexpr (MIX) {
        vj = rnd32(xi * scale);
        w = op_row_k<KIND, double, true, true>(op, src, ii, scale);
    } else {
        vj = xi * scale;
        w = wraw * scale;
    }
    if (valid) {
        basis[(size_t)(vbase + j) * ld + i] = (BT)vj;
        dst[i] = w;
    } else {
        w = 0.0;
    }
    // Column products q_c w for every column (no per-column select); the columns of v_j and of
    // ||w||^2 sit at runtime positions, so their sums come from wave sums, which pair the lanes in
    // the reduce-scatter's order (the same bits), and replace the sum of the lane that holds each.
    // Columns past ncol hold products of no meaning; the block sums write them as zero.
    const double vw = wave_sum(vj * w), ww = wave_sum(w * w);
    const int lane = lane_id();
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = (c < NL) ? q[c < NL ? c : 0] * w : 0.0;
    double s = wave_reduce_scatter<NR>(acc);
    s = (lane == nst) ? vw : ((lane == ncol) ? ww : s);
    if constexpr (NR2 > 0) {
        double acc2[NR2];
#pragma unroll
        for (int c = 0; c < NR2; ++c) acc2[c] = (64 + c < NL) ? q[64 + c < NL ? 64 + c : 0] * w : 0.0;
        double s2 = wave_reduce_scatter<NR2>(acc2);
        s2 = (lane + 64 == nst) ? vw : ((lane + 64 == ncol) ? ww : s2);
        block_partials<NR2, 64>(s2, sh + NWAVE * 64, part_a, lb, ncol);
    }
    block_partials<NR>(s, sh, part_a, lb, ncol);
}
template <int NL, int KIND, typename BT>
__global__ __launch_bounds__(ROWS) void k_step_a(DevOp op, const double* __restrict__ src,
                                                 double* __restrict__ dst, BT* __restrict__ basis,
                                                 int ld, int kc, int vbase, int j, int nblk, int npn,
                                                 const double* __restrict__ part_n, double* __restrict__ part_a,
                                                 const double* __restrict__ red1, const double* __restrict__ red2,
                                                 double* H, double* Bm, Ctrl* ctrl) {
    k_step_a_body<NL, KIND, BT>(op, src, dst, basis, ld, kc, vbase, j, nblk, npn, part_n, part_a, red1, red2, H, Bm, ctrl);
}


// Pass B: h1 = Q^T w (sum of pass A's partials, also stored for the step's closing), w -= Q h1,
// partials of Q^T w; with NORM also of ||w||^2 (reduction column ncol), which the merged kernel
// below needs in place of a pass C. Without NORM the coefficients come from a copy of h1 padded
// with zeros past ncol and the products of the re-read columns past ncol are formed and dropped
// (their partials are written as zero): no per-column select, which would otherwise keep a
// selected coefficient and a lane mask per column live beside the basis values (spilling past
// 256 registers from 64 columns on). The column sums are those of the masked form, bit for bit.
template <int NL, typename BT, bool FOLDED, bool NORM = false>
__device__ __forceinline__ void k_step_b_body(double* __restrict__ w_io, const BT* __restrict__ basis,
                                                 int n, int ld, int kc, int vbase, int j, int nblk, int npa,
                                                 const double* __restrict__ part_a, double* __restrict__ part_b,
                                                 double* __restrict__ red1, const Ctrl* ctrl) {
    constexpr int NR = Width<NL>::NR, NR2 = Width<NL>::NR2;
    __shared__ double sh[NWAVE * NC];
    __shared__ double hs[NC];
    __shared__ double hz[NC];
    const int ncol = kc + j + 1;
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    double q[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) q[c] = (double)basis[qoff(c < ncol ? c : ncol - 1, kc, vbase, ld) + ii];
    double w = w_io[ii];
    const int stopped = ctrl->stop;
    sum_partials<FOLDED ? 16 : 64>(part_a, npa, ncol + 1, sh, hs);
    if (stopped) return;
    if (blockIdx.x == 0 && threadIdx.x <= ncol) red1[threadIdx.x] = hs[threadIdx.x];
    if constexpr (NORM) {
        // h1 padded with zeros past ncol (no per-column select); the products past ncol have no
        // meaning and the block sums write them as zero
        if (threadIdx.x < NC) hz[threadIdx.x] = threadIdx.x < ncol ? hs[threadIdx.x] : 0.0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NL; ++c) w = fma(-q[c], hz[c], w);
        if (valid) w_io[i] = w;
        else w = 0.0;
        // ||w||^2 from a wave sum (the reduce-scatter's lane pairing, so the same bits) in the lane
        // of column ncol, as in pass A
        const double ww = wave_sum(w * w);
        const int lane = lane_id();
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = (c < NL) ? q[c < NL ? c : 0] * w : 0.0;
        double s = wave_reduce_scatter<NR>(acc);
        s = (lane == ncol) ? ww : s;
        if constexpr (NR2 > 0) {
            double acc2[NR2];
#pragma unroll
            for (int c = 0; c < NR2; ++c) acc2[c] = (64 + c < NL) ? q[64 + c < NL ? 64 + c : 0] * w : 0.0;
            double s2 = wave_reduce_scatter<NR2>(acc2);
            s2 = (lane + 64 == ncol) ? ww : s2;
            block_partials<NR2, 64>(s2, sh + NWAVE * 64, part_b, lb, ncol);
        }
        block_partials<NR>(s, sh, part_b, lb, ncol);
    } else {
        if (threadIdx.x < NC) hz[threadIdx.x] = threadIdx.x < ncol ? hs[threadIdx.x] : 0.0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NL; ++c) w = fma(-q[c], hz[c], w);
        if (valid) w_io[i] = w;
        else w = 0.0;
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = c < NL ? q[c] * w : 0.0;
        const double s = wave_reduce_scatter<NR>(acc);
        double s2 = 0.0;
        if constexpr (NR2 > 0) {
            double acc2[NR2];
#pragma unroll
            for (int c = 0; c < NR2; ++c) acc2[c] = 64 + c < NL ? q[64 + c] * w : 0.0;
            s2 = wave_reduce_scatter<NR2>(acc2);
        }
        // block sums as in block_partials, with the columns from ncol on written as zero
        if (lane_id() < NR) sh[wave_id() * NR + lane_id()] = s;
        if constexpr (NR2 > 0)
            if (lane_id() < NR2) sh[NWAVE * 64 + wave_id() * NR2 + lane_id()] = s2;
        __syncthreads();
        const int c = threadIdx.x;
        if (c < NR) {
            double t = sh[c];
#pragma unroll
            for (int q2 = 1; q2 < NWAVE; ++q2) t += sh[q2 * NR + c];
            part_b[lb * NC + c] = c < ncol ? t : 0.0;
        } else if (NR2 > 0 && c >= 64 && c < 64 + NR2) {
            double t = sh[NWAVE * 64 + (c - 64)];
#pragma unroll
            for (int q2 = 1; q2 < NWAVE; ++q2) t += sh[NWAVE * 64 + q2 * NR2 + (c - 64)];
            part_b[lb * NC + c] = c < ncol ? t : 0.0;
        }
    }
}
template <int NL, typename BT, bool FOLDED, bool NORM = false>
__global__ __launch_bounds__(ROWS) void k_step_b(double* __restrict__ w_io, const BT* __restrict__ basis,
                                                 int n, int ld, int kc, int vbase, int j, int nblk, int npa,
                                                 const double* __restrict__ part_a, double* __restrict__ part_b,
                                                 double* __restrict__ red1, const Ctrl* ctrl) {
    k_step_b_body<NL, BT, FOLDED, NORM>(w_io, basis, n, ld, kc, vbase, j, nblk, npa, part_a, part_b, red1, ctrl);
}


// Pass C: h2 = Q^T w (sum of pass B's partials, stored), w -= Q h2, partials of ||w||^2.
template <int NL, typename BT, bool FOLDED>
__device__ __forceinline__ void k_step_c_body(double* __restrict__ w_io, const BT* __restrict__ basis,
                                                 int n, int ld, int kc, int vbase, int j, int nblk, int npb,
                                                 const double* __restrict__ part_b, double* __restrict__ part_n,
                                                 double* __restrict__ red2, const Ctrl* ctrl) {
    __shared__ double sh[NWAVE * NC];
    __shared__ double hs[NC];
    __shared__ double hz[NC];
    const int ncol = kc + j + 1;
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    double q[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) q[c] = (double)basis[qoff(c < ncol ? c : ncol - 1, kc, vbase, ld) + ii];
    double w = w_io[ii];
    const int stopped = ctrl->stop;
    sum_partials<FOLDED ? 16 : 64>(part_b, npb, ncol, sh, hs);
    if (stopped) return;
    if (blockIdx.x == 0 && threadIdx.x < ncol) red2[threadIdx.x] = hs[threadIdx.x];
    // h2 padded with zeros past ncol (as in pass B: no per-column select)
    if (threadIdx.x < NC) hz[threadIdx.x] = threadIdx.x < ncol ? hs[threadIdx.x] : 0.0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NL; ++c) w = fma(-q[c], hz[c], w);
    if (valid) w_io[i] = w;
    else w = 0.0;
    block_partial1(w * w, part_n, lb, sh);
}
template <int NL, typename BT, bool FOLDED>
__global__ __launch_bounds__(ROWS) void k_step_c(double* __restrict__ w_io, const BT* __restrict__ basis,
                                                 int n, int ld, int kc, int vbase, int j, int nblk, int npb,
                                                 const double* __restrict__ part_b, double* __restrict__ part_n,
                                                 double* __restrict__ red2, const Ctrl* ctrl) {
    k_step_c_body<NL, BT, FOLDED>(w_io, basis, n, ld, kc, vbase, j, nblk, npb, part_b, part_n, red2, ctrl);
}


// Merged pass C of step j-1 and pass A of step j (FP64 basis, 1 <= j). Pass B of step j-1 left
// w_B = A v_{j-1} - Q h1 and the partials of h2 = Q^T w_B and ||w_B||^2, Q = [C, v_0..v_{j-1}]
// (ncolp = kc + j columns). CGS2 then forms w_C = w_B - Q h2 and v_j = w_C / h with
// h^2 = ||w_C||^2 = ||w_B||^2 - ||h2||^2 (Q orthonormal). The product A v_j cannot wait for v_j in
// the other rows, so it is formed from the complete w_B by linearity: A v_j = (A w_B - A Q h2) / h.
// With A C = Z (a product formed once per cycle) and the Arnoldi relation of the V columns (Eq. 6:
// A v_l = C B(:, l) + V Hbar(:, l)), A Q h2 = Z h2_C + Q' g, Q' = [Q, v_j], g = [B h2_V; Hbar h2_V].
// The term Q' g / h lies in the span the next projection removes, so the kernel continues with
// w' = (A w_B - Z h2_C) / h, and CGS2 of w' against Q' gives the same vectors as CGS2 of A v_j, with
// coefficients larger by exactly g / h: the closing of step j subtracts g / h from the column it
// assembles. The writer workgroup forms g / h after its rows are done and leaves it in gnext for
// the next kernel; gprev holds the one of step j-1 (none at j-1 = 0, which pass A formed directly).
// Every quantity is as in CGS2 in exact arithmetic; the relation's rounding, like the FP32 rounding
// of Z, enters multiplied by h2, a second-order term. LAST: the cycle's final closing (no product).
//
// The stop flag: a kernel of step j sets ctrl->stop = j + 1, so its own workgroups that read the flag
// after the writer set it still see a stop of a later step than theirs; every other kernel treats
// any nonzero value as stopped.
template <int NL, int KIND, int KZ, bool LAST>
__device__ __forceinline__ void k_step_m_body(DevOp op, const double* __restrict__ wb, double* __restrict__ dst,
                                                 double* __restrict__ basis, const float* __restrict__ Z, int ld,
                                                 int kc, int vbase, int j, int nblk, int npb,
                                                 const double* __restrict__ part_b, double* __restrict__ part_a,
                                                 const double* __restrict__ red1, const double* __restrict__ gprev,
                                                 double* __restrict__ gnext, double* H, double* Bm, Ctrl* ctrl) {
    constexpr int NR = Width<NL>::NR, NR2 = Width<NL>::NR2;
    __shared__ double sh[NWAVE * NC];
    __shared__ double hs[NC];      // h2 (ncolp entries), ||w_B||^2 at ncolp
    __shared__ double hc[NC];      // h2 padded with zeros past ncolp
    __shared__ double hz[KZ > 0 ? KZ : 1];   // h2_C padded with zeros past kc
    __shared__ double gp[NC];      // correction of the column closed here (zero at j - 1 = 0)
    __shared__ double s_scale;
    __shared__ int s_stop;
    const bool writer = blockIdx.x == 0;
    const int n = op.n;
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    const int jj = j - 1;               // the step closed here
    const int ncolp = kc + j;           // columns of Q before v_j
    const int ncol = ncolp + 1;         // with v_j
    const int st = ctrl->stop;
    // loads before the first wait: the basis row, the row of Z, w_B and its product with A
    double q[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) q[c] = basis[qoff(c < ncolp ? c : ncolp - 1, kc, vbase, ld) + ii];
    float z[KZ > 0 ? KZ : 1];
#pragma unroll
    for (int c = 0; c < (KZ > 0 ? KZ : 1); ++c) z[c] = KZ > 0 ? Z[(size_t)min(c, kc - 1) * ld + ii] : 0.0f;
    const double wbi = wb[ii];
    double aw = 0.0;
    if constexpr (!LAST) aw = op_row_k<KIND>(op, wb, ii, 1.0);
    if (threadIdx.x < NC) gp[threadIdx.x] = (jj > 0 && (int)threadIdx.x < ncolp) ? gprev[threadIdx.x] : 0.0;
    CloseIn ci;
    if (threadIdx.x < 64) ci.load(jj, kc, red1, ctrl);
    if (st != 0 && st <= j) return;     // the cycle stopped at an earlier step
    sum_partials<64>(part_b, npb, ncolp + 1, sh, hs);
    if (threadIdx.x < NC) {
        const int t = threadIdx.x;
        const double v = hs[t];
        hc[t] = t < ncolp ? v : 0.0;
        if (KZ > 0 && t < (KZ > 0 ? KZ : 1)) hz[t < (KZ > 0 ? KZ : 1) ? t : 0] = t < kc ? v : 0.0;
    }
    if (threadIdx.x < 64) {
        // ||w_C||^2 = ||w_B||^2 - ||h2||^2, summed in a fixed order (the same bits in every workgroup)
        const int t = threadIdx.x;
        const double a0 = hs[t], a1 = hs[t + 64];
        double q2 = (t < ncolp) ? a0 * a0 : 0.0;
        q2 += (t + 64 < ncolp) ? a1 * a1 : 0.0;
        const double tot = fmax(hs[ncolp] - wave_sum(q2), 0.0);
        int brk;
        double hn;
        double h2c[2], h2b[2];
        load_h2(jj, kc, hs, h2c, h2b);
        const double est = close_step(jj, kc, tot, ci, h2c, h2b, H, Bm, ctrl, writer, brk, hn, sh + 64, gp);
        if (t == 0) {
            const int stop = (brk || !(est > ctrl->tol_abs)) ? 1 : 0;
            s_stop = stop;
            s_scale = brk ? 0.0 : 1.0 / hn;
            if (writer) {
                ctrl->inv_h = s_scale;
                if (stop || LAST) {
                    ctrl->j_done = j;
                    ctrl->breakdown = brk;
                }
                if (stop) ctrl->stop = j + 1;
            }
        }
    }
    __syncthreads();
    const double scale = s_scale;
    // The writer's loads of the earlier columns of B and Hbar (for g / h, below) go out now, so that
    // their latency overlaps the row work. The four waves take interleaved columns l = w, w + 4, ...
    // < jj, each lane one row (two past 64).
    constexpr int LQ = (MMAX + NWAVE - 1) / NWAVE;
    const int wv = wave_id(), lane = lane_id();
    double gm[LAST ? 1 : 2][LAST ? 1 : LQ];
    if (!LAST && writer && !s_stop) {
#pragma unroll
        for (int half = 0; half < (LAST ? 1 : 2); ++half) {
            const int rr = min(lane + 64 * half, ncol - 1);
#pragma unroll
            for (int u = 0; u < (LAST ? 1 : LQ); ++u) {
                const int l = min(wv + NWAVE * u, max(jj - 1, 0));
                gm[half][u] = rr < kc ? Bm[rr + l * KMAX] : H[(rr - kc) + l * LDH];
            }
        }
    }
    // w_C = w_B - Q h2 and v_j = w_C / h
    double wc = wbi;
#pragma unroll
    for (int c = 0; c < NL; ++c) wc = fma(-q[c], hc[c], wc);
    const double vj = wc * scale;
    if (valid) basis[(size_t)(vbase + j) * ld + i] = vj;
    if (s_stop || LAST) return;
    // w' = (A w_B - Z h2_C) / h
    double corr = 0.0;
    if constexpr (KZ > 0) {
#pragma unroll
        for (int c = 0; c < KZ; ++c) corr = fma((double)z[c], hz[c], corr);
    }
    double w = (aw - corr) * scale;
    if (valid) dst[i] = w;
    else w = 0.0;
    // column products without per-column selects; v_j w and ||w||^2 from wave sums, as in pass A
    const double vw = wave_sum(vj * w), ww = wave_sum(w * w);
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = (c < NL) ? q[c < NL ? c : 0] * w : 0.0;
    double s = wave_reduce_scatter<NR>(acc);
    s = (lane == ncolp) ? vw : ((lane == ncol) ? ww : s);
    if constexpr (NR2 > 0) {
        double acc2[NR2];
#pragma unroll
        for (int c = 0; c < NR2; ++c) acc2[c] = (64 + c < NL) ? q[64 + c < NL ? 64 + c : 0] * w : 0.0;
        double s2 = wave_reduce_scatter<NR2>(acc2);
        s2 = (lane + 64 == ncolp) ? vw : ((lane + 64 == ncol) ? ww : s2);
        block_partials<NR2, 64>(s2, sh + NWAVE * 64, part_a, lb, ncol);
    }
    block_partials<NR>(s, sh, part_a, lb, ncol);
    if (!writer) return;
    __syncthreads();
    // g / h for the closing of step j: row t < kc is (B h2_V)_t, row kc + e is (Hbar h2_V)_e, e <= j.
    // Columns l < jj of B and Hbar were loaded above from the stores of the steps they closed;
    // column jj is the one closed here (h1 + h2 - correction, and h below the diagonal). The wave
    // sums are added in wave order, then column jj.
    if constexpr (LAST) return;
    double part2[2];
#pragma unroll
    for (int half = 0; half < (LAST ? 1 : 2); ++half) {
        const int rr = min(lane + 64 * half, ncol - 1);
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < (LAST ? 1 : LQ); ++u) {
            const int l = wv + NWAVE * u;
            const bool ok = l < jj && (rr < kc || l + 1 >= rr - kc);
            a = fma(ok ? gm[half][u] : 0.0, hs[kc + min(l, max(jj - 1, 0))], a);
        }
        part2[half] = a;
    }
    __syncthreads();
    sh[wv * 128 + lane] = part2[0];
    sh[wv * 128 + 64 + lane] = part2[1];
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NC) {
        double a = sh[t];
#pragma unroll
        for (int q2 = 1; q2 < NWAVE; ++q2) a += sh[q2 * 128 + t];
        const int tt = min(t, ncolp);
        const double colj = t < ncolp ? red1[tt] + hs[tt] - gp[tt] : 1.0 / scale;
        a = fma(colj, hs[kc + jj], a);
        gnext[t] = t < ncol ? a * scale : 0.0;
    }
}
template <int NL, int KIND, int KZ, bool LAST>
__global__ __launch_bounds__(ROWS) void k_step_m(DevOp op, const double* __restrict__ wb, double* __restrict__ dst,
                                                 double* __restrict__ basis, const float* __restrict__ Z, int ld,
                                                 int kc, int vbase, int j, int nblk, int npb,
                                                 const double* __restrict__ part_b, double* __restrict__ part_a,
                                                 const double* __restrict__ red1, const double* __restrict__ gprev,
                                                 double* __restrict__ gnext, double* H, double* Bm, Ctrl* ctrl) {
    k_step_m_body<NL, KIND, KZ, LAST>(op, wb, dst, basis, Z, ld, kc, vbase, j, nblk, npb, part_b, part_a, red1, gprev, gnext, H, Bm, ctrl);
}


// Cycle end: closes the last step when no pass A did (the cycle ran all s_cycle steps), then stores
// v_{j_done} = w_last * inv_h (zero after a breakdown), the last column of the cycle's basis.
template <typename BT>
__device__ __forceinline__ void k_close_basis_body(const double* __restrict__ w0, const double* __restrict__ w1,
                                                      BT* __restrict__ basis, int n, int ld, int kc, int vbase,
                                                      int s_cycle, int npn, const double* __restrict__ part_n,
                                                      const double* __restrict__ red1, const double* __restrict__ red2,
                                                      double* H, double* Bm, Ctrl* ctrl) {
    __shared__ double sh[NWAVE * NC];
    __shared__ double s_scale;
    __shared__ int s_jd, s_brk;
    const bool writer = blockIdx.x == 0;
    if (!ctrl->stop) {
        CloseIn ci;
        double h2c[2], h2b[2];
        if (threadIdx.x < 64) {
            ci.load(s_cycle - 1, kc, red1, ctrl);
            load_h2(s_cycle - 1, kc, red2, h2c, h2b);
        }
        const double tot = sum_partials1(part_n, npn, sh);
        if (threadIdx.x < 64) {
            int brk;
            double hn;
            close_step(s_cycle - 1, kc, tot, ci, h2c, h2b, H, Bm, ctrl, writer, brk, hn, sh + 64);
            if (threadIdx.x == 0) {
                s_jd = s_cycle;
                s_brk = brk;
                s_scale = brk ? 0.0 : 1.0 / hn;
                if (writer) {
                    ctrl->j_done = s_cycle;
                    ctrl->breakdown = brk;
                    ctrl->inv_h = s_scale;
                }
            }
        }
    } else if (threadIdx.x == 0) {
        s_jd = ctrl->j_done;
        s_brk = ctrl->breakdown;
        s_scale = ctrl->inv_h;
    }
    __syncthreads();
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i >= n) return;
    const double* wl = ((s_jd - 1) & 1) ? w1 : w0;
    basis[(size_t)(vbase + s_jd) * ld + i] = (BT)(s_brk ? 0.0 : wl[i] * s_scale);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void k_close_basis(const double* __restrict__ w0, const double* __restrict__ w1,
                                                      BT* __restrict__ basis, int n, int ld, int kc, int vbase,
                                                      int s_cycle, int npn, const double* __restrict__ part_n,
                                                      const double* __restrict__ red1, const double* __restrict__ red2,
                                                      double* H, double* Bm, Ctrl* ctrl) {
    k_close_basis_body<BT>(w0, w1, basis, n, ld, kc, vbase, s_cycle, npn, part_n, red1, red2, H, Bm, ctrl);
}


// ---------------------------------------------------------------------------------------------
// Tall-skinny Gram products out = L^T R over all rows (L, R: lists of columns), used for
// [C V]^T U, C^T r, U^T U at a cycle end and for the start-up CholQR.
// ---------------------------------------------------------------------------------------------
constexpr int GCHUNK = 32;               // rows staged per LDS chunk
constexpr int GL_MAX = 2 * KMAX + MMAX + 2;   // max columns on the left
constexpr int GR_MAX = KMAX + 1;              // max columns on the right

template <typename T>
__device__ __forceinline__ const T* col_of(const ColList& L, int a, int ld) {
    int base = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (a < base + L.cnt[s]) return (const T*)L.seg[s] + (size_t)(a - base) * ld;
        base += L.cnt[s];
    }
    return nullptr;
}

// Block partial of L^T R over rows [r0, r1) on the FP64 matrix cores. The output is cut into 16 x 16
// tiles (TA x TB); each wave takes a quarter of the block's rows and accumulates every tile with
// v_mfma_f64_16x16x4f64, four rows per instruction, so each loaded operand feeds TB (A) or TA (B)
// instructions. Operand layout of that instruction: lane l holds A[l % 16][l / 16] (here
// L[row + l / 16][16 ta + l % 16]) and B[l / 16][l % 16] (R[row + l / 16][16 tb + l % 16]); item t of the
// result holds D[4 t + l / 16][l % 16]. Operands of four row steps are loaded while the previous four
// are multiplied; rows past the block end are zeroed in A. The four waves' tiles are added in LDS
// in a fixed order at the end.
typedef double skr_d4 __attribute__((ext_vector_type(4)));
template <int TA, int TB, typename LT, typename RT>
__device__ __forceinline__ void k_gram_partial_body(ColList L, int nl, ColList R, int nr, int n, int ld,
                                                       int rows_per_block, double* __restrict__ gpart) {
    constexpr int NT = TA * TB, KS = NT > 12 ? 2 : 4;   // row steps (of 4 rows) per operand batch
    __shared__ double red[(NWAVE - 1) * NT * 4 * 64];
    const int w = wave_id(), l = lane_id();
    const int rsub = l >> 4, csub = l & 15;
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    const int per = (rows_per_block / NWAVE + 3) / 4 * 4;
    const int w0 = r0 + w * per, w1 = min(r1, w0 + per);
    const LT* lp[TA];
    const RT* rp[TB];
#pragma unroll
    for (int ta = 0; ta < TA; ++ta) lp[ta] = col_of<LT>(L, min(16 * ta + csub, nl - 1), ld);
#pragma unroll
    for (int tb = 0; tb < TB; ++tb) rp[tb] = col_of<RT>(R, min(16 * tb + csub, nr - 1), ld);
    skr_d4 acc[TA][TB];
#pragma unroll
    for (int ta = 0; ta < TA; ++ta)
#pragma unroll
        for (int tb = 0; tb < TB; ++tb) acc[ta][tb] = skr_d4{0.0, 0.0, 0.0, 0.0};
    double av[KS][TA], bv[KS][TB];
    auto fetch = [&](int row0) {
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int row = row0 + 4 * u + rsub;
            const int rc = min(row, r1 - 1);
#pragma unroll
            for (int ta = 0; ta < TA; ++ta) av[u][ta] = (double)lp[ta][rc];
#pragma unroll
            for (int tb = 0; tb < TB; ++tb) bv[u][tb] = (double)rp[tb][rc];
        }
    };
    if (w0 < w1) fetch(w0);
    for (int row0 = w0; row0 < w1; row0 += 4 * KS) {
        double ac[KS][TA], bc[KS][TB];
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const bool rok = row0 + 4 * u + rsub < w1;
#pragma unroll
            for (int ta = 0; ta < TA; ++ta) ac[u][ta] = rok ? av[u][ta] : 0.0;
#pragma unroll
            for (int tb = 0; tb < TB; ++tb) bc[u][tb] = bv[u][tb];
        }
        if (row0 + 4 * KS < w1) fetch(row0 + 4 * KS);
#pragma unroll
        for (int u = 0; u < KS; ++u)
#pragma unroll
            for (int ta = 0; ta < TA; ++ta)
#pragma unroll
                for (int tb = 0; tb < TB; ++tb)
                    acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u][ta], bc[u][tb], acc[ta][tb], 0, 0, 0);
    }
    // waves 1..3 hand their tiles to wave 0, which adds them in wave order and stores the partial
    if (w > 0) {
#pragma unroll
        for (int ta = 0; ta < TA; ++ta)
#pragma unroll
            for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                for (int i2 = 0; i2 < 4; ++i2) red[(((w - 1) * NT + ta * TB + tb) * 4 + i2) * 64 + l] = acc[ta][tb][i2];
    }
    __syncthreads();
    if (w == 0) {
        const int E = nl * nr;
#pragma unroll
        for (int ta = 0; ta < TA; ++ta)
#pragma unroll
            for (int tb = 0; tb < TB; ++tb)
#pragma unroll
                for (int i2 = 0; i2 < 4; ++i2) {
                    double v = acc[ta][tb][i2];
#pragma unroll
                    for (int q = 1; q < NWAVE; ++q) v += red[(((q - 1) * NT + ta * TB + tb) * 4 + i2) * 64 + l];
                    const int a = 16 * ta + 4 * i2 + rsub, b = 16 * tb + csub;
                    if (a < nl && b < nr) gpart[(size_t)blockIdx.x * E + a * nr + b] = v;
                }
    }
}
template <int TA, int TB, typename LT, typename RT>
__global__ __launch_bounds__(ROWS) void k_gram_partial(ColList L, int nl, ColList R, int nr, int n, int ld,
                                                       int rows_per_block, double* __restrict__ gpart) {
    k_gram_partial_body<TA, TB, LT, RT>(L, nl, R, nr, n, ld, rows_per_block, gpart);
}


// out[(e / nr) * ostride + e % nr] = sum_b gpart[b][e]: one workgroup per 64 outputs; wave w sums a
// contiguous quarter of the partials (loads issued 16 at a time), then the quarters are added in
// order.
__device__ __forceinline__ void k_gram_reduce_body(const double* __restrict__ gpart, int nb, int E, int nr,
                                                      int ostride, double* __restrict__ out) {
    __shared__ double sh[NWAVE * 64];
    const int lane = lane_id(), w = wave_id();
    const int e = blockIdx.x * 64 + lane;
    const int per = (nb + NWAVE - 1) / NWAVE;
    const int b0 = w * per, b1 = min(nb, b0 + per);
    double s = 0.0;
    if (e < E) {
        int b = b0;
        for (; b + 16 <= b1; b += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = gpart[(size_t)(b + u) * E + e];
#pragma unroll
            for (int u = 0; u < 16; ++u) s += v[u];
        }
        for (; b < b1; ++b) s += gpart[(size_t)b * E + e];
    }
    sh[w * 64 + lane] = s;
    __syncthreads();
    if (w == 0 && e < E) {
        double t = sh[lane];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q) t += sh[q * 64 + lane];
        out[(e / nr) * ostride + e % nr] = t;
    }
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_gram_reduce(const double* __restrict__ gpart, int nb, int E, int nr,
                                                      int ostride, double* __restrict__ out) {
    k_gram_reduce_body(gpart, nb, E, nr, ostride, out);
}
#endif


// ---------------------------------------------------------------------------------------------
// Cycle end (Alg. 2): x += V-hat y, r -= W-hat G y, C <- W-hat Qc, U <- V-hat P_k R^{-1} (all
// row-wise and in place), as one tall-skinny product [C, U, V] W with W held in LDS: row q of W
// maps input column q to the outputs (C_new[0..KB), U_new[0..KB), dx, dr). KB is the bucket of
// the new recycle size (0, 8, 16, 24 or 32). The partials of ||r_new||^2 are left for the next
// cycle's first pass A.
// ---------------------------------------------------------------------------------------------
// Cycle update in one pass over the basis rows: [C_new | U_new | dx | dr] = [C U V] W, then
// x += dx, r += dr (W carries the signs), the new C and U overwrite the old, and the partials of
// ||r||^2 are written for the next cycle. W (ncl x NO, row q = input column q, zero-padded to
// KP x NP) is gathered into LDS: every entry is one load from the flat coefficient block at an
// index chosen by integer selects, so no load sits inside a divergent branch. The product runs on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64): each wave owns 64 rows (four 16-row tiles) and steps
// over the input columns four at a time; lane l supplies A[l % 16][l / 16] = X[row + l % 16][q + l / 16]
// (16 consecutive rows of one column per 16 lanes) and B[l / 16][l % 16] = W[q + l / 16][o + l % 16],
// and result item t of lane l is output o + l % 16 of row 4 t + l / 16 of the tile. The next four
// column steps load while the current four multiply.
typedef double skr_d4u __attribute__((ext_vector_type(4)));
template <int KB, typename BT>
__device__ __forceinline__ void k_cycle_update_body(double* __restrict__ x, double* __restrict__ r,
                                                       BT* __restrict__ basis, BT* __restrict__ U,
                                                       int n, int ld, int vbase, int kc, int nblk, const Coef* coef,
                                                       double* part_n, Ctrl* ctrl) {
    constexpr int NO = 2 * KB + 2;
    constexpr int NTN = (NO + 15) / 16, NP = 16 * NTN;        // output tiles, padded outputs
    // input columns 2 kc + jd + 1 with jd <= m - kc: at most KMAX + MMAX + 1
    constexpr int MAXQ = KMAX + MMAX + 1, KP = (MAXQ + 3) / 4 * 4;
    constexpr int OQC = offsetof(Coef, Qc) / sizeof(double), OQU = offsetof(Coef, Qu) / sizeof(double);
    constexpr int OYU = offsetof(Coef, yU) / sizeof(double), OYV = offsetof(Coef, yV) / sizeof(double);
    constexpr int ORC = offsetof(Coef, rC) / sizeof(double), ORV = offsetof(Coef, rV) / sizeof(double);
    constexpr int RT = ROWS / NWAVE / 16;                     // 16-row tiles per wave
    constexpr int KSB = 4;                                    // column steps per operand batch
    __shared__ double Wc[KP * NP];
    __shared__ double sh[NWAVE * NC];
    const int jd = ctrl->j_done, brk = ctrl->breakdown, kn = ctrl->k_new;
    const int nv = jd + (brk ? 0 : 1);     // V columns of W-hat (v_{jd} is zero after a breakdown)
    const int ncl = 2 * kc + nv;           // input columns: C (kc), U (kc), V (nv)
    const int nks = (ncl + 3) / 4;         // column steps
    const int w = wave_id(), l = lane_id();
    const int lrow = l & 15, lk = l >> 4;
    const int lb = logical_block(blockIdx.x, nblk);
    const int wrow0 = lb * ROWS + w * 16 * RT;               // first row of this wave
    auto colp = [&](int q) {
        return q < kc ? basis + (size_t)q * ld
                      : (q < 2 * kc ? U + (size_t)(q - kc) * ld : basis + (size_t)(vbase + q - 2 * kc) * ld);
    };
    // The first operand batch, and x or r at the rows of the lanes that update them (outputs 2 KB and
    // 2 KB + 1), are loaded before W is gathered, so that their latency overlaps the gather's.
    double av[KSB][RT];
    auto fetch = [&](int ks0) {
#pragma unroll
        for (int u = 0; u < KSB; ++u) {
            const BT* cp = colp(min(4 * (ks0 + u) + lk, ncl - 1));
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) av[u][rt] = (double)cp[min(wrow0 + 16 * rt + lrow, n - 1)];
        }
    };
    fetch(0);
    const bool ownx = lrow == (2 * KB) % 16, ownr = lrow == (2 * KB + 1) % 16;
    double xr0[RT][4];
    if (ownx || ownr) {
        const double* src = ownx ? x : r;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) xr0[rt][t2] = src[min(wrow0 + 16 * rt + 4 * t2 + lk, n - 1)];
    }
    const double* cf = reinterpret_cast<const double*>(coef);
    for (int e0 = 0; e0 < nks * 4 * NP; e0 += 8 * ROWS) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * ROWS + threadIdx.x;
            const int q = e / NP, o = e - q * NP;
            const bool inC = q < kc, inU = !inC && q < 2 * kc;
            const int c = q - kc, t = q - 2 * kc;
            const bool oC = o < KB, oU = o >= KB && o < 2 * KB, oX = o == 2 * KB, oR = o == 2 * KB + 1;
            int idx = 0;
            bool ok = false;
            double sg = 1.0;
            if (inC) {
                idx = oC ? OQC + q + o * LDQC : ORC + q;
                ok = (oC && o < kn) || oR;
                sg = oR ? -1.0 : 1.0;
            } else if (inU) {
                idx = oU ? OQU + c + (o - KB) * LDQU : OYU + c;
                ok = (oU && (o - KB) < kn) || oX;
            } else {
                idx = oC ? OQC + kc + t + o * LDQC
                         : (oU ? OQU + kc + t + (o - KB) * LDQU : (oX ? OYV + t : ORV + t));
                ok = (oC && o < kn) || (oU && t < jd && (o - KB) < kn) || (oX && t < jd) || oR;
                sg = oR ? -1.0 : 1.0;
            }
            ok = ok && q < ncl;
            const double ld_ = cf[ok ? idx : 0];
            v[u] = ok ? sg * ld_ : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * ROWS + threadIdx.x;
            if (e < nks * 4 * NP) Wc[e] = v[u];
        }
    }
    __syncthreads();
    skr_d4u acc[RT][NTN];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt) acc[rt][nt] = skr_d4u{0.0, 0.0, 0.0, 0.0};
    for (int ks0 = 0; ks0 < nks; ks0 += KSB) {
        double ac[KSB][RT];
#pragma unroll
        for (int u = 0; u < KSB; ++u)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) ac[u][rt] = av[u][rt];
        if (ks0 + KSB < nks) fetch(ks0 + KSB);
#pragma unroll
        for (int u = 0; u < KSB; ++u) {
            if (ks0 + u < nks) {
                const int q = 4 * (ks0 + u) + lk;
                double bv[NTN];
#pragma unroll
                for (int nt = 0; nt < NTN; ++nt) bv[nt] = Wc[q * NP + 16 * nt + lrow];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int nt = 0; nt < NTN; ++nt)
                        acc[rt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u][rt], bv[nt], acc[rt][nt], 0, 0, 0);
            }
        }
    }
    // results: item t of lane l is output o = 16 nt + (l % 16) of row wrow0 + 16 rt + 4 t + l / 16
    double rn2 = 0.0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt) {
            const int o = 16 * nt + lrow;
#pragma unroll
            for (int t2 = 0; t2 < 4; ++t2) {
                const int row = wrow0 + 16 * rt + 4 * t2 + lk;
                if (row < n) {
                    const double val = acc[rt][nt][t2];
                    if (o < KB) {
                        if (o < kn) basis[(size_t)o * ld + row] = (BT)val;
                    } else if (o < 2 * KB) {
                        if (o - KB < kn) U[(size_t)(o - KB) * ld + row] = (BT)val;
                    } else if (o == 2 * KB) {
                        x[row] = xr0[rt][t2] + val;
                    } else if (o == 2 * KB + 1) {
                        const double rn = xr0[rt][t2] + val;
                        r[row] = rn;
                        rn2 = fma(rn, rn, rn2);
                    }
                }
            }
        }
    // partials of ||r||^2: the first pass A of the next cycle forms beta from them
    block_partial1(rn2, part_n, lb, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->stop = 0;
}
// spec_kc >= 0: the host launches the next cycle's opening for spec_kc recycled columns before it
// reads this cycle end; spec_skip tells those kernels whether the next cycle starts as assumed (the
// same test the host applies to the values it reads: a finite estimate above the tolerance, no
// breakdown, k_new == spec_kc).
template <int KB, typename BT>
__global__ __launch_bounds__(ROWS) void k_cycle_update(double* __restrict__ x, double* __restrict__ r,
                                                       BT* __restrict__ basis, BT* __restrict__ U,
                                                       int n, int ld, int vbase, int kc, int nblk, const Coef* coef,
                                                       double* part_n, Ctrl* ctrl, int spec_kc) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double est = ctrl->est;
        const bool go = spec_kc >= 0 && ctrl->k_new == spec_kc && !ctrl->breakdown && isfinite(est) &&
                        est > ctrl->tol_abs;
        ctrl->spec_skip = go ? 0 : 1;
    }
    k_cycle_update_body<KB, BT>(x, r, basis, U, n, ld, vbase, kc, nblk, coef, part_n, ctrl);
}


// ---------------------------------------------------------------------------------------------
// True residual r = b - A x (overwrites r) and the partials of ||r||^2 (closed by k_norm_finish).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void k_true_residual_body(DevOp op, const double* __restrict__ b,
                                                        const double* __restrict__ x, double* __restrict__ r,
                                                        int nblk, double* part_n) {
    __shared__ double sh[NWAVE];
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double v = 0.0;
    if (i < op.n) {
        const double ri = b[i] - op_row(op, x, i, 1.0);
        r[i] = ri;
        v = ri * ri;
    }
    block_partial1(v, part_n, lb, sh);
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_true_residual(DevOp op, const double* __restrict__ b,
                                                        const double* __restrict__ x, double* __restrict__ r,
                                                        int nblk, double* part_n, const int* __restrict__ gate) {
    if (gate && *gate) return;
    k_true_residual_body(op, b, x, r, nblk, part_n);
}
#endif


// ---------------------------------------------------------------------------------------------
// Start-up with a carried recycle space (App. B.1): Z = A Y, CholQR2 of Z with column drops,
// C = Q, U = Y R^{-1}, x1 = U C^T r0, r1 = r0 - C C^T r0. The same projection starts every
// refinement step of the mixed-precision mode (x += U C^T r, r -= C C^T r).
// ---------------------------------------------------------------------------------------------
template <typename BT>
__device__ __forceinline__ void k_spmm_body(DevOp op, const BT* __restrict__ Y, BT* __restrict__ Z,
                                               int ld, int kin) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i >= op.n) return;
    for (int c = 0; c < kin; ++c)
        Z[(size_t)c * ld + i] = (BT)op_row_k<-1, BT, false, sizeof(BT) == 4>(op, Y + (size_t)c * ld, i, 1.0);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void k_spmm(DevOp op, const BT* __restrict__ Y, BT* __restrict__ Z,
                                               int ld, int kin) {
    k_spmm_body<BT>(op, Y, Z, ld, kin);
}


// FP32 copy of an operator array (round to nearest even): the mixed mode's inner operator.
__device__ __forceinline__ void k_to_f32_body(const double* __restrict__ src, float* __restrict__ dst, long count) {
    for (long e = blockIdx.x * (long)ROWS + threadIdx.x; e < count; e += (long)gridDim.x * ROWS) dst[e] = (float)src[e];
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, long count) {
    k_to_f32_body(src, dst, count);
}
#endif


// Z = A C for the kc <= KB recycled columns C = basis columns 0..kc-1 (FP64), the product the merged
// Arnoldi kernel takes A C from. Z is stored in FP32: the kernel only multiplies it by second-pass
// Gram-Schmidt coefficients, which are of the order of the rounding of the first pass, so its
// relative rounding 2^-24 changes that term far below FP64 rounding. One row per thread; the
// operator row (CSR entries or stencil faces) is loaded once and applied to every column, each
// column's terms added in the order of op_row_k.
template <int KIND, int KB>
__device__ __forceinline__ void k_apply_c_body(DevOp op, const double* __restrict__ C, float* __restrict__ Z,
                                                  int ld, int kc, int nblk) {
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    if (i >= op.n) return;
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    if constexpr (KIND == SKR_OP_CSR) {
        const int e0 = op.rowptr[i], e1 = op.rowptr[i + 1];
        for (int e = e0; e < e1; e += 8) {
            int cl[8];
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = min(e + u, e1 - 1);
                cl[u] = op.colind[q];
                v[u] = op.val[q];
            }
#pragma unroll
            for (int c = 0; c < KB; ++c) {
                if (c < kc) {
                    double xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) xv[u] = C[(size_t)c * ld + cl[u]];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (e + u < e1) acc[c] = fma(v[u], xv[u], acc[c]);
                }
            }
        }
    } else if constexpr (KIND == SKR_OP_STENCIL7) {
        const int nx = op.nx, ny = op.ny, nz = op.nz, nxy = nx * ny;
        const int gz = i / nxy, gyx = i - gz * nxy, gy = gyx / nx, gx = gyx - gy * nx;
        const int fx = (gz * ny + gy) * (nx + 1) + gx, fy = (gz * (ny + 1) + gy) * nx + gx, fz = gz * nxy + gyx;
        const double aw = op.ax[fx], ae = op.ax[fx + 1];
        const double as = op.ay[fy], an = op.ay[fy + nx];
        const double ad = op.az[fz], au = op.az[fz + nxy];
        const bool hw = gx > 0, he = gx < nx - 1, hs = gy > 0, hn = gy < ny - 1, hd = gz > 0, hu = gz < nz - 1;
        const double dg = (aw + ae) + (as + an) + (ad + au);
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < kc) {
                const double* x = C + (size_t)c * ld;
                const double xc = x[i];
                const double xw = x[hw ? i - 1 : i], xe = x[he ? i + 1 : i];
                const double xs = x[hs ? i - nx : i], xn = x[hn ? i + nx : i];
                const double xd = x[hd ? i - nxy : i], xu = x[hu ? i + nxy : i];
                double t = dg * xc;
                t = hw ? fma(-aw, xw, t) : t;
                t = he ? fma(-ae, xe, t) : t;
                t = hs ? fma(-as, xs, t) : t;
                t = hn ? fma(-an, xn, t) : t;
                t = hd ? fma(-ad, xd, t) : t;
                t = hu ? fma(-au, xu, t) : t;
                acc[c] = t * op.inv_h2;
            }
        }
    } else {
        const int nx = op.nx, ny = op.ny;
        const int r = i / nx, cc = i - r * nx;
        const double aw = op.ax[r * (nx + 1) + cc], ae = op.ax[r * (nx + 1) + cc + 1];
        const double an = op.ay[r * nx + cc], as = op.ay[(r + 1) * nx + cc];
        const bool hw = cc > 0, he = cc < nx - 1, hn = r > 0, hs = r < ny - 1;
        const double dg = aw + ae + an + as;
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < kc) {
                const double* x = C + (size_t)c * ld;
                const double xc = x[i];
                const double xw = x[hw ? i - 1 : i], xe = x[he ? i + 1 : i];
                const double xn = x[hn ? i - nx : i], xs = x[hs ? i + nx : i];
                double t = dg * xc;
                t = hw ? fma(-aw, xw, t) : t;
                t = he ? fma(-ae, xe, t) : t;
                t = hn ? fma(-an, xn, t) : t;
                t = hs ? fma(-as, xs, t) : t;
                acc[c] = t * op.inv_h2;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < KB; ++c)
        if (c < kc) Z[(size_t)c * ld + i] = (float)acc[c];
}
template <int KIND, int KB>
__global__ __launch_bounds__(ROWS) void k_apply_c(DevOp op, const double* __restrict__ C, float* __restrict__ Z,
                                                  int ld, int kc, int nblk) {
    k_apply_c_body<KIND, KB>(op, C, Z, ld, kc, nblk);
}


// Row-wise triangular solves z <- z R^{-1} (R upper, k x k, ld KMAX) on Z (kept columns gathered
// through keep[]) and on U, compacting both to the first k_eff columns.
template <typename BT>
__device__ __forceinline__ void k_startup_apply_body(BT* __restrict__ Z, BT* __restrict__ U, int n,
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
        z[c] = c < ke ? (double)Z[(size_t)ks[c] * ld + i] : 0.0;
        u[c] = c < ke ? (double)U[(size_t)ks[c] * ld + i] : 0.0;
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
            Z[(size_t)c * ld + i] = (BT)z[c];
            U[(size_t)c * ld + i] = (BT)u[c];
        }
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void k_startup_apply(BT* __restrict__ Z, BT* __restrict__ U, int n,
                                                        int ld, const Coef* coef, int use_keep, int second) {
    k_startup_apply_body<BT>(Z, U, n, ld, coef, use_keep, second);
}


// x = x0 + U c, r -= C c with c = C^T r (ke entries, from a Gram product), and the partials of
// ||r||^2 (closed by k_norm_finish). x0 = 0 at a system start, the current iterate at a refinement
// step. The columns are taken eight at a time, every load of a group in flight together at clamped
// column indices (a coefficient of zero past ke), products added in column order.
template <typename BT>
__device__ __forceinline__ void k_startup_project_body(double* __restrict__ x, double* __restrict__ r,
                                                          const BT* __restrict__ C, const BT* __restrict__ U,
                                                          int n, int ld, int nblk, int ke, int add_x,
                                                          const double* __restrict__ cvec, double* part_n) {
    __shared__ double sh[NWAVE];
    __shared__ double cs[KMAX];
    if (threadIdx.x < KMAX) cs[threadIdx.x] = (int)threadIdx.x < ke ? cvec[threadIdx.x] : 0.0;
    __syncthreads();
    const int lb = logical_block(blockIdx.x, nblk);
    const int i = lb * ROWS + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        double xi = add_x ? x[i] : 0.0, ri = r[i];
        for (int c0 = 0; c0 < ke; c0 += 8) {
            double uc[8], cc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const size_t off = (size_t)min(c0 + u, ke - 1) * ld + i;
                uc[u] = (double)U[off];
                cc[u] = (double)C[off];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double cu = (c0 + u < KMAX) ? cs[min(c0 + u, KMAX - 1)] : 0.0;
                xi = fma(uc[u], cu, xi);
                ri = fma(-cc[u], cu, ri);
            }
        }
        x[i] = xi;
        r[i] = ri;
        v = ri * ri;
    }
    block_partial1(v, part_n, lb, sh);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void k_startup_project(double* __restrict__ x, double* __restrict__ r,
                                                          const BT* __restrict__ C, const BT* __restrict__ U,
                                                          int n, int ld, int nblk, int ke, int add_x,
                                                          const double* __restrict__ cvec, double* part_n,
                                                          const int* __restrict__ gate) {
    if (gate && *gate) return;
    k_startup_project_body<BT>(x, r, C, U, n, ld, nblk, ke, add_x, cvec, part_n);
}


// ---------------------------------------------------------------------------------------------
// Plain y = A x (the sparse product alone, for the SpMV entry point).
// ---------------------------------------------------------------------------------------------
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_spmv(DevOp op, const double* __restrict__ x, double* __restrict__ y) {
    const int i = blockIdx.x * ROWS + threadIdx.x;
    if (i < op.n) y[i] = op_row(op, x, i, 1.0);
}
#endif

// ---------------------------------------------------------------------------------------------
// Partial folding for large grids. Every workgroup of a step kernel re-sums the partials of the
// kernel before it; with many workgroups that costs O(nblk^2) reads. Above FOLD_MIN workgroups
// (or on request) a fold kernel first sums the nblk partial rows into NFOLD rows: workgroup g adds
// rows [g per, (g + 1) per) in a fixed order (lane = column, the four waves take contiguous quarters,
// added in wave order), and the consumer re-sums the NFOLD rows.
// ---------------------------------------------------------------------------------------------
// Columns [0, width) (width <= NC), 64 per pass.
__device__ __forceinline__ void k_fold_body(const double* __restrict__ part, int nblk, int width,
                                               double* __restrict__ out) {
    __shared__ double sh[NWAVE * 64];
    const int lane = lane_id(), w = wave_id();
    const int per = (nblk + NFOLD - 1) / NFOLD;
    const int g0 = blockIdx.x * per, g1 = min(nblk, g0 + per);
    const int q = (per + NWAVE - 1) / NWAVE;
    const int b0 = min(g1, g0 + w * q), b1 = min(g1, b0 + q);
    for (int c0 = 0; c0 < width; c0 += 64) {
        const int col = c0 + lane;
        double s = 0.0;
        if (col < width) {
            for (int b = b0; b < b1; b += 16) {
                double v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = part[(size_t)min(b + u, b1 - 1) * NC + col];
#pragma unroll
                for (int u = 0; u < 16; ++u) s += (b + u < b1) ? v[u] : 0.0;
            }
        }
        sh[w * 64 + lane] = s;
        __syncthreads();
        if (threadIdx.x < 64 && col < width) {
            double t = sh[threadIdx.x];
#pragma unroll
            for (int q2 = 1; q2 < NWAVE; ++q2) t += sh[q2 * 64 + threadIdx.x];
            out[blockIdx.x * NC + col] = t;
        }
        __syncthreads();
    }
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_fold(const double* __restrict__ part, int nblk, int width,
                                               double* __restrict__ out) {
    k_fold_body(part, nblk, width, out);
}
#endif

__device__ __forceinline__ void k_fold1_body(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    __shared__ double sh[NWAVE];
    const int per = (nblk + NFOLD - 1) / NFOLD;
    const int g0 = blockIdx.x * per, g1 = min(nblk, g0 + per);
    double s = 0.0;
    for (int b = g0 + (int)threadIdx.x; b < g1; b += ROWS) s += part[b];
    const double ws = wave_sum(s);
    if (lane_id() == 0) sh[wave_id()] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
#pragma unroll
        for (int q2 = 1; q2 < NWAVE; ++q2) t += sh[q2];
        out[blockIdx.x] = t;
    }
}
#ifndef SKR_CHAINS_UNIT
__global__ __launch_bounds__(ROWS) void k_fold1(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    k_fold1_body(part, nblk, out);
}
#endif

// Host helpers of both launcher sets.
static inline int blocks_for(long n) { return (int)((n + ROWS - 1) / ROWS); }
static inline int bucket8(int c) { return c <= 8 ? 8 : ((c + 7) / 8) * 8; }
#define SKR_DISPATCH8(NLV, CALL)                        \
    switch (NLV) {                                      \
        case 8: CALL(8); break;                         \
        case 16: CALL(16); break;                       \
        case 24: CALL(24); break;                       \
        case 32: CALL(32); break;                       \
        case 40: CALL(40); break;                       \
        case 48: CALL(48); break;                       \
        case 56: CALL(56); break;                       \
        case 64: CALL(64); break;                       \
        case 72: CALL(72); break;                       \
        case 80: CALL(80); break;                       \
        default: CALL(88); break;                       \
    }

// This file is compiled twice. Without SKR_CHAINS_UNIT it gives the single-chain kernels and their
// launchers; with it, the batched kernels of skr_solve_chains (one grid row per chain) and theirs.
// Both wrap the same device bodies above, so the arithmetic of a chain is the same either way.
#ifndef SKR_CHAINS_UNIT
// ---------------------------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------------------------
static inline const double* pn_src(const Work& w) { return w.fold ? w.fold_n : w.part_n; }
static inline int pn_cnt(const Work& w) { return w.fold ? NFOLD : w.nblk; }
void launch_fold_n(hipStream_t s, const Work& w) {
    if (w.fold) hipLaunchKernelGGL(k_fold1, dim3(NFOLD), dim3(ROWS), 0, s, (const double*)w.part_n, w.nblk, w.fold_n);
}

static void launch_norm_finish(hipStream_t s, const Work& w, int mode, double rtol, int ke,
                               const int* gate = nullptr) {
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(ROWS), 0, s, pn_src(w), pn_cnt(w), mode, rtol, ke, w.ctrl, gate);
}
const int* spec_gate(const Work& w) {
    return reinterpret_cast<const int*>(reinterpret_cast<const char*>(w.ctrl) + offsetof(Ctrl, spec_skip));
}
void launch_init(hipStream_t s, const Work& w, const double* b, double* x, double rtol) {
    hipLaunchKernelGGL(k_init, dim3(w.nblk), dim3(ROWS), 0, s, b, x, w.r, w.n, w.nblk, w.part_n);
    launch_fold_n(s, w);
    launch_norm_finish(s, w, FIN_INIT, rtol, 0);
}
void launch_clear_nonfinite(hipStream_t s, const Work& w) {
    hipLaunchKernelGGL(k_clear_nonfinite, dim3(1), dim3(1), 0, s, w.ctrl);
}
void launch_check_sym(hipStream_t s, const Work& w, const DevOp& op) {
    if (op.kind == SKR_OP_CSR)
        hipLaunchKernelGGL(k_check_sym_csr, dim3(blocks_for(op.n)), dim3(ROWS), 0, s, op, w.ctrl);
}
void launch_to_f32(hipStream_t s, const double* src, float* dst, long count) {
    if (count <= 0) return;
    const int g = (int)std::min<long>(2048, (count + ROWS - 1) / ROWS);
    hipLaunchKernelGGL(k_to_f32, dim3(g), dim3(ROWS), 0, s, src, dst, count);
}
void launch_check_finite(hipStream_t s, const Work& w, const double* v, long count) {
    if (count <= 0) return;
    const int g = (int)std::min<long>(1024, (count + ROWS - 1) / ROWS);
    hipLaunchKernelGGL(k_check_finite, dim3(g), dim3(ROWS), 0, s, v, count, w.ctrl);
}
void launch_zero(hipStream_t s, double* x, int n) {
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n)), dim3(ROWS), 0, s, x, n);
}
template <typename BT>
static inline BT* bas(const Work& w) { return reinterpret_cast<BT*>(w.basis); }
template <typename BT>
static inline BT* ucols(const Work& w) { return reinterpret_cast<BT*>(w.U); }

// With e0/e1 non-null the launch goes through hipExtLaunchKernelGGL, whose events take the start
// and end timestamps of the kernel's own dispatch (no marker packets around it).
template <int NL, int KIND, typename BT>
static void step_a_k(hipStream_t s, const Work& w, const DevOp& op, const double* src, double* dst, int kc, int j,
                     hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL((k_step_a<NL, KIND, BT>), dim3(w.nblk), dim3(ROWS), 0, s, e0, e1, 0, op, src, dst,
                          bas<BT>(w), w.ld, kc, w.k, j, w.nblk, pn_cnt(w), pn_src(w), w.part_a,
                          (const double*)w.red1, (const double*)w.red2, w.H, w.Bm, w.ctrl);
}
template <int NL, typename BT>
static void step_a(hipStream_t s, const Work& w, const DevOp& op, const double* src, double* dst, int kc, int j,
                   hipEvent_t e0, hipEvent_t e1) {
    if (op.kind == SKR_OP_CSR)
        step_a_k<NL, SKR_OP_CSR, BT>(s, w, op, src, dst, kc, j, e0, e1);
    else if (op.kind == SKR_OP_STENCIL7)
        step_a_k<NL, SKR_OP_STENCIL7, BT>(s, w, op, src, dst, kc, j, e0, e1);
    else
        step_a_k<NL, SKR_OP_STENCIL5, BT>(s, w, op, src, dst, kc, j, e0, e1);
}
// Passes B and C re-sum NFOLD folded partial rows (w.fold) or one row per workgroup.
template <int NL, typename BT, bool NORM = false>
static void step_b(hipStream_t s, const Work& w, double* dst, int kc, int j, hipEvent_t e0, hipEvent_t e1) {
    if (w.fold)
        hipExtLaunchKernelGGL((k_step_b<NL, BT, true, NORM>), dim3(w.nblk), dim3(ROWS), 0, s, e0, e1, 0, dst,
                              (const BT*)bas<BT>(w), w.n, w.ld, kc, w.k, j, w.nblk, NFOLD, (const double*)w.fold_a,
                              w.part_b, w.red1, (const Ctrl*)w.ctrl);
    else
        hipExtLaunchKernelGGL((k_step_b<NL, BT, false, NORM>), dim3(w.nblk), dim3(ROWS), 0, s, e0, e1, 0, dst,
                              (const BT*)bas<BT>(w), w.n, w.ld, kc, w.k, j, w.nblk, w.nblk, (const double*)w.part_a,
                              w.part_b, w.red1, (const Ctrl*)w.ctrl);
}
// Merged kernel of step j (closes step j-1): reads pass B's partials (folded or not).
template <int NL, int KIND, int KZ, bool LAST>
static void step_m_k(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, hipEvent_t e0, hipEvent_t e1) {
    const double* wb = w.W[(j - 1) & 1];
    double* dst = w.W[j & 1];
    hipExtLaunchKernelGGL((k_step_m<NL, KIND, KZ, LAST>), dim3(w.nblk), dim3(ROWS), 0, s, e0, e1, 0, op, wb, dst,
                          bas<double>(w), (const float*)w.Z, w.ld, kc, w.k, j, w.nblk, w.fold ? NFOLD : w.nblk,
                          (const double*)(w.fold ? w.fold_b : w.part_b), w.part_a, (const double*)w.red1,
                          (const double*)(w.gcorr + ((j - 1) & 1) * NC), w.gcorr + (j & 1) * NC, w.H, w.Bm,
                          w.ctrl);
}
template <int NL, int KZ, bool LAST>
static void step_m_z(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, hipEvent_t e0, hipEvent_t e1) {
    if (op.kind == SKR_OP_CSR)
        step_m_k<NL, SKR_OP_CSR, KZ, LAST>(s, w, op, kc, j, e0, e1);
    else if (op.kind == SKR_OP_STENCIL7)
        step_m_k<NL, SKR_OP_STENCIL7, KZ, LAST>(s, w, op, kc, j, e0, e1);
    else
        step_m_k<NL, SKR_OP_STENCIL5, KZ, LAST>(s, w, op, kc, j, e0, e1);
}
template <int NL, bool LAST>
static void step_m(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, hipEvent_t e0, hipEvent_t e1) {
    // the closing form forms no product: one instance per NL
    if constexpr (LAST) step_m_k<NL, SKR_OP_CSR, 0, true>(s, w, op, kc, j, e0, e1);
    else if (kc == 0) step_m_z<NL, 0, LAST>(s, w, op, kc, j, e0, e1);
    else if (kc <= 8) step_m_z<NL, 8, LAST>(s, w, op, kc, j, e0, e1);
    else if (kc <= 16) step_m_z<NL, 16, LAST>(s, w, op, kc, j, e0, e1);
    else if (kc <= 24) step_m_z<NL, 24, LAST>(s, w, op, kc, j, e0, e1);
    else step_m_z<NL, 32, LAST>(s, w, op, kc, j, e0, e1);
}
template <int NL, typename BT>
static void step_c(hipStream_t s, const Work& w, double* dst, int kc, int j, hipEvent_t e0, hipEvent_t e1) {
    if (w.fold)
        hipExtLaunchKernelGGL((k_step_c<NL, BT, true>), dim3(w.nblk), dim3(ROWS), 0, s, e0, e1, 0, dst,
                              (const BT*)bas<BT>(w), w.n, w.ld, kc, w.k, j, w.nblk, NFOLD, (const double*)w.fold_b,
                              w.part_n, w.red2, (const Ctrl*)w.ctrl);
    else
        hipExtLaunchKernelGGL((k_step_c<NL, BT, false>), dim3(w.nblk), dim3(ROWS), 0, s, e0, e1, 0, dst,
                              (const BT*)bas<BT>(w), w.n, w.ld, kc, w.k, j, w.nblk, w.nblk, (const double*)w.part_b,
                              w.part_n, w.red2, (const Ctrl*)w.ctrl);
}


// One Arnoldi step (three kernels). With ev != nullptr, ev[2q], ev[2q+1] take the start and end of
// kernel q (A, B, C).
template <typename BT>
static void launch_step_t(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, hipEvent_t* ev) {
    const double* src = (j == 0) ? w.r : w.W[(j - 1) & 1];
    double* dst = w.W[j & 1];
    const int ncol = kc + j + 1;
    const int nla = bucket8(ncol + 1), nlb = bucket8(ncol);
    hipEvent_t e[6] = {};
    if (ev)
        for (int q = 0; q < 6; ++q) e[q] = ev[q];
#define CALL_A(NL) step_a<NL, BT>(s, w, op, src, dst, kc, j, e[0], e[1])
    SKR_DISPATCH8(nla, CALL_A)
#undef CALL_A
    if (w.fold) hipLaunchKernelGGL(k_fold, dim3(NFOLD), dim3(ROWS), 0, s, (const double*)w.part_a, w.nblk, ncol + 1, w.fold_a);
#define CALL_B(NL) step_b<NL, BT>(s, w, dst, kc, j, e[2], e[3])
    SKR_DISPATCH8(nlb, CALL_B)
#undef CALL_B
    if (w.fold) hipLaunchKernelGGL(k_fold, dim3(NFOLD), dim3(ROWS), 0, s, (const double*)w.part_b, w.nblk, ncol, w.fold_b);
#define CALL_C(NL) step_c<NL, BT>(s, w, dst, kc, j, e[4], e[5])
    SKR_DISPATCH8(nlb, CALL_C)
#undef CALL_C
    launch_fold_n(s, w);
}
// One Arnoldi step with an FP64 basis, two kernels: step 0 is pass A (from r) and pass B; a later
// step j is the merged kernel (pass C of step j-1 with pass A of step j) and pass B. Pass B leaves
// ||w_B||^2 beside Q^T w_B. With ev != nullptr, ev[0..1] time the first kernel and ev[2..3] pass B.
static void launch_step_2k(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, hipEvent_t* ev) {
    const int ncol = kc + j + 1;
    const int nla = bucket8(ncol + 1);
    hipEvent_t e[4] = {};
    if (ev)
        for (int q = 0; q < 4; ++q) e[q] = ev[q];
    if (j == 0) {
#define CALL_A(NL) step_a<NL, double>(s, w, op, w.r, w.W[0], kc, 0, e[0], e[1])
        SKR_DISPATCH8(nla, CALL_A)
#undef CALL_A
    } else {
#define CALL_M(NL) step_m<NL, false>(s, w, op, kc, j, e[0], e[1])
        SKR_DISPATCH8(nla, CALL_M)
#undef CALL_M
    }
    if (w.fold) hipLaunchKernelGGL(k_fold, dim3(NFOLD), dim3(ROWS), 0, s, (const double*)w.part_a, w.nblk, ncol + 1, w.fold_a);
#define CALL_B(NL) step_b<NL, double, true>(s, w, w.W[j & 1], kc, j, e[2], e[3])
    SKR_DISPATCH8(nla, CALL_B)
#undef CALL_B
    if (w.fold) hipLaunchKernelGGL(k_fold, dim3(NFOLD), dim3(ROWS), 0, s, (const double*)w.part_b, w.nblk, ncol + 1, w.fold_b);
}
void launch_step(hipStream_t s, const Work& w, const DevOp& op, int kc, int j, int s_cycle, hipEvent_t* ev) {
    (void)s_cycle;
    if (w.merged)
        launch_step_2k(s, w, op, kc, j, ev);
    else if (w.mixed)
        launch_step_t<float>(s, w, op, kc, j, ev);
    else
        launch_step_t<double>(s, w, op, kc, j, ev);
}
// Z = A C for the kc recycled columns (the merged Arnoldi kernel reads it).
void launch_apply_c(hipStream_t s, const Work& w, const DevOp& op, int kc) {
    if (!w.merged || kc <= 0) return;
#define SKR_AC(KIND, KB)                                                                                  \
    hipLaunchKernelGGL((k_apply_c<KIND, KB>), dim3(w.nblk), dim3(ROWS), 0, s, op, (const double*)w.basis, (float*)w.Z, \
                       w.ld, kc, w.nblk)
#define SKR_AC_K(KIND)                       \
    if (kc <= 8) SKR_AC(KIND, 8);            \
    else if (kc <= 16) SKR_AC(KIND, 16);     \
    else if (kc <= 24) SKR_AC(KIND, 24);     \
    else SKR_AC(KIND, 32);
    if (op.kind == SKR_OP_CSR) {
        SKR_AC_K(SKR_OP_CSR)
    } else if (op.kind == SKR_OP_STENCIL7) {
        SKR_AC_K(SKR_OP_STENCIL7)
    } else {
        SKR_AC_K(SKR_OP_STENCIL5)
    }
#undef SKR_AC_K
#undef SKR_AC
}
// Cycle end: closes the last step when the cycle did not stop early and stores the last basis
// vector v_{s_cycle}; with an FP64 basis this is the merged kernel in its closing form.
void launch_close_basis(hipStream_t s, const Work& w, const DevOp& op, int kc, int s_cycle) {
    if (w.merged) {
        const int nla = bucket8(kc + s_cycle + 2);
#define CALL_L(NL) step_m<NL, true>(s, w, op, kc, s_cycle, nullptr, nullptr)
        SKR_DISPATCH8(nla, CALL_L)
#undef CALL_L
        return;
    }
    else if (w.mixed)
        hipLaunchKernelGGL(k_close_basis<float>, dim3(w.nblk), dim3(ROWS), 0, s, (const double*)w.W[0],
                           (const double*)w.W[1], bas<float>(w), w.n, w.ld, kc, w.k, s_cycle, pn_cnt(w), pn_src(w),
                           (const double*)w.red1, (const double*)w.red2, w.H, w.Bm, w.ctrl);
    else
        hipLaunchKernelGGL(k_close_basis<double>, dim3(w.nblk), dim3(ROWS), 0, s, (const double*)w.W[0],
                           (const double*)w.W[1], bas<double>(w), w.n, w.ld, kc, w.k, s_cycle, pn_cnt(w), pn_src(w),
                           (const double*)w.red1, (const double*)w.red2, w.H, w.Bm, w.ctrl);
}
// out[a * ostride + b] = L_a^T R_b (a < nl, b < nr); LT, RT: element types of the two lists.
template <typename LT, typename RT>
static void launch_gram_t(hipStream_t s, const Work& w, const ColList& L, int nl, const ColList& R, int nr,
                          double* out, int ostride) {
    const int E = nl * nr;
    const int rpb = ((w.n + w.ngblk - 1) / w.ngblk + GCHUNK - 1) / GCHUNK * GCHUNK;
    const int nb = (w.n + rpb - 1) / rpb;
    const int la = nl <= 32 ? 2 : (nl <= 64 ? 4 : (nl <= 96 ? 6 : 8));
    const int lbk = nr <= 16 ? 1 : (nr <= 32 ? 2 : 3);
#define SKR_GP(LA, LB)                                                                                      \
    hipLaunchKernelGGL((k_gram_partial<LA, LB, LT, RT>), dim3(nb), dim3(ROWS), 0, s, L, nl, R, nr, w.n, w.ld, \
                       rpb, w.gpart)
#define SKR_GP_B(LA)                            \
    switch (lbk) {                              \
        case 1: SKR_GP(LA, 1); break;           \
        case 2: SKR_GP(LA, 2); break;           \
        default: SKR_GP(LA, 3); break;          \
    }
    switch (la) {
        case 2: SKR_GP_B(2); break;
        case 4: SKR_GP_B(4); break;
        case 6: SKR_GP_B(6); break;
        default: SKR_GP_B(8); break;
    }
#undef SKR_GP_B
#undef SKR_GP
    hipLaunchKernelGGL(k_gram_reduce, dim3((E + 63) / 64), dim3(ROWS), 0, s, (const double*)w.gpart, nb, E, nr,
                       ostride, out);
}
// Both lists in the basis storage type.
void launch_gram(hipStream_t s, const Work& w, const ColList& L, int nl, const ColList& R, int nr, double* out) {
    if (w.mixed)
        launch_gram_t<float, float>(s, w, L, nl, R, nr, out, nr);
    else
        launch_gram_t<double, double>(s, w, L, nl, R, nr, out, nr);
}
// Left list in the basis storage type, one FP64 right column (r): out[a * ostride] = L_a^T r.
static void launch_gram_r(hipStream_t s, const Work& w, const ColList& L, int nl, double* out, int ostride) {
    ColList R = {{w.r, nullptr, nullptr, nullptr}, {1, 0, 0, 0}};
    if (w.mixed)
        launch_gram_t<float, double>(s, w, L, nl, R, 1, out, ostride);
    else
        launch_gram_t<double, double>(s, w, L, nl, R, 1, out, ostride);
}
// Column offsets inside the basis buffer, in elements of the storage type.
static inline const void* bcol(const Work& w, int c) {
    return w.mixed ? (const void*)(bas<float>(w) + (size_t)c * w.ld) : (const void*)(bas<double>(w) + (size_t)c * w.ld);
}
void launch_cycle_gram(hipStream_t s, const Work& w, int kc, int jd_max) {
    // L = [C (kc), V_0..V_jd (jd+1), U (kc)], R = [U (kc), r]; jd is bounded on the host by the
    // cycle length, the columns past j_done only add products that nobody reads. In FP64 storage
    // this is one product; with an FP32 basis the FP64 column r is a product of its own.
    ColList L = {{bcol(w, 0), bcol(w, w.k), w.U, nullptr}, {kc, jd_max + 1, kc, 0}};
    const int nl = 2 * kc + jd_max + 1;
    if (!w.mixed) {
        ColList R = {{w.U, w.r, nullptr, nullptr}, {kc, 1, 0, 0}};
        launch_gram(s, w, L, nl, R, kc + 1, w.gram);
    } else {
        ColList R = {{w.U, nullptr, nullptr, nullptr}, {kc, 0, 0, 0}};
        launch_gram_t<float, float>(s, w, L, nl, R, kc, w.gram, kc + 1);
        launch_gram_r(s, w, L, nl, w.gram + kc, kc + 1);
    }
}
void launch_cycle_update(hipStream_t s, const Work& w, double* x, int kc, int k_bucket, int spec_kc) {
#define SKR_UPD(KB, BT)                                                                                      \
    hipLaunchKernelGGL((k_cycle_update<KB, BT>), dim3(w.nblk), dim3(ROWS), 0, s, x, w.r, bas<BT>(w), ucols<BT>(w), \
                       w.n, w.ld, w.k, kc, w.nblk, (const Coef*)w.coef, w.part_n, w.ctrl, spec_kc)
#define SKR_UPD_K(BT)                           \
    switch (k_bucket) {                         \
        case 0: SKR_UPD(0, BT); break;          \
        case 8: SKR_UPD(8, BT); break;          \
        case 16: SKR_UPD(16, BT); break;        \
        case 20: SKR_UPD(20, BT); break;        \
        case 24: SKR_UPD(24, BT); break;        \
        default: SKR_UPD(32, BT); break;        \
    }
    if (w.mixed) {
        SKR_UPD_K(float)
    } else {
        SKR_UPD_K(double)
    }
#undef SKR_UPD_K
#undef SKR_UPD
    launch_fold_n(s, w);
}
void launch_true_residual(hipStream_t s, const Work& w, const DevOp& op, const double* b, const double* x,
                          const int* gate) {
    hipLaunchKernelGGL(k_true_residual, dim3(w.nblk), dim3(ROWS), 0, s, op, b, x, w.r, w.nblk, w.part_n, gate);
    launch_fold_n(s, w);
    launch_norm_finish(s, w, FIN_TRUE_RES, 0.0, 0, gate);
}
void launch_spmm(hipStream_t s, const Work& w, const DevOp& op, int kin) {
    if (w.mixed)
        hipLaunchKernelGGL(k_spmm<float>, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, op, (const float*)ucols<float>(w),
                           bas<float>(w), w.ld, kin);
    else
        hipLaunchKernelGGL(k_spmm<double>, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, op,
                           (const double*)ucols<double>(w), bas<double>(w), w.ld, kin);
}
void launch_startup_gram(hipStream_t s, const Work& w, int kcols) {
    ColList L = {{bcol(w, 0), nullptr, nullptr, nullptr}, {kcols, 0, 0, 0}};
    launch_gram(s, w, L, kcols, L, kcols, w.gram);
}
void launch_startup_apply(hipStream_t s, const Work& w, int use_keep, int second) {
    if (w.mixed)
        hipLaunchKernelGGL(k_startup_apply<float>, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, bas<float>(w),
                           ucols<float>(w), w.n, w.ld, (const Coef*)w.coef, use_keep, second);
    else
        hipLaunchKernelGGL(k_startup_apply<double>, dim3(blocks_for(w.n)), dim3(ROWS), 0, s, bas<double>(w),
                           ucols<double>(w), w.n, w.ld, (const Coef*)w.coef, use_keep, second);
}
// c = C^T r (ke columns, on the matrix cores), then x = x0 + U c, r -= C c and ||r||.
// gate: see k_norm_finish (the Gram product before it only fills scratch that every later use
// recomputes first)
void launch_startup_project(hipStream_t s, const Work& w, double* x, int ke, int add_x, const int* gate) {
    ColList L = {{bcol(w, 0), nullptr, nullptr, nullptr}, {ke, 0, 0, 0}};
    launch_gram_r(s, w, L, ke, w.red1, 1);
    if (w.mixed)
        hipLaunchKernelGGL(k_startup_project<float>, dim3(w.nblk), dim3(ROWS), 0, s, x, w.r,
                           (const float*)bas<float>(w), (const float*)ucols<float>(w), w.n, w.ld, w.nblk, ke, add_x,
                           (const double*)w.red1, w.part_n, gate);
    else
        hipLaunchKernelGGL(k_startup_project<double>, dim3(w.nblk), dim3(ROWS), 0, s, x, w.r,
                           (const double*)bas<double>(w), (const double*)ucols<double>(w), w.n, w.ld, w.nblk, ke,
                           add_x, (const double*)w.red1, w.part_n, gate);
    launch_fold_n(s, w);
    launch_norm_finish(s, w, FIN_PROJECT, 0.0, ke, gate);
}
void launch_spmv(hipStream_t s, const DevOp& op, const double* x, double* y) {
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(op.n)), dim3(ROWS), 0, s, op, x, y);
}
void launch_spmv_repeat(hipStream_t s, const DevOp& op, const double* x, double* y, int repeats) {
    for (int q = 0; q < repeats; ++q)
        hipLaunchKernelGGL(k_spmv, dim3(blocks_for(op.n)), dim3(ROWS), 0, s, op, x, y);
}

int gram_cols_max(int m, int k) { return (2 * k + m + 2) * (k + 1); }

#endif  // !SKR_CHAINS_UNIT

#ifdef SKR_CHAINS_UNIT
// ---------------------------------------------------------------------------------------------
// Batched launches: chain blockIdx.y of the table, the same bodies as the single-chain kernels, so
// that every chain's arithmetic is that of the chain solved alone. A chain with `on` clear, or past
// the steps of its cycle, returns at once.
// ---------------------------------------------------------------------------------------------
#define SKR_CD const ChainDesc& cd = tab[blockIdx.y]; if (!cd.on) return; const Work& w = cd.w
__device__ __forceinline__ const double* pn_src_d(const Work& w) { return w.fold ? w.fold_n : w.part_n; }
__device__ __forceinline__ int pn_cnt_d(const Work& w) { return w.fold ? NFOLD : w.nblk; }

__global__ void kb_clear_nonfinite(const ChainDesc* tab) {
    SKR_CD;
    if (threadIdx.x == 0) k_clear_nonfinite_body(w.ctrl);
}
__global__ __launch_bounds__(ROWS) void kb_init(const ChainDesc* tab) {
    SKR_CD;
    k_init_body(cd.b, cd.x, w.r, w.n, w.nblk, w.part_n);
}
__global__ __launch_bounds__(ROWS) void kb_fold1(const ChainDesc* tab, int j) {
    SKR_CD;
    if (j >= 0 && j >= cd.scyc) return;
    k_fold1_body(w.part_n, w.nblk, w.fold_n);
}
__global__ __launch_bounds__(ROWS) void kb_norm_finish(const ChainDesc* tab, int mode, double rtol) {
    SKR_CD;
    k_norm_finish_body(pn_src_d(w), pn_cnt_d(w), mode, rtol, cd.kc, w.ctrl);
}
__global__ __launch_bounds__(ROWS) void kb_check_finite(const ChainDesc* tab) {
    SKR_CD;
    k_check_finite_body(cd.arr[cd.part], cd.cnt[cd.part], w.ctrl);
}
__global__ __launch_bounds__(ROWS) void kb_to_f32(const ChainDesc* tab) {
    SKR_CD;
    k_to_f32_body(cd.arr[cd.part], cd.arr32[cd.part], cd.cnt[cd.part]);
}
__global__ __launch_bounds__(ROWS) void kb_check_sym(const ChainDesc* tab) {
    SKR_CD;
    if (cd.op.kind == SKR_OP_CSR) k_check_sym_csr_body(cd.op, w.ctrl);
}
__global__ __launch_bounds__(ROWS) void kb_zero(const ChainDesc* tab) {
    SKR_CD;
    k_zero_body(cd.x, w.n);
}
__global__ __launch_bounds__(ROWS) void kb_true_residual(const ChainDesc* tab) {
    SKR_CD;
    k_true_residual_body(cd.op, cd.b, cd.x, w.r, w.nblk, w.part_n);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void kb_spmm(const ChainDesc* tab) {
    SKR_CD;
    k_spmm_body<BT>(cd.op, (const BT*)w.U, (BT*)w.basis, w.ld, cd.kin);
}
// which: 0 the cycle end (Lg, Rg), 1 the start-up (Ls, Ls), 2 the projection (Lp, r), 3 (Lg, r)
template <int TA, int TB, typename LT, typename RT>
__global__ __launch_bounds__(ROWS) void kb_gram_partial(const ChainDesc* tab, int which, int nl, int nr, int rpb) {
    SKR_CD;
    const ColList Rr = {{w.r, nullptr, nullptr, nullptr}, {1, 0, 0, 0}};
    const ColList& L = which == 0 || which == 3 ? cd.Lg : (which == 1 ? cd.Ls : cd.Lp);
    const ColList& R = which == 0 ? cd.Rg : (which == 1 ? cd.Ls : Rr);
    k_gram_partial_body<TA, TB, LT, RT>(L, nl, R, nr, w.n, w.ld, rpb, w.gpart);
}
// out: the Gram block (+ offset) or, with to_red1, red1 (the projection's C^T r)
__global__ __launch_bounds__(ROWS) void kb_gram_reduce(const ChainDesc* tab, int nb, int E, int nr, int ostride,
                                                       int to_red1, int off) {
    SKR_CD;
    k_gram_reduce_body(w.gpart, nb, E, nr, ostride, to_red1 ? w.red1 : w.gram + off);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void kb_startup_apply(const ChainDesc* tab, int use_keep, int second) {
    SKR_CD;
    k_startup_apply_body<BT>((BT*)w.basis, (BT*)w.U, w.n, w.ld, w.coef, use_keep, second);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void kb_startup_project(const ChainDesc* tab, int add_x) {
    SKR_CD;
    k_startup_project_body<BT>(cd.x, w.r, (const BT*)w.basis, (const BT*)w.U, w.n, w.ld, w.nblk, cd.kc, add_x,
                               w.red1, w.part_n);
}
template <int KIND, int KB>
__global__ __launch_bounds__(ROWS) void kb_apply_c(const ChainDesc* tab) {
    SKR_CD;
    k_apply_c_body<KIND, KB>(cd.op, (const double*)w.basis, (float*)w.Z, w.ld, cd.kc, w.nblk);
}
template <int NL, int KIND, typename BT>
__global__ __launch_bounds__(ROWS) void kb_step_a(const ChainDesc* tab, int j) {
    SKR_CD;
    if (j >= cd.scyc) return;
    const double* src = (j == 0) ? w.r : w.W[(j - 1) & 1];
    k_step_a_body<NL, KIND, BT>(cd.op, src, w.W[j & 1], (BT*)w.basis, w.ld, cd.kc, w.k, j, w.nblk, pn_cnt_d(w),
                                pn_src_d(w), w.part_a, w.red1, w.red2, w.H, w.Bm, w.ctrl);
}
template <int NL, typename BT, bool FOLDED, bool NORM>
__global__ __launch_bounds__(ROWS) void kb_step_b(const ChainDesc* tab, int j) {
    SKR_CD;
    if (j >= cd.scyc) return;
    k_step_b_body<NL, BT, FOLDED, NORM>(w.W[j & 1], (const BT*)w.basis, w.n, w.ld, cd.kc, w.k, j, w.nblk,
                                        FOLDED ? NFOLD : w.nblk, FOLDED ? w.fold_a : w.part_a, w.part_b, w.red1,
                                        w.ctrl);
}
template <int NL, typename BT, bool FOLDED>
__global__ __launch_bounds__(ROWS) void kb_step_c(const ChainDesc* tab, int j) {
    SKR_CD;
    if (j >= cd.scyc) return;
    k_step_c_body<NL, BT, FOLDED>(w.W[j & 1], (const BT*)w.basis, w.n, w.ld, cd.kc, w.k, j, w.nblk,
                                  FOLDED ? NFOLD : w.nblk, FOLDED ? w.fold_b : w.part_b, w.part_n, w.red2, w.ctrl);
}
// which 0: part_a -> fold_a, 1: part_b -> fold_b
__global__ __launch_bounds__(ROWS) void kb_fold(const ChainDesc* tab, int j, int which, int width) {
    SKR_CD;
    if (j >= cd.scyc) return;
    k_fold_body(which ? w.part_b : w.part_a, w.nblk, width, which ? w.fold_b : w.fold_a);
}
// LAST: the cycle's final closing at j = scyc of each chain (j is ignored)
template <int NL, int KIND, int KZ, bool LAST>
__global__ __launch_bounds__(ROWS) void kb_step_m(const ChainDesc* tab, int j) {
    SKR_CD;
    if (LAST) j = cd.scyc;
    else if (j >= cd.scyc) return;
    k_step_m_body<NL, KIND, KZ, LAST>(cd.op, w.W[(j - 1) & 1], w.W[j & 1], (double*)w.basis, (const float*)w.Z,
                                      w.ld, cd.kc, w.k, j, w.nblk, w.fold ? NFOLD : w.nblk,
                                      w.fold ? w.fold_b : w.part_b, w.part_a, w.red1,
                                      w.gcorr + ((j - 1) & 1) * NC, w.gcorr + (j & 1) * NC, w.H, w.Bm, w.ctrl);
}
template <typename BT>
__global__ __launch_bounds__(ROWS) void kb_close_basis(const ChainDesc* tab) {
    SKR_CD;
    k_close_basis_body<BT>(w.W[0], w.W[1], (BT*)w.basis, w.n, w.ld, cd.kc, w.k, cd.scyc, pn_cnt_d(w), pn_src_d(w),
                           w.red1, w.red2, w.H, w.Bm, w.ctrl);
}
template <int KB, typename BT>
__global__ __launch_bounds__(ROWS) void kb_cycle_update(const ChainDesc* tab) {
    SKR_CD;
    k_cycle_update_body<KB, BT>(cd.x, w.r, (BT*)w.basis, (BT*)w.U, w.n, w.ld, w.k, cd.kc, w.nblk, w.coef,
                                w.part_n, w.ctrl);
}
// The control snapshot of every chain (and the start-up's k_eff) into one host-readable array.
__global__ void kb_gather(const ChainDesc* tab, CtrlHost* out, int* keff) {
    const ChainDesc& cd = tab[blockIdx.y];
    constexpr int NW = sizeof(CtrlHost) / sizeof(int);
    const int t = threadIdx.x;
    if (t < NW) ((int*)&out[blockIdx.y])[t] = ((const int*)cd.w.ctrl)[t];
    if (t == 0) keff[blockIdx.y] = cd.w.coef->k_eff;
}
#undef SKR_CD

// Launchers of the batched kernels, mirroring the single-chain launchers above.
static inline dim3 grid_b(int x, const Batch& B) { return dim3((unsigned)x, (unsigned)B.C); }
void blaunch_gather(const Batch& B, CtrlHost* out, int* keff) {
    hipLaunchKernelGGL(kb_gather, grid_b(1, B), dim3(64), 0, B.s, B.cd, out, keff);
}
void blaunch_fold_n(const Batch& B, int j) {
    if (B.w0.fold) hipLaunchKernelGGL(kb_fold1, grid_b(NFOLD, B), dim3(ROWS), 0, B.s, B.cd, j);
}
void blaunch_norm_finish(const Batch& B, int mode, double rtol) {
    hipLaunchKernelGGL(kb_norm_finish, grid_b(1, B), dim3(ROWS), 0, B.s, B.cd, mode, rtol);
}
void blaunch_clear_nonfinite(const Batch& B) {
    hipLaunchKernelGGL(kb_clear_nonfinite, grid_b(1, B), dim3(1), 0, B.s, B.cd);
}
void blaunch_init(const Batch& B, double rtol) {
    hipLaunchKernelGGL(kb_init, grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd);
    blaunch_fold_n(B, -1);
    blaunch_norm_finish(B, FIN_INIT, rtol);
}
// checks (finite, and symmetric for CSR) of operator array `part` of every chain; grid as the single path
void blaunch_check_finite(const Batch& B, long count_max) {
    if (count_max <= 0) return;
    const int g = (int)std::min<long>(1024, (count_max + ROWS - 1) / ROWS);
    hipLaunchKernelGGL(kb_check_finite, grid_b(g, B), dim3(ROWS), 0, B.s, B.cd);
}
void blaunch_to_f32(const Batch& B, long count_max) {
    if (count_max <= 0) return;
    const int g = (int)std::min<long>(2048, (count_max + ROWS - 1) / ROWS);
    hipLaunchKernelGGL(kb_to_f32, grid_b(g, B), dim3(ROWS), 0, B.s, B.cd);
}
void blaunch_check_sym(const Batch& B) {
    hipLaunchKernelGGL(kb_check_sym, grid_b(blocks_for(B.w0.n), B), dim3(ROWS), 0, B.s, B.cd);
}
void blaunch_zero(const Batch& B) {
    hipLaunchKernelGGL(kb_zero, grid_b(blocks_for(B.w0.n), B), dim3(ROWS), 0, B.s, B.cd);
}
void blaunch_true_residual(const Batch& B) {
    hipLaunchKernelGGL(kb_true_residual, grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd);
    blaunch_fold_n(B, -1);
    blaunch_norm_finish(B, FIN_TRUE_RES, 0.0);
}
void blaunch_spmm(const Batch& B) {
    if (B.w0.mixed)
        hipLaunchKernelGGL(kb_spmm<float>, grid_b(blocks_for(B.w0.n), B), dim3(ROWS), 0, B.s, B.cd);
    else
        hipLaunchKernelGGL(kb_spmm<double>, grid_b(blocks_for(B.w0.n), B), dim3(ROWS), 0, B.s, B.cd);
}
template <typename LT, typename RT>
static void blaunch_gram_t(const Batch& B, int which, int nl, int nr, int ostride, int to_red1, int off) {
    const Work& w = B.w0;
    const int E = nl * nr;
    const int rpb = ((w.n + w.ngblk - 1) / w.ngblk + GCHUNK - 1) / GCHUNK * GCHUNK;
    const int nb = (w.n + rpb - 1) / rpb;
    const int la = nl <= 32 ? 2 : (nl <= 64 ? 4 : (nl <= 96 ? 6 : 8));
    const int lbk = nr <= 16 ? 1 : (nr <= 32 ? 2 : 3);
#define SKR_BGP(LA, LB)                                                                                     \
    hipLaunchKernelGGL((kb_gram_partial<LA, LB, LT, RT>), grid_b(nb, B), dim3(ROWS), 0, B.s, B.cd, which, nl, nr, rpb)
#define SKR_BGP_B(LA)                           \
    switch (lbk) {                              \
        case 1: SKR_BGP(LA, 1); break;          \
        case 2: SKR_BGP(LA, 2); break;          \
        default: SKR_BGP(LA, 3); break;         \
    }
    switch (la) {
        case 2: SKR_BGP_B(2); break;
        case 4: SKR_BGP_B(4); break;
        case 6: SKR_BGP_B(6); break;
        default: SKR_BGP_B(8); break;
    }
#undef SKR_BGP_B
#undef SKR_BGP
    hipLaunchKernelGGL(kb_gram_reduce, grid_b((E + 63) / 64, B), dim3(ROWS), 0, B.s, B.cd, nb, E, nr, ostride,
                       to_red1, off);
}
// start-up Gram of kcols columns (uniform over the chains launched)
void blaunch_startup_gram(const Batch& B, int kcols) {
    if (B.w0.mixed) blaunch_gram_t<float, float>(B, 1, kcols, kcols, kcols, 0, 0);
    else blaunch_gram_t<double, double>(B, 1, kcols, kcols, kcols, 0, 0);
}
void blaunch_startup_apply(const Batch& B, int use_keep, int second) {
    if (B.w0.mixed)
        hipLaunchKernelGGL(kb_startup_apply<float>, grid_b(blocks_for(B.w0.n), B), dim3(ROWS), 0, B.s, B.cd,
                           use_keep, second);
    else
        hipLaunchKernelGGL(kb_startup_apply<double>, grid_b(blocks_for(B.w0.n), B), dim3(ROWS), 0, B.s, B.cd,
                           use_keep, second);
}
// c = C^T r over cd.kc = ke columns (uniform), then x (+)= U c, r -= C c and ||r||
void blaunch_startup_project(const Batch& B, int ke, int add_x) {
    if (B.w0.mixed) {
        blaunch_gram_t<float, double>(B, 2, ke, 1, 1, 1, 0);
        hipLaunchKernelGGL(kb_startup_project<float>, grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, add_x);
    } else {
        blaunch_gram_t<double, double>(B, 2, ke, 1, 1, 1, 0);
        hipLaunchKernelGGL(kb_startup_project<double>, grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, add_x);
    }
    blaunch_fold_n(B, -1);
    blaunch_norm_finish(B, FIN_PROJECT, 0.0);
}
void blaunch_apply_c(const Batch& B, int kind, int kc) {
    if (!B.w0.merged || kc <= 0) return;
#define SKR_BAC(KIND, KB) hipLaunchKernelGGL((kb_apply_c<KIND, KB>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd)
#define SKR_BAC_K(KIND)                      \
    if (kc <= 8) SKR_BAC(KIND, 8);           \
    else if (kc <= 16) SKR_BAC(KIND, 16);    \
    else if (kc <= 24) SKR_BAC(KIND, 24);    \
    else SKR_BAC(KIND, 32);
    if (kind == SKR_OP_CSR) {
        SKR_BAC_K(SKR_OP_CSR)
    } else if (kind == SKR_OP_STENCIL7) {
        SKR_BAC_K(SKR_OP_STENCIL7)
    } else {
        SKR_BAC_K(SKR_OP_STENCIL5)
    }
#undef SKR_BAC_K
#undef SKR_BAC
}
// one Arnoldi step of every chain launched (uniform kc and operator kind): the single path's kernels
template <int NL, int KIND, typename BT>
static void bstep_a(const Batch& B, int j) {
    hipLaunchKernelGGL((kb_step_a<NL, KIND, BT>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, j);
}
template <int NL, typename BT>
static void bstep_a_k(const Batch& B, int kind, int j) {
    if (kind == SKR_OP_CSR) bstep_a<NL, SKR_OP_CSR, BT>(B, j);
    else if (kind == SKR_OP_STENCIL7) bstep_a<NL, SKR_OP_STENCIL7, BT>(B, j);
    else bstep_a<NL, SKR_OP_STENCIL5, BT>(B, j);
}
template <int NL, typename BT, bool NORM>
static void bstep_b(const Batch& B, int j) {
    if (B.w0.fold)
        hipLaunchKernelGGL((kb_step_b<NL, BT, true, NORM>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, j);
    else
        hipLaunchKernelGGL((kb_step_b<NL, BT, false, NORM>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, j);
}
template <int NL, typename BT>
static void bstep_c(const Batch& B, int j) {
    if (B.w0.fold)
        hipLaunchKernelGGL((kb_step_c<NL, BT, true>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, j);
    else
        hipLaunchKernelGGL((kb_step_c<NL, BT, false>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd, j);
}
static void bfold(const Batch& B, int j, int which, int width) {
    if (B.w0.fold) hipLaunchKernelGGL(kb_fold, grid_b(NFOLD, B), dim3(ROWS), 0, B.s, B.cd, j, which, width);
}
template <int NL, int KZ, bool LAST>
static void bstep_m_z(const Batch& B, int kind, int j) {
    if (LAST || kind == SKR_OP_CSR)
        hipLaunchKernelGGL((kb_step_m<NL, SKR_OP_CSR, LAST ? 0 : KZ, LAST>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s,
                           B.cd, j);
    else if (kind == SKR_OP_STENCIL7)
        hipLaunchKernelGGL((kb_step_m<NL, SKR_OP_STENCIL7, KZ, LAST>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s,
                           B.cd, j);
    else
        hipLaunchKernelGGL((kb_step_m<NL, SKR_OP_STENCIL5, KZ, LAST>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s,
                           B.cd, j);
}
template <int NL, bool LAST>
static void bstep_m(const Batch& B, int kind, int kc, int j) {
    if (LAST) bstep_m_z<NL, 0, true>(B, kind, j);
    else if (kc == 0) bstep_m_z<NL, 0, false>(B, kind, j);
    else if (kc <= 8) bstep_m_z<NL, 8, false>(B, kind, j);
    else if (kc <= 16) bstep_m_z<NL, 16, false>(B, kind, j);
    else if (kc <= 24) bstep_m_z<NL, 24, false>(B, kind, j);
    else bstep_m_z<NL, 32, false>(B, kind, j);
}
// With ev != nullptr, ev[2q], ev[2q+1] take the start and end of kernel q of the step (A or the
// merged kernel, B, C), as in the single-chain launcher.
void blaunch_step(const Batch& B, int kind, int kc, int j, hipEvent_t* ev) {
    const int ncol = kc + j + 1;
    auto rec = [&](int e) {
        if (ev) (void)hipEventRecord(ev[e], B.s);
    };
    if (B.w0.merged) {
        const int nla = bucket8(ncol + 1);
        rec(0);
        if (j == 0) {
#define CALL_A(NL) bstep_a_k<NL, double>(B, kind, 0)
            SKR_DISPATCH8(nla, CALL_A)
#undef CALL_A
        } else {
#define CALL_M(NL) bstep_m<NL, false>(B, kind, kc, j)
            SKR_DISPATCH8(nla, CALL_M)
#undef CALL_M
        }
        rec(1);
        bfold(B, j, 0, ncol + 1);
        rec(2);
#define CALL_B(NL) bstep_b<NL, double, true>(B, j)
        SKR_DISPATCH8(nla, CALL_B)
#undef CALL_B
        rec(3);
        bfold(B, j, 1, ncol + 1);
        return;
    }
    const int nla = bucket8(ncol + 1), nlb = bucket8(ncol);
    if (B.w0.mixed) {
        rec(0);
#define CALL_A(NL) bstep_a_k<NL, float>(B, kind, j)
        SKR_DISPATCH8(nla, CALL_A)
#undef CALL_A
        rec(1);
        bfold(B, j, 0, ncol + 1);
        rec(2);
#define CALL_B(NL) bstep_b<NL, float, false>(B, j)
        SKR_DISPATCH8(nlb, CALL_B)
#undef CALL_B
        rec(3);
        bfold(B, j, 1, ncol);
        rec(4);
#define CALL_C(NL) bstep_c<NL, float>(B, j)
        SKR_DISPATCH8(nlb, CALL_C)
#undef CALL_C
        rec(5);
    } else {
        rec(0);
#define CALL_A(NL) bstep_a_k<NL, double>(B, kind, j)
        SKR_DISPATCH8(nla, CALL_A)
#undef CALL_A
        rec(1);
        bfold(B, j, 0, ncol + 1);
        rec(2);
#define CALL_B(NL) bstep_b<NL, double, false>(B, j)
        SKR_DISPATCH8(nlb, CALL_B)
#undef CALL_B
        rec(3);
        bfold(B, j, 1, ncol);
        rec(4);
#define CALL_C(NL) bstep_c<NL, double>(B, j)
        SKR_DISPATCH8(nlb, CALL_C)
#undef CALL_C
        rec(5);
    }
    if (B.w0.fold) hipLaunchKernelGGL(kb_fold1, grid_b(NFOLD, B), dim3(ROWS), 0, B.s, B.cd, j);
}
void blaunch_close_basis(const Batch& B, int kind, int kc, int s_cycle) {
    if (B.w0.merged) {
        const int nla = bucket8(kc + s_cycle + 2);
#define CALL_L(NL) bstep_m<NL, true>(B, kind, kc, 0)
        SKR_DISPATCH8(nla, CALL_L)
#undef CALL_L
    } else if (B.w0.mixed) {
        hipLaunchKernelGGL(kb_close_basis<float>, grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd);
    } else {
        hipLaunchKernelGGL(kb_close_basis<double>, grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd);
    }
}
void blaunch_cycle_gram(const Batch& B, int kc, int jd_max) {
    const int nl = 2 * kc + jd_max + 1;
    if (!B.w0.mixed) {
        blaunch_gram_t<double, double>(B, 0, nl, kc + 1, kc + 1, 0, 0);
    } else {
        blaunch_gram_t<float, float>(B, 0, nl, kc, kc + 1, 0, 0);
        blaunch_gram_t<float, double>(B, 3, nl, 1, kc + 1, 0, kc);
    }
}
void blaunch_cycle_update(const Batch& B, int k_bucket) {
#define SKR_BUPD(KB, BT) hipLaunchKernelGGL((kb_cycle_update<KB, BT>), grid_b(B.w0.nblk, B), dim3(ROWS), 0, B.s, B.cd)
#define SKR_BUPD_K(BT)                           \
    switch (k_bucket) {                          \
        case 0: SKR_BUPD(0, BT); break;          \
        case 8: SKR_BUPD(8, BT); break;          \
        case 16: SKR_BUPD(16, BT); break;        \
        case 20: SKR_BUPD(20, BT); break;        \
        case 24: SKR_BUPD(24, BT); break;        \
        default: SKR_BUPD(32, BT); break;        \
    }
    if (B.w0.mixed) {
        SKR_BUPD_K(float)
    } else {
        SKR_BUPD_K(double)
    }
#undef SKR_BUPD_K
#undef SKR_BUPD
    blaunch_fold_n(B, -1);
}

#endif  // SKR_CHAINS_UNIT

}  // namespace skr
