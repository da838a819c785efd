// Internal declarations shared by the libskr translation units (device helpers, workspace
// layout, launch wrappers). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/skr.h"

namespace skr {

// ---------------------------------------------------------------------------------------------
// Fixed sizes
// ---------------------------------------------------------------------------------------------
constexpr int ROWS = 256;        // rows per workgroup in every row-parallel kernel (1 row / thread)
constexpr int NWAVE = ROWS / 64; // wavefronts per row workgroup
constexpr int NC = 128;          // stride of the per-workgroup column partials (two 64-lane groups)
constexpr int MMAX = 86;         // largest m: the basis [C V] has kc + j + 1 <= m + 1 columns, and a
                                 // pass-A reduction (those plus ||w||^2) m + 2 <= 88 columns
constexpr int KMAX = 32;         // largest k (recycled vectors)
constexpr int LDH = MMAX + 2;    // leading dimension of the Hessenberg store (rows)
constexpr int DMAX = MMAX + 2;   // leading dimension of the projected matrices (d = kc + j <= m)
constexpr int DSM = 62;          // largest d of the one-row-per-lane dense kernels (larger d: the
                                 // row-looped kernels)
constexpr int DS = 64;           // LDS dimension of the one-row-per-lane dense kernels
constexpr int NFOLD = 64;        // rows of folded partials (large grids)
constexpr int FOLD_MIN = 256;    // grids above this many workgroups fold their partials

// ---------------------------------------------------------------------------------------------
// Operator (device view of skr_op)
// ---------------------------------------------------------------------------------------------
struct DevOp {
    int kind;
    int n;
    const int* rowptr;
    const int* colind;
    const double* val;
    int nx, ny, nz;
    double inv_h2;
    const double* ax;
    const double* ay;
    const double* az;
    // FP32 copies of the values (CSR) or faces (stencils) for the products of the mixed mode's inner
    // cycle (set only there)
    const float* val32;
    const float* ax32;
    const float* ay32;
    const float* az32;
};

// Round to the nearest FP32 value (ties to even), held in FP64.
__device__ __forceinline__ double rnd32(double v) { return (double)(float)v; }

// One row of y = scale * (A x): CSR, 2-D 5-point or 3-D 7-point harmonic-mean stencil. KIND is the
// operator kind when the caller knows it at compile time (each kind then gets its own register
// allocation), or -1 to branch on op.kind. XT is the element type of x. With RND the row is that of
// A v with v = rnd32(scale * x) (the FP32-stored vector the product is defined on), and no scaling
// follows. With OP32 the operator's values are its FP32 copies (op.val32, op.ax32, ...); the
// arithmetic stays FP64.
template <int KIND, typename XT = double, bool RND = false, bool OP32 = false>
__device__ __forceinline__ double op_row_k(const DevOp& op, const XT* __restrict__ x, int i, double scale) {
    const int kind = KIND >= 0 ? KIND : op.kind;
    auto X = [&](int idx) -> double {
        const double v = (double)x[idx];
        return RND ? rnd32(v * scale) : v;
    };
    auto VAL = [&](int q) -> double { return OP32 ? (double)op.val32[q] : op.val[q]; };
    auto FX = [&](int q) -> double { return OP32 ? (double)op.ax32[q] : op.ax[q]; };
    auto FY = [&](int q) -> double { return OP32 ? (double)op.ay32[q] : op.ay[q]; };
    auto FZ = [&](int q) -> double { return OP32 ? (double)op.az32[q] : op.az[q]; };
    double s = 0.0;
    if (kind == SKR_OP_CSR) {
        // Entries in groups of 8: every index, value and gather load of a group is in flight before
        // the first product, at clamped indices; the products are added in entry order.
        const int e0 = op.rowptr[i], e1 = op.rowptr[i + 1];
        for (int e = e0; e < e1; e += 8) {
            int c[8];
            double v[8], xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = min(e + u, e1 - 1);
                c[u] = op.colind[q];
                v[u] = VAL(q);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) xv[u] = X(c[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e + u < e1) s = fma(v[u], xv[u], s);
        }
    } else if (kind == SKR_OP_STENCIL7) {
        const int nx = op.nx, ny = op.ny, nz = op.nz, nxy = nx * ny;
        const int gz = i / nxy, gyx = i - gz * nxy, gy = gyx / nx, gx = gyx - gy * nx;
        const int fx = (gz * ny + gy) * (nx + 1) + gx, fy = (gz * (ny + 1) + gy) * nx + gx, fz = gz * nxy + gyx;
        const double aw = FX(fx), ae = FX(fx + 1);
        const double as = FY(fy), an = FY(fy + nx);
        const double ad = FZ(fz), au = FZ(fz + nxy);
        // neighbour loads at clamped indices (a missing neighbour reads x[i]); its term is selected away
        const bool hw = gx > 0, he = gx < nx - 1, hs = gy > 0, hn = gy < ny - 1, hd = gz > 0, hu = gz < nz - 1;
        const double xc = X(i);
        const double xw = X(hw ? i - 1 : i), xe = X(he ? i + 1 : i);
        const double xs = X(hs ? i - nx : i), xn = X(hn ? i + nx : i);
        const double xd = X(hd ? i - nxy : i), xu = X(hu ? i + nxy : i);
        s = ((aw + ae) + (as + an) + (ad + au)) * xc;
        s = hw ? fma(-aw, xw, s) : s;
        s = he ? fma(-ae, xe, s) : s;
        s = hs ? fma(-as, xs, s) : s;
        s = hn ? fma(-an, xn, s) : s;
        s = hd ? fma(-ad, xd, s) : s;
        s = hu ? fma(-au, xu, s) : s;
        s *= op.inv_h2;
    } else {
        const int nx = op.nx, ny = op.ny;
        const int r = i / nx, c = i - r * nx;
        const double aw = FX(r * (nx + 1) + c), ae = FX(r * (nx + 1) + c + 1);
        const double an = FY(r * nx + c), as = FY((r + 1) * nx + c);
        const bool hw = c > 0, he = c < nx - 1, hn = r > 0, hs = r < ny - 1;
        const double xc = X(i);
        const double xw = X(hw ? i - 1 : i), xe = X(he ? i + 1 : i);
        const double xn = X(hn ? i - nx : i), xs = X(hs ? i + nx : i);
        s = (aw + ae + an + as) * xc;
        s = hw ? fma(-aw, xw, s) : s;
        s = he ? fma(-ae, xe, s) : s;
        s = hn ? fma(-an, xn, s) : s;
        s = hs ? fma(-as, xs, s) : s;
        s *= op.inv_h2;
    }
    return RND ? s : s * scale;
}
__device__ __forceinline__ double op_row(const DevOp& op, const double* __restrict__ x, int i, double scale) {
    return op_row_k<-1, double, false>(op, x, i, scale);
}

// ---------------------------------------------------------------------------------------------
// Control block: per-solve device state read and written by the step kernels.
// ---------------------------------------------------------------------------------------------
struct Ctrl {
    int stop;        // nonzero: the remaining Arnoldi steps of this cycle are skipped
    int j_done;      // Arnoldi steps completed in the current cycle
    int breakdown;   // happy breakdown at step j_done
    int kc;          // recycled columns currently held in C and U
    int k_new;       // recycled columns produced by the last cycle end
    int nonfinite;   // NaN/Inf seen in b or A
    int eig_fail;    // the small eigen solve did not converge (recycle space kept from before)
    int nonsym;      // the operator is not exactly symmetric (CSR check at the system start;
                     // the stencil kinds are symmetric by construction)
    int route;       // eigen stage that formed the last recycle space: 1 symmetric, 2 general, 0 none
    int spec_skip;   // set by each cycle end: nonzero when the kernels the host launched ahead of
                     // its read of that cycle end (the next cycle's opening) must return at once
    double bnorm;    // ||b||
    double tol_abs;  // rtol * ||b||
    double beta;     // ||r|| at the start of the current cycle
    double inv_h;    // scale of the pending Krylov vector (1/beta, then 1/h_{j+1,j})
    double est;      // least-squares residual estimate after the last step
    double res2;     // squared norm from the last true-residual kernel
    double g[MMAX + 2];   // rotated right-hand side of the progressive Givens QR
    double cs[MMAX + 1];
    double sn[MMAX + 1];
};

// Snapshot read back by the host after a cycle.
struct CtrlHost {
    int stop, j_done, breakdown, kc, k_new, nonfinite, eig_fail, nonsym, route, spec_skip;
    double bnorm, tol_abs, beta, inv_h, est, res2;
};

// Coefficients produced by the small dense kernel at a cycle end (device).
struct Coef {
    double yU[KMAX];                      // x += U yU + V yV
    double yV[MMAX + 1];
    double rC[KMAX];                      // r -= C rC + V rV
    double rV[MMAX + 2];
    double Qc[(KMAX + MMAX + 2) * KMAX];  // C_new = [C V] Qc      ((kc+j+1) x k_new, col-major, ld KMAX+MMAX+2)
    double Qu[(KMAX + MMAX + 1) * KMAX];  // U_new = [U V] Qu      ((kc+j) x k_new, ld KMAX+MMAX+1)
    double R[KMAX * KMAX];                // start-up triangular factors
    double R2[KMAX * KMAX];
    double Rinv[KMAX * KMAX];
    int keep[KMAX];
    int k_eff;
    int pad;
};
// Hand-over from the first cycle-end stage to the eigen stages (device).
// DW_PENDING_L, DW_GEN_L: d > DSM, X holds X'' (each large-d stage forms M itself).
enum { DW_NONE = 0, DW_PENDING = 1, DW_GEN = 2, DW_DONE = 3, DW_GEN_L = 4, DW_PENDING_L = 5 };
struct DenseWork {
    int mode, d, kc, pad;
    double Dk[KMAX];
    double gcs[DMAX], gsn[DMAX];
    double R[DMAX * DMAX];    // R_G (upper triangular), column-major, ld DMAX
    double X[DMAX * DMAX];    // top d rows of Q_G^T X, then M = X'' R_G^{-1} for the general stage
};
constexpr int LDQC = KMAX + MMAX + 2;
constexpr int LDQU = KMAX + MMAX + 1;

// ---------------------------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// ---------------------------------------------------------------------------------------------
// Cross-lane exchanges without the LDS crossbar. A double moves as two 32-bit halves.
//  * swap32(a, b): v_permlane32_swap: r0 = (a in lanes 0-31 | b of lanes 0-31 in lanes 32-63),
//    r1 = (a of lanes 32-63 in lanes 0-31 | b in lanes 32-63). With a = the values a lane keeps when
//    it is in the lower half and b = those it keeps when in the upper half, r0 + r1 is, in every
//    lane, its kept value plus the partner's (lane l ^ 32) value of the same column.
//  * swap16: the same between the 16-lane rows 0<->1 and 2<->3 (partner l ^ 16).
//  * DPP row_ror:8 (partner l ^ 8), row_half_mirror (partner 7 - (l % 8) in each group of 8),
//    quad_perm (partners l ^ 2, l ^ 1).
// Every stage adds a value and its partner's, and addition commutes, so both partners hold the
// same bits: the reductions are deterministic and identical in every lane that holds a result.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void swap32_f64(double a, double b, double& r0, double& r1) {
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    r0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    r1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap16_f64(double a, double b, double& r0, double& r1) {
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    r0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    r1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Value of the first active lane (lane 0 when the whole wavefront is active), in every lane.
__device__ __forceinline__ double first_lane(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr int DPP_ROW_ROR8 = 0x128, DPP_ROW_HALF_MIRROR = 0x141, DPP_QP_XOR2 = 0x4E, DPP_QP_XOR1 = 0xB1;

// Partner value at a stage whose partner lies inside a 16-lane row (HALF = 8, 4, 2, 1).
template <int HALF>
__device__ __forceinline__ double row_partner(double x) {
    if constexpr (HALF == 8) return dpp_f64<DPP_ROW_ROR8>(x);
    else if constexpr (HALF == 4) return dpp_f64<DPP_ROW_HALF_MIRROR>(x);
    else if constexpr (HALF == 2) return dpp_f64<DPP_QP_XOR2>(x);
    else return dpp_f64<DPP_QP_XOR1>(x);
}

// Sum over the wavefront; every lane gets the same bits.
__device__ __forceinline__ double wave_sum(double x) {
    double r0, r1;
    swap32_f64(x, x, r0, r1);
    x = r0 + r1;
    swap16_f64(x, x, r0, r1);
    x = r0 + r1;
    x += row_partner<8>(x);
    x += row_partner<4>(x);
    x += row_partner<2>(x);
    x += row_partner<1>(x);
    return x;
}
__device__ __forceinline__ double wave_max(double x) {
    double r0, r1;
    swap32_f64(x, x, r0, r1);
    x = fmax(r0, r1);
    swap16_f64(x, x, r0, r1);
    x = fmax(r0, r1);
    x = fmax(x, row_partner<8>(x));
    x = fmax(x, row_partner<4>(x));
    x = fmax(x, row_partner<2>(x));
    x = fmax(x, row_partner<1>(x));
    return x;
}

// Butterfly reduce-scatter over one wavefront of NR (a power of two <= 64) column values per lane:
// on return lane l holds the wave-wide sum of column (l mod NR) in v[0]. Stages with HALF >= NR
// are plain all-reduce stages; the remaining stages halve the columns each lane keeps (a lane whose
// HALF bit is set keeps the upper half). The order of additions is fixed, so results are bitwise
// reproducible. Every register index is a compile-time constant.
template <int HALF, int NR>
__device__ __forceinline__ void rs_stage(double (&v)[NR], int lane) {
    if constexpr (HALF >= 16) {
#pragma unroll
        for (int i = 0; i < HALF; ++i) {
            double r0, r1;
            if constexpr (HALF == 32) swap32_f64(v[i], v[i + HALF], r0, r1);
            else swap16_f64(v[i], v[i + HALF], r0, r1);
            v[i] = r0 + r1;
        }
    } else {
        const bool upper = (lane & HALF) != 0;
#pragma unroll
        for (int i = 0; i < HALF; ++i) {
            const double send = upper ? v[i] : v[i + HALF];
            const double keep = upper ? v[i + HALF] : v[i];
            v[i] = keep + row_partner<HALF>(send);
        }
    }
}

template <int OFF, int NR>
__device__ __forceinline__ void allreduce_stage(double (&v)[NR]) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        double r0, r1;
        if constexpr (OFF == 32) swap32_f64(v[i], v[i], r0, r1);
        else swap16_f64(v[i], v[i], r0, r1);
        v[i] = r0 + r1;
    }
}

template <int NR>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[NR]) {
    static_assert(NR >= 16, "reduction widths are 16, 32 or 64");
    const int lane = lane_id();
    if constexpr (NR <= 16) {
        allreduce_stage<32, NR>(v);
        allreduce_stage<16, NR>(v);
    } else if constexpr (NR == 32) {
        allreduce_stage<32, NR>(v);
    }
    if constexpr (NR >= 64) rs_stage<32, NR>(v, lane);
    if constexpr (NR >= 32) rs_stage<16, NR>(v, lane);
    rs_stage<8, NR>(v, lane);
    rs_stage<4, NR>(v, lane);
    rs_stage<2, NR>(v, lane);
    rs_stage<1, NR>(v, lane);
    return v[0];
}



// Arrive at the end of a grid-wide reduction. Returns true in exactly one workgroup, the last
// one to arrive, after which it may read every workgroup's partials. The caller's partial stores
// must precede the call. The counter is reset by the last workgroup.
__device__ __forceinline__ bool last_block_arrive(unsigned* counter, unsigned nblocks) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(counter, 1u);
        is_last = (t == nblocks - 1) ? 1 : 0;
        if (is_last) atomicExch(counter, 0u);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// ---------------------------------------------------------------------------------------------
// Fence-free grid reductions. A kernel writes one partial per workgroup; every workgroup of the
// next kernel (launched on the same stream, so the partials are visible) sums all partials itself
// in the same fixed order, so all workgroups hold bitwise identical totals. This avoids device-scope
// fences and atomics, which cost far more than a kernel boundary on a multi-XCD GPU.
// ---------------------------------------------------------------------------------------------

// Per-workgroup sum of one value per thread into part[lb] (fixed order).
__device__ __forceinline__ void block_partial1(double v, double* part, int lb, double* sh) {
    const double ws = wave_sum(v);
    if (lane_id() == 0) sh[wave_id()] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q) t += sh[q];
        part[lb] = t;
    }
    __syncthreads();
}

// Sum of part[0..nblk) in a fixed order (lane-strided, four loads in flight per lane, then a
// wave butterfly). Called by all threads of a workgroup; every thread gets the total.
__device__ __forceinline__ double sum_partials1(const double* part, int nblk, double* sh) {
    if (threadIdx.x < 64) {
        double s = 0.0;
        int b = threadIdx.x;
        for (; b + 192 < nblk; b += 256) {
            const double v0 = part[b], v1 = part[b + 64], v2 = part[b + 128], v3 = part[b + 192];
            s += v0; s += v1; s += v2; s += v3;
        }
        for (; b < nblk; b += 64) s += part[b];
        s = wave_sum(s);
        if (threadIdx.x == 0) sh[0] = s;
    }
    __syncthreads();
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Column sums of part[b * NC + c] (b < nblk, c < nr <= NC) into out[0..nr) (LDS), fixed order: each
// wave sums a contiguous quarter of the workgroups (up to 64 loads in flight per lane), then the
// quarters are added in order. Columns 64.. (nr > 64) are a second pass of the same form. BATCH loads
// are issued together (16 suffice for folded partials, 16 rows per wave, and keep registers free).
// Columns start at cfirst (a multiple of 64). Called by all threads of a workgroup; sh holds
// NWAVE * 64 doubles.
template <int BATCH = 64>
__device__ __forceinline__ void sum_partials(const double* part, int nblk, int nr, double* sh, double* out,
                                             int cfirst = 0) {
    const int lane = lane_id(), w = wave_id();
    const int per = (nblk + NWAVE - 1) / NWAVE;
    const int b0 = w * per, b1 = min(nblk, b0 + per);
    for (int c0 = cfirst; c0 < nr; c0 += 64) {
        const int col = c0 + lane;
        double s = 0.0;
        if (col < nr) {
            for (int b = b0; b < b1; b += BATCH) {
                double v[BATCH];
                if (b + BATCH <= b1) {
                    // a full batch (wave-uniform test): one row pointer and constant offsets, no
                    // per-load guard (a guarded load compiles into an exec-mask branch of its own)
                    const double* pb = part + (size_t)b * NC + (unsigned)col;
#pragma unroll
                    for (int u = 0; u < BATCH; ++u) v[u] = pb[u * NC];
                } else {
#pragma unroll
                    for (int u = 0; u < BATCH; ++u) v[u] = (b + u < b1) ? part[(b + u) * NC + col] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < BATCH; ++u) s += v[u];
            }
        }
        sh[w * 64 + lane] = s;
        __syncthreads();
        if (threadIdx.x < 64 && col < nr) {
            double t = sh[lane];
#pragma unroll
            for (int q = 1; q < NWAVE; ++q) t += sh[q * 64 + lane];
            out[col] = t;
        }
        __syncthreads();
    }
}

// Sum of one value per thread over the grid, for kernels that run once per system: the partial of
// each workgroup goes to part[lb] (so a following kernel may re-sum it with sum_partials1) and the
// last workgroup to arrive forms the total in the same order. Returns true in that workgroup.
__device__ __forceinline__ bool grid_sum1(double v, double* part, unsigned* counter, int nblk, int lb,
                                          double* sh, double* result) {
    block_partial1(v, part, lb, sh);
    if (!last_block_arrive(counter, (unsigned)nblk)) return false;
    *result = sum_partials1(part, nblk, sh);
    return true;
}

// Logical row-block index for hardware workgroup id b. Workgroups are dispatched round-robin over
// the 8 XCDs; when the grid divides evenly, consecutive logical blocks are kept on one XCD so
// that a block's stencil/CSR neighbours mostly sit in the same L2.
__device__ __forceinline__ int logical_block(int b, int nblk) {
    if ((nblk & 7) != 0) return b;
    const int per = nblk >> 3;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------------------------
// Workspace (device buffers owned by a context)
// ---------------------------------------------------------------------------------------------
struct Work {
    int n = 0, ld = 0, nblk = 0, m = 0, k = 0;
    void* block = nullptr;       // the one device block every buffer below lives in
    // [C (k cols) | V (m+1 cols)] and U (k cols), column-major, leading dim ld; the elements are
    // doubles, or floats when mixed (the buffers are sized for doubles either way)
    double* basis = nullptr;
    double* U = nullptr;
    double* Z = nullptr;         // A C (k columns stored as FP32, FP64 basis only): the merged Arnoldi
                                 // kernel's A C
    int mixed = 0;
    double* W[2] = {nullptr, nullptr};
    double* r = nullptr;
    double* part_a = nullptr;    // nblk * NC partials written by step pass A (read by pass B)
    double* part_b = nullptr;    // nblk * NC partials written by step pass B (read by pass C)
    double* part_n = nullptr;    // nblk scalar partials of a squared norm (read by the next kernel)
    double* part = nullptr;      // nblk * NC partials of the start-up projection
    double* gpart = nullptr;     // Gram partials: ngblk * gram_max
    double* gram = nullptr;      // reduced Gram result
    double* fold_a = nullptr;    // NFOLD * NC folded partials of pass A (large grids)
    double* fold_b = nullptr;    // NFOLD * NC folded partials of pass B
    double* fold_n = nullptr;    // NFOLD folded norm partials
    int fold = 0;                // nonzero: partials are folded before every re-sum
    int merged = 0;              // nonzero: two kernels per Arnoldi step (FP64 basis, no folding)
    double* red1 = nullptr;      // NC
    double* red2 = nullptr;      // NC
    double* gcorr = nullptr;     // 2 x NC: column corrections of the merged Arnoldi kernel (alternating)
    double* H = nullptr;         // LDH x MMAX
    double* Bm = nullptr;        // KMAX x MMAX
    Ctrl* ctrl = nullptr;
    Coef* coef = nullptr;
    DenseWork* dense = nullptr;
    unsigned* counters = nullptr;  // 8 counters
    size_t gram_max = 0;
    int ngblk = 0;
};

int gram_cols_max(int m, int k);

// Up to four column segments for the tall-skinny Gram products; segment s has cnt[s] columns at
// seg[s] (stride ld), all of the element type the kernel takes for the list.
struct ColList {
    const void* seg[4];
    int cnt[4];
};

// ---------------------------------------------------------------------------------------------
// Batched launches (skr_solve_chains): several chains of one shape advance in one launch, chain c
// in grid row blockIdx.y. Each chain keeps its own workspace; its descriptor holds the device
// pointers and the values that differ between chains. A launch's template parameters are uniform
// over the chains it covers; `on` masks the chains a launch leaves alone.
// ---------------------------------------------------------------------------------------------
struct ChainDesc {
    Work w;                 // the chain's workspace (device pointers) and sizes
    DevOp op;               // operator of the chain's current system
    const double* b;
    double* x;
    ColList Lg, Rg;         // cycle-end Gram lists ([C V U] and [U r]) of the current cycle
    ColList Ls;             // start-up columns (kin or ke)
    ColList Lp;             // C columns for C^T r (projection)
    int on;                 // the launch touches this chain
    int kc;                 // recycled columns (C, U) of the current cycle / projection
    int kin;                // carried columns at the start-up
    int ke;                 // columns kept by the start-up drop
    int scyc;               // steps of the current cycle
    int part;               // which operator array a check / conversion launch touches (0..2)
    long cnt[3];            // operator array lengths: CSR values, or faces ax, ay, az
    const double* arr[3];   // the operator arrays
    float* arr32[3];        // their FP32 copies (mixed mode)
};

// A batched launch: the device table of C chain descriptors and the sizes shared by every chain
// (a representative workspace: n, ld, nblk, m, k, fold, mixed, merged).
struct Batch {
    hipStream_t s;
    const ChainDesc* cd;
    int C;
    Work w0;
};

}  // namespace skr
