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
constexpr int NC = 64;           // width of the column reductions of the Arnoldi step
constexpr int MMAX = 62;         // largest m: the basis [C V] has kc + j + 1 <= m + 1 < NC columns
constexpr int KMAX = 32;         // largest k (recycled vectors)
constexpr int LDH = MMAX + 2;    // leading dimension of the Hessenberg store (rows)
constexpr int DMAX = 64;         // largest projected dimension d = kc + j (<= m) plus one
constexpr int NORM_COL = NC - 1; // reduction column that carries ||A v_j||^2 in the first pass

// ---------------------------------------------------------------------------------------------
// Operator (device view of skr_op)
// ---------------------------------------------------------------------------------------------
struct DevOp {
    int kind;
    int n;
    const int* rowptr;
    const int* colind;
    const double* val;
    int nx, ny;
    double inv_h2;
    const double* ax;
    const double* ay;
};

// One row of y = scale * (A x).
__device__ __forceinline__ double op_row(const DevOp& op, const double* __restrict__ x, int i, double scale) {
    double s = 0.0;
    if (op.kind == SKR_OP_CSR) {
        const int e0 = op.rowptr[i], e1 = op.rowptr[i + 1];
        for (int e = e0; e < e1; ++e) s = fma(op.val[e], x[op.colind[e]], s);
    } else {
        const int nx = op.nx, ny = op.ny;
        const int r = i / nx, c = i - r * nx;
        const double aw = op.ax[r * (nx + 1) + c], ae = op.ax[r * (nx + 1) + c + 1];
        const double an = op.ay[r * nx + c], as = op.ay[(r + 1) * nx + c];
        s = (aw + ae + an + as) * x[i];
        if (c > 0) s = fma(-aw, x[i - 1], s);
        if (c < nx - 1) s = fma(-ae, x[i + 1], s);
        if (r > 0) s = fma(-an, x[i - nx], s);
        if (r < ny - 1) s = fma(-as, x[i + nx], s);
        s *= op.inv_h2;
    }
    return s * scale;
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
    int pad0;
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
    int stop, j_done, breakdown, kc, k_new, nonfinite, eig_fail, pad0;
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
constexpr int LDQC = KMAX + MMAX + 2;
constexpr int LDQU = KMAX + MMAX + 1;

// ---------------------------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Butterfly reduce-scatter over one wavefront: on return lane l holds the wave-wide sum of
// column l (v[0]). The order of additions is fixed, so results are bitwise reproducible. Each
// stage is a separate template instance so that every register index is a compile-time constant.
template <int HALF>
__device__ __forceinline__ void rs_stage(double (&v)[NC], int lane) {
    const bool upper = (lane & HALF) != 0;
#pragma unroll
    for (int i = 0; i < HALF; ++i) {
        const double send = upper ? v[i] : v[i + HALF];
        const double keep = upper ? v[i + HALF] : v[i];
        v[i] = keep + __shfl_xor(send, HALF, 64);
    }
}

__device__ __forceinline__ double wave_reduce_scatter64(double (&v)[NC]) {
    const int lane = lane_id();
    rs_stage<32>(v, lane);
    rs_stage<16>(v, lane);
    rs_stage<8>(v, lane);
    rs_stage<4>(v, lane);
    rs_stage<2>(v, lane);
    rs_stage<1>(v, lane);
    return v[0];
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
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

// Column sums over the per-workgroup partials part[b * NC + c] (b < nblk), fixed order:
// each wave sums a contiguous range of workgroups, then the waves are added in order.
// Must be called by all ROWS threads of the last workgroup; result in out[0..NC).
__device__ __forceinline__ void final_reduce64(const double* part, int nblk, double* sh, double* out) {
    const int lane = lane_id(), w = wave_id();
    const int per = (nblk + NWAVE - 1) / NWAVE;
    const int b0 = w * per, b1 = min(nblk, b0 + per);
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += __builtin_nontemporal_load(&part[b * NC + lane]);
    sh[w * NC + lane] = s;
    __syncthreads();
    if (threadIdx.x < NC) {
        double t = sh[lane];
#pragma unroll
        for (int q = 1; q < NWAVE; ++q) t += sh[q * NC + lane];
        out[lane] = t;
    }
    __syncthreads();
}

// Sum of one value per thread over the grid: partial per workgroup, fixed-order final sum in the
// last workgroup. Returns true in the last workgroup, where *result holds the total.
__device__ __forceinline__ bool grid_sum1(double v, double* part, unsigned* counter, int nblk, int lb,
                                          double* sh, double* result) {
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
    if (!last_block_arrive(counter, (unsigned)nblk)) return false;
    // fixed order: each lane sums a strided subset, then a fixed butterfly over the wave
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) s += __builtin_nontemporal_load(&part[b]);
        s = wave_sum(s);
        if (threadIdx.x == 0) sh[0] = s;
    }
    __syncthreads();
    *result = sh[0];
    __syncthreads();
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
    double* basis = nullptr;     // [C (k cols) | V (m+1 cols)], column-major, leading dim ld
    double* U = nullptr;         // k cols
    double* W[2] = {nullptr, nullptr};
    double* r = nullptr;
    double* part = nullptr;      // nblk * NC partials
    double* part1 = nullptr;     // nblk scalar partials
    double* gpart = nullptr;     // Gram partials: ngblk * gram_max
    double* gram = nullptr;      // reduced Gram result
    double* red1 = nullptr;      // NC
    double* red2 = nullptr;      // NC
    double* H = nullptr;         // LDH x MMAX
    double* Bm = nullptr;        // KMAX x MMAX
    Ctrl* ctrl = nullptr;
    Coef* coef = nullptr;
    unsigned* counters = nullptr;  // 8 counters
    size_t gram_max = 0;
    int ngblk = 0;
};

int gram_cols_max(int m, int k);

}  // namespace skr
