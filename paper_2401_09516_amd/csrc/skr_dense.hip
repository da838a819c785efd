// Small dense FP64 work of a GCRO-DR cycle end and of the start-up QR.
//
// Cycle end (Alg. 2, cycle body): with kc recycled columns and jd Arnoldi steps, d = kc + jd,
//   G = [[D_k, B], [0, Hbar]]             ((d+1) x d),   W-hat = [C, V_{jd+1}],  V-hat = [U D_k, V_jd]
//   y = argmin || W-hat^T r - G y ||,  x += V-hat y,  r -= W-hat G y
//   harmonic Ritz pairs  G^T G z = theta G^T (W-hat^T V-hat) z,  k smallest |theta|  ->  P_k
//   [Q, R] = qr(G P_k),  C <- W-hat Q,  U <- V-hat P_k R^{-1}
// Formulation used here (equal in exact arithmetic): Givens rotations give G = Q_G [R_G; 0];
// then the pencil is R_G z = theta X'' z with X'' the top d rows of Q_G^T (W-hat^T V-hat), so
// with w = R_G z the eigenvectors of M = X'' R_G^{-1} with the largest |mu| = 1/|theta| are
// wanted. G P_k = Q_G [W_sel; 0] with W_sel = R_G P_k, so if W_sel = Q_w R_w then
// Q = Q_G [Q_w; 0] and U_new = V-hat R_G^{-1} Q_w. The eigenproblem is solved by Householder
// reduction to Hessenberg form, the Francis double-shift QR iteration (real Schur form) and
// back-substitution for the selected eigenvectors.
#include "skr_internal.hpp"

namespace skr {

constexpr int LDG = DMAX + 1;   // leading dimension of G and X/M in LDS
constexpr int LDW = DMAX + 1;   // leading dimension of the eigenvector / Q_w / Qu work arrays

__device__ __forceinline__ double wave_sum64(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}
__device__ __forceinline__ double wave_max64(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

// Copy a rows x cols column-major block from global (leading dimension lds) to LDS (leading
// dimension ldd) with nthr threads, eight loads in flight per thread.
__device__ __forceinline__ void stage_block(double* dst, int ldd, const double* src, int lds, int rows, int cols,
                                            int t, int nthr) {
    const int total = rows * cols;
    for (int e0 = 0; e0 < total; e0 += 8 * nthr) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * nthr + t;
            v[u] = (e < total) ? src[(e % rows) + (e / rows) * lds] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * nthr + t;
            if (e < total) dst[(e % rows) + (e / rows) * ldd] = v[u];
        }
    }
}

// Householder reflector P = I - tau v v^T, v = (1, v1, v2), with P (x, y, z)^T = (alpha, 0, 0)^T.
__device__ __forceinline__ void house3(double x, double y, double z, double& v1, double& v2, double& tau,
                                       double& alpha) {
    const double sc = fabs(x) + fabs(y) + fabs(z);
    if (sc == 0.0) { v1 = v2 = tau = 0.0; alpha = 0.0; return; }
    x /= sc; y /= sc; z /= sc;
    const double sig = y * y + z * z;
    if (sig == 0.0) { v1 = v2 = tau = 0.0; alpha = x * sc; return; }
    const double mu = sqrt(x * x + sig);
    const double v0 = (x <= 0.0) ? x - mu : -sig / (x + mu);
    tau = 2.0 * v0 * v0 / (sig + v0 * v0);
    v1 = y / v0;
    v2 = z / v0;
    alpha = mu * sc;
}

// complex helpers
__device__ __forceinline__ void cdiv(double ar, double ai, double br, double bi, double& cr, double& ci) {
    if (fabs(br) >= fabs(bi)) {
        const double r = bi / br, den = br + bi * r;
        cr = (ar + ai * r) / den;
        ci = (ai - ar * r) / den;
    } else {
        const double r = br / bi, den = bi + br * r;
        cr = (ar * r + ai) / den;
        ci = (ai * r - ar) / den;
    }
}

// Stage 1 of a cycle end (one wavefront): G, X = W-hat^T V-hat, Givens QR of G, least-squares
// solution and the coefficients of the x and r updates. When a recycle space is to be formed, R_G,
// the top d rows of Q_G^T X, the rotations and D_k are handed to the eigen stage through dw.
__global__ __launch_bounds__(64) void k_dense_prep(const double* __restrict__ H, const double* __restrict__ Bm,
                                                   const double* __restrict__ gram, int kc, int jd_max, int k_target,
                                                   Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    __shared__ double G[LDG * DMAX];
    __shared__ double X[LDG * DMAX];
    __shared__ double rhs[DMAX + 1], gcs[DMAX], gsn[DMAX], Dk[KMAX], hv[DMAX + 1];
    const int t = threadIdx.x;
    const int jd = ctrl->j_done;
    const double beta = ctrl->beta;
    const int d = kc + jd;
    const int nr = kc + 1;

    // ---- D_k, G, X = W-hat^T V-hat (structured), right-hand side W-hat^T r. Global inputs are
    //      staged with eight loads in flight per lane.
    if (t < kc) Dk[t] = 1.0 / sqrt(gram[(kc + jd_max + 1 + t) * nr + t]);
    for (int c = 0; c < d; ++c)
        if (t <= d) {
            G[t + c * LDG] = 0.0;
            X[t + c * LDG] = (c >= kc && t == c) ? 1.0 : 0.0;   // V_{jd+1}^T V_jd = I_{jd+1,jd}, C^T V = 0
        }
    __syncthreads();
    {
        // Hbar (rows 0..jd, columns 0..jd-1, Hessenberg) -> G[kc + r][kc + c]
        const int nh = (jd + 1) * jd;
        for (int e0 = 0; e0 < nh; e0 += 64 * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + t, c = e / (jd + 1), r = e - c * (jd + 1);
                v[u] = (e < nh && r <= c + 1) ? H[r + c * LDH] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + t, c = e / (jd + 1), r = e - c * (jd + 1);
                if (e < nh) G[kc + r + (kc + c) * LDG] = v[u];
            }
        }
        // B (kc x jd) -> G[r][kc + c]
        const int nbm = kc * jd;
        for (int e0 = 0; e0 < nbm; e0 += 64 * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + t, c = e / max(kc, 1), r = e - c * kc;
                v[u] = (e < nbm) ? Bm[r + c * KMAX] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + t, c = e / max(kc, 1), r = e - c * kc;
                if (e < nbm) G[r + (kc + c) * LDG] = v[u];
            }
        }
        __syncthreads();
        // [C V]^T U (rows 0..d, columns 0..kc-1) -> X[r][c] D_c;  D_k -> G[c][c]
        const int ng = (d + 1) * kc;
        for (int e0 = 0; e0 < ng; e0 += 64 * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + t, c = e / (d + 1), r = e - c * (d + 1);
                v[u] = (e < ng) ? gram[r * nr + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + t, c = e / (d + 1), r = e - c * (d + 1);
                if (e < ng) X[r + c * LDG] = v[u] * Dk[c];
            }
        }
        if (t < kc) G[t + t * LDG] = Dk[t];
    }
    if (t <= d) rhs[t] = (t < kc) ? gram[t * nr + kc] : (t == kc ? beta : 0.0);
    __syncthreads();

    // ---- Givens QR of G (the Hessenberg block only; the D_k block is already triangular)
    for (int c = kc; c < d; ++c) {
        const double a = G[c + c * LDG], b = G[c + 1 + c * LDG];
        const double rho = hypot(a, b);
        const double cs = rho > 0.0 ? a / rho : 1.0, sn = rho > 0.0 ? b / rho : 0.0;
        if (t >= c && t < d) {
            const double g0 = G[c + t * LDG], g1 = G[c + 1 + t * LDG];
            G[c + t * LDG] = cs * g0 + sn * g1;
            G[c + 1 + t * LDG] = -sn * g0 + cs * g1;
        }
        if (t < d) {
            const double x0 = X[c + t * LDG], x1 = X[c + 1 + t * LDG];
            X[c + t * LDG] = cs * x0 + sn * x1;
            X[c + 1 + t * LDG] = -sn * x0 + cs * x1;
        }
        if (t == 0) {
            const double r0 = rhs[c], r1 = rhs[c + 1];
            rhs[c] = cs * r0 + sn * r1;
            rhs[c + 1] = -sn * r0 + cs * r1;
            gcs[c] = cs;
            gsn[c] = sn;
        }
        __syncthreads();
        if (t == 0) G[c + 1 + c * LDG] = 0.0;
        __syncthreads();
    }

    // ---- least squares: y = R_G^{-1} rhs[0:d]
    double yv = (t < d) ? rhs[t] : 0.0;
    for (int c = d - 1; c >= 0; --c) {
        const double yc = __shfl(yv, c, 64) / G[c + c * LDG];
        if (t == c) yv = yc;
        if (t < c) yv = fma(-G[t + c * LDG], yc, yv);
    }
    if (t < kc) coef->yU[t] = Dk[t] * yv;
    if (t >= kc && t < d) coef->yV[t - kc] = yv;
    // G y = Q_G [rhs[0:d]; 0]
    if (t <= d) hv[t] = (t < d) ? rhs[t] : 0.0;
    __syncthreads();
    if (t == 0) {
        for (int c = d - 1; c >= kc; --c) {
            const double a = hv[c], b = hv[c + 1];
            hv[c] = gcs[c] * a - gsn[c] * b;
            hv[c + 1] = gsn[c] * a + gcs[c] * b;
        }
    }
    __syncthreads();
    if (t < kc) coef->rC[t] = hv[t];
    if (t >= kc && t <= d) coef->rV[t - kc] = hv[t];

    const bool recycle = k_target > 0 && (kc > 0 || jd > k_target);
    if (!recycle) {
        if (t == 0) { ctrl->k_new = 0; ctrl->eig_fail = 0; dw->mode = DW_NONE; }
        return;
    }
    // hand over R_G (d x d, upper), X'' (d x d), rotations and D_k
    for (int c = 0; c < d; ++c)
        if (t < d) {
            dw->R[t + c * DMAX] = (t <= c) ? G[t + c * LDG] : 0.0;
            dw->X[t + c * DMAX] = X[t + c * LDG];
        }
    if (t < d) { dw->gcs[t] = gcs[t]; dw->gsn[t] = gsn[t]; }
    if (t < kc) dw->Dk[t] = Dk[t];
    if (t == 0) { dw->d = d; dw->kc = kc; dw->mode = DW_PENDING; }
}

// Stage 2, symmetric case (4 wavefronts). M = X'' R_G^{-1} is formed; for symmetric A it is
// symmetric in exact arithmetic (G^T G and G^T W-hat^T V-hat = V-hat^T A V-hat are), and when the
// computed M is symmetric to 1e-10 relative, the eigenpairs of (M + M^T)/2 are found by the cyclic
// Jacobi method (round-robin ordering: each round rotates d/2 disjoint pairs in parallel). Its
// eigenvectors are orthonormal, so the selected ones form Q_w directly. Otherwise M is handed to
// the general stage.
constexpr int DT = 256;         // threads of the symmetric stage
constexpr int LDS_ = DMAX + 1;  // leading dimension of S and V in LDS

__global__ __launch_bounds__(DT) void k_dense_sym(int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    if (dw->mode != DW_PENDING) return;
    __shared__ double S[LDS_ * DMAX];
    __shared__ double V[LDS_ * DMAX];
    __shared__ double R[LDS_ * DMAX];
    __shared__ double Wq[LDS_ * KMAX];
    __shared__ double gcs[DMAX], gsn[DMAX], Dk[KMAX];
    __shared__ double red[DT / 64], red2[DT / 64];
    __shared__ double jc[DMAX / 2], js[DMAX / 2];
    __shared__ int jp[DMAX / 2], jq[DMAX / 2];
    __shared__ int sel[KMAX];
    __shared__ int nsel_s, sym_s;
    const int t = threadIdx.x;
    const int d = dw->d, kc = dw->kc;
    const int dp = d + (d & 1);                 // even size (a zero row/column pads an odd d)
    // load R_G, X'', the rotations of Q_G and D_k
    stage_block(R, LDS_, dw->R, DMAX, d, d, t, DT);
    stage_block(S, LDS_, dw->X, DMAX, d, d, t, DT);
    if (t < d) { gcs[t] = dw->gcs[t]; gsn[t] = dw->gsn[t]; }
    if (t < kc) Dk[t] = dw->Dk[t];
    __syncthreads();
    // M = X'' R^{-1}: column c of M = (X''_c - sum_{q<c} M_q R_qc) / R_cc, right-looking over c
    for (int c = 0; c < d; ++c) {
        const double inv = 1.0 / R[c + c * LDS_];
        for (int r = t; r < d; r += DT) S[r + c * LDS_] *= inv;
        __syncthreads();
        for (int e = t; e < d * (d - c - 1); e += DT) {
            const int r = e % d, c2 = c + 1 + e / d;
            S[r + c2 * LDS_] = fma(-S[r + c * LDS_], R[c + c2 * LDS_], S[r + c2 * LDS_]);
        }
        __syncthreads();
    }
    // symmetry test: max |M - M^T| <= 1e-10 max |M|
    double amax = 0.0, dmax = 0.0;
    for (int e = t; e < d * d; e += DT) {
        const int r = e % d, c = e / d;
        const double a = S[r + c * LDS_];
        amax = fmax(amax, fabs(a));
        dmax = fmax(dmax, fabs(a - S[c + r * LDS_]));
    }
    amax = wave_max64(amax);
    dmax = wave_max64(dmax);
    if ((t & 63) == 0) { red[t >> 6] = amax; red2[t >> 6] = dmax; }
    __syncthreads();
    if (t == 0) {
        double ga = red[0], gd = red2[0];
        for (int q = 1; q < DT / 64; ++q) { ga = fmax(ga, red[q]); gd = fmax(gd, red2[q]); }
        sym_s = (gd <= 1e-10 * ga) ? 1 : 0;
    }
    __syncthreads();
    if (!sym_s) {
        for (int e = t; e < d * d; e += DT) {
            const int r = e % d, c = e / d;
            dw->X[r + c * DMAX] = S[r + c * LDS_];
        }
        if (t == 0) dw->mode = DW_GEN;
        return;
    }
    // S = (M + M^T) / 2 in place (each unordered pair by one thread), padded to dp; V = I
    for (int e = t; e < dp * dp; e += DT) {
        const int r = e % dp, c = e / dp;
        V[r + c * LDS_] = (r == c) ? 1.0 : 0.0;
        if (r < c) {
            const double v = (c < d) ? 0.5 * (S[r + c * LDS_] + S[c + r * LDS_]) : 0.0;
            S[r + c * LDS_] = v;
            S[c + r * LDS_] = v;
        } else if (r == c && c >= d) {
            S[r + c * LDS_] = 0.0;
        }
    }
    __syncthreads();
    // cyclic Jacobi sweeps until off(S) <= 1e-13 ||diag(S)|| (a rotation is skipped when
    // |S_pq| <= 1e-16 sqrt(|S_pp S_qq|)). Thread t works on pair t >> 3 and every 8th row/column
    // starting at t & 7.
    const int np = dp / 2;
    const int my_pair = t >> 3, my_g = t & 7;
    for (int sweep = 0; sweep < 20; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int c = my_pair; c < dp; c += DT / 8)
            for (int r = my_g; r < dp; r += 8) {
                const double a = S[r + c * LDS_];
                if (r != c) off = fma(a, a, off);
                else dia = fma(a, a, dia);
            }
        off = wave_sum64(off);
        dia = wave_sum64(dia);
        if ((t & 63) == 0) { red[t >> 6] = off; red2[t >> 6] = dia; }
        __syncthreads();
        double offt = 0.0, diat = 0.0;
        for (int q = 0; q < DT / 64; ++q) { offt += red[q]; diat += red2[q]; }
        __syncthreads();
        if (!(offt > 1e-26 * diat)) break;
        for (int round = 0; round < dp - 1; ++round) {
            if (t < np) {
                // circle method: position 0 fixed, the others rotate
                const int a = t, b = dp - 1 - t;
                const int pa = (a == 0) ? 0 : 1 + (a - 1 + round) % (dp - 1);
                const int pb = (b == 0) ? 0 : 1 + (b - 1 + round) % (dp - 1);
                const int p = min(pa, pb), q = max(pa, pb);
                const double spq = S[p + q * LDS_], spp = S[p + p * LDS_], sqq = S[q + q * LDS_];
                double c = 1.0, s = 0.0;
                if (fabs(spq) > 1e-16 * sqrt(fabs(spp * sqq))) {
                    const double tau = (sqq - spp) / (2.0 * spq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                jp[t] = p; jq[t] = q; jc[t] = c; js[t] = s;
            }
            __syncthreads();
            if (my_pair < np && js[my_pair] != 0.0) {
                const int p = jp[my_pair], q = jq[my_pair];
                const double c = jc[my_pair], s = js[my_pair];
                // rows: S <- J^T S
                for (int col = my_g; col < dp; col += 8) {
                    const double sp = S[p + col * LDS_], sq = S[q + col * LDS_];
                    S[p + col * LDS_] = c * sp - s * sq;
                    S[q + col * LDS_] = s * sp + c * sq;
                }
            }
            __syncthreads();
            if (my_pair < np && js[my_pair] != 0.0) {
                const int p = jp[my_pair], q = jq[my_pair];
                const double c = jc[my_pair], s = js[my_pair];
                // columns: S <- S J, V <- V J
                for (int row = my_g; row < dp; row += 8) {
                    const double sp = S[row + p * LDS_], sq = S[row + q * LDS_];
                    S[row + p * LDS_] = c * sp - s * sq;
                    S[row + q * LDS_] = s * sp + c * sq;
                    const double vp = V[row + p * LDS_], vq = V[row + q * LDS_];
                    V[row + p * LDS_] = c * vp - s * vq;
                    V[row + q * LDS_] = s * vp + c * vq;
                }
            }
            __syncthreads();
        }
    }
    // select the k_target eigenvalues of largest |mu| (smallest |theta| = 1/|mu|), ties by index
    if (t < 64) {
        int ns = 0;
        unsigned long long used = 0ull;
        for (int it = 0; it < k_target; ++it) {
            double key = -1.0;
            int idx = t;
            if (t < d && !((used >> t) & 1ull)) {
                const double mag = fabs(S[t + t * LDS_]);
                if (mag > 0.0) key = mag;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ok = __shfl_xor(key, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (ok > key || (ok == key && oi < idx)) { key = ok; idx = oi; }
            }
            if (key <= 0.0) break;
            used |= 1ull << idx;
            if (t == 0) sel[ns] = idx;
            ++ns;
        }
        if (t == 0) nsel_s = ns;
    }
    __syncthreads();
    const int kn = nsel_s;
    // Qu = R_G^{-1} Q_w with Q_w = V[:, sel]: back-substitution, parallel over (row, column)
    for (int e = t; e < d * kn; e += DT) {
        const int r = e % d, o = e / d;
        Wq[r + o * LDS_] = V[r + sel[o] * LDS_];
    }
    __syncthreads();
    for (int c = d - 1; c >= 0; --c) {
        const double rcc = R[c + c * LDS_];
        for (int o = t; o < kn; o += DT) Wq[c + o * LDS_] /= rcc;
        __syncthreads();
        for (int e = t; e < c * kn; e += DT) {
            const int r = e % c, o = e / c;
            Wq[r + o * LDS_] = fma(-R[r + c * LDS_], Wq[c + o * LDS_], Wq[r + o * LDS_]);
        }
        __syncthreads();
    }
    for (int e = t; e < d * kn; e += DT) {
        const int r = e % d, o = e / d;
        coef->Qu[r + o * LDQU] = (r < kc ? Dk[r] : 1.0) * Wq[r + o * LDS_];
    }
    // Qc = Q_G [Q_w; 0] (one thread per column, rotations in reverse order)
    if (t < kn) {
        const int o = t, col = sel[o];
        double carry = 0.0;
        for (int c = d - 1; c >= kc; --c) {
            const double a = V[c + col * LDS_];
            coef->Qc[c + 1 + o * LDQC] = gsn[c] * a + gcs[c] * carry;
            carry = gcs[c] * a - gsn[c] * carry;
        }
        coef->Qc[kc + o * LDQC] = carry;
        for (int c = 0; c < kc; ++c) coef->Qc[c + o * LDQC] = V[c + col * LDS_];
    }
    if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 0; dw->mode = DW_DONE; }
}

// Stage 2, general (nonsymmetric) case, one wavefront: M = X'' R_G^{-1} was formed by the
// symmetric stage, which found it nonsymmetric. Householder reduction to Hessenberg form, Francis
// double-shift QR, eigenvectors of the selected eigenvalues by back-substitution, an orthonormal
// basis Q_w of them, and the recycle-space coefficients Qu = R_G^{-1} Q_w, Qc = Q_G [Q_w; 0].
__global__ __launch_bounds__(64) void k_dense_gen(int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    if (dw->mode != DW_GEN) return;
    __shared__ double G[LDG * DMAX];
    __shared__ double X[LDG * DMAX];
    __shared__ double Z[DMAX * DMAX];
    __shared__ double Wv[LDW * KMAX];
    __shared__ double Uq[LDW * KMAX];
    __shared__ double gcs[DMAX], gsn[DMAX], Dk[KMAX], wr[DMAX], wi[DMAX], hv[DMAX + 1];
    __shared__ int taken[DMAX], sel_pos[KMAX], sel_cplx[KMAX], sel_col[KMAX];
    const int t = threadIdx.x;
    const int d = dw->d, kc = dw->kc;
    const double eps = 2.220446049250313e-16;
    stage_block(G, LDG, dw->R, DMAX, d, d, t, 64);
    stage_block(X, LDG, dw->X, DMAX, d, d, t, 64);
    if (t < d) { gcs[t] = dw->gcs[t]; gsn[t] = dw->gsn[t]; }
    if (t < kc) Dk[t] = dw->Dk[t];
    __syncthreads();
    // Z = I
    for (int c = 0; c < d; ++c)
        if (t < d) Z[t + c * DMAX] = (t == c) ? 1.0 : 0.0;
    __syncthreads();

    // ---- Householder reduction of M to upper Hessenberg form, Z accumulates the reflectors
    for (int c = 0; c + 2 < d; ++c) {
        const double xr = (t >= c + 1 && t < d) ? X[t + c * LDG] : 0.0;
        const double sig = wave_sum64((t >= c + 2 && t < d) ? xr * xr : 0.0);
        const double x0 = X[c + 1 + c * LDG];
        if (sig == 0.0) continue;
        const double mu = sqrt(x0 * x0 + sig);
        const double v0 = (x0 <= 0.0) ? x0 - mu : -sig / (x0 + mu);
        const double tau = 2.0 * v0 * v0 / (sig + v0 * v0);
        if (t >= c + 1 && t < d) hv[t] = (t == c + 1) ? 1.0 : xr / v0;
        __syncthreads();
        if (t >= c && t < d) {
            double s = 0.0;
            for (int r = c + 1; r < d; ++r) s = fma(hv[r], X[r + t * LDG], s);
            s *= tau;
            for (int r = c + 1; r < d; ++r) X[r + t * LDG] = fma(-s, hv[r], X[r + t * LDG]);
        }
        __syncthreads();
        if (t < d) {
            double s = 0.0, sz = 0.0;
            for (int q = c + 1; q < d; ++q) {
                s = fma(X[t + q * LDG], hv[q], s);
                sz = fma(Z[t + q * DMAX], hv[q], sz);
            }
            s *= tau;
            sz *= tau;
            for (int q = c + 1; q < d; ++q) {
                X[t + q * LDG] = fma(-s, hv[q], X[t + q * LDG]);
                Z[t + q * DMAX] = fma(-sz, hv[q], Z[t + q * DMAX]);
            }
        }
        __syncthreads();
        if (t >= c + 2 && t < d) X[t + c * LDG] = 0.0;
        if (t == 0) X[c + 1 + c * LDG] = mu;
        __syncthreads();
    }

    // ---- Francis double-shift QR to real Schur form (T in X, Z accumulated)
    double tnorm = 0.0;
    if (t < d)
        for (int c = 0; c < d; ++c) tnorm = fmax(tnorm, fabs(X[t + c * LDG]));
    tnorm = wave_max64(tnorm);
    int hi = d - 1, its = 0, total = 0;
    bool failed = false;
    while (hi >= 0) {
        bool small = false;
        if (t >= 1 && t <= hi) {
            double sc = fabs(X[t - 1 + (t - 1) * LDG]) + fabs(X[t + t * LDG]);
            if (sc == 0.0) sc = tnorm;
            small = fabs(X[t + (t - 1) * LDG]) <= eps * sc;
        }
        const unsigned long long mask = __ballot(small);
        const int l = mask ? 63 - __clzll(mask) : 0;
        __syncthreads();
        if (l > 0 && t == 0) X[l + (l - 1) * LDG] = 0.0;
        __syncthreads();
        if (l == hi) {
            if (t == 0) { wr[hi] = X[hi + hi * LDG]; wi[hi] = 0.0; }
            hi -= 1;
            its = 0;
            __syncthreads();
            continue;
        }
        if (l == hi - 1) {
            const int p = hi - 1, q = hi;
            const double a = X[p + p * LDG], b = X[p + q * LDG], c = X[q + p * LDG], dd = X[q + q * LDG];
            const double pp = 0.5 * (a - dd), bc = b * c, disc = pp * pp + bc;
            if (disc >= 0.0) {
                const double zz = pp + copysign(sqrt(disc), pp);
                const double rho = hypot(zz, c);
                const double cs = rho > 0.0 ? zz / rho : 1.0, sn = rho > 0.0 ? c / rho : 0.0;
                __syncthreads();
                if (t >= p && t < d) {
                    const double r0 = X[p + t * LDG], r1 = X[q + t * LDG];
                    X[p + t * LDG] = cs * r0 + sn * r1;
                    X[q + t * LDG] = -sn * r0 + cs * r1;
                }
                __syncthreads();
                if (t <= q) {
                    const double c0 = X[t + p * LDG], c1 = X[t + q * LDG];
                    X[t + p * LDG] = cs * c0 + sn * c1;
                    X[t + q * LDG] = -sn * c0 + cs * c1;
                }
                if (t < d) {
                    const double z0 = Z[t + p * DMAX], z1 = Z[t + q * DMAX];
                    Z[t + p * DMAX] = cs * z0 + sn * z1;
                    Z[t + q * DMAX] = -sn * z0 + cs * z1;
                }
                __syncthreads();
                if (t == 0) {
                    X[q + p * LDG] = 0.0;
                    wr[p] = X[p + p * LDG];
                    wr[q] = X[q + q * LDG];
                    wi[p] = 0.0;
                    wi[q] = 0.0;
                }
            } else {
                if (t == 0) {
                    wr[p] = wr[q] = dd + pp;
                    wi[p] = sqrt(-disc);
                    wi[q] = -wi[p];
                }
            }
            hi -= 2;
            its = 0;
            __syncthreads();
            continue;
        }
        if (total >= 30 * d) { failed = true; break; }
        ++its;
        ++total;
        double h11, h12, h21, h22;
        if (its == 10) {
            const double s = fabs(X[l + 1 + l * LDG]) + fabs(X[l + 2 + (l + 1) * LDG]);
            h11 = 0.75 * s + X[l + l * LDG]; h12 = -0.4375 * s; h21 = s; h22 = h11;
        } else if (its == 20) {
            const double s = fabs(X[hi + (hi - 1) * LDG]) + fabs(X[hi - 1 + (hi - 2) * LDG]);
            h11 = 0.75 * s + X[hi + hi * LDG]; h12 = -0.4375 * s; h21 = s; h22 = h11;
        } else {
            h11 = X[hi - 1 + (hi - 1) * LDG]; h12 = X[hi - 1 + hi * LDG];
            h21 = X[hi + (hi - 1) * LDG]; h22 = X[hi + hi * LDG];
        }
        const double str = h11 + h22, sdet = h11 * h22 - h12 * h21;
        const double a00 = X[l + l * LDG], a01 = X[l + (l + 1) * LDG];
        const double a10 = X[l + 1 + l * LDG], a11 = X[l + 1 + (l + 1) * LDG], a21 = X[l + 2 + (l + 1) * LDG];
        double px = a00 * a00 + a01 * a10 - str * a00 + sdet;
        double py = a10 * (a00 + a11 - str);
        double pz = a10 * a21;
        for (int kk = l; kk <= hi - 2; ++kk) {
            double v1, v2, tau, alpha;
            house3(px, py, pz, v1, v2, tau, alpha);
            __syncthreads();
            if (tau != 0.0) {
                const int c0 = (kk > l) ? kk - 1 : l;
                if (t >= c0 && t < d) {
                    const double a = X[kk + t * LDG], b = X[kk + 1 + t * LDG], c = X[kk + 2 + t * LDG];
                    const double s = tau * (a + v1 * b + v2 * c);
                    X[kk + t * LDG] = a - s;
                    X[kk + 1 + t * LDG] = b - s * v1;
                    X[kk + 2 + t * LDG] = c - s * v2;
                }
                __syncthreads();
                const int r1 = min(kk + 3, hi);
                if (t <= r1) {
                    const double a = X[t + kk * LDG], b = X[t + (kk + 1) * LDG], c = X[t + (kk + 2) * LDG];
                    const double s = tau * (a + v1 * b + v2 * c);
                    X[t + kk * LDG] = a - s;
                    X[t + (kk + 1) * LDG] = b - s * v1;
                    X[t + (kk + 2) * LDG] = c - s * v2;
                }
                if (t < d) {
                    const double a = Z[t + kk * DMAX], b = Z[t + (kk + 1) * DMAX], c = Z[t + (kk + 2) * DMAX];
                    const double s = tau * (a + v1 * b + v2 * c);
                    Z[t + kk * DMAX] = a - s;
                    Z[t + (kk + 1) * DMAX] = b - s * v1;
                    Z[t + (kk + 2) * DMAX] = c - s * v2;
                }
                __syncthreads();
            }
            if (kk > l && t == 0) {
                X[kk + (kk - 1) * LDG] = alpha;
                X[kk + 1 + (kk - 1) * LDG] = 0.0;
                X[kk + 2 + (kk - 1) * LDG] = 0.0;
            }
            __syncthreads();
            px = X[kk + 1 + kk * LDG];
            py = X[kk + 2 + kk * LDG];
            pz = (kk < hi - 2) ? X[kk + 3 + kk * LDG] : 0.0;
        }
        // closing 2-element reflector on rows/columns hi-1, hi
        {
            const int kk = hi - 1;
            double v1, v2, tau, alpha;
            house3(px, py, 0.0, v1, v2, tau, alpha);
            __syncthreads();
            if (tau != 0.0) {
                const int c0 = kk - 1;
                if (t >= c0 && t < d) {
                    const double a = X[kk + t * LDG], b = X[kk + 1 + t * LDG];
                    const double s = tau * (a + v1 * b);
                    X[kk + t * LDG] = a - s;
                    X[kk + 1 + t * LDG] = b - s * v1;
                }
                __syncthreads();
                if (t <= hi) {
                    const double a = X[t + kk * LDG], b = X[t + (kk + 1) * LDG];
                    const double s = tau * (a + v1 * b);
                    X[t + kk * LDG] = a - s;
                    X[t + (kk + 1) * LDG] = b - s * v1;
                }
                if (t < d) {
                    const double a = Z[t + kk * DMAX], b = Z[t + (kk + 1) * DMAX];
                    const double s = tau * (a + v1 * b);
                    Z[t + kk * DMAX] = a - s;
                    Z[t + (kk + 1) * DMAX] = b - s * v1;
                }
                __syncthreads();
            }
            if (t == 0) {
                X[kk + (kk - 1) * LDG] = alpha;
                X[kk + 1 + (kk - 1) * LDG] = 0.0;
            }
            __syncthreads();
        }
    }

    if (failed) {
        // keep the current recycle space: C_new = C, U_new = U
        const int kn = kc;
        for (int o = 0; o < kn; ++o)
            for (int r = t; r <= d; r += 64) {
                coef->Qc[r + o * LDQC] = (r == o) ? 1.0 : 0.0;
                if (r < d) coef->Qu[r + o * LDQU] = (r == o) ? 1.0 : 0.0;
            }
        if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 1; dw->mode = DW_DONE; }
        return;
    }

    // ---- select the k eigenvalues of largest |mu| (smallest |theta|); a conjugate pair counts two
    if (t < d) taken[t] = 0;
    __syncthreads();
    int nsel = 0, ncols = 0;
    while (ncols < k_target) {
        double key = -1.0;
        if (t < d && !taken[t] && wi[t] >= 0.0) {
            const double mag = hypot(wr[t], wi[t]);
            if (mag > 0.0) key = mag;
        }
        int idx = t;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ok = __shfl_xor(key, off, 64);
            const int oi = __shfl_xor(idx, off, 64);
            if (ok > key || (ok == key && oi < idx)) { key = ok; idx = oi; }
        }
        if (key <= 0.0) break;
        const int cplx = wi[idx] > 0.0 ? 1 : 0;
        if (ncols + 1 + cplx > k_target) break;
        if (t == 0) {
            sel_pos[nsel] = idx;
            sel_cplx[nsel] = cplx;
            sel_col[nsel] = ncols;
            taken[idx] = 1;
        }
        __syncthreads();
        ++nsel;
        ncols += 1 + cplx;
    }
    __syncthreads();

    // ---- eigenvectors of the quasi-triangular T by back-substitution (one lane per selection),
    //      written to Wv in the Schur basis
    const double smin = fmax(eps * tnorm, 1e-290);
    if (t < nsel) {
        const int p = sel_pos[t], col = sel_col[t];
        double* xr = Wv + col * LDW;
        if (!sel_cplx[t]) {
            const double lam = wr[p];
            for (int r = 0; r < d; ++r) xr[r] = 0.0;
            xr[p] = 1.0;
            int r = p - 1;
            while (r >= 0) {
                if (r > 0 && X[r + (r - 1) * LDG] != 0.0) {
                    double s1 = 0.0, s2 = 0.0;
                    for (int c = r + 1; c <= p; ++c) {
                        s1 = fma(X[r - 1 + c * LDG], xr[c], s1);
                        s2 = fma(X[r + c * LDG], xr[c], s2);
                    }
                    const double a = X[r - 1 + (r - 1) * LDG] - lam, b = X[r - 1 + r * LDG];
                    const double c = X[r + (r - 1) * LDG], dd = X[r + r * LDG] - lam;
                    double det = a * dd - b * c;
                    if (fabs(det) < smin * smin) det = copysign(smin * smin, det);
                    xr[r - 1] = (-s1 * dd + b * s2) / det;
                    xr[r] = (-a * s2 + c * s1) / det;
                    r -= 2;
                } else {
                    double s = 0.0;
                    for (int c = r + 1; c <= p; ++c) s = fma(X[r + c * LDG], xr[c], s);
                    double den = X[r + r * LDG] - lam;
                    if (fabs(den) < smin) den = copysign(smin, den);
                    xr[r] = -s / den;
                    r -= 1;
                }
            }
        } else {
            // pair at (p, p+1), lambda = wr + i wi: x_p = lambda - T_{p+1,p+1}, x_{p+1} = T_{p+1,p}
            const double lr = wr[p], li = wi[p];
            double* xi = Wv + (col + 1) * LDW;
            for (int r = 0; r < d; ++r) { xr[r] = 0.0; xi[r] = 0.0; }
            xr[p] = lr - X[p + 1 + (p + 1) * LDG];
            xi[p] = li;
            xr[p + 1] = X[p + 1 + p * LDG];
            xi[p + 1] = 0.0;
            int r = p - 1;
            while (r >= 0) {
                if (r > 0 && X[r + (r - 1) * LDG] != 0.0) {
                    double s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
                    for (int c = r + 1; c <= p + 1; ++c) {
                        s1r = fma(X[r - 1 + c * LDG], xr[c], s1r);
                        s1i = fma(X[r - 1 + c * LDG], xi[c], s1i);
                        s2r = fma(X[r + c * LDG], xr[c], s2r);
                        s2i = fma(X[r + c * LDG], xi[c], s2i);
                    }
                    // [[a - lam, b], [c, dd - lam]] [x1; x2] = -[s1; s2]
                    const double ar = X[r - 1 + (r - 1) * LDG] - lr, ai = -li;
                    const double b = X[r - 1 + r * LDG], c = X[r + (r - 1) * LDG];
                    const double dr = X[r + r * LDG] - lr, di = -li;
                    double detr = ar * dr - ai * di - b * c, deti = ar * di + ai * dr;
                    if (fabs(detr) + fabs(deti) < smin * smin) detr = smin * smin;
                    // x1 = (-s1 * (dd - lam) + b * s2) / det ; x2 = (-(a - lam) * s2 + c * s1) / det
                    const double n1r = -(s1r * dr - s1i * di) + b * s2r, n1i = -(s1r * di + s1i * dr) + b * s2i;
                    const double n2r = -(ar * s2r - ai * s2i) + c * s1r, n2i = -(ar * s2i + ai * s2r) + c * s1i;
                    cdiv(n1r, n1i, detr, deti, xr[r - 1], xi[r - 1]);
                    cdiv(n2r, n2i, detr, deti, xr[r], xi[r]);
                    r -= 2;
                } else {
                    double sr = 0.0, si = 0.0;
                    for (int c = r + 1; c <= p + 1; ++c) {
                        sr = fma(X[r + c * LDG], xr[c], sr);
                        si = fma(X[r + c * LDG], xi[c], si);
                    }
                    double denr = X[r + r * LDG] - lr, deni = -li;
                    if (fabs(denr) + fabs(deni) < smin) denr = smin;
                    cdiv(-sr, -si, denr, deni, xr[r], xi[r]);
                    r -= 1;
                }
            }
        }
    }
    __syncthreads();
    // back to the basis of M: w = Z x (lane = row), into Uq
    for (int o = 0; o < ncols; ++o) {
        if (t < d) {
            double s = 0.0;
            for (int c = 0; c < d; ++c) s = fma(Z[t + c * DMAX], Wv[c + o * LDW], s);
            Uq[t + o * LDW] = s;
        }
    }
    __syncthreads();

    // ---- orthonormal basis Q_w of the selected vectors (modified Gram-Schmidt, two passes)
    int kn = 0;
    for (int o = 0; o < ncols; ++o) {
        double w = (t < d) ? Uq[t + o * LDW] : 0.0;
        const double n0 = sqrt(wave_sum64(w * w));
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < kn; ++q) {
                const double qv = (t < d) ? Wv[t + q * LDW] : 0.0;
                const double h = wave_sum64(qv * w);
                w = fma(-h, qv, w);
            }
        const double nw = sqrt(wave_sum64(w * w));
        __syncthreads();
        if (nw > 1e-12 * n0 && n0 > 0.0) {
            if (t < d) Wv[t + kn * LDW] = w / nw;
            ++kn;
        }
        __syncthreads();
    }

    // ---- Qu = R_G^{-1} Q_w with D_k folded into the rows of U (lane = column)
    if (t < kn) {
        double* u = Uq + t * LDW;
        for (int r = d - 1; r >= 0; --r) {
            double s = Wv[r + t * LDW];
            for (int c = r + 1; c < d; ++c) s = fma(-G[r + c * LDG], u[c], s);
            u[r] = s / G[r + r * LDG];
        }
        for (int r = 0; r < d; ++r) coef->Qu[r + t * LDQU] = (r < kc ? Dk[r] : 1.0) * u[r];
        // Qc = Q_G [Q_w; 0]
        double carry = 0.0;
        for (int c = d - 1; c >= kc; --c) {
            const double a = Wv[c + t * LDW];
            coef->Qc[c + 1 + t * LDQC] = gsn[c] * a + gcs[c] * carry;
            carry = gcs[c] * a - gsn[c] * carry;
        }
        if (kc < d || d == 0) coef->Qc[kc + t * LDQC] = carry;
        for (int c = 0; c < kc; ++c) coef->Qc[c + t * LDQC] = Wv[c + t * LDW];
    }
    if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 0; dw->mode = DW_DONE; }
}

// ---------------------------------------------------------------------------------------------
// Start-up CholQR: Cholesky of the Gram matrix Z^T Z (kin x kin, row-major in gram). With drops,
// a column whose pivot falls to <= 1e-14 ||z_j||^2 (R_jj <= 1e-7 ||z_j||) is left out.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_chol(const double* __restrict__ gram, int kin, int with_drop, Coef* coef) {
    __shared__ double A[KMAX * KMAX];
    __shared__ double Rf[KMAX * KMAX];
    __shared__ double d0[KMAX];
    __shared__ int keep[KMAX];
    __shared__ int pos[KMAX];
    const int t = threadIdx.x;
    for (int e = t; e < KMAX * KMAX; e += 64) {
        const int r = e % KMAX, c = e / KMAX;
        A[e] = (r < kin && c < kin) ? gram[r * kin + c] : 0.0;
        Rf[e] = 0.0;
    }
    __syncthreads();
    if (t < kin) d0[t] = A[t + t * KMAX];
    __syncthreads();
    int ke = 0;
    for (int j = 0; j < kin; ++j) {
        double piv = A[j + j * KMAX];
        const bool drop = with_drop ? !(piv > 1e-14 * d0[j]) : false;
        if (!with_drop && !(piv > 0.0)) piv = 1e-300;
        __syncthreads();
        if (drop) continue;
        const double rjj = sqrt(piv);
        if (t == 0) { keep[ke] = j; pos[j] = ke; Rf[j + j * KMAX] = rjj; }
        if (t > j && t < kin) Rf[j + t * KMAX] = A[j + t * KMAX] / rjj;
        __syncthreads();
        if (t > j && t < kin) {
            const double rt = Rf[j + t * KMAX];
            for (int c = j + 1; c < kin; ++c) A[c + t * KMAX] = fma(-Rf[j + c * KMAX], rt, A[c + t * KMAX]);
        }
        __syncthreads();
        ++ke;
    }
    // compact R to the kept columns (upper triangular, ld KMAX)
    double* Rout = with_drop ? coef->R : coef->R2;
    for (int e = t; e < KMAX * KMAX; e += 64) {
        const int r = e % KMAX, c = e / KMAX;
        Rout[e] = (r < ke && c < ke) ? Rf[keep[r] + keep[c] * KMAX] : 0.0;
    }
    if (with_drop) {
        if (t < KMAX) coef->keep[t] = t < ke ? keep[t] : 0;
        if (t == 0) coef->k_eff = ke;
    }
}

void launch_cycle_dense(hipStream_t s, const Work& w, int kc, int jd_max, int k_target) {
    hipLaunchKernelGGL(k_dense_prep, dim3(1), dim3(64), 0, s, (const double*)w.H, (const double*)w.Bm,
                       (const double*)w.gram, kc, jd_max, k_target, w.coef, w.dense, w.ctrl);
    if (k_target > 0) {
        hipLaunchKernelGGL(k_dense_sym, dim3(1), dim3(DT), 0, s, k_target, w.coef, w.dense, w.ctrl);
        hipLaunchKernelGGL(k_dense_gen, dim3(1), dim3(64), 0, s, k_target, w.coef, w.dense, w.ctrl);
    }
}
void launch_chol(hipStream_t s, const Work& w, int kin, int with_drop) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(64), 0, s, (const double*)w.gram, kin, with_drop, w.coef);
}

}  // namespace skr
