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

constexpr int LDG = DS + 1;   // leading dimension of G and X/M in LDS
constexpr int LDW = DS + 1;   // leading dimension of the eigenvector / Q_w / Qu work arrays

__device__ __forceinline__ double wave_sum64(double x) { return wave_sum(x); }
__device__ __forceinline__ double wave_max64(double x) { return wave_max(x); }
// Sums over aligned groups of 4 and 8 lanes (every lane of a group gets the same bits).
__device__ __forceinline__ double group4_sum(double x) {
    x += row_partner<1>(x);
    return x + row_partner<2>(x);
}
__device__ __forceinline__ double group8_sum(double x) {
    x = group4_sum(x);
    return x + row_partner<4>(x);
}

// Copy a rows x cols column-major block from global (leading dimension lds) to LDS (leading
// dimension ldd) with nthr threads (a multiple of 64): lane t % 64 takes rows t % 64 (+ 64 ...), the
// wave t / 64 every (nthr / 64)-th column, eight loads in flight per thread (all unconditional).
__device__ __forceinline__ void stage_block(double* dst, int ldd, const double* src, int lds, int rows, int cols,
                                            int t, int nthr) {
    const int cstep = nthr >> 6;
    for (int rb = 0; rb < rows; rb += 64) {
        const int rr = rb + (t & 63), rc = min(rr, rows - 1);
        for (int c0 = t >> 6; c0 < cols; c0 += 8 * cstep) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[rc + min(c0 + u * cstep, cols - 1) * lds];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u * cstep;
                if (rr < rows && c < cols) dst[rr + c * ldd] = v[u];
            }
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
__device__ __forceinline__ void k_dense_prep_body(const double* __restrict__ H, const double* __restrict__ Bm,
                                                   const double* __restrict__ gram, int kc, int jd_max, int k_target,
                                                   Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    __shared__ double G[LDG * DS];
    __shared__ double X[LDG * DS];
    __shared__ double rhs[DS + 1], gcs[DS], gsn[DS], Dk[KMAX], hv[DS + 1];
    const int t = threadIdx.x;
    const int jd = ctrl->j_done;
    const double beta = ctrl->beta;
    const int d = kc + jd;
    const int nr = kc + 1;
    if (d > DSM) return;       // the row-looped kernels take it

    // ---- D_k, G, X = W-hat^T V-hat (structured), right-hand side W-hat^T r. Global inputs are
    //      staged with eight loads in flight per lane.
    if (t < kc) Dk[t] = 1.0 / sqrt(gram[(kc + jd_max + 1 + t) * nr + t]);
    if (t < kc) { gcs[t] = 1.0; gsn[t] = 0.0; }     // no rotation on the D_k rows (handed over as such)
    for (int c = 0; c < d; ++c)
        if (t <= d) {
            G[t + c * LDG] = 0.0;
            X[t + c * LDG] = (c >= kc && t == c) ? 1.0 : 0.0;   // V_{jd+1}^T V_jd = I_{jd+1,jd}, C^T V = 0
        }
    __syncthreads();
    {
        // Lane t takes row t of each block (every block has at most 63 rows here), eight columns'
        // loads in flight, no integer division.
        // Hbar (rows 0..jd, columns 0..jd-1, Hessenberg) -> G[kc + r][kc + c]
        const int rh = min(t, jd);
        for (int c0 = 0; c0 < jd; c0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = H[rh + min(c0 + u, jd - 1) * LDH];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u;
                if (t <= jd && c < jd) G[kc + t + (kc + c) * LDG] = (t <= c + 1) ? v[u] : 0.0;
            }
        }
        // B (kc x jd) -> G[r][kc + c]
        if (kc > 0) {
            const int rb = min(t, kc - 1);
            for (int c0 = 0; c0 < jd; c0 += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = Bm[rb + min(c0 + u, jd - 1) * KMAX];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = c0 + u;
                    if (t < kc && c < jd) G[t + (kc + c) * LDG] = v[u];
                }
            }
        }
        __syncthreads();
        // [C V]^T U (rows 0..d, columns 0..kc-1) -> X[r][c] D_c;  D_k -> G[c][c]
        if (kc > 0) {
            const int rg = min(t, d);
            for (int c0 = 0; c0 < kc; c0 += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = gram[rg * nr + min(c0 + u, kc - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = c0 + u;
                    if (t <= d && c < kc) X[t + c * LDG] = v[u] * Dk[c];
                }
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
        // G[c + 1, c] is left at its rounding-level value: only the upper triangle is read after this
        __syncthreads();
    }

    // ---- least squares: y = R_G^{-1} rhs[0:d]
    double yv = (t < d) ? rhs[t] : 0.0;
    for (int c = d - 1; c >= 0; --c) {
        // y_c from lane c (a uniform lane: two lane reads, no LDS round trip)
        const unsigned long long yu = (unsigned long long)__double_as_longlong(yv);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)yu, c);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(yu >> 32), c);
        const double yc = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo)) / G[c + c * LDG];
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
        if (t == 0) { ctrl->k_new = 0; ctrl->eig_fail = 0; ctrl->route = 0; dw->mode = DW_NONE; }
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
__global__ __launch_bounds__(64) void k_dense_prep(const double* __restrict__ H, const double* __restrict__ Bm,
                                                   const double* __restrict__ gram, int kc, int jd_max, int k_target,
                                                   Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    k_dense_prep_body(H, Bm, gram, kc, jd_max, k_target, coef, dw, ctrl);
}


// Stage 2, symmetric case (4 wavefronts). M = X'' R_G^{-1} is formed; for symmetric A it is
// symmetric in exact arithmetic (G^T G and G^T W-hat^T V-hat = V-hat^T A V-hat are). The route is
// taken only for an operator that is exactly symmetric (ctrl->nonsym clear: a stencil kind, or a
// CSR matrix that passed the check at the system start), and only when the computed M is also
// symmetric to sym_tol relative (1e-10 with an FP64 basis, 1e-4 with an FP32 one, far above the
// rounding of the stored columns). Then the wanted eigenpairs of S = (M + M^T)/2 are found by
// Householder reduction to tridiagonal form T, multisection with Sturm counts for the eigenvalues
// of T, twisted factorizations of T - lambda I for their eigenvectors, back-transformation through
// the reflectors and modified Gram-Schmidt (a second pass when a column lost more than 30 % of
// its norm). Otherwise, or when an eigenvector comes out dependent on the others (a cluster) or
// not finite, M is handed to the general stage.
constexpr int DT = 256;         // threads of the symmetric stage
constexpr int LDS_ = DS + 1;  // leading dimension of S and V in LDS
constexpr int NSLOT = 2 * DT;   // multisection: Sturm counts per round (two recurrences per thread)

// Sturm counts of T - sh[s] I (s = 0, 1; two interleaved recurrences): the number of negative
// pivots D_i of its LDL^T factorization, D_i = (a_i - sh) - b_{i-1}^2 / D_{i-1}, a pivot of
// magnitude below pivmin taken as -pivmin. The quotient uses v_rcp_f64 with two Newton steps.
__device__ __forceinline__ void sturm2(const double* ta, const double* tb2, int d, double pivmin,
                                       const double sh[2], int cnt[2]) {
    double D[2];
#pragma unroll
    for (int s4 = 0; s4 < 2; ++s4) {
        D[s4] = ta[0] - sh[s4];
        if (fabs(D[s4]) < pivmin) D[s4] = -pivmin;
        cnt[s4] = D[s4] < 0.0;
    }
    for (int m0 = 1; m0 < d; m0 += 8) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int mm = min(m0 + u, d - 1);
            av[u] = ta[mm];
            bv[u] = tb2[mm - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (m0 + u < d) {
#pragma unroll
                for (int s4 = 0; s4 < 2; ++s4) {
                    double rc = __builtin_amdgcn_rcp(D[s4]);
                    rc = fma(rc, fma(-D[s4], rc, 1.0), rc);
                    rc = fma(rc, fma(-D[s4], rc, 1.0), rc);
                    D[s4] = fma(-bv[u], rc, av[u] - sh[s4]);
                    if (fabs(D[s4]) < pivmin) D[s4] = -pivmin;
                    cnt[s4] += D[s4] < 0.0;
                }
            }
        }
    }
}

// The eigenvalues of the symmetric tridiagonal T (diagonal ta, off-diagonal tb, squares tb2, in LDS)
// that the eigen stage keeps: the k_target of largest magnitude (smallest |theta| = 1/|mu|), by
// multisection with Sturm counts (count(sigma) = number of eigenvalues below sigma), DT threads.
// * Round 0 counts at 511 points spread evenly over the widened Gershgorin interval and at 0.
// * The wanted eigenvalues are among the candidates: the min(k_target, n_neg) lowest and the
//   min(k_target, d - n_neg) highest, n_neg = count(0) (at most k_target can come from either
//   end). Each candidate takes its bracket from round 0 by a binary search for the point where the
//   count passes its index (so the bracket always holds a change of the count across the index).
// * Every later round splits each candidate's bracket at NSLOT / ncand points until all brackets
//   are below 2e-8 ||T||.
// * Selection from both ends by magnitude (the eigenvalues ascend); at equal magnitude the upper
//   one first; a zero eigenvalue (theta infinite) is never taken.
// Returns the number selected; lsel[o] is the o-th selected eigenvalue (bracket midpoint) and
// isel[o] the candidate slot whose bracket [blo, bhi] holds it. tnorm and pivmin are set for the
// eigenvector stage. Every thread of the block calls it.
__device__ __forceinline__ int multisect_select(int d, int k_target, const double* ta, const double* tb,
                                                const double* tb2, double* blo, double* bhi, double* lam,
                                                double* bsh, int* bcnt, int* isel, double* lsel,
                                                double& tnorm, double& pivmin) {
    __shared__ int nb_s, nc_s, ns_s;
    const int t = threadIdx.x;
    const double eps = 2.220446049250313e-16;
    double glo = __builtin_inf(), ghi = -__builtin_inf(), bm2 = 0.0;
    for (int i = 0; i < d; ++i) {
        const double rad = (i > 0 ? fabs(tb[i - 1]) : 0.0) + (i + 1 < d ? fabs(tb[i]) : 0.0);
        glo = fmin(glo, ta[i] - rad);
        ghi = fmax(ghi, ta[i] + rad);
        if (i + 1 < d) bm2 = fmax(bm2, tb2[i]);
    }
    tnorm = fmax(fabs(glo), fabs(ghi));
    pivmin = 2.2250738585072014e-308 * fmax(1.0, bm2);
    const double widen = 2.0 * eps * tnorm * d + 2.0 * pivmin;
    glo -= widen;
    ghi += widen;
    const double tol = 2e-8 * tnorm;
    double sh[2];
    int cnt[2];
    // round 0: points glo + (ghi - glo) p / NSLOT (p = 1 .. NSLOT - 1) in slots 0 .. NSLOT - 2, and 0
#pragma unroll
    for (int s4 = 0; s4 < 2; ++s4) {
        const int slot = t + DT * s4;
        sh[s4] = (slot == NSLOT - 1) ? 0.0 : glo + (ghi - glo) * ((double)(slot + 1) / (double)NSLOT);
    }
    sturm2(ta, tb2, d, pivmin, sh, cnt);
#pragma unroll
    for (int s4 = 0; s4 < 2; ++s4) {
        bsh[t + DT * s4] = sh[s4];
        bcnt[t + DT * s4] = cnt[s4];
    }
    __syncthreads();
    if (t == 0) {
        const int nneg = bcnt[NSLOT - 1];
        const int nb = min(k_target, nneg), nt = min(k_target, d - nneg);
        nb_s = nb;
        nc_s = nb + nt;
    }
    __syncthreads();
    const int nb = nb_s, nc = nc_s;
    // candidate c is eigenvalue index c (c < nb) or d - nc + c
    int open = 0;
    if (t < nc) {
        const int i = t < nb ? t : d - nc + t;
        int lo = -1, hi = NSLOT - 1;     // point lo has count <= i (-1: glo), point hi count > i (ghi)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bcnt[mid] > i) hi = mid;
            else lo = mid;
        }
        const double nl = lo < 0 ? glo : bsh[lo];
        double nh = hi == NSLOT - 1 ? ghi : bsh[hi];
        if (nh < nl) nh = nl;
        blo[t] = nl;
        bhi[t] = nh;
        open = (nh - nl) > tol;
    }
    // later rounds: slot -> (candidate, point); slots past ns * nc repeat the last candidate unused
    const int ns = nc > 0 ? NSLOT / nc : 1;
    int cs[2], ps[2];
#pragma unroll
    for (int s4 = 0; s4 < 2; ++s4) {
        const int slot = t + DT * s4, c = slot / ns;
        cs[s4] = min(c, max(nc - 1, 0));
        ps[s4] = slot - c * ns;
    }
    for (int round = 0; round < 48 && __syncthreads_or(open); ++round) {
#pragma unroll
        for (int s4 = 0; s4 < 2; ++s4) {
            const double lo = blo[cs[s4]];
            sh[s4] = lo + (bhi[cs[s4]] - lo) * ((double)(ps[s4] + 1) / (double)(ns + 1));
        }
        sturm2(ta, tb2, d, pivmin, sh, cnt);
#pragma unroll
        for (int s4 = 0; s4 < 2; ++s4) {
            bsh[t + DT * s4] = sh[s4];
            bcnt[t + DT * s4] = cnt[s4];
        }
        __syncthreads();
        open = 0;
        if (t < nc) {
            const int i = t < nb ? t : d - nc + t, base = t * ns;
            int lo = -1, hi = ns;        // the bracket's ends stand for points -1 and ns
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (bcnt[base + mid] > i) hi = mid;
                else lo = mid;
            }
            const double nl = lo < 0 ? blo[t] : bsh[base + lo];
            double nh = hi == ns ? bhi[t] : bsh[base + hi];
            if (nh < nl) nh = nl;
            blo[t] = nl;
            bhi[t] = nh;
            open = (nh - nl) > tol;
        }
    }
    if (t < nc) lam[t] = 0.5 * (blo[t] + bhi[t]);
    __syncthreads();
    if (t == 0) {
        int lo = 0, hi = nc - 1, nsel = 0;   // lo over the lower candidates, hi over the upper ones
        while (nsel < k_target && (lo < nb || hi >= nb)) {
            const int pick = lo >= nb ? hi-- : (hi < nb ? lo++ : (fabs(lam[hi]) >= fabs(lam[lo]) ? hi-- : lo++));
            if (!(fabs(lam[pick]) > 0.0)) break;
            isel[nsel] = pick;
            lsel[nsel++] = lam[pick];
        }
        ns_s = nsel;
    }
    __syncthreads();
    return ns_s;
}

// Forward substitution m R = x'' for one row of M held in registers (acc), over chunks of at most
// 16 entries of the rows of R: chunk (C, S0) holds R[C, S0 .. S0 + N - 1]. Column C sets m_C to
// the product of acc[C] with the reciprocal of R[C, C]; every later entry s then takes
// -m_C R[C, s] as one FMA, in increasing C. The chunk after this one (the next chunk of row C, or
// the first of row C + 1 with its reciprocal) is read from LDS before this chunk's FMAs, and
// scheduling barriers keep that order, so the reads overlap the arithmetic. Template parameters
// make every index into acc a constant.
template <int S0>
constexpr int mchunk_n() { return (DS - S0) < 16 ? (DS - S0) : 16; }
template <int C, int S0, int N>
__device__ __forceinline__ void msolve_chunk(double (&acc)[DS], const double* R, const double* Rd, int d,
                                             double mc, const double (&cur)[N]) {
    constexpr bool row_end = S0 + N >= DS;
    constexpr int NC = row_end ? C + 1 : C;
    constexpr int NS0 = row_end ? C + 2 : S0 + N;
    constexpr bool more = NS0 < DS;
    constexpr int NN = more ? mchunk_n<NS0>() : 1;
    double nxt[NN];
    double rdn = 0.0;
    if constexpr (more) {
#pragma unroll
        for (int u = 0; u < NN; ++u) nxt[u] = R[NC + (NS0 + u) * LDS_];
        if constexpr (row_end) rdn = Rd[NC];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < N; ++u) acc[S0 + u] = fma(-mc, cur[u], acc[S0 + u]);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (more) {
        if constexpr (row_end) {
            if (NC < d) {
                const double mn = acc[NC] * rdn;
                acc[NC] = mn;
                msolve_chunk<NC, NS0, NN>(acc, R, Rd, d, mn, nxt);
            }
        } else {
            msolve_chunk<NC, NS0, NN>(acc, R, Rd, d, mc, nxt);
        }
    }
}

__device__ __forceinline__ void k_dense_sym_body(int k_target, double sym_tol, Coef* coef, DenseWork* dw,
                                                  Ctrl* ctrl) {
    if (dw->mode != DW_PENDING) return;
    __shared__ double S[LDS_ * DS];
    __shared__ double V[LDS_ * DS];
    __shared__ double R[LDS_ * DS];
    __shared__ double gcs[DS], gsn[DS], Dk[KMAX], Rd[DS];
    __shared__ double red[DT / 64], red2[DT / 64];
    __shared__ double ta[DS], tb[DS], tb2[DS], hb[DS];
    __shared__ double blo[DS], bhi[DS], lam[DS], lsel[KMAX];
    __shared__ double bsh[NSLOT];
    __shared__ int bcnt[NSLOT];
    __shared__ int sel[KMAX], isel[KMAX];
    __shared__ int sym_s, need2_s, fail_s;
    const int t = threadIdx.x;
    const int d = dw->d, kc = dw->kc;
    const int dp = d + (d & 1);                 // even size (a zero row/column pads an odd d)
    // load R_G, X'', the rotations of Q_G and D_k
    stage_block(R, LDS_, dw->R, DMAX, d, d, t, DT);
    stage_block(S, LDS_, dw->X, DMAX, d, d, t, DT);
    if (t < d) { gcs[t] = dw->gcs[t]; gsn[t] = dw->gsn[t]; }
    if (t < kc) Dk[t] = dw->Dk[t];
    __syncthreads();
    // M = X'' R^{-1}: row r of M solves m R = x'' by forward substitution over the columns. The rows
    // are independent: one lane per row (d <= 62 rows, wave 0) keeps its whole row in registers, and
    // row c of R reaches every lane as an LDS broadcast, so no value moves between lanes. Entry s
    // takes the terms m_c R[c, s] for c < s in increasing c, one FMA each, and m_s is the product of
    // the result with the reciprocal of R[s, s]. Columns past d compute on padding and are not
    // stored. The diagonal of R is then zeroed in LDS for the triangular solve of the Qu formation.
    if (t < d) Rd[t] = 1.0 / R[t + t * LDS_];
    __syncthreads();
    if (t < 64) {
        const int rr = min(t, d - 1);
        double acc[DS];
#pragma unroll
        for (int s2 = 0; s2 < DS; ++s2) acc[s2] = S[rr + min(s2, d - 1) * LDS_];
        {
            double cur[mchunk_n<1>()];
#pragma unroll
            for (int u = 0; u < mchunk_n<1>(); ++u) cur[u] = R[(1 + u) * LDS_];
            const double m0 = acc[0] * Rd[0];
            acc[0] = m0;
            msolve_chunk<0, 1>(acc, R, Rd, d, m0, cur);
        }
        if (t < d) {
#pragma unroll
            for (int s2 = 0; s2 < DS; ++s2)
                if (s2 < d) S[t + s2 * LDS_] = acc[s2];
        }
    }
    __syncthreads();
    if (t < d) R[t + t * LDS_] = 0.0;
    __syncthreads();
    // symmetry test: max |M - M^T| <= sym_tol max |M|
    double amax = 0.0, dmax = 0.0;
    const int rl = t & 63, cw = t >> 6;     // row, first column of this thread in the d x d loops below
    if (rl < d) {
        for (int c = cw; c < d; c += DT / 64) {
            const double a = S[rl + c * LDS_];
            amax = fmax(amax, fabs(a));
            dmax = fmax(dmax, fabs(a - S[c + rl * LDS_]));
        }
    }
    amax = wave_max64(amax);
    dmax = wave_max64(dmax);
    if ((t & 63) == 0) { red[t >> 6] = amax; red2[t >> 6] = dmax; }
    __syncthreads();
    if (t == 0) {
        double ga = red[0], gd = red2[0];
        for (int q = 1; q < DT / 64; ++q) { ga = fmax(ga, red[q]); gd = fmax(gd, red2[q]); }
        sym_s = (!ctrl->nonsym && gd <= sym_tol * ga) ? 1 : 0;
    }
    __syncthreads();
    // M goes to the general stage's input in any case: that stage takes over if this one declines
    if (rl < d)
        for (int c = cw; c < d; c += DT / 64) dw->X[rl + c * DMAX] = S[rl + c * LDS_];
    if (!sym_s) {
        if (t == 0) dw->mode = DW_GEN;
        return;
    }
    // S = (M + M^T) / 2 in place (each unordered pair by one thread)
    if (rl < d) {
        for (int c = cw; c < d; c += DT / 64) {
            if (rl < c) {
                const double v = 0.5 * (S[rl + c * LDS_] + S[c + rl * LDS_]);
                S[rl + c * LDS_] = v;
                S[c + rl * LDS_] = v;
            }
        }
    }
    __syncthreads();

    // ---- Householder tridiagonalization. Step j maps x = S[j+1:d, j] to alpha e_1 with
    // H_j = I - beta v v^T, v = x - alpha e_1 (zero above row j + 1): v is kept whole in column j of
    // S (LDS, for the back-transformation). The trailing matrix lives in registers: thread
    // t holds row r = t % 64 at the columns c = t / 64 + 4u (u < 16). Step j: the wave holding column
    // j forms the reflector and publishes v (double-buffered); every thread adds its part of
    // p = beta S' v; every wave then sums the four parts of its rows in the same order, so all waves
    // hold the same p and K = beta p^T v / 2, and w = p - K v. The update S' -= v w^T + w v^T takes w
    // at its columns from the wave's own copy of w in LDS, and adds the two products without
    // contraction so that S stays exactly symmetric.
    __shared__ double hvb[2][64], hbeta[2], ppart[DT / 64][64], wsh[DT / 64][64];
    {
        const int r = t & 63;
        const int wv = __builtin_amdgcn_readfirstlane(t >> 6);   // this wave's column class
        double s[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = wv + 4 * u;
            s[u] = (r < d && c < d) ? S[r + c * LDS_] : 0.0;
        }
        for (int j = 0; j + 2 < d; ++j) {
            const int j1 = j + 1, buf = j & 1;
            if (wv == (j & 3)) {
                double x = 0.0;    // S[r, j]
#pragma unroll
                for (int u = 0; u < 16; ++u) x = (u == (j >> 2)) ? s[u] : x;
                const double sig = wave_sum64((r >= j + 2 && r < d) ? x * x : 0.0);
                const double xh = __shfl(x, j1, 64), diag = __shfl(x, j, 64);
                double beta = 0.0, v0 = 0.0, alpha = xh;
                if (sig > 0.0) {
                    const double mu = sqrt(fma(xh, xh, sig));
                    v0 = (xh >= 0.0) ? xh + mu : xh - mu;
                    alpha = (xh >= 0.0) ? -mu : mu;
                    beta = 2.0 / fma(v0, v0, sig);
                }
                const double vrow = (r == j1) ? v0 : ((r > j1 && r < d) ? x : 0.0);
                hvb[buf][r] = vrow;
                if (r < LDS_) S[r + j * LDS_] = vrow;      // the whole reflector, for the back-transformation
                if (r == 0) { ta[j] = diag; tb[j] = alpha; hb[j] = beta; hbeta[buf] = beta; }
            }
            __syncthreads();
            const double beta = hbeta[buf];
            if (beta != 0.0) {   // same in every thread
                double vc[16];
                double pp = 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    vc[u] = hvb[buf][min(wv + 4 * u, 63)];
                    pp = fma(s[u], vc[u], pp);
                }
                ppart[wv][r] = pp;
                __syncthreads();
                const double pr = beta * ((ppart[0][r] + ppart[1][r]) + (ppart[2][r] + ppart[3][r]));
                const double vr = hvb[buf][r];
                const double kp = wave_sum64((r >= j1 && r < d) ? pr * vr : 0.0);
                const double K = 0.5 * beta * kp;
                const double wr = fma(-K, vr, pr);
                // w at this thread's columns: each wave passes its own copy of w through LDS (the
                // reads of one column are a broadcast)
                wsh[wv][r] = wr;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                double wcv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) wcv[u] = wsh[wv][min(wv + 4 * u, 63)];
                // every entry is updated: those outside the trailing block (row or column < j1, or
                // padding) are never read again except as factors of an exact zero of v, and stay
                // finite, so they change no value that is used (a select per entry cost more than
                // the update itself)
#pragma unroll
                for (int u = 0; u < 16; ++u) s[u] = s[u] - __dadd_rn(__dmul_rn(vr, wcv[u]), __dmul_rn(wr, vc[u]));
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        // the last 2 x 2 block: T(d-2, d-2), T(d-1, d-2), T(d-1, d-1)
        if (d >= 2) {
            const int c2 = d - 2, c1 = d - 1;
            if (wv == (c2 & 3)) {
                double x = 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) x = (u == (c2 >> 2)) ? s[u] : x;
                if (r == c2) ta[c2] = x;
                if (r == c1) tb[c2] = x;
            }
            if (wv == (c1 & 3)) {
                double x = 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) x = (u == (c1 >> 2)) ? s[u] : x;
                if (r == c1) ta[c1] = x;
            }
        } else if (d == 1 && t == 0) {
            ta[0] = S[0];
        }
    }
    __syncthreads();
    if (t < d - 1) tb2[t] = tb[t] * tb[t];
    __syncthreads();

    // ---- the wanted eigenvalues of T (multisection over the candidates at both ends)
    double tnorm = 0.0, pivmin = 0.0;
    const int kn = multisect_select(d, k_target, ta, tb, tb2, blo, bhi, lam, bsh, bcnt, isel, lsel, tnorm, pivmin);
    if (t == 0) {
        need2_s = 0;
        fail_s = 0;
    }
    __syncthreads();

    // ---- eigenvectors of T (wave 0 and wave 1, lane o for selected eigenvalue o): T - lambda I =
    // L+ D+ L+^T = U- D- U-^T, twist index r = argmin |gamma_r|, gamma_r = D+_r + D-_r - (a_r - lambda),
    // then z_r = 1 and z_i = -b_i z_{i+1} / D+_i (i < r), z_{i+1} = -b_i z_i / D-_{i+1} (i >= r), so that
    // (T - lambda I) z = gamma_r e_r. Wave 0 forms D+ and the upper part of z, wave 1 D- and the lower
    // part, side by side on two SIMDs (the other waves only join the barriers). The eigenvalue from
    // multisection (to 2e-8 ||T||) is refined by one Rayleigh-quotient step, lambda += gamma_r / ||z||^2
    // (cubically convergent), kept inside its bisection interval; the second pass gives the
    // eigenvector. D+ and D- live in V (columns of 32), z overwrites D+. Quotients use v_rcp_f64 with
    // two Newton steps.
    double* Fp = V;
    double* Fm = V + DS * KMAX;
    __shared__ double nzs[2][KMAX];
    {
        const int o = t & 63, side = t >> 6;
        const bool act = side < 2 && o < kn;
        const int oc = min(o, KMAX - 1);
        const int ie = act ? isel[oc] : 0;
        const double lo_ = blo[ie], hi_ = bhi[ie];
        double lm = act ? lsel[oc] : 0.0;
        auto frcp = [](double v) {
            double rc = __builtin_amdgcn_rcp(v);
            rc = fma(rc, fma(-v, rc, 1.0), rc);
            return fma(rc, fma(-v, rc, 1.0), rc);
        };
        for (int pass = 0; pass < 2; ++pass) {
            if (act) {
                if (side == 0) {
                    double dp = ta[0] - lm;
                    if (fabs(dp) < pivmin) dp = -pivmin;
                    Fp[o] = dp;
                    for (int s2 = 1; s2 < d; ++s2) {
                        dp = fma(-tb2[s2 - 1], frcp(dp), ta[s2] - lm);
                        if (fabs(dp) < pivmin) dp = -pivmin;
                        Fp[s2 * KMAX + o] = dp;
                    }
                } else {
                    double dm = ta[d - 1] - lm;
                    if (fabs(dm) < pivmin) dm = -pivmin;
                    Fm[(d - 1) * KMAX + o] = dm;
                    for (int ib = d - 2; ib >= 0; --ib) {
                        dm = fma(-tb2[ib], frcp(dm), ta[ib] - lm);
                        if (fabs(dm) < pivmin) dm = -pivmin;
                        Fm[ib * KMAX + o] = dm;
                    }
                }
            }
            __syncthreads();
            int rt = 0;
            double gam = 0.0, nz = 0.0;
            if (act) {
                // the same search in both waves (same operands and order, so the same twist index)
                double gb = __builtin_inf();
                for (int i = 0; i < d; ++i) {
                    const double g = Fp[i * KMAX + o] + Fm[i * KMAX + o] - (ta[i] - lm);
                    if (fabs(g) < gb) { gb = fabs(g); gam = g; rt = i; }
                }
            }
            __syncthreads();    // wave 1 has read D+ before wave 0 overwrites it with z
            if (act) {
                double z = 1.0;
                if (side == 0) {
                    for (int i = rt - 1; i >= 0; --i) {
                        z = -tb[i] * z * frcp(Fp[i * KMAX + o]);
                        Fp[i * KMAX + o] = z;
                        nz = fma(z, z, nz);
                    }
                    Fp[rt * KMAX + o] = 1.0;
                } else {
                    for (int i = rt; i + 1 < d; ++i) {
                        z = -tb[i] * z * frcp(Fm[(i + 1) * KMAX + o]);
                        Fp[(i + 1) * KMAX + o] = z;
                        nz = fma(z, z, nz);
                    }
                }
                nzs[side][o] = nz;
            }
            __syncthreads();
            // ||z||^2 = 1 + upper part + lower part, added in the same order in both waves
            if (act) {
                const double nzo = nzs[side ^ 1][o];
                const double nz2 = 1.0 + (side == 0 ? nz + nzo : nzo + nz);
                if (pass == 0) {
                    const double ln = lm + gam / nz2;
                    if (ln == ln) lm = fmin(fmax(ln, lo_), hi_);
                }
            }
            __syncthreads();
        }
    }

    // ---- back-transformation z <- H_0 ... H_{d-3} z and modified Gram-Schmidt, eight lanes per
    // column (column c = t / 8, rows t % 8 + 8 i in registers); the finished columns go to V.
    const int zc = t >> 3, part = t & 7;
    double zr[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = part + 8 * i;
        zr[i] = (zc < kn && r < d) ? Fp[r * KMAX + zc] : 0.0;
    }
    __syncthreads();
    for (int j = d - 3; j >= 0; --j) {
        const double beta = hb[j];
        if (beta == 0.0) continue;
        double vr[8];     // column j of S holds the whole reflector (zero outside rows j+1 .. d-1)
#pragma unroll
        for (int i = 0; i < 8; ++i) vr[i] = S[min(part + 8 * i, LDS_ - 1) + j * LDS_];
        double dt0 = 0.0, dt1 = 0.0;
#pragma unroll
        for (int i = 0; i < 8; i += 2) { dt0 = fma(vr[i], zr[i], dt0); dt1 = fma(vr[i + 1], zr[i + 1], dt1); }
        double dot = dt0 + dt1;
        dot = group8_sum(dot);
        dot *= beta;
#pragma unroll
        for (int i = 0; i < 8; ++i) zr[i] = fma(-dot, vr[i], zr[i]);
    }
    double n0;
    {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < 8; i += 2) { a0 = fma(zr[i], zr[i], a0); a1 = fma(zr[i + 1], zr[i + 1], a1); }
        n0 = a0 + a1;
        n0 = group8_sum(n0);
        n0 = sqrt(n0);
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < kn; ++j) {
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int i = 0; i < 8; i += 2) { a0 = fma(zr[i], zr[i], a0); a1 = fma(zr[i + 1], zr[i + 1], a1); }
            double nr = a0 + a1;
            nr = group8_sum(nr);
            nr = sqrt(nr);
            if (zc == j) {
                if (pass == 0) {
                    if (!(nr > 1e-8 * n0) || !(n0 < __builtin_inf())) fail_s = 1;
                    else if (nr < 0.7 * n0) need2_s = 1;
                }
                const double inv = (nr > 0.0) ? 1.0 / nr : 0.0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    zr[i] *= inv;
                    const int r = part + 8 * i;
                    if (r < d) V[r + j * LDS_] = zr[i];
                }
            }
            __syncthreads();
            double qv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int r = part + 8 * i;
                qv[i] = (r < d) ? V[r + j * LDS_] : 0.0;
            }
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int i = 0; i < 8; i += 2) { d0 = fma(qv[i], zr[i], d0); d1 = fma(qv[i + 1], zr[i + 1], d1); }
            double dot = d0 + d1;
            dot = group8_sum(dot);
            const double f = (zc > j && zc < kn) ? dot : 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) zr[i] = fma(-f, qv[i], zr[i]);
        }
        __syncthreads();
        if (fail_s || !need2_s) break;
    }
    if (fail_s) {
        if (t == 0) dw->mode = DW_GEN;
        return;
    }
    if (t < kn) sel[t] = t;
    __syncthreads();
    // Qc = Q_G [Q_w; 0], Q_w = V[:, sel]: one lane per column, the rotations of Q_G in reverse order
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
    // Qu = R_G^{-1} Q_w by back-substitution, eight lanes per column with lane part p holding rows
    // 8p..8p+7 in registers (y_i broadcast from its owner); the rows of the recycled part carry D_k
    {
        const int o = t >> 3, p = t & 7;
        const int col = sel[min(o, KMAX - 1)];
        double y[8];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
            const int r = 8 * p + s2;
            y[s2] = (o < kn && r < d) ? V[r + col * LDS_] : 0.0;
        }
        for (int i0 = ((d - 1) >> 3) << 3; i0 >= 0; i0 -= 8) {
            const int owner = i0 >> 3;
#pragma unroll
            for (int s1 = 7; s1 >= 0; --s1) {
                const int i = i0 + s1;
                if (i < d) {
                    double rq[8];
#pragma unroll
                    for (int s2 = 0; s2 < 8; ++s2) rq[s2] = R[8 * p + s2 + i * LDS_];
                    const double yl = y[s1] * Rd[i];
                    y[s1] = (p == owner) ? yl : y[s1];
                    const double yi = __shfl(yl, (t & ~7) | owner, 64);
                    // rows i and below of column i of R are zero in LDS: no mask
#pragma unroll
                    for (int s2 = 0; s2 < 8; ++s2) y[s2] = fma(-yi, rq[s2], y[s2]);
                }
            }
        }
        if (o < kn) {
#pragma unroll
            for (int s2 = 0; s2 < 8; ++s2) {
                const int r = 8 * p + s2;
                if (r < d) coef->Qu[r + o * LDQU] = (r < kc ? Dk[r < KMAX ? r : 0] : 1.0) * y[s2];
            }
        }
    }
    __syncthreads();
    if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 0; ctrl->route = 1; dw->mode = DW_DONE; }
}
__global__ __launch_bounds__(DT) void k_dense_sym(int k_target, double sym_tol, Coef* coef, DenseWork* dw,
                                                  Ctrl* ctrl) {
    k_dense_sym_body(k_target, sym_tol, coef, dw, ctrl);
}


// Stage 2, general (nonsymmetric) case, one wavefront: M = X'' R_G^{-1} was formed by the
// symmetric stage, which found it nonsymmetric. Householder reduction to Hessenberg form, Francis
// double-shift QR, eigenvectors of the selected eigenvalues by back-substitution, an orthonormal
// basis Q_w of them, and the recycle-space coefficients Qu = R_G^{-1} Q_w, Qc = Q_G [Q_w; 0].
__device__ __forceinline__ void k_dense_gen_body(int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    if (dw->mode != DW_GEN) return;
    __shared__ double G[LDG * DS];
    __shared__ double X[LDG * DS];
    __shared__ double Z[DS * DS];
    __shared__ double Wv[LDW * KMAX];
    __shared__ double Uq[LDW * KMAX];
    __shared__ double gcs[DS], gsn[DS], Dk[KMAX], wr[DS], wi[DS], hv[DS + 1];
    __shared__ int taken[DS], sel_pos[KMAX], sel_cplx[KMAX], sel_col[KMAX];
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
        if (t < d) Z[t + c * DS] = (t == c) ? 1.0 : 0.0;
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
                sz = fma(Z[t + q * DS], hv[q], sz);
            }
            s *= tau;
            sz *= tau;
            for (int q = c + 1; q < d; ++q) {
                X[t + q * LDG] = fma(-s, hv[q], X[t + q * LDG]);
                Z[t + q * DS] = fma(-sz, hv[q], Z[t + q * DS]);
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
                    const double z0 = Z[t + p * DS], z1 = Z[t + q * DS];
                    Z[t + p * DS] = cs * z0 + sn * z1;
                    Z[t + q * DS] = -sn * z0 + cs * z1;
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
                    const double a = Z[t + kk * DS], b = Z[t + (kk + 1) * DS], c = Z[t + (kk + 2) * DS];
                    const double s = tau * (a + v1 * b + v2 * c);
                    Z[t + kk * DS] = a - s;
                    Z[t + (kk + 1) * DS] = b - s * v1;
                    Z[t + (kk + 2) * DS] = c - s * v2;
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
                    const double a = Z[t + kk * DS], b = Z[t + (kk + 1) * DS];
                    const double s = tau * (a + v1 * b);
                    Z[t + kk * DS] = a - s;
                    Z[t + (kk + 1) * DS] = b - s * v1;
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
        if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 1; ctrl->route = 2; dw->mode = DW_DONE; }
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
            for (int c = 0; c < d; ++c) s = fma(Z[t + c * DS], Wv[c + o * LDW], s);
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
    if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 0; ctrl->route = 2; dw->mode = DW_DONE; }
}
__global__ __launch_bounds__(64) void k_dense_gen(int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    k_dense_gen_body(k_target, coef, dw, ctrl);
}


// ---------------------------------------------------------------------------------------------
// Cycle end for DSM < d <= MMAX: the same three stages with their thread mappings stretched to
// d <= MMAX (rows looped over the lanes where one row per lane no longer fits). Each large-d eigen
// stage forms M = X'' R_G^{-1} itself; the symmetric one hands over to the general one exactly as
// in the small case. LDS holds two or three d x d regions, each reused across the phases.
// ---------------------------------------------------------------------------------------------
constexpr int LDP = MMAX + 2;   // leading dimension of G and X ((d + 1) x d) in the first stage
constexpr int LDL = MMAX + 1;   // leading dimension of the d x d arrays of the general stage

__device__ __forceinline__ void k_dense_prep_L_body(const double* __restrict__ H, const double* __restrict__ Bm,
                                                     const double* __restrict__ gram, int kc, int jd_max,
                                                     int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    __shared__ double G[LDP * MMAX];
    __shared__ double X[LDP * MMAX];
    __shared__ double rhs[MMAX + 2], gcs[MMAX + 1], gsn[MMAX + 1], Dk[KMAX], hv[MMAX + 2], yv[MMAX + 1];
    const int t = threadIdx.x;
    const int jd = ctrl->j_done;
    const double beta = ctrl->beta;
    const int d = kc + jd;
    const int nr = kc + 1;
    if (d <= DSM) return;       // the one-row-per-lane kernels take it

    // ---- D_k, G = [[D_k, B], [0, Hbar]], X = W-hat^T V-hat, right-hand side W-hat^T r
    if (t < kc) Dk[t] = 1.0 / sqrt(gram[(kc + jd_max + 1 + t) * nr + t]);
    for (int c = 0; c < d; ++c)
        for (int r = t; r <= d; r += 64) {
            G[r + c * LDP] = 0.0;
            X[r + c * LDP] = (c >= kc && r == c) ? 1.0 : 0.0;   // V_{jd+1}^T V_jd = I_{jd+1,jd}, C^T V = 0
        }
    __syncthreads();
    for (int e = t; e < (jd + 1) * jd; e += 64) {
        const int c = e / (jd + 1), r = e - c * (jd + 1);
        if (r <= c + 1) G[kc + r + (kc + c) * LDP] = H[r + c * LDH];
    }
    for (int e = t; e < kc * jd; e += 64) {
        const int c = e / kc, r = e - c * kc;
        G[r + (kc + c) * LDP] = Bm[r + c * KMAX];
    }
    __syncthreads();
    for (int e = t; e < (d + 1) * kc; e += 64) {
        const int c = e / (d + 1), r = e - c * (d + 1);
        X[r + c * LDP] = gram[r * nr + c] * Dk[c];
    }
    if (t < kc) G[t + t * LDP] = Dk[t];
    for (int r = t; r <= d; r += 64) rhs[r] = (r < kc) ? gram[r * nr + kc] : (r == kc ? beta : 0.0);
    __syncthreads();

    // ---- Givens QR of G (the Hessenberg block)
    for (int c = kc; c < d; ++c) {
        const double a = G[c + c * LDP], b = G[c + 1 + c * LDP];
        const double rho = hypot(a, b);
        const double cs = rho > 0.0 ? a / rho : 1.0, sn = rho > 0.0 ? b / rho : 0.0;
        __syncthreads();
        for (int q = t; q < d; q += 64) {
            if (q >= c) {
                const double g0 = G[c + q * LDP], g1 = G[c + 1 + q * LDP];
                G[c + q * LDP] = cs * g0 + sn * g1;
                G[c + 1 + q * LDP] = -sn * g0 + cs * g1;
            }
            const double x0 = X[c + q * LDP], x1 = X[c + 1 + q * LDP];
            X[c + q * LDP] = cs * x0 + sn * x1;
            X[c + 1 + q * LDP] = -sn * x0 + cs * x1;
        }
        if (t == 0) {
            const double r0 = rhs[c], r1 = rhs[c + 1];
            rhs[c] = cs * r0 + sn * r1;
            rhs[c + 1] = -sn * r0 + cs * r1;
            gcs[c] = cs;
            gsn[c] = sn;
        }
        // G[c + 1, c] is left at its rounding-level value: only the upper triangle is read after this
        __syncthreads();
    }

    // ---- least squares: y = R_G^{-1} rhs[0:d] (column-oriented back-substitution)
    for (int r = t; r < d; r += 64) yv[r] = rhs[r];
    __syncthreads();
    for (int c = d - 1; c >= 0; --c) {
        const double yc = yv[c] / G[c + c * LDP];
        __syncthreads();
        if (t == 0) yv[c] = yc;
        for (int r = t; r < c; r += 64) yv[r] = fma(-G[r + c * LDP], yc, yv[r]);
        __syncthreads();
    }
    for (int r = t; r < d; r += 64) {
        if (r < kc) coef->yU[r] = Dk[r] * yv[r];
        else coef->yV[r - kc] = yv[r];
    }
    // G y = Q_G [rhs[0:d]; 0]
    for (int r = t; r <= d; r += 64) hv[r] = (r < d) ? rhs[r] : 0.0;
    __syncthreads();
    if (t == 0) {
        for (int c = d - 1; c >= kc; --c) {
            const double a = hv[c], b = hv[c + 1];
            hv[c] = gcs[c] * a - gsn[c] * b;
            hv[c + 1] = gsn[c] * a + gcs[c] * b;
        }
    }
    __syncthreads();
    for (int r = t; r <= d; r += 64) {
        if (r < kc) coef->rC[r] = hv[r];
        else coef->rV[r - kc] = hv[r];
    }

    const bool recycle = k_target > 0 && (kc > 0 || jd > k_target);
    if (!recycle) {
        if (t == 0) { ctrl->k_new = 0; ctrl->eig_fail = 0; ctrl->route = 0; dw->mode = DW_NONE; }
        return;
    }
    // hand over R_G (d x d, upper), X'' (d x d), rotations and D_k
    for (int c = 0; c < d; ++c)
        for (int r = t; r < d; r += 64) {
            dw->R[r + c * DMAX] = (r <= c) ? G[r + c * LDP] : 0.0;
            dw->X[r + c * DMAX] = X[r + c * LDP];
        }
    for (int r = t; r < d; r += 64) { dw->gcs[r] = gcs[r]; dw->gsn[r] = gsn[r]; }
    if (t < kc) dw->Dk[t] = Dk[t];
    if (t == 0) { dw->d = d; dw->kc = kc; dw->mode = DW_PENDING_L; }
}
__global__ __launch_bounds__(64) void k_dense_prep_L(const double* __restrict__ H, const double* __restrict__ Bm,
                                                     const double* __restrict__ gram, int kc, int jd_max,
                                                     int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    k_dense_prep_L_body(H, Bm, gram, kc, jd_max, k_target, coef, dw, ctrl);
}


// Symmetric stage for d > DSM (DT threads): the route of k_dense_sym (M, symmetry test,
// Householder tridiagonalization, multisection, twisted factorizations, back-transformation and
// Gram-Schmidt, Qc and Qu) with every thread mapping stretched to d <= MMAX. Two LDS regions: S
// (X'', then M, then S = (M + M^T)/2 reduced to tridiagonal form with the reflectors below the
// subdiagonal, then R_G again for Qu) and V (R_G while M is formed, then the pivots of the twisted
// factorizations and the eigenvectors). dw->X keeps X'' for the general stage if this one declines.
constexpr int RPL = (MMAX + 7) / 8;   // rows per lane when eight lanes share a column

__device__ __forceinline__ void k_dense_sym_L_body(int k_target, double sym_tol, Coef* coef, DenseWork* dw,
                                                    Ctrl* ctrl) {
    if (dw->mode != DW_PENDING_L) return;
    __shared__ double S[LDL * MMAX];
    __shared__ double V[LDL * MMAX];
    __shared__ double gcs[MMAX], gsn[MMAX], Dk[KMAX], Rd[MMAX];
    __shared__ double red[DT / 64], red2[DT / 64];
    __shared__ double ta[MMAX], tb[MMAX], tb2[MMAX], hb[MMAX], hv0[MMAX], hP[MMAX];
    __shared__ double blo[MMAX], bhi[MMAX], lam[MMAX], lsel[KMAX], hsig[1], hkp[DT / 64];
    __shared__ double bsh[NSLOT];
    __shared__ int bcnt[NSLOT];
    __shared__ int sel[KMAX], isel[KMAX];
    __shared__ int sym_s, need2_s, fail_s;
    const int t = threadIdx.x;
    const int d = dw->d, kc = dw->kc;
    double* R = V;
    stage_block(R, LDL, dw->R, DMAX, d, d, t, DT);
    stage_block(S, LDL, dw->X, DMAX, d, d, t, DT);
    if (t < d) { gcs[t] = dw->gcs[t]; gsn[t] = dw->gsn[t]; }
    if (t < kc) Dk[t] = dw->Dk[t];
    __syncthreads();
    if (t < d) Rd[t] = 1.0 / R[t + t * LDL];
    __syncthreads();
    // ---- M = X'' R^{-1}: thread r solves m R = x'' for row r (right-looking over the columns)
    if (t < d) {
        for (int c = 0; c < d; ++c) {
            const double mc = S[t + c * LDL] * Rd[c];
            S[t + c * LDL] = mc;
            for (int q = c + 1; q < d; ++q) S[t + q * LDL] = fma(-mc, R[c + q * LDL], S[t + q * LDL]);
        }
    }
    __syncthreads();
    // ---- symmetry test: max |M - M^T| <= sym_tol max |M|
    double amax = 0.0, dmax = 0.0;
    for (int e = t; e < d * d; e += DT) {
        const int r = e % d, c = e / d;
        const double a = S[r + c * LDL];
        amax = fmax(amax, fabs(a));
        dmax = fmax(dmax, fabs(a - S[c + r * LDL]));
    }
    amax = wave_max64(amax);
    dmax = wave_max64(dmax);
    if ((t & 63) == 0) { red[t >> 6] = amax; red2[t >> 6] = dmax; }
    __syncthreads();
    if (t == 0) {
        double ga = red[0], gd = red2[0];
        for (int q = 1; q < DT / 64; ++q) { ga = fmax(ga, red[q]); gd = fmax(gd, red2[q]); }
        sym_s = (!ctrl->nonsym && gd <= sym_tol * ga) ? 1 : 0;
    }
    __syncthreads();
    if (!sym_s) {
        if (t == 0) dw->mode = DW_GEN_L;
        return;
    }
    // S = (M + M^T) / 2 in place (each unordered pair by one thread)
    for (int e = t; e < d * d; e += DT) {
        const int r = e % d, c = e / d;
        if (r < c) {
            const double v = 0.5 * (S[r + c * LDL] + S[c + r * LDL]);
            S[r + c * LDL] = v;
            S[c + r * LDL] = v;
        }
    }
    __syncthreads();

    // ---- Householder tridiagonalization (as in k_dense_sym): p = beta S' v with two threads per
    // row, the rank-2 update strided over all threads (products added without contraction, so S
    // stays exactly symmetric), sigma of the next step from column j + 1 by wave 0.
    if (t < 64) {
        double x2 = 0.0;
        for (int r = 2 + t; r < d; r += 64) x2 = fma(S[r], S[r], x2);
        const double sg = wave_sum64(x2);
        if (t == 0) hsig[0] = sg;
    }
    __syncthreads();
    for (int j = 0; j + 2 < d; ++j) {
        const int j1 = j + 1;
        const double sig = hsig[0];
        const double xh = S[j1 + j * LDL];
        double beta = 0.0, v0 = 0.0, alpha = xh;
        if (sig > 0.0) {
            const double mu = sqrt(fma(xh, xh, sig));
            v0 = (xh >= 0.0) ? xh + mu : xh - mu;
            alpha = (xh >= 0.0) ? -mu : mu;
            beta = 2.0 / fma(v0, v0, sig);
        }
        if (t == 0) { ta[j] = S[j + j * LDL]; tb[j] = alpha; hb[j] = beta; hv0[j] = v0; }
        if (beta != 0.0) {   // same in every thread
            {
                const int r = j1 + (t >> 1), q = t & 1;
                const int rr = min(r, d - 1);
                double acc0 = 0.0, acc1 = 0.0;
                int u = 0;
                for (int c = j1 + q; c < d; c += 2, ++u) {
                    const double vc = (c == j1) ? v0 : S[c + j * LDL];
                    const double sv = S[rr + c * LDL];
                    if (u & 1) acc1 = fma(sv, vc, acc1);
                    else acc0 = fma(sv, vc, acc0);
                }
                double acc = acc0 + acc1;
                acc += row_partner<1>(acc);
                const double pr = beta * acc;
                const double vr = (rr == j1) ? v0 : S[rr + j * LDL];
                const double kp = wave_sum64((q == 0 && r < d) ? pr * vr : 0.0);
                if (q == 0 && r < d) hP[r] = pr;
                if ((t & 63) == 0) hkp[t >> 6] = kp;
            }
            __syncthreads();
            {
                const double K = 0.5 * beta * ((hkp[0] + hkp[1]) + (hkp[2] + hkp[3]));
                const int nt = d - j1;
                for (int e = t; e < nt * nt; e += DT) {
                    const int r = j1 + e % nt, c = j1 + e / nt;
                    const double vr = (r == j1) ? v0 : S[r + j * LDL];
                    const double vc = (c == j1) ? v0 : S[c + j * LDL];
                    const double wr = fma(-K, vr, hP[r]);
                    const double wc = fma(-K, vc, hP[c]);
                    S[r + c * LDL] = S[r + c * LDL] - __dadd_rn(__dmul_rn(vr, wc), __dmul_rn(wr, vc));
                }
            }
        }
        __syncthreads();
        if (t < 64) {
            double x2 = 0.0;
            for (int r = j1 + 2 + t; r < d; r += 64) x2 = fma(S[r + j1 * LDL], S[r + j1 * LDL], x2);
            const double sg = wave_sum64(x2);
            if (t == 0) hsig[0] = sg;
        }
        __syncthreads();
    }
    if (t == 0) {
        ta[d - 2] = S[d - 2 + (d - 2) * LDL];
        tb[d - 2] = S[d - 1 + (d - 2) * LDL];
        ta[d - 1] = S[d - 1 + (d - 1) * LDL];
    }
    __syncthreads();
    if (t < d - 1) tb2[t] = tb[t] * tb[t];
    __syncthreads();

    // ---- the wanted eigenvalues of T (as in k_dense_sym)
    double tnorm = 0.0, pivmin = 0.0;
    const int kn = multisect_select(d, k_target, ta, tb, tb2, blo, bhi, lam, bsh, bcnt, isel, lsel, tnorm, pivmin);
    if (t == 0) {
        need2_s = 0;
        fail_s = 0;
    }
    __syncthreads();

    // ---- eigenvectors of T by twisted factorizations (as in k_dense_sym), pivots in V
    double* Fp = V;
    double* Fm = V + DMAX * KMAX;
    if (t < 64) {
        const int o = t >> 1, side = t & 1;
        const bool act = o < kn;
        const int oc = min(o, KMAX - 1);
        const int ie = act ? isel[oc] : 0;
        const double lo_ = blo[ie], hi_ = bhi[ie];
        double lm = act ? lsel[oc] : 0.0;
        auto frcp = [](double v) {
            double rc = __builtin_amdgcn_rcp(v);
            rc = fma(rc, fma(-v, rc, 1.0), rc);
            return fma(rc, fma(-v, rc, 1.0), rc);
        };
        for (int pass = 0; pass < 2; ++pass) {
            if (act) {
                if (side == 0) {
                    double dp = ta[0] - lm;
                    if (fabs(dp) < pivmin) dp = -pivmin;
                    Fp[o] = dp;
                    for (int s2 = 1; s2 < d; ++s2) {
                        dp = fma(-tb2[s2 - 1], frcp(dp), ta[s2] - lm);
                        if (fabs(dp) < pivmin) dp = -pivmin;
                        Fp[s2 * KMAX + o] = dp;
                    }
                } else {
                    double dm = ta[d - 1] - lm;
                    if (fabs(dm) < pivmin) dm = -pivmin;
                    Fm[(d - 1) * KMAX + o] = dm;
                    for (int ib = d - 2; ib >= 0; --ib) {
                        dm = fma(-tb2[ib], frcp(dm), ta[ib] - lm);
                        if (fabs(dm) < pivmin) dm = -pivmin;
                        Fm[ib * KMAX + o] = dm;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int rt = 0;
            double gam = 0.0, nz = 0.0;
            if (act) {
                double gb = __builtin_inf();
                for (int i = 0; i < d; ++i) {
                    const double g = Fp[i * KMAX + o] + Fm[i * KMAX + o] - (ta[i] - lm);
                    if (fabs(g) < gb) { gb = fabs(g); gam = g; rt = i; }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (act) {
                double z = 1.0;
                if (side == 0) {
                    for (int i = rt - 1; i >= 0; --i) {
                        z = -tb[i] * z * frcp(Fp[i * KMAX + o]);
                        Fp[i * KMAX + o] = z;
                        nz = fma(z, z, nz);
                    }
                    Fp[rt * KMAX + o] = 1.0;
                } else {
                    for (int i = rt; i + 1 < d; ++i) {
                        z = -tb[i] * z * frcp(Fm[(i + 1) * KMAX + o]);
                        Fp[(i + 1) * KMAX + o] = z;
                        nz = fma(z, z, nz);
                    }
                }
            }
            const double nzo = row_partner<1>(nz);
            const double nz2 = 1.0 + (side == 0 ? nz + nzo : nzo + nz);
            if (act && pass == 0) {
                const double ln = lm + gam / nz2;
                if (ln == ln) lm = fmin(fmax(ln, lo_), hi_);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();

    // ---- back-transformation and modified Gram-Schmidt, eight lanes per column (column c = t / 8,
    // rows t % 8 + 8 i, i < RPL, in registers); the finished columns go to V
    const int zc = t >> 3, part = t & 7;
    double zr[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int r = part + 8 * i;
        zr[i] = (zc < kn && r < d) ? Fp[r * KMAX + zc] : 0.0;
    }
    __syncthreads();
    for (int j = d - 3; j >= 0; --j) {
        const double beta = hb[j];
        if (beta == 0.0) continue;
        const double v0 = hv0[j];
        double vr[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = part + 8 * i;
            const double sv = S[min(r, d - 1) + j * LDL];
            const double m1 = (r > j + 1 && r < d) ? 1.0 : 0.0, m0 = (r == j + 1) ? 1.0 : 0.0;
            vr[i] = fma(m1, sv, m0 * v0);
        }
        double dt0 = 0.0, dt1 = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            if (i & 1) dt1 = fma(vr[i], zr[i], dt1);
            else dt0 = fma(vr[i], zr[i], dt0);
        }
        double dot = dt0 + dt1;
        dot = group8_sum(dot);
        dot *= beta;
#pragma unroll
        for (int i = 0; i < RPL; ++i) zr[i] = fma(-dot, vr[i], zr[i]);
    }
    auto sq8 = [&]() {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            if (i & 1) a1 = fma(zr[i], zr[i], a1);
            else a0 = fma(zr[i], zr[i], a0);
        }
        return sqrt(group8_sum(a0 + a1));
    };
    const double n0 = sq8();
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < kn; ++j) {
            const double nr = sq8();
            if (zc == j) {
                if (pass == 0) {
                    if (!(nr > 1e-8 * n0) || !(n0 < __builtin_inf())) fail_s = 1;
                    else if (nr < 0.7 * n0) need2_s = 1;
                }
                const double inv = (nr > 0.0) ? 1.0 / nr : 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    zr[i] *= inv;
                    const int r = part + 8 * i;
                    if (r < d) V[r + j * LDL] = zr[i];
                }
            }
            __syncthreads();
            double qv[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int r = part + 8 * i;
                qv[i] = (r < d) ? V[r + j * LDL] : 0.0;
            }
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                if (i & 1) d1 = fma(qv[i], zr[i], d1);
                else d0 = fma(qv[i], zr[i], d0);
            }
            double dot = d0 + d1;
            dot = group8_sum(dot);
            const double f = (zc > j && zc < kn) ? dot : 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) zr[i] = fma(-f, qv[i], zr[i]);
        }
        __syncthreads();
        if (fail_s || !need2_s) break;
    }
    if (fail_s) {
        if (t == 0) dw->mode = DW_GEN_L;
        return;
    }
    if (t < kn) sel[t] = t;
    // R_G again, in S (the reflectors are no longer needed)
    stage_block(S, LDL, dw->R, DMAX, d, d, t, DT);
    __syncthreads();
    // Qc = Q_G [Q_w; 0]: one lane per column, the rotations of Q_G in reverse order
    if (t < kn) {
        const int o = t, col = sel[o];
        double carry = 0.0;
        for (int c = d - 1; c >= kc; --c) {
            const double a = V[c + col * LDL];
            coef->Qc[c + 1 + o * LDQC] = gsn[c] * a + gcs[c] * carry;
            carry = gcs[c] * a - gsn[c] * carry;
        }
        coef->Qc[kc + o * LDQC] = carry;
        for (int c = 0; c < kc; ++c) coef->Qc[c + o * LDQC] = V[c + col * LDL];
    }
    // Qu = R_G^{-1} Q_w by back-substitution, eight lanes per column with lane part p holding rows
    // RPL p .. RPL p + RPL - 1 (y_i broadcast from its owner); the rows of the recycled part carry D_k
    {
        const int o = t >> 3, p = t & 7;
        const int col = sel[min(o, KMAX - 1)];
        double y[RPL];
#pragma unroll
        for (int s2 = 0; s2 < RPL; ++s2) {
            const int r = RPL * p + s2;
            y[s2] = (o < kn && r < d) ? V[r + col * LDL] : 0.0;
        }
        for (int i0 = ((d - 1) / RPL) * RPL; i0 >= 0; i0 -= RPL) {
            const int owner = i0 / RPL;
#pragma unroll
            for (int s1 = RPL - 1; s1 >= 0; --s1) {
                const int i = i0 + s1;
                if (i < d) {
                    double rq[RPL];
#pragma unroll
                    for (int s2 = 0; s2 < RPL; ++s2) rq[s2] = S[min(RPL * p + s2, d - 1) + i * LDL];
                    const double yl = y[s1] * Rd[i];
                    y[s1] = (p == owner) ? yl : y[s1];
                    const double yi = __shfl(yl, (t & ~7) | owner, 64);
#pragma unroll
                    for (int s2 = 0; s2 < RPL; ++s2) {
                        const double f = (RPL * p + s2 < i) ? yi : 0.0;
                        y[s2] = fma(-f, rq[s2], y[s2]);
                    }
                }
            }
        }
        if (o < kn) {
#pragma unroll
            for (int s2 = 0; s2 < RPL; ++s2) {
                const int r = RPL * p + s2;
                if (r < d) coef->Qu[r + o * LDQU] = (r < kc ? Dk[r < KMAX ? r : 0] : 1.0) * y[s2];
            }
        }
    }
    __syncthreads();
    if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 0; ctrl->route = 1; dw->mode = DW_DONE; }
}
__global__ __launch_bounds__(DT) void k_dense_sym_L(int k_target, double sym_tol, Coef* coef, DenseWork* dw,
                                                    Ctrl* ctrl) {
    k_dense_sym_L_body(k_target, sym_tol, coef, dw, ctrl);
}


// General stage for d > DSM. LDS regions: XR (X'', then M, then the Schur form T, then the
// back-transformed vectors and the back-substitution scratch), ZR (R_G, then the Schur vectors,
// then R_G again), WV (the selected eigenvectors in the Schur basis, then Q_w).
__device__ __forceinline__ void k_dense_gen_L_body(int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    if (dw->mode != DW_GEN_L) return;
    __shared__ double XR[LDL * MMAX];
    __shared__ double ZR[LDL * MMAX];
    __shared__ double WV[LDL * KMAX];
    __shared__ double gcs[MMAX], gsn[MMAX], Dk[KMAX], wr[MMAX], wi[MMAX], hv[MMAX + 1], Rd[MMAX];
    __shared__ int taken[MMAX], sel_pos[KMAX], sel_cplx[KMAX], sel_col[KMAX];
    double* X = XR;
    double* Z = ZR;
    double* Wv = WV;
    double* Uq = XR;
    const int t = threadIdx.x;
    const int d = dw->d, kc = dw->kc;
    const double eps = 2.220446049250313e-16;
    stage_block(X, LDL, dw->X, DMAX, d, d, t, 64);
    stage_block(Z, LDL, dw->R, DMAX, d, d, t, 64);
    for (int r = t; r < d; r += 64) { gcs[r] = dw->gcs[r]; gsn[r] = dw->gsn[r]; }
    if (t < kc) Dk[t] = dw->Dk[t];
    __syncthreads();

    // ---- M = X'' R_G^{-1}: row r solves m R = x'' (right-looking over the columns)
    for (int r = t; r < d; r += 64) Rd[r] = 1.0 / Z[r + r * LDL];
    __syncthreads();
    for (int r = t; r < d; r += 64)
        for (int c = 0; c < d; ++c) {
            const double mc = X[r + c * LDL] * Rd[c];
            X[r + c * LDL] = mc;
            for (int q = c + 1; q < d; ++q) X[r + q * LDL] = fma(-mc, Z[c + q * LDL], X[r + q * LDL]);
        }
    __syncthreads();
    // Z = I
    for (int c = 0; c < d; ++c)
        for (int r = t; r < d; r += 64) Z[r + c * LDL] = (r == c) ? 1.0 : 0.0;
    __syncthreads();

    // ---- Householder reduction of M to upper Hessenberg form, Z accumulates the reflectors
    for (int c = 0; c + 2 < d; ++c) {
        double sp = 0.0;
        for (int r = t; r < d; r += 64)
            if (r >= c + 2) sp = fma(X[r + c * LDL], X[r + c * LDL], sp);
        const double sig = wave_sum64(sp);
        const double x0 = X[c + 1 + c * LDL];
        if (sig == 0.0) continue;
        const double mu = sqrt(x0 * x0 + sig);
        const double v0 = (x0 <= 0.0) ? x0 - mu : -sig / (x0 + mu);
        const double tau = 2.0 * v0 * v0 / (sig + v0 * v0);
        for (int r = t; r < d; r += 64)
            if (r >= c + 1) hv[r] = (r == c + 1) ? 1.0 : X[r + c * LDL] / v0;
        __syncthreads();
        for (int q = t; q < d; q += 64)
            if (q >= c) {
                double s = 0.0;
                for (int r = c + 1; r < d; ++r) s = fma(hv[r], X[r + q * LDL], s);
                s *= tau;
                for (int r = c + 1; r < d; ++r) X[r + q * LDL] = fma(-s, hv[r], X[r + q * LDL]);
            }
        __syncthreads();
        for (int r = t; r < d; r += 64) {
            double s = 0.0, sz = 0.0;
            for (int q = c + 1; q < d; ++q) {
                s = fma(X[r + q * LDL], hv[q], s);
                sz = fma(Z[r + q * LDL], hv[q], sz);
            }
            s *= tau;
            sz *= tau;
            for (int q = c + 1; q < d; ++q) {
                X[r + q * LDL] = fma(-s, hv[q], X[r + q * LDL]);
                Z[r + q * LDL] = fma(-sz, hv[q], Z[r + q * LDL]);
            }
        }
        __syncthreads();
        for (int r = t; r < d; r += 64)
            if (r >= c + 2) X[r + c * LDL] = 0.0;
        if (t == 0) X[c + 1 + c * LDL] = mu;
        __syncthreads();
    }

    // ---- Francis double-shift QR to real Schur form (T in X, Z accumulated)
    double tn = 0.0;
    for (int r = t; r < d; r += 64)
        for (int c = 0; c < d; ++c) tn = fmax(tn, fabs(X[r + c * LDL]));
    const double tnorm = wave_max64(tn);
    int hi = d - 1, its = 0, total = 0;
    bool failed = false;
    while (hi >= 0) {
        // l: the largest row index in 1..hi whose subdiagonal entry is negligible (0 if none)
        bool small0 = false, small1 = false;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int r = t + 64 * half;
            bool sm = false;
            if (r >= 1 && r <= hi) {
                double sc = fabs(X[r - 1 + (r - 1) * LDL]) + fabs(X[r + r * LDL]);
                if (sc == 0.0) sc = tnorm;
                sm = fabs(X[r + (r - 1) * LDL]) <= eps * sc;
            }
            if (half == 0) small0 = sm;
            else small1 = sm;
        }
        const unsigned long long m0 = __ballot(small0), m1 = __ballot(small1);
        const int l = m1 ? 64 + 63 - __clzll(m1) : (m0 ? 63 - __clzll(m0) : 0);
        __syncthreads();
        if (l > 0 && t == 0) X[l + (l - 1) * LDL] = 0.0;
        __syncthreads();
        if (l == hi) {
            if (t == 0) { wr[hi] = X[hi + hi * LDL]; wi[hi] = 0.0; }
            hi -= 1;
            its = 0;
            __syncthreads();
            continue;
        }
        if (l == hi - 1) {
            const int p = hi - 1, q = hi;
            const double a = X[p + p * LDL], b = X[p + q * LDL], c = X[q + p * LDL], dd = X[q + q * LDL];
            const double pp = 0.5 * (a - dd), bc = b * c, disc = pp * pp + bc;
            if (disc >= 0.0) {
                const double zz = pp + copysign(sqrt(disc), pp);
                const double rho = hypot(zz, c);
                const double cs = rho > 0.0 ? zz / rho : 1.0, sn = rho > 0.0 ? c / rho : 0.0;
                __syncthreads();
                for (int e = t; e < d; e += 64)
                    if (e >= p) {
                        const double r0 = X[p + e * LDL], r1 = X[q + e * LDL];
                        X[p + e * LDL] = cs * r0 + sn * r1;
                        X[q + e * LDL] = -sn * r0 + cs * r1;
                    }
                __syncthreads();
                for (int e = t; e <= q; e += 64) {
                    const double c0 = X[e + p * LDL], c1 = X[e + q * LDL];
                    X[e + p * LDL] = cs * c0 + sn * c1;
                    X[e + q * LDL] = -sn * c0 + cs * c1;
                }
                for (int e = t; e < d; e += 64) {
                    const double z0 = Z[e + p * LDL], z1 = Z[e + q * LDL];
                    Z[e + p * LDL] = cs * z0 + sn * z1;
                    Z[e + q * LDL] = -sn * z0 + cs * z1;
                }
                __syncthreads();
                if (t == 0) {
                    X[q + p * LDL] = 0.0;
                    wr[p] = X[p + p * LDL];
                    wr[q] = X[q + q * LDL];
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
            const double s = fabs(X[l + 1 + l * LDL]) + fabs(X[l + 2 + (l + 1) * LDL]);
            h11 = 0.75 * s + X[l + l * LDL]; h12 = -0.4375 * s; h21 = s; h22 = h11;
        } else if (its == 20) {
            const double s = fabs(X[hi + (hi - 1) * LDL]) + fabs(X[hi - 1 + (hi - 2) * LDL]);
            h11 = 0.75 * s + X[hi + hi * LDL]; h12 = -0.4375 * s; h21 = s; h22 = h11;
        } else {
            h11 = X[hi - 1 + (hi - 1) * LDL]; h12 = X[hi - 1 + hi * LDL];
            h21 = X[hi + (hi - 1) * LDL]; h22 = X[hi + hi * LDL];
        }
        const double str = h11 + h22, sdet = h11 * h22 - h12 * h21;
        const double a00 = X[l + l * LDL], a01 = X[l + (l + 1) * LDL];
        const double a10 = X[l + 1 + l * LDL], a11 = X[l + 1 + (l + 1) * LDL], a21 = X[l + 2 + (l + 1) * LDL];
        double px = a00 * a00 + a01 * a10 - str * a00 + sdet;
        double py = a10 * (a00 + a11 - str);
        double pz = a10 * a21;
        for (int kk = l; kk <= hi - 2; ++kk) {
            double v1, v2, tau, alpha;
            house3(px, py, pz, v1, v2, tau, alpha);
            __syncthreads();
            if (tau != 0.0) {
                const int c0 = (kk > l) ? kk - 1 : l;
                for (int e = t; e < d; e += 64)
                    if (e >= c0) {
                        const double a = X[kk + e * LDL], b = X[kk + 1 + e * LDL], c = X[kk + 2 + e * LDL];
                        const double s = tau * (a + v1 * b + v2 * c);
                        X[kk + e * LDL] = a - s;
                        X[kk + 1 + e * LDL] = b - s * v1;
                        X[kk + 2 + e * LDL] = c - s * v2;
                    }
                __syncthreads();
                const int r1 = min(kk + 3, hi);
                for (int e = t; e <= r1; e += 64) {
                    const double a = X[e + kk * LDL], b = X[e + (kk + 1) * LDL], c = X[e + (kk + 2) * LDL];
                    const double s = tau * (a + v1 * b + v2 * c);
                    X[e + kk * LDL] = a - s;
                    X[e + (kk + 1) * LDL] = b - s * v1;
                    X[e + (kk + 2) * LDL] = c - s * v2;
                }
                for (int e = t; e < d; e += 64) {
                    const double a = Z[e + kk * LDL], b = Z[e + (kk + 1) * LDL], c = Z[e + (kk + 2) * LDL];
                    const double s = tau * (a + v1 * b + v2 * c);
                    Z[e + kk * LDL] = a - s;
                    Z[e + (kk + 1) * LDL] = b - s * v1;
                    Z[e + (kk + 2) * LDL] = c - s * v2;
                }
                __syncthreads();
            }
            if (kk > l && t == 0) {
                X[kk + (kk - 1) * LDL] = alpha;
                X[kk + 1 + (kk - 1) * LDL] = 0.0;
                X[kk + 2 + (kk - 1) * LDL] = 0.0;
            }
            __syncthreads();
            px = X[kk + 1 + kk * LDL];
            py = X[kk + 2 + kk * LDL];
            pz = (kk < hi - 2) ? X[kk + 3 + kk * LDL] : 0.0;
        }
        // closing 2-element reflector on rows/columns hi-1, hi
        {
            const int kk = hi - 1;
            double v1, v2, tau, alpha;
            house3(px, py, 0.0, v1, v2, tau, alpha);
            __syncthreads();
            if (tau != 0.0) {
                const int c0 = kk - 1;
                for (int e = t; e < d; e += 64)
                    if (e >= c0) {
                        const double a = X[kk + e * LDL], b = X[kk + 1 + e * LDL];
                        const double s = tau * (a + v1 * b);
                        X[kk + e * LDL] = a - s;
                        X[kk + 1 + e * LDL] = b - s * v1;
                    }
                __syncthreads();
                for (int e = t; e <= hi; e += 64) {
                    const double a = X[e + kk * LDL], b = X[e + (kk + 1) * LDL];
                    const double s = tau * (a + v1 * b);
                    X[e + kk * LDL] = a - s;
                    X[e + (kk + 1) * LDL] = b - s * v1;
                }
                for (int e = t; e < d; e += 64) {
                    const double a = Z[e + kk * LDL], b = Z[e + (kk + 1) * LDL];
                    const double s = tau * (a + v1 * b);
                    Z[e + kk * LDL] = a - s;
                    Z[e + (kk + 1) * LDL] = b - s * v1;
                }
                __syncthreads();
            }
            if (t == 0) {
                X[kk + (kk - 1) * LDL] = alpha;
                X[kk + 1 + (kk - 1) * LDL] = 0.0;
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
        if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 1; ctrl->route = 2; dw->mode = DW_DONE; }
        return;
    }

    // ---- select the k eigenvalues of largest |mu| (smallest |theta|); a conjugate pair counts two.
    // Each lane takes the better of its two rows (the lower index on a tie), then a butterfly picks
    // the largest key, ties to the lower index.
    for (int r = t; r < d; r += 64) taken[r] = 0;
    __syncthreads();
    int nsel = 0, ncols = 0;
    while (ncols < k_target) {
        double key = -1.0;
        int idx = t;
        for (int r = t; r < d; r += 64) {
            if (!taken[r] && wi[r] >= 0.0) {
                const double mag = hypot(wr[r], wi[r]);
                if (mag > 0.0 && mag > key) { key = mag; idx = r; }
            }
        }
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
        double* xr = Wv + col * LDL;
        if (!sel_cplx[t]) {
            const double lam = wr[p];
            for (int r = 0; r < d; ++r) xr[r] = 0.0;
            xr[p] = 1.0;
            int r = p - 1;
            while (r >= 0) {
                if (r > 0 && X[r + (r - 1) * LDL] != 0.0) {
                    double s1 = 0.0, s2 = 0.0;
                    for (int c = r + 1; c <= p; ++c) {
                        s1 = fma(X[r - 1 + c * LDL], xr[c], s1);
                        s2 = fma(X[r + c * LDL], xr[c], s2);
                    }
                    const double a = X[r - 1 + (r - 1) * LDL] - lam, b = X[r - 1 + r * LDL];
                    const double c = X[r + (r - 1) * LDL], dd = X[r + r * LDL] - lam;
                    double det = a * dd - b * c;
                    if (fabs(det) < smin * smin) det = copysign(smin * smin, det);
                    xr[r - 1] = (-s1 * dd + b * s2) / det;
                    xr[r] = (-a * s2 + c * s1) / det;
                    r -= 2;
                } else {
                    double s = 0.0;
                    for (int c = r + 1; c <= p; ++c) s = fma(X[r + c * LDL], xr[c], s);
                    double den = X[r + r * LDL] - lam;
                    if (fabs(den) < smin) den = copysign(smin, den);
                    xr[r] = -s / den;
                    r -= 1;
                }
            }
        } else {
            // pair at (p, p+1), lambda = wr + i wi: x_p = lambda - T_{p+1,p+1}, x_{p+1} = T_{p+1,p}
            const double lr = wr[p], li = wi[p];
            double* xi = Wv + (col + 1) * LDL;
            for (int r = 0; r < d; ++r) { xr[r] = 0.0; xi[r] = 0.0; }
            xr[p] = lr - X[p + 1 + (p + 1) * LDL];
            xi[p] = li;
            xr[p + 1] = X[p + 1 + p * LDL];
            xi[p + 1] = 0.0;
            int r = p - 1;
            while (r >= 0) {
                if (r > 0 && X[r + (r - 1) * LDL] != 0.0) {
                    double s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
                    for (int c = r + 1; c <= p + 1; ++c) {
                        s1r = fma(X[r - 1 + c * LDL], xr[c], s1r);
                        s1i = fma(X[r - 1 + c * LDL], xi[c], s1i);
                        s2r = fma(X[r + c * LDL], xr[c], s2r);
                        s2i = fma(X[r + c * LDL], xi[c], s2i);
                    }
                    const double ar = X[r - 1 + (r - 1) * LDL] - lr, ai = -li;
                    const double b = X[r - 1 + r * LDL], c = X[r + (r - 1) * LDL];
                    const double dr = X[r + r * LDL] - lr, di = -li;
                    double detr = ar * dr - ai * di - b * c, deti = ar * di + ai * dr;
                    if (fabs(detr) + fabs(deti) < smin * smin) detr = smin * smin;
                    const double n1r = -(s1r * dr - s1i * di) + b * s2r, n1i = -(s1r * di + s1i * dr) + b * s2i;
                    const double n2r = -(ar * s2r - ai * s2i) + c * s1r, n2i = -(ar * s2i + ai * s2r) + c * s1i;
                    cdiv(n1r, n1i, detr, deti, xr[r - 1], xi[r - 1]);
                    cdiv(n2r, n2i, detr, deti, xr[r], xi[r]);
                    r -= 2;
                } else {
                    double sr = 0.0, si = 0.0;
                    for (int c = r + 1; c <= p + 1; ++c) {
                        sr = fma(X[r + c * LDL], xr[c], sr);
                        si = fma(X[r + c * LDL], xi[c], si);
                    }
                    double denr = X[r + r * LDL] - lr, deni = -li;
                    if (fabs(denr) + fabs(deni) < smin) denr = smin;
                    cdiv(-sr, -si, denr, deni, xr[r], xi[r]);
                    r -= 1;
                }
            }
        }
    }
    __syncthreads();
    // back to the basis of M: w = Z x (lane = row), into Uq (T is no longer needed)
    for (int o = 0; o < ncols; ++o)
        for (int r = t; r < d; r += 64) {
            double s = 0.0;
            for (int c = 0; c < d; ++c) s = fma(Z[r + c * LDL], Wv[c + o * LDL], s);
            Uq[r + o * LDL] = s;
        }
    __syncthreads();

    // ---- orthonormal basis Q_w of the selected vectors (modified Gram-Schmidt, two passes)
    const int r0 = t, r1 = t + 64;
    const bool v0 = r0 < d, v1 = r1 < d;
    int kn = 0;
    for (int o = 0; o < ncols; ++o) {
        double w0 = v0 ? Uq[r0 + o * LDL] : 0.0, w1 = v1 ? Uq[r1 + o * LDL] : 0.0;
        const double n0 = sqrt(wave_sum64(fma(w0, w0, w1 * w1)));
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < kn; ++q) {
                const double q0 = v0 ? Wv[r0 + q * LDL] : 0.0, q1 = v1 ? Wv[r1 + q * LDL] : 0.0;
                const double h = wave_sum64(fma(q0, w0, q1 * w1));
                w0 = fma(-h, q0, w0);
                w1 = fma(-h, q1, w1);
            }
        const double nw = sqrt(wave_sum64(fma(w0, w0, w1 * w1)));
        __syncthreads();
        if (nw > 1e-12 * n0 && n0 > 0.0) {
            if (v0) Wv[r0 + kn * LDL] = w0 / nw;
            if (v1) Wv[r1 + kn * LDL] = w1 / nw;
            ++kn;
        }
        __syncthreads();
    }

    // ---- Qu = R_G^{-1} Q_w with D_k folded into the rows of U (lane = column), R_G staged again
    stage_block(Z, LDL, dw->R, DMAX, d, d, t, 64);
    __syncthreads();
    if (t < kn) {
        double* u = Uq + t * LDL;
        for (int r = d - 1; r >= 0; --r) {
            double s = Wv[r + t * LDL];
            for (int c = r + 1; c < d; ++c) s = fma(-Z[r + c * LDL], u[c], s);
            u[r] = s / Z[r + r * LDL];
        }
        for (int r = 0; r < d; ++r) coef->Qu[r + t * LDQU] = (r < kc ? Dk[r] : 1.0) * u[r];
        // Qc = Q_G [Q_w; 0]
        double carry = 0.0;
        for (int c = d - 1; c >= kc; --c) {
            const double a = Wv[c + t * LDL];
            coef->Qc[c + 1 + t * LDQC] = gsn[c] * a + gcs[c] * carry;
            carry = gcs[c] * a - gsn[c] * carry;
        }
        if (kc < d || d == 0) coef->Qc[kc + t * LDQC] = carry;
        for (int c = 0; c < kc; ++c) coef->Qc[c + t * LDQC] = Wv[c + t * LDL];
    }
    if (t == 0) { ctrl->k_new = kn; ctrl->eig_fail = 0; ctrl->route = 2; dw->mode = DW_DONE; }
}
__global__ __launch_bounds__(64) void k_dense_gen_L(int k_target, Coef* coef, DenseWork* dw, Ctrl* ctrl) {
    k_dense_gen_L_body(k_target, coef, dw, ctrl);
}


// ---------------------------------------------------------------------------------------------
// Start-up CholQR: Cholesky of the Gram matrix Z^T Z (kin x kin, row-major in gram). With drops,
// a column whose pivot falls to <= 1e-14 ||z_j||^2 (R_jj <= 1e-7 ||z_j||) is left out.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void k_chol_body(const double* __restrict__ gram, int kin, int with_drop, Coef* coef) {
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
__global__ __launch_bounds__(64) void k_chol(const double* __restrict__ gram, int kin, int with_drop, Coef* coef) {
    k_chol_body(gram, kin, with_drop, coef);
}


void launch_cycle_dense(hipStream_t s, const Work& w, int kc, int jd_max, int k_target) {
    hipLaunchKernelGGL(k_dense_prep, dim3(1), dim3(64), 0, s, (const double*)w.H, (const double*)w.Bm,
                       (const double*)w.gram, kc, jd_max, k_target, w.coef, w.dense, w.ctrl);
    if (k_target > 0) {
        // The symmetric stage runs only for an exactly symmetric operator (ctrl->nonsym). For one,
        // M is symmetric in exact arithmetic and its computed asymmetry is the rounding of the
        // stored columns (FP64 storage: ~1e-15 relative, FP32 storage: up to ~1e-6 on the Darcy
        // workloads); the tolerance is a guard far above that.
        const double sym_tol = w.mixed ? 1e-4 : 1e-10;
        hipLaunchKernelGGL(k_dense_sym, dim3(1), dim3(DT), 0, s, k_target, sym_tol, w.coef, w.dense, w.ctrl);
        hipLaunchKernelGGL(k_dense_gen, dim3(1), dim3(64), 0, s, k_target, w.coef, w.dense, w.ctrl);
    }
    if (w.m > DSM) {
        // d = kc + j_done is known on the device only: the kernels of both sizes are queued and each
        // returns at once unless d falls in its range (the mode set by the first stage selects the
        // general stage)
        hipLaunchKernelGGL(k_dense_prep_L, dim3(1), dim3(64), 0, s, (const double*)w.H, (const double*)w.Bm,
                           (const double*)w.gram, kc, jd_max, k_target, w.coef, w.dense, w.ctrl);
        if (k_target > 0) {
            const double sym_tol = w.mixed ? 1e-4 : 1e-10;
            hipLaunchKernelGGL(k_dense_sym_L, dim3(1), dim3(DT), 0, s, k_target, sym_tol, w.coef, w.dense, w.ctrl);
            hipLaunchKernelGGL(k_dense_gen_L, dim3(1), dim3(64), 0, s, k_target, w.coef, w.dense, w.ctrl);
        }
    }
}
void launch_chol(hipStream_t s, const Work& w, int kin, int with_drop) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(64), 0, s, (const double*)w.gram, kin, with_drop, w.coef);
}

// Batched forms (skr_solve_chains): one workgroup per chain, chain blockIdx.y, the same bodies.
#define SKR_CD const ChainDesc& cd = tab[blockIdx.y]; if (!cd.on) return; const Work& w = cd.w
__global__ __launch_bounds__(64) void kb_dense_prep(const ChainDesc* tab, int k_target) {
    SKR_CD;
    k_dense_prep_body(w.H, w.Bm, w.gram, cd.kc, cd.scyc, k_target, w.coef, w.dense, w.ctrl);
}
__global__ __launch_bounds__(DT) void kb_dense_sym(const ChainDesc* tab, int k_target, double sym_tol) {
    SKR_CD;
    k_dense_sym_body(k_target, sym_tol, w.coef, w.dense, w.ctrl);
}
__global__ __launch_bounds__(64) void kb_dense_gen(const ChainDesc* tab, int k_target) {
    SKR_CD;
    k_dense_gen_body(k_target, w.coef, w.dense, w.ctrl);
}
__global__ __launch_bounds__(64) void kb_dense_prep_L(const ChainDesc* tab, int k_target) {
    SKR_CD;
    k_dense_prep_L_body(w.H, w.Bm, w.gram, cd.kc, cd.scyc, k_target, w.coef, w.dense, w.ctrl);
}
__global__ __launch_bounds__(DT) void kb_dense_sym_L(const ChainDesc* tab, int k_target, double sym_tol) {
    SKR_CD;
    k_dense_sym_L_body(k_target, sym_tol, w.coef, w.dense, w.ctrl);
}
__global__ __launch_bounds__(64) void kb_dense_gen_L(const ChainDesc* tab, int k_target) {
    SKR_CD;
    k_dense_gen_L_body(k_target, w.coef, w.dense, w.ctrl);
}
__global__ __launch_bounds__(64) void kb_chol(const ChainDesc* tab, int with_drop) {
    SKR_CD;
    k_chol_body(w.gram, with_drop ? cd.kin : cd.ke, with_drop, w.coef);
}
#undef SKR_CD
void blaunch_cycle_dense(const Batch& B, int k_target) {
    const dim3 g(1, (unsigned)B.C);
    const double sym_tol = B.w0.mixed ? 1e-4 : 1e-10;
    hipLaunchKernelGGL(kb_dense_prep, g, dim3(64), 0, B.s, B.cd, k_target);
    if (k_target > 0) {
        hipLaunchKernelGGL(kb_dense_sym, g, dim3(DT), 0, B.s, B.cd, k_target, sym_tol);
        hipLaunchKernelGGL(kb_dense_gen, g, dim3(64), 0, B.s, B.cd, k_target);
    }
    if (B.w0.m > DSM) {
        hipLaunchKernelGGL(kb_dense_prep_L, g, dim3(64), 0, B.s, B.cd, k_target);
        if (k_target > 0) {
            hipLaunchKernelGGL(kb_dense_sym_L, g, dim3(DT), 0, B.s, B.cd, k_target, sym_tol);
            hipLaunchKernelGGL(kb_dense_gen_L, g, dim3(64), 0, B.s, B.cd, k_target);
        }
    }
}
void blaunch_chol(const Batch& B, int with_drop) {
    hipLaunchKernelGGL(kb_chol, dim3(1, (unsigned)B.C), dim3(64), 0, B.s, B.cd, with_drop);
}

}  // namespace skr
