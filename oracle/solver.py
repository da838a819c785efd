"""GCRO-DR along a sequence of systems, plain FP64 NumPy/SciPy (oracle, test infrastructure only).

Follows Alg. 2 ("GCRO-DR", App. B.2) with the recycle-space adaptation of App. B.1, the
Arnoldi relation Eq. 3 and the projected Arnoldi relation Eq. 6 (Sec. 4.2). GMRES(m) is this
routine with k = 0 (Sec. 4.2: GMRES is the special case of GCRO-DR with k set to zero).

Readings adopted where the paper is silent or loose (each is mirrored by the GPU library):
* Real arithmetic: the conjugate transposes of the paper become transposes.
* x0 = 0 for every system; the stopping test is relative, ||r|| <= rtol * ||b||.
* Orthogonalisation: classical Gram-Schmidt with one full re-orthogonalisation (CGS2) against
  [C_k, V_j]; B and H accumulate the coefficients of both passes.
* Convergence is tested after every Arnoldi step on the least-squares residual of the
  Hessenberg block (the rows belonging to C_k can always be satisfied exactly, so this is the
  residual of the whole projected problem). ``full_cycles=True`` instead tests only between
  cycles, as printed in Alg. 2.
* The cycle that stops early still updates x, r and the recycle space (when it ran >= 1 step).
* Happy breakdown: h_{j+1,j} <= 1e-14 * ||A v_j|| ends the cycle with an exact projected solve.
* On exit the true residual b - A x is computed; if it is above the tolerance the solve goes on
  from that residual.
* ``maxit`` bounds the Arnoldi steps of one system.
* Start-up QR of A*Y (App. B.1): R has a positive diagonal. A column j with
  R_jj <= 1e-7 * ||(A Y)_j|| is treated as dependent and dropped (fewer recycled vectors).
* Harmonic Ritz selection: the k eigenvalues of smallest modulus (ties by index, infinite
  values never chosen). A complex pair is represented by the real and imaginary parts of one
  eigenvector; when the k-th chosen value is one half of a conjugate pair, that half is dropped.
* A first system (or any system without a recycle space) starts with a GMRES(m) cycle and takes
  the k harmonic Ritz vectors of the standard form (Alg. 2, else branch) when that cycle ran more
  than k steps; otherwise no recycle space is formed.
* A system whose right-hand side is zero returns x = 0 and passes the incoming recycle space on.

Mixed-precision mode (``basis_fp32=True``; the FP32-inner / FP64-refinement variant of the method,
an extension that the paper does not describe):
* Every column kept in the subspace stores is rounded to FP32 when it is stored: the Arnoldi
  vectors v_j and the recycle pair C_k, U_k (after the start-up QR and after each cycle).
* The inner cycle's operator is A with its stored values rounded to FP32 (``A_inner``; by default
  the CSR values rounded, for a matrix-free stencil the matrix assembled from its rounded faces):
  it is applied to the stored (rounded) vectors in the Arnoldi steps and in the start-up product
  A Y. All arithmetic, x, r, Hbar, G, the least-squares and eigen problems stay FP64, and every true
  residual b - A x uses the FP64 operator.
* Iterative refinement at cycle granularity: every cycle starts from the true residual
  r = b - A x computed in FP64 (not at the very first cycle from x = 0, where r = b already),
  projected onto range(C) as at a system start (x += U C^T r, r -= C C^T r), so each cycle
  computes an FP32-stored correction to an FP64 iterate. The projection keeps r orthogonal to C,
  which the cycle's least-squares problem on [C, V] relies on; a true residual is only
  orthogonal to the FP32-stored C up to rounding, and without the projection that component
  grows from cycle to cycle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

CONVERGED = 0
MAXIT = 1
BREAKDOWN = 2      # happy breakdown: converged through an exact projected solve
NONFINITE = 3

RANK_DROP_TOL = 1e-7
BREAKDOWN_TOL = 1e-14


def fp32_store(v: np.ndarray) -> np.ndarray:
    """Round to the nearest FP32 value (ties to even), held in FP64."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def _keep(v: np.ndarray) -> np.ndarray:
    return v


@dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iters: int                 # Arnoldi steps
    cycles: int
    spmv: int                  # all products with A (Arnoldi, start-up A*Y, true residuals)
    relres_true: float
    relres_est: float
    k_start: int = 0           # recycled vectors kept by the start-up QR
    rank_dropped: int = 0      # recycled vectors dropped by the start-up QR
    Y_next: np.ndarray | None = None
    C_last: np.ndarray | None = None                   # C_k matching Y_next (A Y_next = C_last)
    res_history: list = field(default_factory=list)   # ||r|| after the start and after each cycle
    restarts: int = 0          # cycles started from a true residual after a failed exit test
    cycle_log: list = field(default_factory=list)     # keep_cycles: (||r|| at the cycle start, C after it)


def qr_pos(M: np.ndarray):
    """Reduced QR with a non-negative diagonal of R (the unique factorisation when M has full rank)."""
    Q, R = np.linalg.qr(M, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def ls_residual(Hbar: np.ndarray, beta: float) -> float:
    """min_y ||beta e1 - Hbar y||: beta times the first entry of the unit vector orthogonal to range(Hbar)."""
    Qf = np.linalg.qr(Hbar, mode="complete")[0]
    return float(beta * abs(Qf[0, -1]))


# ----------------------------------------------------------------------------------------------
# Harmonic Ritz vectors
# ----------------------------------------------------------------------------------------------
def select_smallest(theta: np.ndarray, Z: np.ndarray, k: int):
    """Real basis P of the eigenvectors of the k smallest-modulus eigenvalues (see module readings).

    Eigenvalues are visited by increasing modulus (ties by index). A complex eigenvalue is taken
    together with its conjugate partner (the remaining eigenvalue closest to its conjugate) as the
    two columns Re z, Im z; when only one slot is left for a pair, the selection stops there.
    """
    theta = np.asarray(theta)
    cand = [i for i in range(theta.size) if np.isfinite(theta[i])]
    cand.sort(key=lambda i: (abs(theta[i]), i))
    cols, vals, used = [], [], set()
    for i in cand:
        if len(cols) >= k:
            break
        if i in used:
            continue
        if np.imag(theta[i]) == 0.0:
            cols.append(np.real(Z[:, i]))
            vals.append(theta[i])
            used.add(i)
            continue
        others = [p for p in cand if p not in used and p != i
                  and np.sign(np.imag(theta[p])) == -np.sign(np.imag(theta[i]))]
        if not others:
            continue
        p = min(others, key=lambda q: (abs(theta[q] - np.conj(theta[i])), q))
        if len(cols) + 2 > k:
            break
        cols.append(np.real(Z[:, i]))
        cols.append(np.imag(Z[:, i]))
        vals.extend([theta[i], theta[p]])
        used.update([i, p])
    P = np.column_stack(cols) if cols else np.zeros((Z.shape[0], 0))
    return P, np.asarray(vals)


def harmonic_ritz_standard(Hbar: np.ndarray, k: int):
    """k harmonic Ritz vectors of H_m + h_{m+1,m}^2 H_m^{-T} e_m e_m^T (Alg. 2, else branch)."""
    j = Hbar.shape[1]
    H = Hbar[:j, :]
    h = Hbar[j, j - 1]
    e = np.zeros(j)
    e[-1] = 1.0
    f = np.linalg.solve(H.T, e)
    M = H.copy()
    M[:, -1] += h * h * f
    theta, Z = np.linalg.eig(M)
    return select_smallest(theta, Z, k)


def harmonic_ritz_generalized(G: np.ndarray, WtV: np.ndarray, k: int):
    """k vectors of G^T G z = theta G^T (W^T V) z with smallest |theta| (Alg. 2, cycle body)."""
    theta, Z = sla.eig(G.T @ G, G.T @ WtV)
    return select_smallest(theta, Z, k)


# ----------------------------------------------------------------------------------------------
# Arnoldi with (I - C C^T) A and CGS2 (Eq. 3 when C is empty, Eq. 6 otherwise)
# ----------------------------------------------------------------------------------------------
def arnoldi_cycle(A, r: np.ndarray, C, s: int, tol_abs: float, full_cycles: bool = False, store=_keep):
    """Up to s Arnoldi steps from v1 = r/||r||.

    Returns (V, Hbar, B, est, breakdown): V is n x (j+1), Hbar (j+1) x j, B kc x j for the j steps
    taken, est the least-squares residual of Hbar against ||r|| e1. ``store`` is applied to every
    Arnoldi vector as it is stored (identity, or FP32 rounding in the mixed-precision mode).
    """
    n = r.size
    kc = 0 if C is None else C.shape[1]
    beta = float(np.linalg.norm(r))
    basis = np.zeros((n, kc + s + 1), order="F")       # [C, v1, v2, ...]
    if kc:
        basis[:, :kc] = C
    basis[:, kc] = store(r / beta)
    Hbar = np.zeros((s + 1, s))
    B = np.zeros((kc, s))
    est = beta
    breakdown = False
    j_done = 0
    for j in range(s):
        w = A @ basis[:, kc + j]
        wn0 = float(np.linalg.norm(w))
        Qb = basis[:, :kc + j + 1]
        c1 = Qb.T @ w
        w = w - Qb @ c1
        c2 = Qb.T @ w
        w = w - Qb @ c2
        c = c1 + c2
        B[:, j] = c[:kc]
        Hbar[:j + 1, j] = c[kc:]
        hn = float(np.linalg.norm(w))
        j_done = j + 1
        if hn <= BREAKDOWN_TOL * wn0:
            breakdown = True
            Hbar[j + 1, j] = 0.0
        else:
            Hbar[j + 1, j] = hn
            basis[:, kc + j + 1] = store(w / hn)
        est = ls_residual(Hbar[:j + 2, :j + 1], beta)
        if breakdown:
            break
        if not full_cycles and est <= tol_abs:
            break
    j = j_done
    return basis[:, kc:kc + j + 1], Hbar[:j + 1, :j], B[:, :j], est, breakdown


# ----------------------------------------------------------------------------------------------
# Start-up with a recycled space (App. B.1; Alg. 2, if branch)
# ----------------------------------------------------------------------------------------------
def startup(A, Y: np.ndarray, r0: np.ndarray, store=_keep):
    """[Q,R] = qr(A Y); C = Q; U = Y R^-1; x1 = U C^T r0; r1 = r0 - C C^T r0 (with column drops).
    C and U pass through ``store`` before they are used."""
    Z = A @ Y
    keep = list(range(Y.shape[1]))
    while keep:
        Q, R = qr_pos(Z[:, keep])
        bad = [t for t in range(len(keep))
               if not R[t, t] > RANK_DROP_TOL * np.linalg.norm(Z[:, keep[t]])]
        if not bad:
            break
        del keep[bad[0]]
    dropped = Y.shape[1] - len(keep)
    if not keep:
        return np.zeros_like(r0), r0.copy(), None, None, dropped
    C = store(Q)
    U = store(sla.solve_triangular(R, Y[:, keep].T, trans="T", lower=False).T)    # Y R^{-1}
    c = C.T @ r0
    x1 = U @ c
    r1 = r0 - C @ c
    return x1, r1, C, U, dropped


def project_onto_c(x: np.ndarray, r: np.ndarray, C, U):
    """x + U C^T r and r - C C^T r (App. B.1, the projection of a system start); identity without C."""
    if C is None:
        return x, r
    c = C.T @ r
    return x + U @ c, r - C @ c


# ----------------------------------------------------------------------------------------------
# Cycle-end matrices (Alg. 2, while body)
# ----------------------------------------------------------------------------------------------
def cycle_matrices(C: np.ndarray, U: np.ndarray, V: np.ndarray, Hbar: np.ndarray, B: np.ndarray):
    """G, W^ and V^ of a GCRO-DR cycle of j steps: D_k scales U to unit columns, V^ = [U D_k, V_j],
    W^ = [C, V_{j+1}] and G = [[D_k, B], [0, Hbar]], so that A V^ = W^ G (Eq. 6 with A U = C)."""
    kc = C.shape[1]
    j = Hbar.shape[1]
    d = 1.0 / np.linalg.norm(U, axis=0)               # D_k: U D_k has unit columns
    Vhat = np.hstack([U * d[None, :], V[:, :j]])
    What = np.hstack([C, V])
    G = np.zeros((kc + j + 1, kc + j))
    G[:kc, :kc] = np.diag(d)
    G[:kc, kc:] = B
    G[kc:, kc:] = Hbar
    return G, What, Vhat


# ----------------------------------------------------------------------------------------------
# One system
# ----------------------------------------------------------------------------------------------
def fp32_operator(A):
    """A with its stored values rounded to FP32 (the mixed mode's inner operator of a CSR matrix)."""
    Ai = A.copy()
    Ai.data = fp32_store(Ai.data)
    return Ai


def gcrodr(A, b: np.ndarray, Y: np.ndarray | None = None, m: int = 30, k: int = 10,
           rtol: float = 1e-8, maxit: int = 10000, full_cycles: bool = False,
           basis_fp32: bool = False, keep_cycles: bool = False, A_inner=None) -> SolveResult:
    """Solve A x = b from x0 = 0, recycling span(Y) (App. B.2, Alg. 2). Returns the next Y in Y_next.
    ``basis_fp32`` selects the mixed-precision mode described in the module notes, with inner operator
    ``A_inner`` (default: fp32_operator(A)); ``keep_cycles`` records, per cycle, the residual norm it
    started from and the recycle space C it left."""
    if k < 0 or m <= k or rtol <= 0:
        raise ValueError("need 0 <= k < m and rtol > 0")
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n)
    if not (np.all(np.isfinite(b)) and np.all(np.isfinite(A.data))):
        return SolveResult(x, NONFINITE, 0, 0, 0, np.nan, np.nan, Y_next=Y)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return SolveResult(x, CONVERGED, 0, 0, 0, 0.0, 0.0, Y_next=Y)
    tol_abs = rtol * bnorm
    store = fp32_store if basis_fp32 else _keep
    Ai = (A_inner if A_inner is not None else fp32_operator(A)) if basis_fp32 else A
    r = b.copy()
    r_fresh = True                   # r is b - A x computed directly (x = 0 here) or just projected
    C = U = None
    spmv = iters = cycles = 0
    k_start = dropped = 0
    restarts = 0
    cycle_log = []
    if k > 0 and Y is not None and Y.shape[1] > 0:
        x, r, C, U, dropped = startup(Ai, Y, r, store)
        spmv += Y.shape[1]
        k_start = 0 if C is None else C.shape[1]
        # r was just projected; with FP32-stored C and U the first cycle still refines from the
        # true residual (A U equals C only to FP32 rounding)
        r_fresh = C is None or not basis_fp32
    hist = [float(np.linalg.norm(r))]
    est = hist[0]
    status = None
    breakdown = False
    rt_norm = None
    if hist[0] <= tol_abs:           # the projection onto C already solved the system
        rt = b - A @ x
        spmv += 1
        rt_norm = float(np.linalg.norm(rt))
        if rt_norm <= tol_abs:
            status = CONVERGED
        else:
            x, r = project_onto_c(x, rt, C, U)
            r_fresh = True
            restarts += 1
    while status is None:
        if iters >= maxit:
            status = MAXIT
            break
        if not r_fresh:
            if basis_fp32:
                # refinement step: the cycle corrects the FP64 iterate from its true residual,
                # projected onto range(C) as at a system start (App. B.1)
                spmv += 1
                x, r = project_onto_c(x, b - A @ x, C, U)
            else:
                # the same projection of the current residual (x += U C^T r, r -= C C^T r): zero in
                # exact arithmetic, where r stays orthogonal to C; in floating point it removes the
                # rounding-level component along C that a cycle leaves in r, which would otherwise
                # persist at a fixed absolute size and, relative to the shrinking residual, tilt
                # v1 = r/||r|| (and with it the next C) out of orthogonality
                x, r = project_onto_c(x, r, C, U)
        r_fresh = False
        s = m if C is None else m - C.shape[1]
        s = min(s, maxit - iters)
        V, Hbar, B, est, breakdown = arnoldi_cycle(Ai, r, C, s, tol_abs, full_cycles, store)
        j = Hbar.shape[1]
        iters += j
        spmv += j
        cycles += 1
        beta = float(np.linalg.norm(r))
        if C is None:
            # GMRES(m) cycle (Alg. 2, else branch): min ||c - Hbar y||, x += V_j y, r = V_{j+1}(c - Hbar y)
            cvec = np.zeros(j + 1)
            cvec[0] = beta
            y = np.linalg.lstsq(Hbar, cvec, rcond=None)[0]
            x = x + V[:, :j] @ y
            r = V @ (cvec - Hbar @ y)
            if k > 0 and j > k:
                P, _ = harmonic_ritz_standard(Hbar, k)
                if P.shape[1] > 0:
                    Yt = V[:, :j] @ P
                    Q, R = qr_pos(Hbar @ P)
                    C = store(V @ Q)
                    U = store(sla.solve_triangular(R, Yt.T, trans="T", lower=False).T)
        else:
            # GCRO-DR cycle (Alg. 2, while body)
            G, What, Vhat = cycle_matrices(C, U, V, Hbar, B)
            rhs = What.T @ r
            y = np.linalg.lstsq(G, rhs, rcond=None)[0]
            x = x + Vhat @ y
            r = r - What @ (G @ y)
            P, _ = harmonic_ritz_generalized(G, What.T @ Vhat, k)
            if P.shape[1] > 0:
                Yt = Vhat @ P
                Q, R = qr_pos(G @ P)
                C = store(What @ Q)
                U = store(sla.solve_triangular(R, Yt.T, trans="T", lower=False).T)
        hist.append(float(np.linalg.norm(r)))
        if keep_cycles:
            cycle_log.append((beta, None if C is None else C.copy()))
        if est <= tol_abs or breakdown:
            rt = b - A @ x
            spmv += 1
            rt_norm = float(np.linalg.norm(rt))
            if rt_norm <= tol_abs:
                status = BREAKDOWN if breakdown else CONVERGED
                break
            # the estimate met the tolerance but the true residual does not (rounding drift): go on
            # from the true residual, projected onto range(C) as at a system start (App. B.1), so
            # that the next cycle's v1 is orthogonal to C as the cycle's least-squares problem and
            # the structure of W^T V^ assume
            x, r = project_onto_c(x, rt, C, U)
            r_fresh = True
            restarts += 1
    if status == MAXIT:
        rt_norm = float(np.linalg.norm(b - A @ x))
        spmv += 1
    Y_next = U if (k > 0 and U is not None) else None
    return SolveResult(x, status, iters, cycles, spmv, rt_norm / bnorm, float(est / bnorm),
                       k_start, dropped, Y_next, C if Y_next is not None else None, hist, restarts,
                       cycle_log)


def gmres(A, b, m: int = 30, rtol: float = 1e-8, maxit: int = 10000) -> SolveResult:
    """Restarted GMRES(m): GCRO-DR with k = 0 (Sec. 4.2)."""
    return gcrodr(A, b, None, m, 0, rtol, maxit)


def solve_sequence(As, bs, order=None, m: int = 30, k: int = 10, rtol: float = 1e-8,
                   maxit: int = 10000, full_cycles: bool = False, limit: int | None = None,
                   basis_fp32: bool = False, A_inner=None):
    """Solve the systems in ``order`` (identity when None), carrying Y = U_k from each to the next.

    Returns a list of SolveResult indexed by original system index (None for systems not solved
    when ``limit`` stops the sequence early).
    """
    N = len(As)
    order = list(range(N)) if order is None else [int(i) for i in order]
    if limit is not None:
        order = order[:limit]
    results = [None] * N
    Y = None
    for idx in order:
        res = gcrodr(As[idx], bs[idx], Y, m, k, rtol, maxit, full_cycles, basis_fp32,
                     A_inner=None if A_inner is None else A_inner[idx])
        results[idx] = res
        Y = res.Y_next
    return results
