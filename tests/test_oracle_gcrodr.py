"""Pins of the GCRO-DR / GMRES oracle against what the paper and the mathematics fix.

Each pin is chosen so that a plausible slip (a dropped term of Eq. 6, a wrong sign in the residual
update, a transposed operand in the eigenproblem, a mis-applied D_k scaling) breaks at least one.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import (BREAKDOWN, CONVERGED, MAXIT, NONFINITE, gcrodr, gmres,
                    harmonic_ritz_generalized, harmonic_ritz_standard, solve_sequence)
from oracle.solver import arnoldi_cycle, cycle_matrices, qr_pos, select_smallest, startup
from workloads import darcy_sequence


def convdiff(N, peclet=30.0, seed=0):
    """Nonsymmetric upwind convection-diffusion matrix on an N x N grid (test input only)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (N + 1)
    bx, by = peclet * (0.5 + rng.random()), peclet * (rng.random() - 0.5)
    A = sp.lil_matrix((N * N, N * N))
    for i in range(N):
        for j in range(N):
            r = i * N + j
            A[r, r] = 4.0 / h ** 2 + (abs(bx) + abs(by)) / h
            nbrs = ((i, j - 1, -1 / h ** 2 - max(bx, 0) / h), (i, j + 1, -1 / h ** 2 + min(bx, 0) / h),
                    (i - 1, j, -1 / h ** 2 - max(by, 0) / h), (i + 1, j, -1 / h ** 2 + min(by, 0) / h))
            for ii, jj, c in nbrs:
                if 0 <= ii < N and 0 <= jj < N:
                    A[r, ii * N + jj] = c
    return A.tocsr()


@pytest.fixture(scope="module")
def darcy16():
    return darcy_sequence(16, 6)


def test_convdiff_helper_is_what_it_claims():
    A = convdiff(5).toarray()
    assert np.allclose(A.sum(axis=1)[12], 0.0, atol=1e-9)   # interior row of a pure stencil sums to 0
    assert not np.allclose(A, A.T)


# ---------------------------------------------------------------------------- Arnoldi (Eq. 3, Eq. 6)
@pytest.mark.parametrize("kc", [0, 5])
def test_arnoldi_cgs2_relations(darcy16, kc):
    A = darcy16[0].A
    n = A.shape[0]
    rng = np.random.default_rng(3)
    C = None
    if kc:
        C, _ = qr_pos(A @ rng.standard_normal((n, kc)))
    r = rng.standard_normal(n)
    if kc:
        r = r - C @ (C.T @ r)          # GCRO-DR residuals are orthogonal to C (App. B.1)
    s = 25
    V, Hb, B, est, brk = arnoldi_cycle(A, r, C, s, 0.0)
    assert V.shape == (n, s + 1) and Hb.shape == (s + 1, s) and not brk
    assert np.abs(V.T @ V - np.eye(s + 1)).max() <= 1e-12
    assert np.allclose(np.tril(Hb, -2), 0.0)
    AV = A @ V[:, :s]
    normA = spla.norm(A)
    if kc:
        assert np.abs(C.T @ V).max() <= 1e-12
        lhs = AV - C @ (C.T @ AV)
        np.testing.assert_allclose(B, C.T @ AV, atol=1e-12 * normA)
    else:
        lhs = AV
    assert np.linalg.norm(lhs - V @ Hb) <= 1e-12 * normA * np.sqrt(s)


def test_gmres_cycle_estimate_is_true_residual(darcy16):
    # the LS residual of Hbar equals ||b - A x_j|| for the GMRES iterate x_j (Eq. 3)
    A, b = darcy16[1].A, darcy16[1].b
    beta = np.linalg.norm(b)
    for s in (1, 7, 30):
        V, Hb, _, est, _ = arnoldi_cycle(A, b, None, s, 0.0)
        c = np.zeros(s + 1); c[0] = beta
        y = np.linalg.lstsq(Hb, c, rcond=None)[0]
        true = np.linalg.norm(b - A @ (V[:, :s] @ y))
        assert abs(est - true) <= 1e-9 * beta


def test_residuals_monotone(darcy16):
    res = solve_sequence([s.A for s in darcy16], [s.b for s in darcy16], None, 20, 6, 1e-10, 5000)
    for r in res:
        h = r.res_history
        assert all(h[i + 1] <= h[i] * (1 + 1e-12) + 1e-14 * h[0] for i in range(len(h) - 1))


# ------------------------------------------------------------------------------------ GMRES = k 0
def test_gmres_matches_scipy():
    seq = darcy_sequence(32, 3, first_seed=11)
    for s in seq:
        inner = []
        xs, info = spla.gmres(s.A, s.b, rtol=1e-8, atol=0.0, restart=30, maxiter=200,
                              callback=lambda pr: inner.append(pr), callback_type="pr_norm")
        assert info == 0
        r = gmres(s.A, s.b, 30, 1e-8, 20000)
        assert r.status == CONVERGED
        assert abs(r.iters - len(inner)) <= 1
        rel = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
        assert rel <= (1e-10 if r.iters == len(inner) else 1e-7)


# ------------------------------------------------------------------------------- harmonic Ritz
def test_harmonic_ritz_forms_agree_at_k0(darcy16):
    # Alg. 2 uses the standard form for the first cycle and the generalised form afterwards;
    # with an empty C (G = Hbar, W^T V = I_{m+1,m}) both define the same eigenpairs.
    for A in (darcy16[2].A, convdiff(12)):
        n = A.shape[0]
        V, Hb, _, _, _ = arnoldi_cycle(A, np.random.default_rng(5).standard_normal(n), None, 20, 0.0)
        Ps, ts = harmonic_ritz_standard(Hb, 20)
        Pg, tg = harmonic_ritz_generalized(Hb, np.eye(21, 20), 20)
        assert ts.size == tg.size == 20
        for a, b in ((ts, tg), (tg, ts)):
            for t in a:
                assert np.min(np.abs(b - t)) <= 1e-8 * abs(t)


def test_harmonic_ritz_eigen_residual_and_bounds(darcy16):
    A = darcy16[3].A
    n = A.shape[0]
    V, Hb, _, _, _ = arnoldi_cycle(A, np.random.default_rng(6).standard_normal(n), None, 30, 0.0)
    P, th = harmonic_ritz_standard(Hb, 8)
    assert P.shape == (30, 8)
    assert np.all(np.imag(th) == 0)                       # SPD A: real harmonic Ritz values
    lam = np.linalg.eigvalsh(A.toarray())
    assert np.all(np.real(th) >= lam[0] * (1 - 1e-10)) and np.all(np.real(th) <= lam[-1] * (1 + 1e-10))
    # harmonic Ritz condition: A y - theta y is orthogonal to A V_m  (y = V_m z)
    AV = A @ V[:, :30]
    for i in range(8):
        y = V[:, :30] @ P[:, i]
        res = AV.T @ (A @ y - th[i].real * y)
        assert np.linalg.norm(res) <= 1e-8 * np.linalg.norm(AV.T @ (A @ y))
    # smallest moduli were chosen
    Pall, tall = harmonic_ritz_standard(Hb, 30)
    assert np.max(np.abs(th)) <= np.sort(np.abs(tall))[8] * (1 + 1e-12)


# ------------------------------------------------- generalized harmonic Ritz, nonsymmetric, k > 0
def _gcrodr_cycle(seed):
    """One GCRO-DR cycle with a nonempty C on a nonsymmetric operator: C, U from the start-up with the
    recycle space of a neighbouring system, 20 Arnoldi steps, and the cycle-end matrices."""
    A0, A1 = convdiff(12, seed=2 * seed), convdiff(12, seed=2 * seed + 1)
    b = np.ones(A0.shape[0])
    Y = gcrodr(A0, b, None, 30, 8, 1e-10, 3000).Y_next
    _, r1, C, U, _ = startup(A1, Y, b)
    V, Hb, B, _, brk = arnoldi_cycle(A1, r1, C, 20, 0.0)
    assert C.shape[1] >= 6 and not brk
    G, What, Vhat = cycle_matrices(C, U, V, Hb, B)
    return A1, G, What, Vhat


def _harmonic_ritz_violation(A, Vhat, P, theta):
    """Largest relative violation of the harmonic Ritz condition (A y - theta y) orthogonal to
    range(A V^), y = V^ z, with A applied explicitly. A conjugate pair is the column pair (Re z, Im z)
    listed with theta first."""
    AVh = A @ Vhat
    worst, c = 0.0, 0
    while c < P.shape[1]:
        t = theta[c]
        if np.imag(t) != 0.0:
            z, step = P[:, c] + 1j * P[:, c + 1], 2
        else:
            z, step, t = P[:, c], 1, np.real(t)
        y = Vhat @ z
        Ay = A @ y
        worst = max(worst, np.linalg.norm(AVh.T @ (Ay - t * y)) / np.linalg.norm(AVh.T @ Ay))
        c += step
    return worst


@pytest.mark.parametrize("seed", range(3))
def test_cycle_matrices_satisfy_the_cycle_relation(seed):
    # A V^ = W^ G (Alg. 2 while body; Eq. 6 with A U = C), with A applied explicitly: pins D_k, B
    # and Hbar in G and the column order of V^ and W^
    A, G, What, Vhat = _gcrodr_cycle(seed)
    assert np.linalg.norm(A @ Vhat - What @ G) <= 1e-12 * spla.norm(A) * np.linalg.norm(Vhat)


@pytest.mark.parametrize("seed", range(3))
def test_generalized_harmonic_ritz_nonsymmetric(seed):
    A, G, What, Vhat = _gcrodr_cycle(seed)
    k = 8
    P, th = harmonic_ritz_generalized(G, What.T @ Vhat, k)
    assert P.shape[1] in (k - 1, k)
    # each selected pair satisfies the harmonic Ritz condition with the explicit operator
    assert _harmonic_ritz_violation(A, Vhat, P, th) <= 1e-9
    # the selected values are the smallest-modulus eigenvalues of the pencil
    # ((A V^)^T (A V^), (A V^)^T V^) formed from explicit products
    AVh = A @ Vhat
    ev = sla.eigvals(AVh.T @ AVh, AVh.T @ Vhat)
    ev = ev[np.isfinite(ev)]
    ev = ev[np.argsort(np.abs(ev), kind="stable")]
    for t in th:
        assert np.min(np.abs(ev[:P.shape[1] + 1] - t)) <= 1e-8 * abs(t)
    assert np.max(np.abs(th)) <= np.abs(ev[P.shape[1] - 1]) * (1 + 1e-8)
    if P.shape[1] == k - 1:          # only when the k-th is half of a conjugate pair
        assert np.imag(ev[k - 1]) != 0.0 and abs(ev[k - 1] - np.conj(ev[k])) <= 1e-8 * abs(ev[k - 1])


def test_generalized_harmonic_ritz_pin_detects_a_transposed_operand():
    # the same selection from the pencil (G^T G, (W^T V)^T G), whose eigenvalues are the same but
    # whose eigenvectors are not, must fail the harmonic Ritz condition above
    A, G, What, Vhat = _gcrodr_cycle(0)
    WtV = What.T @ Vhat
    Pm, thm = select_smallest(*sla.eig(G.T @ G, WtV.T @ G), 8)
    assert _harmonic_ritz_violation(A, Vhat, Pm, thm) > 1e-3


def test_complex_pair_handling():
    # 2x2 rotation block has eigenvalues +-i (a conjugate pair of modulus 1), plus reals 0.5, 3.
    M = np.zeros((4, 4)); M[0, 1], M[1, 0] = -1.0, 1.0; M[2, 2] = 0.5; M[3, 3] = 3.0
    Hb = np.vstack([M, np.zeros((1, 4))])            # h_{m+1,m} = 0: harmonic Ritz = Ritz values
    P2, t2 = harmonic_ritz_standard(Hb, 2)            # k-th is half of the pair -> dropped
    assert P2.shape[1] == 1 and np.isclose(t2[0], 0.5)
    P3, t3 = harmonic_ritz_standard(Hb, 3)
    assert P3.shape[1] == 3
    span = np.linalg.qr(P3)[0]
    e = np.eye(4)
    for v in (e[:, 0], e[:, 1], e[:, 2]):             # span{Re z, Im z, z_0.5} = span{e0, e1, e2}
        assert np.linalg.norm(v - span @ (span.T @ v)) < 1e-12


# ------------------------------------------------------------------------- start-up and recycling
def test_startup_closed_form(darcy16):
    A = darcy16[0].A
    n = A.shape[0]
    rng = np.random.default_rng(8)
    Y = rng.standard_normal((n, 6))
    w = rng.standard_normal(6)
    b = A @ (Y @ w)
    r = gcrodr(A, b, Y, 20, 6, 1e-8, 100)
    assert r.status == CONVERGED and r.iters == 0 and r.k_start == 6
    np.testing.assert_allclose(r.x, Y @ w, rtol=1e-10, atol=1e-10 * np.linalg.norm(Y @ w))


def test_startup_relations_and_rank_drop(darcy16):
    A = darcy16[0].A
    n = A.shape[0]
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((n, 5))
    Y[:, 3] = Y[:, 1] * 2.0                             # dependent column
    x1, r1, C, U, dropped = startup(A, Y, np.ones(n))
    assert dropped == 1 and C.shape[1] == 4
    assert np.abs(C.T @ C - np.eye(4)).max() <= 1e-12
    assert np.linalg.norm(A @ U - C) <= 1e-10 * spla.norm(A) * np.linalg.norm(U)
    assert np.abs(C.T @ r1).max() <= 1e-12 * np.sqrt(n)
    np.testing.assert_allclose(x1 + 0, U @ (C.T @ np.ones(n)))


@pytest.mark.parametrize("m,k", [(20, 6), (80, 20)])
def test_recycle_space_relations_after_solve(darcy16, m, k):
    A, b = darcy16[0].A, darcy16[0].b
    r = gcrodr(A, b, None, m, k, 1e-10, 5000)
    U, C = r.Y_next, r.C_last
    assert U.shape == (A.shape[0], k) and C.shape == U.shape
    assert np.abs(C.T @ C - np.eye(k)).max() <= 1e-12
    assert np.linalg.norm(A @ U - C) <= 1e-10 * spla.norm(A) * np.linalg.norm(U)


@pytest.mark.parametrize("kind", ["darcy", "convdiff"])
def test_c_orthonormal_after_every_cycle(kind):
    # C^T C = I to 1e-12 after every cycle end of a chain solved to 1e-12 (the projection of r at
    # each cycle start keeps v1 orthogonal to C; without it the loss grows like eps / relres)
    if kind == "darcy":
        seq = darcy_sequence(32, 3)
        As, bs = [s.A for s in seq], [s.b for s in seq]
    else:
        As, bs = [convdiff(14, seed=s) for s in range(3)], [np.ones(196)] * 3
    Y, ncyc = None, 0
    for A, b in zip(As, bs):
        r = gcrodr(A, b, Y, 30, 10, 1e-12, 5000, keep_cycles=True)
        assert r.status == CONVERGED and r.relres_true <= 1e-12
        for _, C in r.cycle_log:
            if C is not None:
                assert np.abs(C.T @ C - np.eye(C.shape[1])).max() <= 1e-12
                ncyc += 1
        Y = r.Y_next
    assert ncyc >= 8


def test_restart_from_true_residual():
    # rtol 1e-13 on 32^2 Darcy: the estimate meets the tolerance before the true residual does, so
    # the solve goes on from the true residual projected onto range(C) (App. B.1), and still
    # converges with C orthonormal
    seq = darcy_sequence(32, 2)
    Y, restarts = None, 0
    for s in seq:
        r = gcrodr(s.A, s.b, Y, 30, 10, 1e-13, 5000, keep_cycles=True)
        assert r.status == CONVERGED and r.relres_true <= 1e-13
        assert all(np.abs(C.T @ C - np.eye(C.shape[1])).max() <= 1e-12 for _, C in r.cycle_log if C is not None)
        restarts += r.restarts
        Y = r.Y_next
    assert restarts >= 1


def test_unattainable_tolerance_stagnates_without_diverging():
    # rtol 1e-15 is below the attainable accuracy of FP64 on this system: the solve must stop at
    # maxit near the attainable residual, not diverge
    s = darcy_sequence(32, 1)[0]
    r = gcrodr(s.A, s.b, None, 30, 10, 1e-15, 600)
    assert r.status == MAXIT and np.isfinite(r.relres_true) and r.relres_true <= 1e-12
    assert max(r.res_history[1:]) <= r.res_history[0]


def test_span_invariance(darcy16):
    A0, A1, b1 = darcy16[0].A, darcy16[1].A, darcy16[1].b
    Y = gcrodr(A0, darcy16[0].b, None, 20, 6, 1e-10, 5000).Y_next
    T = np.random.default_rng(4).standard_normal((6, 6)) + 3 * np.eye(6)
    ra = gcrodr(A1, b1, Y, 20, 6, 1e-10, 5000)
    rb = gcrodr(A1, b1, Y @ T, 20, 6, 1e-10, 5000)
    assert ra.iters == rb.iters
    assert np.linalg.norm(ra.x - rb.x) <= 1e-8 * np.linalg.norm(ra.x)


def test_recycling_reduces_iterations(darcy16):
    As, bs = [s.A for s in darcy16], [s.b for s in darcy16]
    skr = solve_sequence(As, bs, None, 30, 10, 1e-8, 5000)
    gm = solve_sequence(As, bs, None, 30, 0, 1e-8, 5000)
    assert sum(r.iters for r in skr[1:]) < 0.8 * sum(r.iters for r in gm[1:])


# ------------------------------------------------------------------------------- whole solves
@pytest.mark.parametrize("kind", ["darcy", "convdiff"])
def test_tiny_solve_against_dense_lu(kind):
    A = darcy_sequence(8, 1, first_seed=2)[0].A if kind == "darcy" else convdiff(8, seed=3)
    n = A.shape[0]
    rng = np.random.default_rng(10)
    Ad = A.toarray()
    Y = None
    for t in range(3):
        b = rng.standard_normal(n)
        r = gcrodr(A, b, Y, 12, 4, 1e-12, 2000)
        xl = np.linalg.solve(Ad, b)
        assert r.status in (CONVERGED, BREAKDOWN)
        assert np.linalg.norm(r.x - xl) / np.linalg.norm(xl) <= 10 * np.linalg.cond(Ad) * 1e-12
        Y = r.Y_next


@pytest.mark.parametrize("m,k", [(30, 10), (80, 20)])
def test_sequence_solutions_match_direct(darcy16, m, k):
    As, bs = [s.A for s in darcy16], [s.b for s in darcy16]
    res = solve_sequence(As, bs, None, m, k, 1e-8, 5000)
    for A, b, r in zip(As, bs, res):
        xs = spla.spsolve(A.tocsc(), b)
        lam_min = spla.eigsh(A, k=1, sigma=0, return_eigenvectors=False)[0]
        mu = np.linalg.norm(b) / lam_min / np.linalg.norm(xs)
        assert r.relres_true <= 1e-8
        assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= mu * r.relres_true * 1.0001


def test_nonsymmetric_sequence_converges():
    As = [convdiff(14, seed=s) for s in range(4)]
    bs = [np.ones(196)] * 4
    res = solve_sequence(As, bs, None, 25, 8, 1e-9, 3000)
    for A, b, r in zip(As, bs, res):
        assert r.status == CONVERGED
        assert np.linalg.norm(b - A @ r.x) <= 1e-9 * np.linalg.norm(b) * (1 + 1e-9)


# --------------------------------------------------------------------------------- edge cases
def test_edge_cases(darcy16):
    A, b = darcy16[0].A, darcy16[0].b
    n = A.shape[0]
    Y = np.random.default_rng(1).standard_normal((n, 3))
    r = gcrodr(A, np.zeros(n), Y, 10, 3, 1e-8, 100)
    assert r.status == CONVERGED and r.iters == 0 and not r.x.any() and r.Y_next is Y
    bn = b.copy(); bn[5] = np.nan
    assert gcrodr(A, bn, None, 10, 3, 1e-8, 100).status == NONFINITE
    r = gcrodr(A, b, None, 10, 3, 1e-8, 1)
    assert r.status == MAXIT and r.iters == 1 and r.relres_true > 1e-8
    r = gcrodr(sp.identity(n, format="csr"), b, None, 10, 3, 1e-8, 100)
    assert r.status == BREAKDOWN and r.iters == 1
    np.testing.assert_allclose(r.x, b, rtol=1e-14)
    r = gcrodr(A, b, None, 10, 3, 1e-8, 5000, full_cycles=True)
    assert r.status == CONVERGED and r.relres_true <= 1e-8
    with pytest.raises(ValueError):
        gcrodr(A, b, None, 5, 5, 1e-8, 10)
