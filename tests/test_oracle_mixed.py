"""Pins of the oracle's mixed-precision mode: FP32 storage of the subspace columns (Arnoldi vectors,
C_k, U_k) with FP64 arithmetic, and one refinement step (a cycle from the true FP64 residual) per
cycle. The paper fixes the method in exact arithmetic; these pins check what that mode must
preserve and what it must change:
* the stored columns are exactly FP32 values, rounded to nearest (IEEE 754 binary32);
* the inner cycle's operator is A with its values rounded to FP32, while true residuals use A;
* the Arnoldi and recycle relations still hold, to FP32 storage accuracy;
* because x and r stay FP64 and each cycle restarts from the true residual, the solve reaches
  residuals far below what any FP32 iterate can represent, and the solutions match a direct solve;
* the iteration counts stay those of the FP64 method (per-cycle contraction is unchanged while it
  is far above the FP32 floor);
* one extra product with A per refinement step.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import CONVERGED, gcrodr, solve_sequence
from oracle.solver import arnoldi_cycle, fp32_operator, fp32_store, qr_pos
from workloads import darcy_sequence
from workloads.darcy import assemble_csr


@pytest.fixture(scope="module")
def darcy16():
    return darcy_sequence(16, 6)


def is_fp32(v):
    return np.array_equal(v, v.astype(np.float32).astype(np.float64))


def test_fp32_store_is_round_to_nearest_even():
    # binary32 has a 24-bit significand: spacing 2^-23 on [1, 2), 2^-22 on [2, 4)
    cases = [(1.0 + 2.0 ** -24, 1.0),                          # tie, rounds to the even neighbour
             (1.0 + 3 * 2.0 ** -24, 1.0 + 2.0 ** -22),         # tie between 1+2^-23 (odd) and 1+2^-22 (even)
             (1.0 + 2.0 ** -24 + 2.0 ** -40, 1.0 + 2.0 ** -23),   # just above the tie
             (-(1.0 + 2.0 ** -23), -(1.0 + 2.0 ** -23)),       # exact
             (np.pi, 13176795 / 2.0 ** 22),                    # nearest binary32 to pi
             (1e-50, 0.0),                                     # below the subnormal range
             (2.0 ** -149, 2.0 ** -149)]                       # smallest subnormal
    for v, want in cases:
        assert fp32_store(np.array([v]))[0] == want, v


@pytest.mark.parametrize("kc", [0, 4])
def test_arnoldi_relations_on_stored_basis(darcy16, kc):
    A = darcy16[0].A
    n = A.shape[0]
    rng = np.random.default_rng(5)
    C = None
    if kc:
        C = fp32_store(qr_pos(A @ rng.standard_normal((n, kc)))[0])
    r = rng.standard_normal(n)
    if kc:                       # the cycle's residual is orthogonal to C (start-up projection)
        r = r - C @ (C.T @ r)
        r = r - C @ (C.T @ r)
    errs = {}
    for name, store in (("fp64", lambda v: v), ("fp32", fp32_store)):
        V, Hbar, B, est, brk = arnoldi_cycle(A, r, C, 20, 0.0, False, store)
        j = Hbar.shape[1]
        if name == "fp32":
            assert all(is_fp32(V[:, t]) for t in range(j + 1))
        lhs = A @ V[:, :j]
        rhs = V @ Hbar + (C @ B if kc else 0.0)
        errs[name] = np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs)
        # orthogonality of the new vectors against [C, V] (C itself is given)
        errs[name + "_orth"] = np.linalg.norm(V.T @ V - np.eye(j + 1)) + (np.linalg.norm(C.T @ V) if kc else 0.0)
    # FP64: rounding level; FP32 storage: FP32 level, and not better (the rounding really happens)
    assert errs["fp64"] < 1e-13 and errs["fp64_orth"] < 1e-12
    assert 1e-10 < errs["fp32"] < 3e-6
    assert errs["fp32_orth"] < 3e-6


def test_recycle_space_stored_fp32_and_consistent(darcy16):
    As, bs = [s.A for s in darcy16[:3]], [s.b for s in darcy16[:3]]
    res = solve_sequence(As, bs, None, 30, 10, 1e-8, 5000, basis_fp32=True)
    for A, r in zip(As, res):
        U, C = r.Y_next, r.C_last
        assert U is not None and U.shape[1] == 10
        assert is_fp32(U) and is_fp32(C)
        # C = A U with orthonormal columns, up to the FP32 rounding of both
        assert np.linalg.norm(A @ U - C) / np.linalg.norm(C) < 1e-5
        assert np.linalg.norm(C.T @ C - np.eye(10)) < 1e-5


@pytest.mark.parametrize("rtol", [1e-11, 1e-12])
def test_mixed_reaches_fp64_accuracy(darcy16, rtol):
    As, bs = [s.A for s in darcy16[:4]], [s.b for s in darcy16[:4]]
    res = solve_sequence(As, bs, None, 30, 10, rtol, 8000, basis_fp32=True)
    for A, b, r in zip(As, bs, res):
        assert r.status == CONVERGED
        rel = np.linalg.norm(b - A @ r.x) / np.linalg.norm(b)
        assert rel <= rtol * (1 + 1e-6)
        xs = spla.spsolve(A.tocsc(), b)
        lam_min = spla.eigsh(A, k=1, sigma=0, return_eigenvectors=False)[0]
        mu = np.linalg.norm(b) / lam_min / np.linalg.norm(xs)
        assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= mu * rel * 1.0001 + 1e-14
        # an FP32 iterate could not get there: rounding x alone to FP32 leaves a far larger residual
        assert np.linalg.norm(b - A @ fp32_store(r.x)) / np.linalg.norm(b) > 100 * rtol


def test_mixed_iterations_track_fp64(darcy16):
    As, bs = [s.A for s in darcy16], [s.b for s in darcy16]
    r64 = solve_sequence(As, bs, None, 30, 10, 1e-8, 5000)
    r32 = solve_sequence(As, bs, None, 30, 10, 1e-8, 5000, basis_fp32=True)
    for a, b in zip(r64, r32):
        assert b.status == CONVERGED
        assert abs(a.iters - b.iters) <= max(3, 0.15 * a.iters), (a.iters, b.iters)


def test_one_refinement_product_per_cycle(darcy16):
    A, b = darcy16[1].A, darcy16[1].b
    r64 = gcrodr(A, b, None, 10, 0, 1e-8, 5000)
    r32 = gcrodr(A, b, None, 10, 0, 1e-8, 5000, basis_fp32=True)
    assert r64.cycles > 3 and r32.cycles > 3
    # FP64: Arnoldi products + the final true residual; mixed: + one residual per later cycle
    assert r64.spmv == r64.iters + 1
    assert r32.spmv == r32.iters + (r32.cycles - 1) + 1


def test_fp32_operator_rounds_every_value():
    A = darcy_sequence(8, 1)[0].A
    Ai = fp32_operator(A)
    assert (Ai.indptr == A.indptr).all() and (Ai.indices == A.indices).all()
    assert is_fp32(Ai.data) and not is_fp32(A.data)
    assert np.all(np.abs(Ai.data - A.data) <= 2.0 ** -24 * np.abs(A.data))
    assert A.data.dtype == np.float64 and not np.shares_memory(Ai.data, A.data)


def test_inner_operator_is_the_fp32_one(monkeypatch):
    # the operator a mixed-mode solve hands to its Arnoldi cycles and its start-up product is A with
    # its values rounded to FP32 (or the given inner operator: a stencil's is assembled from its
    # rounded faces, which differs from the rounded CSR values); an FP64 solve hands A itself
    import oracle.solver as S
    s = darcy_sequence(24, 2, first_seed=3)
    A = s[1].A
    Ai_csr = fp32_operator(A)
    Ai_st = assemble_csr(fp32_store(s[1].ax), fp32_store(s[1].ay), s[1].inv_h2)
    assert np.abs(Ai_st - Ai_csr).max() > 0.0
    Y = gcrodr(s[0].A, s[0].b, None, 20, 6, 1e-8, 5000).Y_next
    seen = []
    orig_cycle, orig_start = S.arnoldi_cycle, S.startup
    monkeypatch.setattr(S, "arnoldi_cycle", lambda Aop, *a, **kw: (seen.append(Aop), orig_cycle(Aop, *a, **kw))[1])
    monkeypatch.setattr(S, "startup", lambda Aop, *a, **kw: (seen.append(Aop), orig_start(Aop, *a, **kw))[1])
    for inner, want, fp32 in ((None, Ai_csr, True), (Ai_st, Ai_st, True), (None, A, False)):
        seen.clear()
        r = S.gcrodr(A, s[1].b, Y, 20, 6, 1e-8, 5000, basis_fp32=fp32, A_inner=inner)
        assert r.status == CONVERGED and len(seen) >= 2
        for Aop in seen:
            assert (abs(Aop - want)).max() == 0.0
    # the FP32 operator changes the Arnoldi relation at its rounding level only
    V, Hbar, B, est, brk = arnoldi_cycle(Ai_csr, s[1].b, None, 20, 0.0)
    j = Hbar.shape[1]
    ref = np.linalg.norm(Ai_csr @ V[:, :j])
    assert np.linalg.norm(Ai_csr @ V[:, :j] - V @ Hbar) / ref < 1e-13
    assert 1e-10 < np.linalg.norm(A @ V[:, :j] - V @ Hbar) / ref < 1e-6


def test_mixed_solutions_use_fp64_residuals(darcy16):
    # the refinement's true residuals use the FP64 operator: a solve at rtol 1e-11 reaches it with A,
    # which the FP32-rounded operator alone could not certify
    s = darcy16[1]
    r = gcrodr(s.A, s.b, None, 30, 10, 1e-11, 20000, basis_fp32=True)
    assert r.status == CONVERGED
    assert np.linalg.norm(s.b - s.A @ r.x) <= 1e-11 * np.linalg.norm(s.b) * (1 + 1e-9)
    assert np.linalg.norm(s.b - fp32_operator(s.A) @ r.x) > 1e-9 * np.linalg.norm(s.b)
