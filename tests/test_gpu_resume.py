"""Checkpoint and resume of a chain (skr_recycle_get / skr_recycle_set, SKR_FLAG_CONTINUE).

Bars (written in the tests):
* a sorted chain solved in two calls, the second on a fresh context seeded with the recycle space
  read back from the first, gives results (status, counts, residuals) and solutions identical bit
  for bit to the uninterrupted call, with an FP64 and with an FP32-stored basis;
* the oracle's GCRO-DR started from the read-back recycle space (Y = U_k, App. B.1) on the next
  system of the chain needs the same number of Arnoldi steps within max(1, 0.5 %), the bar of a
  system whose recycle space is given exactly, and its solution lies within the residual bound;
* errors: SKR_FLAG_CONTINUE without a carried space or with another k or precision, reading before
  any solve, kcols > k, ld < n; GMRES (k = 0) carries no columns.
"""
import numpy as np
import pytest

import oracle
from gpu_common import same_result as _same, log, make_ctx, need_gpu, solution_bound
from workloads import darcy_sequence, param_matrix
from workloads.device import upload_systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    return torch, skr


def _solve(torch, skr, ctx, systems, m, k, flags):
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=m, k=k, rtol=1e-8, maxit=20000, flags=flags)
    torch.cuda.synchronize()
    return res, [x.cpu().numpy() for x in xs]


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("split", [1, 3])
def test_split_chain_equals_uninterrupted(env, mixed, split):
    torch, skr = env
    log(f"[resume] 32x32 chain of 8, GCRO-DR(30,10), split after {split}, mixed={mixed}")
    flags = skr.SKR_FLAG_MIXED if mixed else 0
    systems = darcy_sequence(32, 8, first_seed=21)
    order = [int(i) for i in oracle.greedy_sort(param_matrix(systems))]
    chain = [systems[i] for i in order]
    n = chain[0].n
    ctx = make_ctx(torch)
    try:
        ref, xref = _solve(torch, skr, ctx, chain, 30, 10, flags)
        k_end = skr.skr_recycle_get(ctx)
        assert 0 < k_end <= 10
    finally:
        skr.skr_ctx_destroy(ctx)
    ctx1, ctx2 = make_ctx(torch), make_ctx(torch)
    try:
        r1, x1 = _solve(torch, skr, ctx1, chain[:split], 30, 10, flags)
        kk = skr.skr_recycle_get(ctx1)
        U = torch.full((max(kk, 1), n), float("nan"), dtype=torch.float64, device="cuda:0")
        assert skr.skr_recycle_get(ctx1, U) == kk
        skr.skr_recycle_set(ctx2, U, n, kk, 30, 10, flags=flags)
        r2, x2 = _solve(torch, skr, ctx2, chain[split:], 30, 10, flags | skr.SKR_FLAG_CONTINUE)
        for pos, (r, x) in enumerate(zip(r1 + r2, x1 + x2)):
            assert _same(r, ref[pos]), (pos, r, ref[pos])
            assert np.array_equal(x, xref[pos]), pos
        assert skr.skr_recycle_get(ctx2) == k_end
        # the oracle started from the read-back space on the next system of the chain
        Uh = U[:kk].cpu().numpy().T.copy()
        s = chain[split]
        o = oracle.gcrodr(s.A, s.b, Uh, 30, 10, 1e-8, 20000, basis_fp32=mixed)
        g = r2[0]
        log(f"  next system: iters gpu {g['iters']} oracle {o.iters}, k_start {g['k_start']}/{o.k_start}")
        assert g["k_start"] == o.k_start
        assert abs(g["iters"] - o.iters) <= max(1, int(0.005 * o.iters))
        bound, _ = solution_bound(s.A, s.b, o.x, g["relres_true"], o.relres_true)
        assert np.linalg.norm(x2[0] - o.x) / np.linalg.norm(o.x) <= bound
    finally:
        skr.skr_ctx_destroy(ctx1)
        skr.skr_ctx_destroy(ctx2)


def test_resume_errors(env):
    torch, skr = env
    log("[resume] argument errors")
    systems = darcy_sequence(16, 2, first_seed=5)
    n = systems[0].n
    ctx = make_ctx(torch)
    try:
        with pytest.raises(skr.SkrError) as e:
            skr.skr_recycle_get(ctx)
        assert e.value.code == skr.SKR_EINVAL
        ops, bs, xs = upload_systems(systems, "cuda:0")
        with pytest.raises(skr.SkrError) as e:
            skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=6, rtol=1e-8, maxit=5000,
                                   flags=skr.SKR_FLAG_CONTINUE)
        assert e.value.code == skr.SKR_EINVAL
        skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=6, rtol=1e-8, maxit=5000)
        kk = skr.skr_recycle_get(ctx)
        assert kk > 0
        U = torch.zeros((kk, n), dtype=torch.float64, device="cuda:0")
        with pytest.raises(skr.SkrError):
            skr.skr_recycle_get(ctx, U, ld=n - 1)
        for flags, k in ((skr.SKR_FLAG_CONTINUE | skr.SKR_FLAG_MIXED, 6), (skr.SKR_FLAG_CONTINUE, 5)):
            with pytest.raises(skr.SkrError) as e:
                skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=k, rtol=1e-8, maxit=5000, flags=flags)
            assert e.value.code == skr.SKR_EINVAL
        with pytest.raises(skr.SkrError):
            skr.skr_recycle_set(ctx, U, n, 7, 20, 6)
        with pytest.raises(skr.SkrError):
            skr.skr_recycle_set(ctx, U, n, kk, 20, 6, ld=n - 1)
        # GMRES carries no columns; a continued GMRES call is accepted
        skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=0, rtol=1e-8, maxit=5000)
        assert skr.skr_recycle_get(ctx) == 0
        rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=0, rtol=1e-8, maxit=5000,
                                         flags=skr.SKR_FLAG_CONTINUE)
        assert rc == skr.SKR_OK and all(r["k_start"] == 0 for r in res)
    finally:
        skr.skr_ctx_destroy(ctx)


def test_split_chain_bench_size(env):
    """256^2 Darcy, the first 4 systems of a seeded chain with GCRO-DR(60,20) (the bench's system size
    and launch configuration), split after 2: bitwise equal to the uninterrupted chain."""
    torch, skr = env
    log("[resume] 256x256, 4 systems, GCRO-DR(60,20), split after 2")
    chain = darcy_sequence(256, 4, first_seed=300)
    n = chain[0].n
    ctx, ctx1, ctx2 = make_ctx(torch), make_ctx(torch), make_ctx(torch)
    try:
        ref, xref = _solve(torch, skr, ctx, chain, 60, 20, 0)
        r1, x1 = _solve(torch, skr, ctx1, chain[:2], 60, 20, 0)
        kk = skr.skr_recycle_get(ctx1)
        U = torch.empty((max(kk, 1), n), dtype=torch.float64, device="cuda:0")
        skr.skr_recycle_get(ctx1, U)
        skr.skr_recycle_set(ctx2, U, n, kk, 60, 20)
        r2, x2 = _solve(torch, skr, ctx2, chain[2:], 60, 20, skr.SKR_FLAG_CONTINUE)
        for pos, (r, x) in enumerate(zip(r1 + r2, x1 + x2)):
            assert _same(r, ref[pos]), (pos, r, ref[pos])
            assert np.array_equal(x, xref[pos]), pos
    finally:
        for c in (ctx, ctx1, ctx2):
            skr.skr_ctx_destroy(c)


def test_rhs_in_recycled_range(env):
    """The start-up's closed form (App. B.1) on the device: a right-hand side b = A U_k c lies in
    range(C_k), so a continued chain solves it by the projection alone (no Arnoldi step,
    x = U_k R^-1 C_k^T b), as the oracle does from the same read-back U_k. The residual left is at
    rounding level; the solution is within the residual bound of both U_k c and the oracle's."""
    import types
    torch, skr = env
    log("[resume] b in range(A U_k): zero Arnoldi steps")
    s = darcy_sequence(32, 1, first_seed=33)[0]
    n = s.n
    ctx = make_ctx(torch)
    try:
        _solve(torch, skr, ctx, [s], 30, 10, 0)
        kk = skr.skr_recycle_get(ctx)
        assert kk == 10
        U = torch.empty((kk, n), dtype=torch.float64, device="cuda:0")
        skr.skr_recycle_get(ctx, U)
        Uh = U.cpu().numpy().T.copy()
        u = Uh @ np.random.default_rng(7).standard_normal(kk)
        b1 = s.A @ u
        sys1 = types.SimpleNamespace(A=s.A, b=b1, n=n, N_g=s.N_g)
        res, xs = _solve(torch, skr, ctx, [sys1], 30, 10, skr.SKR_FLAG_CONTINUE)
        g = res[0]
        o = oracle.gcrodr(s.A, b1, Uh, 30, 10, 1e-8, 20000)
        log(f"  gpu: status {g['status']} iters {g['iters']} k_start {g['k_start']} relres {g['relres_true']:.2e};"
            f" oracle iters {o.iters} relres {o.relres_true:.2e}")
        assert o.status == oracle.CONVERGED and o.iters == 0 and o.k_start == kk
        assert g["status"] == skr.SKR_CONVERGED and g["iters"] == 0 and g["cycles"] == 0
        assert g["k_start"] == kk and g["rank_dropped"] == 0
        assert g["spmv"] == kk + 1            # A U_k at the start-up and the true residual
        assert g["relres_true"] <= 1e-12
        for ref, rr in ((u, np.linalg.norm(b1 - s.A @ u) / np.linalg.norm(b1)), (o.x, o.relres_true)):
            bound, _ = solution_bound(s.A, b1, ref, g["relres_true"], rr)
            assert np.linalg.norm(xs[0] - ref) / np.linalg.norm(ref) <= bound
        assert skr.skr_recycle_get(ctx) == kk
    finally:
        skr.skr_ctx_destroy(ctx)
