"""GPU parity at large cycle lengths (62 < m <= 86) and at the largest k: the Arnoldi steps reduce up
to 88 columns (two 64-lane column groups) and every cycle end with d = kc + j_done > 62 takes the
large-d dense stages (the symmetric tridiagonal route for the Darcy operators, the general Francis
route for the nonsymmetric advection-diffusion chain). A cycle that stops early with d <= 62 takes
the one-row-per-lane stages, so a chain exercises both.

Bars (written in the tests): those of the sequence solver (status equal, relative residual at most
rtol, solution within the residual bound of the oracle's, Arnoldi step counts within max(1, 0.5 %)
for the first two systems of a chain and within max(3, 10 %) further down, 3 % for the chain), and
the ones stated in a test where they differ.
"""
import numpy as np
import pytest

import oracle
from gpu_common import compare_chain, log, make_ctx, need_gpu, solution_bound
from workloads import darcy3d_sequence, darcy_sequence, param_matrix
from workloads.device import upload_systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    ctx = make_ctx(torch)
    yield torch, skr, ctx
    skr.skr_ctx_destroy(ctx)


def _ref(systems, order, m, k, rtol, fp32=False, maxit=40000):
    return oracle.solve_sequence([s.A for s in systems], [s.b for s in systems], order, m, k, rtol, maxit,
                                 basis_fp32=fp32)


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_gcrodr_80_20_chain(env, kind):
    """32x32 Darcy, 8 systems sorted into one chain, GCRO-DR(80,20): d = 80 at every full cycle."""
    torch, skr, ctx = env
    log(f"[large-m] GCRO-DR(80,20) chain kind={kind}")
    systems = darcy_sequence(32, 8)
    order = oracle.greedy_sort(param_matrix(systems))
    ops, bs, xs = upload_systems(systems, "cuda:0", kind)
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=80, k=20, rtol=1e-8, maxit=40000)
    assert rc == skr.SKR_OK
    ref = _ref(systems, order, 80, 20, 1e-8)
    assert max(r.cycles for r in ref) >= 2       # full cycles, so the row-looped stage runs
    compare_chain(systems, res, xs, ref, f"m80-{kind}", order)


def test_gmres_80(env):
    """GMRES(80): full 80-step cycles, no recycling (systems independent, exact counts)."""
    torch, skr, ctx = env
    log("[large-m] GMRES(80)")
    systems = darcy_sequence(32, 3, first_seed=40)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=80, k=0, rtol=1e-8, maxit=40000)
    assert rc == skr.SKR_OK
    ref = _ref(systems, None, 80, 0, 1e-8)
    compare_chain(systems, res, xs, ref, "gmres80", strict=True)
    for g, r in zip(res, ref):
        assert g["spmv"] == r.spmv and g["cycles"] == r.cycles


def test_largest_m_ragged(env):
    """m = 86 (the largest), k = 20, ragged n = 37^2, rtol 1e-10."""
    torch, skr, ctx = env
    log("[large-m] GCRO-DR(86,20), n = 1369, rtol 1e-10")
    systems = darcy_sequence(37, 4, first_seed=70)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=86, k=20, rtol=1e-10, maxit=40000)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, None, 86, 20, 1e-10), "m86", rtol=1e-10)
    with pytest.raises(skr.SkrError):
        skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=87, k=20, rtol=1e-8, maxit=10)


def test_nonsymmetric_large_m(env):
    """Upwind advection-diffusion (nonsymmetric, complex harmonic Ritz pairs possible), GCRO-DR(72,10)."""
    torch, skr, ctx = env
    log("[large-m] advection-diffusion 24x24, 5 systems, GCRO-DR(72,10)")
    from workloads.advdiff import advdiff_sequence
    systems = advdiff_sequence(24, 5, amp=30.0)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=72, k=10, rtol=1e-9, maxit=40000)
    assert rc == skr.SKR_OK
    ref = _ref(systems, None, 72, 10, 1e-9)
    for i, s in enumerate(systems):
        x = xs[i].cpu().numpy()
        g, r = res[i], ref[i]
        rel = np.linalg.norm(x - r.x) / np.linalg.norm(r.x)
        smin = np.linalg.svd(s.A.toarray(), compute_uv=False)[-1]
        mu = np.linalg.norm(s.b) / smin / np.linalg.norm(r.x)
        bound = max(1e-7, 1.01 * mu * (g["relres_true"] + r.relres_true))
        log(f"  advdiff m72 sys {i}: iters gpu {g['iters']} oracle {r.iters}  cycles {g['cycles']}/{r.cycles}"
            f"  rel {rel:.2e} (bound {bound:.1e})")
        assert g["status"] == r.status == oracle.CONVERGED
        assert g["relres_true"] <= 1e-9 * (1 + 1e-9)
        assert rel <= bound
        assert abs(g["iters"] - r.iters) <= (1 if i < 2 else max(3, 0.1 * r.iters))


def test_mixed_80_20_chain(env):
    """FP32-stored basis and recycle space with GCRO-DR(80,20), against the oracle's mixed mode."""
    torch, skr, ctx = env
    log("[large-m] mixed GCRO-DR(80,20) chain")
    systems = darcy_sequence(32, 6, first_seed=3)
    order = oracle.greedy_sort(param_matrix(systems))
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=80, k=20, rtol=1e-8, maxit=40000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, order, 80, 20, 1e-8, fp32=True), "mixed-m80", order, lead=0.02)


def test_3d_80_20_chain(env):
    """3-D Darcy 12^3 (7-point stencil), 5 systems, GCRO-DR(80,20)."""
    torch, skr, ctx = env
    log("[large-m] 3-D 12^3 GCRO-DR(80,20)")
    systems = darcy3d_sequence(12, 5)
    order = oracle.greedy_sort(param_matrix(systems))
    ops, bs, xs = upload_systems(systems, "cuda:0", "stencil")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=80, k=20, rtol=1e-8, maxit=40000)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, order, 80, 20, 1e-8), "3d-m80", order)


def test_fold_large_m(env):
    """The folded partial reductions (forced) with more than 64 reduction columns."""
    torch, skr, ctx = env
    log("[large-m] GCRO-DR(80,20) with folded partials")
    systems = darcy_sequence(32, 4, first_seed=9)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=80, k=20, rtol=1e-8, maxit=40000,
                                     flags=skr.SKR_FLAG_FOLD)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, None, 80, 20, 1e-8), "fold-m80")
    for s, x in zip(systems, xs):
        xh = x.cpu().numpy()
        assert np.linalg.norm(s.b - s.A @ xh) <= 1e-8 * np.linalg.norm(s.b) * (1 + 1e-9)


def test_largest_k():
    """k = 32 (the largest): GCRO-DR(86,32) on 20^2 Darcy reaches d = 86 with 32 selected harmonic Ritz
    vectors (the largest dense case); GCRO-DR(33,32) runs one Arnoldi step per cycle (up to ~200
    cycle ends per system). Against the oracle; for (33,32) the first two systems take two steps, twice
    the oracle's own spread there (it moves by one step when b is perturbed by 1e-15 relative)."""
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    ctx = make_ctx(torch)
    try:
        for N, m, k in ((20, 86, 32), (16, 33, 32)):
            log(f"[large-m] GCRO-DR({m},{k}) on {N}x{N}, 3 systems")
            systems = darcy_sequence(N, 3, first_seed=90)
            ops, bs, xs = upload_systems(systems, "cuda:0")
            rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=m, k=k, rtol=1e-8, maxit=40000)
            assert rc == skr.SKR_OK
            ref = _ref(systems, None, m, k, 1e-8)
            if m == 86:
                compare_chain(systems, res, xs, ref, f"m{m}k{k}")
                continue
            for i, (s, g, r) in enumerate(zip(systems, res, ref)):
                x = xs[i].cpu().numpy()
                bound, _ = solution_bound(s.A, s.b, r.x, g["relres_true"], r.relres_true)
                log(f"  sys {i}: iters gpu {g['iters']} oracle {r.iters} cycles {g['cycles']}/{r.cycles}")
                assert g["status"] == r.status == oracle.CONVERGED
                assert g["relres_true"] <= 1e-8 * (1 + 1e-12)
                assert np.linalg.norm(x - r.x) / np.linalg.norm(r.x) <= bound
                assert abs(g["iters"] - r.iters) <= (2 if i < 2 else max(3, 0.1 * r.iters))
    finally:
        skr.skr_ctx_destroy(ctx)
