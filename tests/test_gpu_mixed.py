"""GPU parity of the mixed-precision mode (SKR_FLAG_MIXED: FP32-stored Arnoldi vectors and recycle
space, FP64 arithmetic, one refinement step per cycle) against the oracle's mixed mode on the same
seeded inputs.

Bars (written in the tests): the same as for the FP64 path, since both sides round the same FP64
values to FP32 and so follow the same trajectory up to the rare value that sits on an FP32 rounding
tie: status equal, relative residual (FP64, of the FP64 solution) at most rtol, solution within the
residual bound of the oracle's, Arnoldi step counts equal up to one step for the first two systems
of a chain and within max(3, 10 %) further down (3 % for the chain), product counts equal where no
recycle space is inherited.
"""
import numpy as np
import pytest

import oracle
from gpu_common import compare_chain, log, make_ctx, need_gpu
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


def _ref(systems, order, m, k, rtol, maxit=20000):
    return oracle.solve_sequence([s.A for s in systems], [s.b for s in systems], order, m, k, rtol, maxit,
                                 basis_fp32=True)


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_mixed_config1(env, kind):
    """32x32 Darcy, 16 systems sorted into one chain, GCRO-DR(30,10), rel-res 1e-8."""
    torch, skr, ctx = env
    log(f"[mixed] config-1 chain kind={kind}")
    systems = darcy_sequence(32, 16)
    order = oracle.greedy_sort(param_matrix(systems))
    ops, bs, xs = upload_systems(systems, "cuda:0", kind)
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=30, k=10, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, order, 30, 10, 1e-8), f"mixed-cfg1-{kind}", order)


def test_mixed_gmres_k0(env):
    """GMRES(30) with an FP32 basis and one refinement step per cycle: systems are independent."""
    torch, skr, ctx = env
    log("[mixed] GMRES(30), k = 0")
    systems = darcy_sequence(32, 3, first_seed=40)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=30, k=0, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    ref = _ref(systems, None, 30, 0, 1e-8)
    compare_chain(systems, res, xs, ref, "mixed-gmres", strict=True)
    for g, r in zip(res, ref):
        assert g["spmv"] == r.spmv and g["cycles"] == r.cycles


@pytest.mark.parametrize("rtol", [1e-10, 1e-11])
def test_mixed_beyond_fp32(env, rtol):
    """Ragged n = 37^2, GCRO-DR(12,5): residuals that no FP32 iterate can represent."""
    torch, skr, ctx = env
    log(f"[mixed] ragged n=1369, GCRO-DR(12,5), rtol {rtol}")
    systems = darcy_sequence(37, 5, first_seed=70)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=12, k=5, rtol=rtol, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, None, 12, 5, rtol), f"mixed-{rtol}", rtol=rtol)
    for s, x in zip(systems, xs):
        xh = x.cpu().numpy()
        rel = np.linalg.norm(s.b - s.A @ xh) / np.linalg.norm(s.b)
        assert rel <= rtol * (1 + 1e-6)
        x32 = xh.astype(np.float32).astype(np.float64)
        assert np.linalg.norm(s.b - s.A @ x32) / np.linalg.norm(s.b) > 10 * rtol


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_mixed_3d_chain(env, kind):
    """3-D Darcy 10^3 (7-point), 6 systems, GCRO-DR(30,10)."""
    torch, skr, ctx = env
    log(f"[mixed] 3-D 10^3 chain kind={kind}")
    systems = darcy3d_sequence(10, 6)
    order = oracle.greedy_sort(param_matrix(systems))
    ops, bs, xs = upload_systems(systems, "cuda:0", kind)
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=30, k=10, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, order, 30, 10, 1e-8), f"mixed-3d-{kind}", order)


def test_mixed_fold_path(env):
    """Config-1 chain with the folded reductions forced on (the large-grid path) in mixed mode."""
    torch, skr, ctx = env
    log("[mixed] config-1 chain, folded reductions")
    systems = darcy_sequence(32, 8)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=30, k=10, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED | skr.SKR_FLAG_FOLD)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, None, 30, 10, 1e-8), "mixed-fold")


def test_mixed_config2_prefix(env):
    """256x256 Darcy, the first 2 systems of the sorted 400-system chain, GCRO-DR(60,20), FP32 basis:
    the bench workload's size and launch configuration, against the oracle's mixed mode."""
    torch, skr, ctx = env
    log("[mixed] config-2 prefix: 256x256, 2 systems of the sorted chain")
    systems = darcy_sequence(256, 400)
    P = param_matrix(systems)
    Pd = torch.from_numpy(np.ascontiguousarray(P)).cuda()
    order, _ = skr.skr_sort(ctx, Pd, P.shape[0], P.shape[1], 0)
    del P, Pd
    pre = [systems[i] for i in order[:2]]
    ops, bs, xs = upload_systems(pre, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=60, k=20, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    compare_chain(pre, res, xs, _ref(pre, None, 60, 20, 1e-8), "mixed-cfg2-prefix")
