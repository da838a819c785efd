"""GPU parity of the mixed-precision mode (SKR_FLAG_MIXED: FP32-stored Arnoldi vectors and recycle
space, the inner products with the operator's values rounded to FP32, FP64 arithmetic, one
refinement step per cycle with the FP64 operator) against the oracle's mixed mode on the same
seeded inputs, with the same inner operator (the rounded CSR values, or for the stencils the
matrix assembled from the rounded faces).

Bars (written in the tests): status equal, relative residual (FP64, of the FP64 solution) at most
rtol, solution within the residual bound of the oracle's, Arnoldi step counts within max(1, 2 %)
for the first two systems of a chain and within max(3, 10 %) further down (3 % for the chain),
product counts equal where no recycle space is inherited. Both sides round the same FP64 values to
FP32, but a long solve amplifies rounding differences: under a 1e-15 relative perturbation of b the
oracle's own first system of the sorted 256^2 chain moves over 1,491..1,505 steps in this mode
(0.94 %), so the first-systems bar is twice that spread; GMRES (no recycling) keeps one step.
"""
import numpy as np
import pytest

import oracle
from gpu_common import compare_chain, log, make_ctx, need_gpu
from oracle.solver import fp32_store
from workloads import darcy3d_sequence, darcy_sequence, param_matrix
from workloads.darcy import assemble_csr
from workloads.darcy3d import assemble_csr3d
from workloads.device import upload_systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    ctx = make_ctx(torch)
    yield torch, skr, ctx
    skr.skr_ctx_destroy(ctx)


def _inner(systems, kind):
    """The inner operator the GPU's mixed mode applies: CSR values rounded to FP32 (the oracle's
    default), or for the matrix-free stencils the matrix assembled from the FP32-rounded faces."""
    if kind == "csr":
        return None
    out = []
    for s in systems:
        if hasattr(s, "az"):
            out.append(assemble_csr3d(fp32_store(s.ax), fp32_store(s.ay), fp32_store(s.az), s.inv_h2))
        else:
            out.append(assemble_csr(fp32_store(s.ax), fp32_store(s.ay), s.inv_h2))
    return out


# bar on the first two systems of a chain: twice the oracle's own spread in this mode (compare_chain)
MIXED_LEAD = 0.02


def _ref(systems, order, m, k, rtol, maxit=20000, kind="csr"):
    return oracle.solve_sequence([s.A for s in systems], [s.b for s in systems], order, m, k, rtol, maxit,
                                 basis_fp32=True, A_inner=_inner(systems, kind))


@pytest.mark.parametrize("kind", ["csr", "stencil"])
def test_mixed_darcy32_chain(env, kind):
    """32x32 Darcy, 16 systems sorted into one chain, GCRO-DR(30,10), rel-res 1e-8."""
    torch, skr, ctx = env
    log(f"[mixed] 32x32 chain of 16 systems kind={kind}")
    systems = darcy_sequence(32, 16)
    order = oracle.greedy_sort(param_matrix(systems))
    ops, bs, xs = upload_systems(systems, "cuda:0", kind)
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=30, k=10, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, order, 30, 10, 1e-8, kind=kind), f"mixed-darcy32-{kind}", order,
                  lead=MIXED_LEAD)


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
        # products besides the Arnoldi steps (one refinement residual per cycle, the exit test) and
        # cycles equal; the step counts themselves are within the one-step bar above
        assert g["spmv"] - g["iters"] == r.spmv - r.iters and g["cycles"] == r.cycles


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
    compare_chain(systems, res, xs, _ref(systems, None, 12, 5, rtol), f"mixed-{rtol}", rtol=rtol, lead=MIXED_LEAD)
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
    compare_chain(systems, res, xs, _ref(systems, order, 30, 10, 1e-8, kind=kind), f"mixed-3d-{kind}", order, lead=MIXED_LEAD)


def test_mixed_fold_path(env):
    """32x32 chain with the folded reductions forced on (the large-grid path) in mixed mode."""
    torch, skr, ctx = env
    log("[mixed] 32x32 chain, folded reductions")
    systems = darcy_sequence(32, 8)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=30, k=10, rtol=1e-8, maxit=20000,
                                     flags=skr.SKR_FLAG_MIXED | skr.SKR_FLAG_FOLD)
    assert rc == skr.SKR_OK
    compare_chain(systems, res, xs, _ref(systems, None, 30, 10, 1e-8), "mixed-fold", lead=MIXED_LEAD)


def test_mixed_darcy256_prefix(env):
    """256x256 Darcy, the first 2 systems of the sorted 400-system chain, GCRO-DR(60,20), FP32 basis:
    the bench workload's size and launch configuration, against the oracle's mixed mode."""
    torch, skr, ctx = env
    log("[mixed] 256x256 prefix: 2 systems of the sorted 400-system chain")
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
    compare_chain(pre, res, xs, _ref(pre, None, 60, 20, 1e-8), "mixed-darcy256-prefix", lead=MIXED_LEAD)


def test_mixed_edge_cases(env):
    """The refinement step around the exits of a solve: b = 0, NaN in b, maxit = 1, a happy breakdown
    (identity operator), a start-up whose projection already solves the system, against the oracle's
    mixed mode where it defines the outcome."""
    torch, skr, ctx = env
    log("[mixed] edge cases")
    import types

    import scipy.sparse as sp
    M = skr.SKR_FLAG_MIXED
    s = darcy_sequence(16, 1, first_seed=5)[0]
    n = s.n
    ops, bs, xs = upload_systems([s, s, s, s], "cuda:0")
    bs[1].zero_()
    bs[2][5] = float("nan")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=6, rtol=1e-8, maxit=5000, flags=M)
    assert rc == skr.SKR_OK
    assert res[0]["status"] == skr.SKR_CONVERGED
    assert res[1]["status"] == skr.SKR_CONVERGED and res[1]["iters"] == 0 and not xs[1].any()
    assert res[2]["status"] == skr.SKR_NONFINITE and not xs[2].any()
    assert res[3]["status"] == skr.SKR_CONVERGED          # recycles the space of system 0
    ref = oracle.solve_sequence([s.A, s.A], [s.b, s.b], None, 20, 6, 1e-8, 5000, basis_fp32=True)
    assert abs(res[0]["iters"] - ref[0].iters) <= 1 and abs(res[3]["iters"] - ref[1].iters) <= 1
    # maxit = 1
    ops1, bs1, xs1 = upload_systems([s], "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops1, bs1, xs1, None, m=20, k=6, rtol=1e-8, maxit=1, flags=M)
    assert rc == skr.SKR_WARN_NOTCONVERGED and res[0]["status"] == skr.SKR_MAXIT and res[0]["iters"] == 1
    r1 = oracle.gcrodr(s.A, s.b, None, 20, 6, 1e-8, 1, basis_fp32=True)
    assert abs(res[0]["relres_true"] - r1.relres_true) <= 1e-6 * r1.relres_true
    # identity: the first step breaks down, x = b up to the FP32 rounding of the stored basis vector
    ident = types.SimpleNamespace(A=sp.identity(n, format="csr"), b=s.b, n=n, N_g=s.N_g)
    ops2, bs2, xs2 = upload_systems([ident], "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops2, bs2, xs2, None, m=20, k=6, rtol=1e-8, maxit=100, flags=M)
    assert res[0]["status"] in (skr.SKR_BREAKDOWN, skr.SKR_CONVERGED)
    assert res[0]["relres_true"] <= 1e-8
    np.testing.assert_allclose(xs2[0].cpu().numpy(), s.b, rtol=1e-7)
    # the same right-hand side twice: the second system starts from a recycle space whose projection
    # already gives a small residual; the result still meets the FP64 tolerance
    ops3, bs3, xs3 = upload_systems([s, s], "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops3, bs3, xs3, None, m=20, k=6, rtol=1e-8, maxit=5000, flags=M)
    for r, x in zip(res, xs3):
        xh = x.cpu().numpy()
        assert r["status"] == skr.SKR_CONVERGED
        assert np.linalg.norm(s.b - s.A @ xh) <= 1e-8 * np.linalg.norm(s.b) * (1 + 1e-9)
