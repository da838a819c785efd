"""Full-size checks of the secondary workloads, where the oracle cannot run in seconds: properties
that hold at any size, recomputed on the CPU from the returned solutions.

* 3-D Darcy at 128^3 (n = 2,097,152; the bench's --dim 3 workload and launch configuration), matrix-free
  7-point operator, GCRO-DR(80,20) with FP64 and FP32-stored basis, and GCRO-DR(60,20): the FP64 residual ||b - A x|| / ||b|| of every
  returned x, recomputed with the assembled CSR matrix, is at most rtol (1 + 1e-9); the 7-point
  operator matches the CSR product row by row on sampled rows, within 8 eps sum_j |a_ij x_j|.
* Darcy 256^2, the whole sorted 400-system chain with GCRO-DR(60,20) (the bench workload in the
  launch configuration the bench times): every returned x has FP64 residual ||b - A x|| / ||b|| at
  most rtol (1 + 1e-9), recomputed on the CPU with the CSR matrix; every system converged and
  reuses a recycle space (k_start > 0 after the first).
* Advection-diffusion time-stepping at 512^2: one chain of 3 backward-Euler steps through the serving runtime;
  every step's residual, recomputed on the CPU, is at most rtol (1 + 1e-9), and the chain keeps its
  recycle space (fewer Arnoldi steps after the first).
"""
import numpy as np
import pytest

from gpu_common import log, make_ctx, need_gpu
from workloads import darcy3d_sequence, param_matrix
from workloads.darcy3d import darcy3d_from_nodes
from workloads.device import upload_systems

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def env():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    ctx = make_ctx(torch)
    yield torch, skr, ctx
    skr.skr_ctx_destroy(ctx)


@pytest.mark.parametrize("m,mixed", [(80, False), (80, True), (60, False)])
def test_3d_128_residuals(env, m, mixed):
    torch, skr, ctx = env
    log(f"[full] 3-D 128^3 stencil, 2 systems of the sorted chain, GCRO-DR({m},20), mixed={mixed}")
    systems = darcy3d_sequence(128, 2, with_csr=False)
    P = param_matrix(systems)
    order, _ = skr.skr_sort(ctx, torch.from_numpy(P).cuda(), P.shape[0], P.shape[1], 0)
    ops, bs, xs = upload_systems(systems, "cuda:0", "stencil")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=m, k=20, rtol=1e-8, maxit=40000,
                                     flags=skr.SKR_FLAG_MIXED if mixed else 0)
    assert rc == skr.SKR_OK
    torch.cuda.synchronize()
    for i in order:
        s = darcy3d_from_nodes(systems[i].a, with_csr=True)
        x = xs[i].cpu().numpy()
        rel = np.linalg.norm(s.b - s.A @ x) / np.linalg.norm(s.b)
        log(f"  sys {i}: iters {res[i]['iters']} relres gpu {res[i]['relres_true']:.3e} cpu {rel:.3e}")
        assert res[i]["status"] == skr.SKR_CONVERGED
        assert rel <= 1e-8 * (1 + 1e-9)
        assert abs(rel - res[i]["relres_true"]) <= 1e-3 * rel + 1e-16
    # 7-point operator against the CSR product on sampled rows
    s = darcy3d_from_nodes(systems[0].a, with_csr=True)
    xr = np.random.default_rng(3).standard_normal(s.n)
    xd = torch.from_numpy(xr).cuda()
    yd = torch.empty_like(xd)
    skr.skr_spmv(ctx, ops[0], xd, yd)
    y = yd.cpu().numpy()
    rows = np.random.default_rng(4).choice(s.n, 4096, replace=False)
    ref = s.A[rows] @ xr
    bound = 8 * EPS * (abs(s.A[rows]) @ np.abs(xr))
    assert np.all(np.abs(y[rows] - ref) <= bound)


def test_darcy256_full_chain_residuals(env):
    torch, skr, ctx = env
    log("[full] 256x256 Darcy, the sorted 400-system chain, GCRO-DR(60,20)")
    from workloads import darcy_sequence
    systems = darcy_sequence(256, 400)
    P = param_matrix(systems)
    order, _ = skr.skr_sort(ctx, torch.from_numpy(P).cuda(), P.shape[0], P.shape[1], 0)
    del P
    ops, bs, xs = upload_systems(systems, "cuda:0")
    rc, res = skr.skr_solve_sequence(ctx, ops, bs, xs, order, m=60, k=20, rtol=1e-8, maxit=40000)
    assert rc == skr.SKR_OK
    torch.cuda.synchronize()
    worst = 0.0
    for pos, i in enumerate(int(v) for v in order):
        s, r = systems[i], res[i]
        x = xs[i].cpu().numpy()
        rel = np.linalg.norm(s.b - s.A @ x) / np.linalg.norm(s.b)
        worst = max(worst, rel)
        assert r["status"] == skr.SKR_CONVERGED, (pos, i, r)
        assert rel <= 1e-8 * (1 + 1e-9), (pos, i, rel)
        assert abs(rel - r["relres_true"]) <= 1e-3 * rel + 1e-16, (pos, i, rel, r["relres_true"])
        assert pos == 0 or r["k_start"] > 0, (pos, i, r)
    log(f"  400 systems converged, worst CPU-recomputed relres {worst:.3e}, "
        f"mean steps {np.mean([r['iters'] for r in res]):.1f}")


def test_advdiff_512_time_stepping(env):
    torch, skr, ctx = env
    log("[full] advection-diffusion chain at 512^2, 3 backward-Euler steps through the serving runtime")
    from workloads.advdiff import advdiff_chains
    ch = advdiff_chains(512, 1, first_seed=0)[0]
    sctx = make_ctx(torch)
    try:
        skr.skr_serve_start(sctx, max_chains=2, workers=1, split_d2_rel=1e-12)
        ops, _, _ = upload_systems([ch], "cuda:0")
        params = torch.from_numpy(ch.params).cuda()
        b = torch.from_numpy(ch.x0 / ch.dt).cuda()
        iters = []
        for t in range(3):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            tk = skr.skr_submit(sctx, ops[0], params, params.numel(), b, x, m=60, k=20, rtol=1e-8, maxit=20000)
            assert skr.skr_ticket_chain(sctx, tk) == (0, t)
            r = skr.skr_wait(sctx, tk)
            xh, bh = x.cpu().numpy(), b.cpu().numpy()
            rel = np.linalg.norm(bh - ch.A @ xh) / np.linalg.norm(bh)
            log(f"  step {t}: iters {r['iters']} relres gpu {r['relres_true']:.3e} cpu {rel:.3e}")
            assert r["status"] == skr.SKR_CONVERGED and rel <= 1e-8 * (1 + 1e-9)
            iters.append(r["iters"])
            b = x / ch.dt
        assert iters[1] < iters[0] and iters[2] < iters[0]
        skr.skr_serve_stop(sctx)
    finally:
        skr.skr_ctx_destroy(sctx)
