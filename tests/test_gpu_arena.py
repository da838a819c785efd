"""GPU tests of the caller-owned arena (skr_ctx_create's arena_dev / arena_bytes).

Bars (written in the tests):
* a context whose arena is smaller than the workspace skr_workspace_bytes reports fails the solve
  with SKR_ENOMEM, and the same arena enlarged to that size (plus the sort's buffers) solves the
  chain with results and solutions identical bit for bit to a context that allocates its own
  memory, in both storage modes;
* serving on a context whose arena holds one chain at a time: a system of a second shape that
  arrives while the first shape's chain runs is deferred (its ticket has no chain yet), the idle
  chain is retired to make room, and every system meets the tolerance; the second shape's results
  equal bit for bit the same systems solved alone.
"""
import math

import numpy as np
import pytest

from gpu_common import log, need_gpu, same_result
from workloads import darcy_sequence
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
    return rc, res, [x.cpu().numpy() for x in xs]


@pytest.mark.parametrize("mixed", [False, True])
def test_arena_solve_and_exhaustion(env, mixed):
    torch, skr = env
    flags = skr.SKR_FLAG_MIXED if mixed else 0
    systems = darcy_sequence(32, 5, first_seed=31)
    n, m, k = systems[0].n, 30, 10
    wb = skr.skr_workspace_bytes(n, m, k, flags)
    op32 = 4 * int(systems[0].A.nnz) + 256 if mixed else 0
    log(f"[arena] workspace {wb} bytes, mixed={mixed}")
    stream = torch.cuda.current_stream().cuda_stream
    # too small: one byte short of the workspace
    small = torch.empty(wb - 1, dtype=torch.uint8, device="cuda:0")
    ctx = skr.skr_ctx_create(0, stream, small)
    try:
        ops, bs, xs = upload_systems(systems[:1], "cuda:0")
        with pytest.raises(skr.SkrError) as e:
            skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=m, k=k, rtol=1e-8, maxit=20000, flags=flags)
        assert e.value.code == skr.SKR_ENOMEM
    finally:
        skr.skr_ctx_destroy(ctx)
    # large enough (the 256-byte alignment of the buffer start may cost one block)
    arena = torch.empty(wb + op32 + 512, dtype=torch.uint8, device="cuda:0")
    ctx_a = skr.skr_ctx_create(0, stream, arena)
    ctx_p = skr.skr_ctx_create(0, stream)
    try:
        rc_a, ra, xa = _solve(torch, skr, ctx_a, systems, m, k, flags)
        rc_p, rp, xp = _solve(torch, skr, ctx_p, systems, m, k, flags)
    finally:
        skr.skr_ctx_destroy(ctx_a)
        skr.skr_ctx_destroy(ctx_p)
    assert rc_a == rc_p == skr.SKR_OK
    for a, p, u, v in zip(ra, rp, xa, xp):
        assert same_result(a, p)
        assert np.array_equal(u, v)
    # a half-given arena is an argument error
    import ctypes
    out = ctypes.c_void_p()
    assert skr.load_library().skr_ctx_create(0, stream, arena.data_ptr(), 0, ctypes.byref(out)) == skr.SKR_EINVAL


def test_arena_serving_defers_and_retires(env):
    torch, skr = env
    a = darcy_sequence(64, 1, first_seed=41)[0]          # the long first system (rtol 1e-11)
    b = darcy_sequence(32, 3, first_seed=42)
    m, k, p_a, p_b = 30, 10, a.a.size, b[0].a.size
    cb_a = skr.skr_workspace_bytes(a.n, m, k, 0) + (8 * p_a + 255) // 256 * 256
    cb_b = skr.skr_workspace_bytes(b[0].n, m, k, 0) + (8 * p_b + 255) // 256 * 256
    size = max(cb_a, cb_b) + min(cb_a, cb_b) // 2 + 1024           # one chain at a time
    log(f"[arena] serving with an arena of {size} bytes (chains of {cb_a} and {cb_b} bytes)")
    arena = torch.empty(size, dtype=torch.uint8, device="cuda:0")
    ctx = skr.skr_ctx_create(0, torch.cuda.current_stream().cuda_stream, arena)
    try:
        skr.skr_serve_start(ctx, max_chains=4, workers=2, split_d2_rel=math.inf)
        ops_a, bs_a, xs_a = upload_systems([a], "cuda:0")
        ops_b, bs_b, xs_b = upload_systems(b, "cuda:0")
        pa = torch.from_numpy(np.ascontiguousarray(a.a.ravel())).cuda()
        pbs = [torch.from_numpy(np.ascontiguousarray(s.a.ravel())).cuda() for s in b]
        t0 = skr.skr_submit(ctx, ops_a[0], pa, p_a, bs_a[0], xs_a[0], m=m, k=k, rtol=1e-11, maxit=40000)
        tb = [skr.skr_submit(ctx, ops_b[i], pbs[i], p_b, bs_b[i], xs_b[i], m=m, k=k, rtol=1e-8, maxit=20000)
              for i in range(3)]
        first = skr.skr_ticket_chain(ctx, tb[0])
        r0 = skr.skr_wait(ctx, t0)
        rb = [skr.skr_wait(ctx, t) for t in tb]
        stats = skr.skr_serve_stats_get(ctx)
        torch.cuda.synchronize()
        log(f"  first b ticket chain {first}; stats {stats}")
        assert r0["status"] == skr.SKR_CONVERGED and all(r["status"] == skr.SKR_CONVERGED for r in rb)
        assert stats["chains_created"] == 2 and stats["chains_retired"] >= 1
        assert stats["bytes_in_use"] <= size
        x0 = xs_a[0].cpu().numpy()
        assert np.linalg.norm(a.b - a.A @ x0) <= 1e-11 * np.linalg.norm(a.b) * (1 + 1e-9)
        xb = [x.cpu().numpy() for x in xs_b]
        skr.skr_serve_stop(ctx)
    finally:
        skr.skr_ctx_destroy(ctx)
    # the b systems formed one fresh chain, in submission order: the same as solving them alone
    ctx2 = skr.skr_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        rc, ref, xref = _solve(torch, skr, ctx2, b, m, k, 0)
    finally:
        skr.skr_ctx_destroy(ctx2)
    for r, q, u, v in zip(rb, ref, xb, xref):
        assert same_result(r, q)
        assert np.array_equal(u, v)
    # the first b system could not get a chain while the 64^2 chain was queued or running
    assert tuple(first) == (-1, -1)
