"""GPU tests of the serving runtime (skr_serve_start / skr_submit / skr_poll).

Bars (written in the tests):
* with one chain, serving gives bit-identical solutions and equal counts to skr_solve_sequence
  over the same systems in submission order (the same kernels, the same recycle hand-over);
* the chain each system joins, and its position there, equal the rule recomputed on the CPU from
  the oracle's exact squared distances (nearest chain of the same shape by d2, ties to the lower
  id, a new chain above split_d2_rel * ||params||^2 or when every chain of the shape holds
  max_chain_systems systems);
* every chain's results meet the oracle's for the same systems in chain order, to the parity bars
  of the sequence solver;
* results are bit-identical with one worker and with four (the interleaving of chains is
  invisible);
* deferred admission (no room for a new chain) completes every system, in a fresh chain;
* argument errors, a non-finite right-hand side and ticket collection behave as documented.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_common import same_result as _same, compare_chain, log, make_ctx, need_gpu
from workloads import darcy_sequence, param_matrix
from workloads.device import upload_systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    return torch, skr


def _stream(seed=7, sizes=(24, 32), count=10):
    """Interleaved submission stream of Darcy systems of two grid sizes (seeded)."""
    rng = np.random.default_rng(seed)
    sys_by_size = {N: darcy_sequence(N, count, first_seed=100 * N) for N in sizes}
    order = []
    left = {N: list(range(count)) for N in sizes}
    while any(left.values()):
        N = sizes[int(rng.integers(len(sizes)))]
        if left[N]:
            order.append(sys_by_size[N][left[N].pop(0)])
    return order


def _upload(torch, systems, kind="csr"):
    ops, bs, xs = upload_systems(systems, "cuda:0", kind)
    params = [torch.from_numpy(np.ascontiguousarray(s.a.ravel())).cuda() for s in systems]
    return ops, bs, xs, params


def _serve(torch, skr, systems, m=20, k=6, rtol=1e-8, flags=None, workers=4, max_chains=8,
           split=math.inf, kind="csr", cap=0):
    ctx = make_ctx(torch)
    try:
        skr.skr_serve_start(ctx, max_chains=max_chains, workers=workers, split_d2_rel=split,
                            max_chain_systems=cap)
        ops, bs, xs, params = _upload(torch, systems, kind)
        flags = flags or [0] * len(systems)
        tickets = [skr.skr_submit(ctx, ops[i], params[i], params[i].numel(), bs[i], xs[i], m=m, k=k, rtol=rtol,
                                  maxit=20000, flags=flags[i]) for i in range(len(systems))]
        where = [skr.skr_ticket_chain(ctx, t) for t in tickets]
        res = [skr.skr_wait(ctx, t) for t in tickets]
        stats = skr.skr_serve_stats_get(ctx)
        torch.cuda.synchronize()
        xh = [x.cpu().numpy() for x in xs]
        skr.skr_serve_stop(ctx)
    finally:
        skr.skr_ctx_destroy(ctx)
    return res, xh, where, stats


def _cpu_rule(systems, split=math.inf, max_chains=8, shape=lambda s: s.n, cap=0):
    """The admission rule of skr.h on the CPU with the oracle's exact d2 (no retirement needed)."""
    tails, shapes, counts, out = [], [], [], []
    for s in systems:
        p = s.a.ravel()
        same = [c for c in range(len(tails)) if shapes[c] == shape(s)]
        cand = [c for c in same if not (cap > 0 and counts[c] >= cap)]
        if same and not cand:                       # every chain of the shape is full
            if len(tails) < max_chains:
                tails.append(p)
                shapes.append(shape(s))
                counts.append(0)
                out.append((len(tails) - 1, 0))
                counts[-1] = 1
                continue
            cand = same
        best, bd = None, math.inf
        for c in cand:
            d = oracle.sq_distance(p, tails[c])
            if d < bd:
                best, bd = c, d
        if best is None and cand:
            best = cand[0]
        pn2 = oracle.sq_distance(p, np.zeros_like(p))
        if best is None or (bd > split * pn2 and len(tails) < max_chains):
            tails.append(p)
            shapes.append(shape(s))
            counts.append(0)
            best = len(tails) - 1
        tails[best] = p
        out.append((best, counts[best]))
        counts[best] += 1
    return out


@pytest.mark.parametrize("m,k", [(20, 6), (80, 20)])
def test_serve_one_chain_equals_solve_sequence(env, m, k):
    torch, skr = env
    log(f"[serve] one chain vs skr_solve_sequence, 32x32, 6 systems, GCRO-DR({m},{k})")
    systems = darcy_sequence(32, 6, first_seed=300)
    res, xh, where, _ = _serve(torch, skr, systems, m=m, k=k, max_chains=1, workers=2)
    assert [w for w in where] == [(0, i) for i in range(6)]
    ctx = make_ctx(torch)
    try:
        ops, bs, xs, _ = _upload(torch, systems)
        rc, ref = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=m, k=k, rtol=1e-8, maxit=20000)
        torch.cuda.synchronize()
        for i in range(6):
            assert _same(res[i], ref[i]), i
            assert np.array_equal(xh[i], xs[i].cpu().numpy()), i
    finally:
        skr.skr_ctx_destroy(ctx)


@pytest.mark.parametrize("split,cap,max_chains", [(math.inf, 0, 8), (0.02, 0, 8), (math.inf, 3, 8),
                                                  (math.inf, 3, 5)])
def test_serve_assignment_and_parity(env, split, cap, max_chains):
    torch, skr = env
    log(f"[serve] two sizes interleaved, split {split}, chain cap {cap}, max_chains {max_chains}")
    systems = _stream()
    res, xh, where, stats = _serve(torch, skr, systems, split=split, cap=cap, max_chains=max_chains)
    want = _cpu_rule(systems, split=split, cap=cap, max_chains=max_chains)
    if cap:
        n_full = sum(1 for c in set(c for c, _ in want) if sum(1 for cc, _ in want if cc == c) > cap)
        assert n_full == 0 or len({c for c, _ in want}) == max_chains     # over the cap only without room
    assert where == want
    assert stats["completed"] == len(systems) and stats["chains_created"] == len({c for c, _ in want})
    # per chain: the oracle's sequence solve over the chain's systems in chain order
    for c in sorted({c for c, _ in want}):
        idx = [i for i, (cc, _) in enumerate(want) if cc == c]
        chain_sys = [systems[i] for i in idx]
        ref = oracle.solve_sequence([s.A for s in chain_sys], [s.b for s in chain_sys], None, 20, 6, 1e-8, 20000)

        class _X:                 # host solutions in the shape compare_chain reads
            def __init__(self, a):
                self.a = a

            def cpu(self):
                return self

            def numpy(self):
                return self.a
        compare_chain(chain_sys, [res[i] for i in idx], [_X(xh[i]) for i in idx], ref, f"serve-chain{c}")


def test_serve_mix_equals_alone(env):
    """Every chain of a served mix (two sizes interleaved, several chains of each size, four workers)
    gives results and solutions identical bit for bit to the same systems solved alone, in chain
    order, by skr_solve_sequence on a fresh context."""
    torch, skr = env
    log("[serve] each chain of the mix against the chain alone")
    systems = _stream(seed=13, count=8)
    res, xh, where, stats = _serve(torch, skr, systems, split=0.02, workers=4)
    chains = sorted({c for c, _ in where})
    assert len(chains) >= 3
    for c in chains:
        idx = sorted((p, i) for i, (cc, p) in enumerate(where) if cc == c)
        idx = [i for _, i in idx]
        ctx = make_ctx(torch)
        try:
            ops, bs, xs, _ = _upload(torch, [systems[i] for i in idx])
            rc, ref = skr.skr_solve_sequence(ctx, ops, bs, xs, None, m=20, k=6, rtol=1e-8, maxit=20000)
            torch.cuda.synchronize()
            for q, i in enumerate(idx):
                assert _same(res[i], ref[q]), (c, q, i)
                assert np.array_equal(xh[i], xs[q].cpu().numpy()), (c, q, i)
        finally:
            skr.skr_ctx_destroy(ctx)


def test_serve_workers_do_not_change_results(env):
    torch, skr = env
    log("[serve] 1 worker vs 4 workers, bitwise")
    systems = _stream(seed=11, count=6)
    r1, x1, w1, _ = _serve(torch, skr, systems, workers=1, split=0.02)
    r4, x4, w4, _ = _serve(torch, skr, systems, workers=4, split=0.02)
    assert w1 == w4
    for i in range(len(systems)):
        assert _same(r1[i], r4[i]), i
        assert np.array_equal(x1[i], x4[i]), i


def test_serve_deferred_admission(env):
    torch, skr = env
    log("[serve] max_chains = 1 with two sizes: deferred admission")
    a, b = darcy_sequence(24, 2, first_seed=500), darcy_sequence(32, 1, first_seed=600)
    systems = [a[0], b[0], a[1]]
    res, xh, where, stats = _serve(torch, skr, systems, max_chains=1, workers=2)
    assert stats["completed"] == 3 and stats["chains_created"] == 3 and stats["chains_retired"] >= 2
    for s, r, x in zip(systems, res, xh):
        ref = oracle.gcrodr(s.A, s.b, None, 20, 6, 1e-8, 20000)     # every system starts a fresh chain
        assert r["status"] == ref.status and abs(r["iters"] - ref.iters) <= 1
        assert np.linalg.norm(s.b - s.A @ x) <= 1e-8 * np.linalg.norm(s.b) * (1 + 1e-9)


def test_serve_mixed_and_fp64_chains_are_separate(env):
    torch, skr = env
    log("[serve] FP32-basis and FP64 systems of one size form separate chains")
    systems = darcy_sequence(32, 6, first_seed=700)
    flags = [skr.SKR_FLAG_MIXED if i % 2 else 0 for i in range(6)]
    res, xh, where, _ = _serve(torch, skr, systems, flags=flags)
    assert {where[i][0] for i in range(0, 6, 2)} == {0} and {where[i][0] for i in range(1, 6, 2)} == {1}
    for c, idx, mixed in ((0, [0, 2, 4], False), (1, [1, 3, 5], True)):
        chain_sys = [systems[i] for i in idx]
        ref = oracle.solve_sequence([s.A for s in chain_sys], [s.b for s in chain_sys], None, 20, 6, 1e-8, 20000,
                                    basis_fp32=mixed)
        for i, r in zip(idx, ref):
            assert res[i]["status"] == r.status
            assert abs(res[i]["iters"] - r.iters) <= max(3, 0.1 * r.iters)
            s = systems[i]
            assert np.linalg.norm(s.b - s.A @ xh[i]) <= 1e-8 * np.linalg.norm(s.b) * (1 + 1e-9)


def test_serve_errors(env):
    torch, skr = env
    log("[serve] argument errors, non-finite b, ticket collection")
    s = darcy_sequence(16, 1, first_seed=800)[0]
    ctx = make_ctx(torch)
    try:
        ops, bs, xs, params = _upload(torch, [s, s])
        with pytest.raises(skr.SkrError) as e:
            skr.skr_submit(ctx, ops[0], params[0], params[0].numel(), bs[0], xs[0])
        assert e.value.code == skr.SKR_EINVAL
        skr.skr_serve_start(ctx, max_chains=2, workers=1, arena_bytes=1000)
        with pytest.raises(skr.SkrError) as e:
            skr.skr_serve_start(ctx)
        assert e.value.code == skr.SKR_EINVAL
        with pytest.raises(skr.SkrError) as e:                   # workspace larger than the arena
            skr.skr_submit(ctx, ops[0], params[0], params[0].numel(), bs[0], xs[0], m=20, k=6)
        assert e.value.code == skr.SKR_ENOMEM
        skr.skr_serve_stop(ctx)
        skr.skr_serve_start(ctx, max_chains=2, workers=1)
        with pytest.raises(skr.SkrError):
            skr.skr_submit(ctx, ops[0], params[0], params[0].numel(), bs[0], xs[0], m=5, k=5)
        bs[1][3] = float("nan")
        t0 = skr.skr_submit(ctx, ops[0], params[0], params[0].numel(), bs[0], xs[0], m=20, k=6)
        t1 = skr.skr_submit(ctx, ops[1], params[1], params[1].numel(), bs[1], xs[1], m=20, k=6)
        r0, r1 = skr.skr_wait(ctx, t0), skr.skr_wait(ctx, t1)
        assert r0["status"] == skr.SKR_CONVERGED and r1["status"] == skr.SKR_NONFINITE
        with pytest.raises(skr.SkrError) as e:                   # collected already
            skr.skr_poll(ctx, t0)
        assert e.value.code == skr.SKR_EINVAL
        with pytest.raises(skr.SkrError):
            skr.skr_poll(ctx, 12345)
        skr.skr_serve_stop(ctx)
    finally:
        skr.skr_ctx_destroy(ctx)


def test_serve_time_stepping_chains(env):
    """Backward-Euler advection-diffusion chains (24x24, 3 chains x 4 steps): the right-hand side
    of step t + 1 is x^t / dt, so each chain's systems are submitted one after another and keep
    their chain (identical parameters, d2 = 0) and its recycle space. Against the oracle stepping
    the same chains from its own solutions."""
    torch, skr = env
    log("[serve] time-stepping advection-diffusion chains")
    from workloads.advdiff import advdiff_chains
    chains = advdiff_chains(24, 3, first_seed=900)
    steps, m, k, rtol = 4, 20, 6, 1e-9
    ctx = make_ctx(torch)
    try:
        skr.skr_serve_start(ctx, max_chains=8, workers=3, split_d2_rel=1e-12)
        ops, _, _ = upload_systems(chains, "cuda:0")
        params = [torch.from_numpy(c.params).cuda() for c in chains]
        xs = [[torch.zeros(c.n, dtype=torch.float64, device="cuda") for _ in range(steps)] for c in chains]
        bs = [torch.empty(c.n, dtype=torch.float64, device="cuda") for c in chains]
        res = [[None] * steps for _ in chains]
        where = [[None] * steps for _ in chains]
        for t in range(steps):
            tickets = []
            for c, ch in enumerate(chains):
                prev = torch.from_numpy(ch.x0).cuda() if t == 0 else xs[c][t - 1]
                torch.div(prev, ch.dt, out=bs[c])
                torch.cuda.synchronize()
                tickets.append(skr.skr_submit(ctx, ops[c], params[c], params[c].numel(), bs[c], xs[c][t], m=m, k=k,
                                              rtol=rtol, maxit=20000))
            for c, tk in enumerate(tickets):
                where[c][t] = skr.skr_ticket_chain(ctx, tk)
                res[c][t] = skr.skr_wait(ctx, tk)
        torch.cuda.synchronize()
        xh = [[x.cpu().numpy() for x in xc] for xc in xs]
        skr.skr_serve_stop(ctx)
    finally:
        skr.skr_ctx_destroy(ctx)
    for c, ch in enumerate(chains):
        assert [w for w in where[c]] == [(c, t) for t in range(steps)]
        smin = np.linalg.svd(ch.A.toarray(), compute_uv=False)[-1]
        Y, b = None, ch.x0 / ch.dt
        for t in range(steps):
            r = oracle.gcrodr(ch.A, b, Y, m, k, rtol, 20000)
            g = res[c][t]
            mu = np.linalg.norm(b) / smin / np.linalg.norm(r.x)
            rel = np.linalg.norm(xh[c][t] - r.x) / np.linalg.norm(r.x)
            log(f"  chain {c} step {t}: iters gpu {g['iters']} oracle {r.iters}  rel {rel:.2e}")
            assert g["status"] == r.status == oracle.CONVERGED
            assert g["relres_true"] <= rtol * (1 + 1e-9)
            # both runs step from their own x^t, which agree to the solve tolerance: mu (rr + rr) per step,
            # accumulated over the steps taken
            assert rel <= max(1e-7, 1.01 * (t + 1) * mu * (g["relres_true"] + r.relres_true))
            assert abs(g["iters"] - r.iters) <= (1 if t < 2 else max(3, 0.1 * r.iters))
            Y, b = r.Y_next, r.x / ch.dt
