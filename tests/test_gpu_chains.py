"""GPU tests of skr_solve_chains: several chains of a sorted order advanced together, one grid row
per chain in every launch (the data-parallel split of the sorted sequence, App. E).

Bar (written in the tests): every chain's results (all fields but the wall-clock seconds) and
solutions equal bit for bit those of the same chain solved alone with skr_solve_sequence on a
context of its own. The batched kernels wrap the same device bodies with the same launch shapes, so
anything short of bitwise equality is a bug. Cases: FP64 CSR (two kernels per Arnoldi step),
FP32 storage with the matrix-free stencil, a nonsymmetric advection-diffusion chain set (general
eigen stage), the folded three-kernel path (n > 65536), m = 72 (two column groups), chains that
stop at maxit at different points, a non-finite right-hand side inside a chain, an empty chain,
and time-stepping chains continued call by call (SKR_FLAG_CONTINUE). The oracle pins the chains
through skr_solve_sequence's own parity tests; here the nonsymmetric case also checks the reported
residuals against ones recomputed on the CPU.
"""
import numpy as np
import pytest

from gpu_common import log, make_ctx, need_gpu, same_result
from workloads import darcy_sequence
from workloads.advdiff import advdiff_chains, advdiff_sequence
from workloads.device import upload_systems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    return torch, skr


def _alone(torch, skr, systems, kind, order, starts, nan_at, **kw):
    """Each chain on a fresh context with one skr_solve_sequence call."""
    N = len(systems)
    res, xs = [None] * N, [None] * N
    for c in range(len(starts) - 1):
        sl = [int(i) for i in order[starts[c]:starts[c + 1]]]
        if not sl:
            continue
        ops, bs, xl = upload_systems([systems[i] for i in sl], "cuda:0", kind)
        for q, i in enumerate(sl):
            if i in nan_at:
                bs[q][nan_at[i]] = float("nan")
        ctx = make_ctx(torch)
        try:
            _, r = skr.skr_solve_sequence(ctx, ops, bs, xl, None, **kw)
        finally:
            torch.cuda.synchronize()
            skr.skr_ctx_destroy(ctx)
        for q, i in enumerate(sl):
            res[i] = r[q]
            xs[i] = xl[q].cpu().numpy()
    return res, xs


def _batched(torch, skr, systems, kind, order, starts, nan_at, **kw):
    ops, bs, xl = upload_systems(systems, "cuda:0", kind)
    for i, e in nan_at.items():
        bs[i][e] = float("nan")
    ctx = make_ctx(torch)
    try:
        rc, res = skr.skr_solve_chains(ctx, starts, ops, bs, xl, order, **kw)
    finally:
        torch.cuda.synchronize()
        skr.skr_ctx_destroy(ctx)
    return rc, res, [x.cpu().numpy() for x in xl], xl


def _same(a, b):
    """same_result with NaN equal to NaN (a non-finite system reports NaN residuals)."""
    fa = {k: v for k, v in a.items() if k != "seconds"}
    fb = {k: v for k, v in b.items() if k != "seconds"}
    nan = [k for k, v in fa.items() if isinstance(v, float) and np.isnan(v)]
    return (all(isinstance(fb[k], float) and np.isnan(fb[k]) for k in nan)
            and same_result({k: v for k, v in fa.items() if k not in nan}, {k: v for k, v in fb.items() if k not in nan}))


def _check_equal(tag, order, starts, res_b, xs_b, res_a, xs_a):
    for c in range(len(starts) - 1):
        for pos in range(starts[c], starts[c + 1]):
            i = int(order[pos])
            assert _same(res_b[i], res_a[i]), (tag, c, pos, i, res_b[i], res_a[i])
            assert np.array_equal(xs_b[i], xs_a[i], equal_nan=True), (tag, c, pos, i)
    log(f"  {tag}: {len(order)} systems in {len(starts) - 1} chains equal the chains solved alone"
        f" (iterations {[res_b[int(i)]['iters'] for i in order]})")


class _Sys:
    def __init__(self, A, b):
        self.A, self.b, self.n = A, b, A.shape[0]


CASES = {
    # tag: (systems factory, operator kind, chain starts, options, {system: NaN entry})
    "darcy-fp64-csr": (lambda: darcy_sequence(32, 10, first_seed=300), "csr", [0, 4, 4, 7, 10],
                       dict(m=30, k=10, rtol=1e-8, maxit=20000, flags=0), {}),
    "darcy-fp32basis-stencil": (lambda: darcy_sequence(32, 9, first_seed=310), "stencil", [0, 2, 5, 9],
                                dict(m=30, k=10, rtol=1e-8, maxit=20000, flags="mixed"), {}),
    "darcy-fp64-m72": (lambda: darcy_sequence(32, 6, first_seed=320), "csr", [0, 3, 6],
                       dict(m=72, k=20, rtol=1e-8, maxit=20000, flags=0), {}),
    "darcy-maxit": (lambda: darcy_sequence(32, 6, first_seed=330), "csr", [0, 1, 3, 6],
                    dict(m=30, k=10, rtol=1e-10, maxit=75, flags=0), {}),
    "darcy-nonfinite": (lambda: darcy_sequence(32, 6, first_seed=340), "csr", [0, 3, 6],
                        dict(m=30, k=10, rtol=1e-8, maxit=20000, flags=0), {1: 17}),
    "darcy-fold-fp64": (lambda: darcy_sequence(288, 4, first_seed=350), "csr", [0, 2, 4],
                        dict(m=30, k=10, rtol=1e-8, maxit=20000, flags=0), {}),
}


@pytest.mark.parametrize("tag", list(CASES))
def test_chains_equal_alone(env, tag):
    torch, skr = env
    make, kind, starts, kw, nan_at = CASES[tag]
    kw = dict(kw)
    if kw["flags"] == "mixed":
        kw["flags"] = skr.SKR_FLAG_MIXED
    systems = make()
    N = len(systems)
    order = np.random.default_rng(7).permutation(N)
    log(f"[chains] {tag}: n {systems[0].n}, chains {np.diff(starts).tolist()}, {kw}")
    rc_b, res_b, xs_b, _ = _batched(torch, skr, systems, kind, order, starts, nan_at, **kw)
    res_a, xs_a = _alone(torch, skr, systems, kind, order, starts, nan_at, **kw)
    _check_equal(tag, order, starts, res_b, xs_b, res_a, xs_a)
    if tag == "darcy-maxit":
        assert rc_b == skr.SKR_WARN_NOTCONVERGED
        assert any(r["status"] == skr.SKR_MAXIT for r in res_b)
    elif tag == "darcy-nonfinite":
        (i,) = nan_at
        assert res_b[i]["status"] == skr.SKR_NONFINITE and not np.any(xs_b[i])
        assert all(r["status"] == skr.SKR_CONVERGED for j, r in enumerate(res_b) if j != i)
    else:
        assert rc_b == skr.SKR_OK and all(r["status"] == skr.SKR_CONVERGED for r in res_b)


def test_nonsymmetric_chains_equal_alone(env):
    torch, skr = env
    systems = [_Sys(s.A, s.b) for s in advdiff_sequence(32, 6, first_seed=360, amp=30.0)]
    order = np.arange(6)
    starts = [0, 3, 6]
    kw = dict(m=20, k=6, rtol=1e-8, maxit=20000, flags=skr.SKR_FLAG_MIXED)
    log("[chains] advection-diffusion 32^2, FP32 storage, 2 chains of 3")
    rc, res_b, xs_b, xl = _batched(torch, skr, systems, "csr", order, starts, {}, **kw)
    res_a, xs_a = _alone(torch, skr, systems, "csr", order, starts, {}, **kw)
    _check_equal("advdiff-mixed", order, starts, res_b, xs_b, res_a, xs_a)
    assert rc == skr.SKR_OK
    for s, r, x in zip(systems, res_b, xs_b):
        # the reported FP64 residual is the true one, recomputed here on the CPU
        rr = np.linalg.norm(s.b - s.A @ x) / np.linalg.norm(s.b)
        assert r["status"] == skr.SKR_CONVERGED and rr <= 1e-8 * (1 + 1e-6), (r, rr)
        assert abs(rr - r["relres_true"]) <= 1e-3 * rr


def test_single_chain_equals_solve_sequence(env):
    torch, skr = env
    systems = darcy_sequence(32, 5, first_seed=370)
    order = np.array([3, 0, 4, 1, 2])
    kw = dict(m=30, k=10, rtol=1e-8, maxit=20000, flags=0)
    _, res_b, xs_b, _ = _batched(torch, skr, systems, "csr", order, [0, 5], {}, **kw)
    res_a, xs_a = _alone(torch, skr, systems, "csr", order, [0, 5], {}, **kw)
    _check_equal("one-chain", order, [0, 5], res_b, xs_b, res_a, xs_a)


def test_time_stepping_chains_continue(env):
    """C backward-Euler chains, one system per chain per call, b^{t+1} = x^t / dt, continued with
    SKR_FLAG_CONTINUE; each chain equals the same steps solved alone call by call."""
    torch, skr = env
    C, T = 3, 3
    chains = advdiff_chains(32, C, first_seed=380)
    ops, _, _ = upload_systems(chains, "cuda:0")
    kw = dict(m=20, k=6, rtol=1e-8, maxit=20000)

    def steps_batched():
        ctx = make_ctx(torch)
        prev = [torch.from_numpy(c.x0).cuda() for c in chains]
        out = []
        try:
            for t in range(T):
                bs = [p / c.dt for p, c in zip(prev, chains)]
                xs = [torch.zeros_like(b) for b in bs]
                flags = skr.SKR_FLAG_MIXED | (skr.SKR_FLAG_CONTINUE if t else 0)
                rc, res = skr.skr_solve_chains(ctx, list(range(C + 1)), ops, bs, xs, None, flags=flags, **kw)
                assert rc == skr.SKR_OK
                out.append((res, [x.cpu().numpy() for x in xs]))
                prev = xs
            # a continuation with another chain count is refused
            with pytest.raises(skr.SkrError) as e:
                skr.skr_solve_chains(ctx, [0, 1, 2], ops[:2], bs[:2], xs[:2], None,
                                     flags=skr.SKR_FLAG_MIXED | skr.SKR_FLAG_CONTINUE, **kw)
            assert e.value.code == skr.SKR_EINVAL
        finally:
            torch.cuda.synchronize()
            skr.skr_ctx_destroy(ctx)
        return out

    def steps_alone(c):
        ctx = make_ctx(torch)
        prev = torch.from_numpy(chains[c].x0).cuda()
        out = []
        try:
            for t in range(T):
                b = prev / chains[c].dt
                x = torch.zeros_like(b)
                flags = skr.SKR_FLAG_MIXED | (skr.SKR_FLAG_CONTINUE if t else 0)
                rc, res = skr.skr_solve_sequence(ctx, [ops[c]], [b], [x], None, flags=flags, **kw)
                out.append((res[0], x.cpu().numpy()))
                prev = x
        finally:
            torch.cuda.synchronize()
            skr.skr_ctx_destroy(ctx)
        return out

    log(f"[chains] {C} time-stepping advection-diffusion chains x {T} steps, continued call by call")
    bat = steps_batched()
    for c in range(C):
        alone = steps_alone(c)
        for t in range(T):
            rb, xb = bat[t][0][c], bat[t][1][c]
            ra, xa = alone[t]
            assert same_result(rb, ra), (c, t, rb, ra)
            assert np.array_equal(xb, xa), (c, t)
            assert rb["status"] == skr.SKR_CONVERGED
        log(f"  chain {c}: iterations per step {[bat[t][0][c]['iters'] for t in range(T)]}, k_start "
            f"{[bat[t][0][c]['k_start'] for t in range(T)]}")


def test_argument_errors(env):
    torch, skr = env
    systems = darcy_sequence(16, 3, first_seed=390)
    ops, bs, xs = upload_systems(systems, "cuda:0")
    ctx = make_ctx(torch)
    try:
        for starts in ([1, 3], [0, 2], [0, 2, 1, 3]):
            with pytest.raises(skr.SkrError) as e:
                skr.skr_solve_chains(ctx, starts, ops, bs, xs, None)
            assert e.value.code == skr.SKR_EINVAL, starts
        with pytest.raises(skr.SkrError) as e:        # nothing to continue on a fresh context
            skr.skr_solve_chains(ctx, [0, 3], ops, bs, xs, None, flags=skr.SKR_FLAG_CONTINUE)
        assert e.value.code == skr.SKR_EINVAL
    finally:
        skr.skr_ctx_destroy(ctx)
