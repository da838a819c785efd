"""skr_sort_noalloc (the allocation-free variant of skr_sort for callers that cannot allocate)
against skr_sort through the C ABI: order and step squared distances identical bit for bit, on two
calls in a row, the second with fewer systems (the shared scratch keeps the first call's contents),
and the size limit reported as SKR_EINVAL."""
import numpy as np
import pytest

from gpu_common import log, make_ctx, need_gpu

pytestmark = pytest.mark.gpu


def _params(N, p, seed):
    rng = np.random.default_rng([2401, 77, seed])
    P = rng.standard_normal((N, p)) * np.exp(rng.standard_normal((1, p)))
    P[N // 3] = P[N // 5]            # an exact duplicate: its tie goes to the lower index
    return P


def test_noalloc_sort_equals_sort():
    torch = need_gpu()
    from paper_2401_09516_amd import skr
    ctx = make_ctx(torch)
    try:
        for N, p, start in ((512, 3000, 7), (300, 70000, 0), (40, 66564, 3)):
            log(f"[noalloc] sort N={N} p={p} start={start}")
            P = _params(N, p, N)
            Pd = torch.from_numpy(P).to("cuda:0")
            o_ref, d_ref = skr.skr_sort(ctx, Pd, N, p, start)
            o_na, d_na = skr.skr_sort_noalloc(ctx, Pd, N, p, start)
            assert o_na[0] == start and sorted(o_na.tolist()) == list(range(N))
            assert np.array_equal(o_na, o_ref)
            assert np.array_equal(d_na.view(np.uint64), d_ref.view(np.uint64))
        Pd = torch.zeros((513, 4), dtype=torch.float64, device="cuda:0")
        with pytest.raises(skr.SkrError) as ei:
            skr.skr_sort_noalloc(ctx, Pd, 513, 4, 0)
        assert ei.value.code == skr.SKR_EINVAL
    finally:
        skr.skr_ctx_destroy(ctx)
