"""Helpers shared by the GPU tests (device set-up, uploads, comparisons with the oracle)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def need_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_09516_amd import skr
    skr.load_library()        # fails loudly when the library is missing
    return torch


def make_ctx(torch):
    from paper_2401_09516_amd import skr
    return skr.skr_ctx_create(0, torch.cuda.current_stream().cuda_stream)


def solution_bound(A, b, x_ref, rr_a, rr_b):
    """Bound on ||x_a - x_b|| / ||x_b|| for two iterates with relative residuals rr_a, rr_b.

    ||x_a - x_b|| <= ||A^-1|| (||r_a|| + ||r_b||), so the relative difference is at most
    mu (rr_a + rr_b) with mu = ||A^-1||_2 ||b|| / ||x||; the parity target 1e-7 is used unless that
    bound is larger.
    """
    import scipy.sparse.linalg as spla
    lam = spla.eigsh(A, k=1, sigma=0, return_eigenvectors=False)[0]
    mu = np.linalg.norm(b) / abs(lam) / np.linalg.norm(x_ref)
    return max(1e-7, 1.01 * mu * (rr_a + rr_b)), mu
