"""Sorting Krylov Recycling on MI355X (gfx950): greedy-sorted sequences of sparse systems solved
with GCRO-DR and a recycled subspace, all compute in hand-written HIP kernels behind a C ABI
(``include/skr.h``, ``libskr.so``). ``skr`` is the thin ctypes binding.
"""
from . import skr  # noqa: F401
from .skr import (Operator, SkrError, csr_op, load_library, skr_ctx_create, skr_ctx_destroy, skr_profile_get,
                  skr_profile_reset, skr_solve_sequence, skr_sort, skr_spmv, skr_spmv_repeat, skr_version, stencil_op)

__all__ = ["Operator", "SkrError", "csr_op", "load_library", "skr_ctx_create", "skr_ctx_destroy",
           "skr_profile_get", "skr_profile_reset", "skr_solve_sequence", "skr_sort", "skr_spmv", "skr_spmv_repeat",
           "skr_version", "stencil_op"]
