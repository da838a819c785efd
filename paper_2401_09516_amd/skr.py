"""ctypes binding of libskr (include/skr.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libskr.so``; this module converts Python objects
into the C structures and pointers of the ABI. Device buffers are passed as objects with a
``data_ptr()`` method (PyTorch tensors on a ROCm device) or as raw integer addresses. Loading
fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libskr.so")

SKR_OK = 0
SKR_EINVAL = -1
SKR_ENOMEM = -2
SKR_EHIP = -3
SKR_ENONFINITE = -4
SKR_WARN_NOTCONVERGED = 1
SKR_PENDING = 2

SKR_CONVERGED = 0
SKR_MAXIT = 1
SKR_BREAKDOWN = 2
SKR_NONFINITE = 3

SKR_OP_CSR = 0
SKR_OP_STENCIL5 = 1
SKR_OP_STENCIL7 = 2

SKR_FLAG_PROFILE = 1
SKR_FLAG_FOLD = 2
SKR_FLAG_MIXED = 4
SKR_FLAG_CONTINUE = 8

EXPORTED = ("skr_ctx_create", "skr_ctx_destroy", "skr_last_error", "skr_version", "skr_sort", "skr_sort_noalloc",
            "skr_solve_sequence", "skr_solve_chains", "skr_spmv", "skr_spmv_repeat", "skr_profile_get", "skr_profile_reset",
            "skr_serve_start", "skr_submit", "skr_poll", "skr_wait", "skr_ticket_chain", "skr_serve_stats_get",
            "skr_serve_stop", "skr_recycle_get", "skr_recycle_set", "skr_workspace_bytes")


class SkrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libskr error {code}: {msg}")
        self.code = code


class skr_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("inv_h2", ctypes.c_double),
                ("ax", ctypes.c_void_p), ("ay", ctypes.c_void_p), ("nz", ctypes.c_int32),
                ("az", ctypes.c_void_p)]


class skr_opts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("k", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class skr_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32), ("k_start", ctypes.c_int32),
                ("rank_dropped", ctypes.c_int32), ("iters", ctypes.c_int64), ("spmv", ctypes.c_int64),
                ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double), ("seconds", ctypes.c_double)]


class skr_kernel_stat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class skr_profile(ctypes.Structure):
    _fields_ = [("step_a", skr_kernel_stat), ("step_b", skr_kernel_stat), ("step_c", skr_kernel_stat),
                ("steps", ctypes.c_int64), ("cycles", ctypes.c_int64), ("step_bytes", ctypes.c_double),
                ("eig_symmetric", ctypes.c_int64), ("eig_general", ctypes.c_int64)]


class skr_serve_opts(ctypes.Structure):
    _fields_ = [("max_chains", ctypes.c_int32), ("workers", ctypes.c_int32), ("arena_bytes", ctypes.c_uint64),
                ("split_d2_rel", ctypes.c_double), ("max_chain_systems", ctypes.c_int32), ("pad0", ctypes.c_int32)]


class skr_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("chains_live", ctypes.c_int32),
                ("chains_created", ctypes.c_int32), ("chains_retired", ctypes.c_int32),
                ("deferred", ctypes.c_int32), ("bytes_in_use", ctypes.c_uint64)]


_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libskr.so and declare the prototypes of include/skr.h."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.skr_ctx_create.argtypes = [i32, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.skr_ctx_create.restype = i32
    lib.skr_ctx_destroy.argtypes = [vp]
    lib.skr_ctx_destroy.restype = i32
    lib.skr_last_error.argtypes = []
    lib.skr_last_error.restype = ctypes.c_char_p
    lib.skr_version.argtypes = []
    lib.skr_version.restype = ctypes.c_char_p
    lib.skr_sort.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(dbl)]
    lib.skr_sort.restype = i32
    lib.skr_sort_noalloc.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(dbl)]
    lib.skr_sort_noalloc.restype = i32
    lib.skr_solve_sequence.argtypes = [vp, ctypes.POINTER(skr_op), ctypes.POINTER(vp), ctypes.POINTER(vp), i64,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(skr_opts),
                                       ctypes.POINTER(skr_result)]
    lib.skr_solve_sequence.restype = i32
    lib.skr_solve_chains.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(skr_op),
                                     ctypes.POINTER(vp), ctypes.POINTER(vp), i64, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(skr_opts), ctypes.POINTER(skr_result)]
    lib.skr_solve_chains.restype = i32
    lib.skr_spmv.argtypes = [vp, ctypes.POINTER(skr_op), vp, vp]
    lib.skr_spmv.restype = i32
    lib.skr_spmv_repeat.argtypes = [vp, ctypes.POINTER(skr_op), vp, vp, ctypes.c_int32, ctypes.POINTER(dbl)]
    lib.skr_spmv_repeat.restype = i32
    lib.skr_profile_get.argtypes = [vp, ctypes.POINTER(skr_profile)]
    lib.skr_profile_get.restype = i32
    lib.skr_profile_reset.argtypes = [vp]
    lib.skr_profile_reset.restype = i32
    lib.skr_serve_start.argtypes = [vp, ctypes.POINTER(skr_serve_opts)]
    lib.skr_serve_start.restype = i32
    lib.skr_submit.argtypes = [vp, ctypes.POINTER(skr_op), vp, i64, vp, vp, ctypes.POINTER(skr_opts),
                               ctypes.POINTER(ctypes.c_uint64)]
    lib.skr_submit.restype = i32
    lib.skr_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(skr_result)]
    lib.skr_poll.restype = i32
    lib.skr_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(skr_result)]
    lib.skr_wait.restype = i32
    lib.skr_ticket_chain.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.skr_ticket_chain.restype = i32
    lib.skr_serve_stats_get.argtypes = [vp, ctypes.POINTER(skr_serve_stats)]
    lib.skr_serve_stats_get.restype = i32
    lib.skr_serve_stop.argtypes = [vp]
    lib.skr_serve_stop.restype = i32
    lib.skr_workspace_bytes.argtypes = [i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]
    lib.skr_workspace_bytes.restype = ctypes.c_size_t
    lib.skr_recycle_get.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp, i64]
    lib.skr_recycle_get.restype = i32
    lib.skr_recycle_set.argtypes = [vp, ctypes.POINTER(skr_opts), i64, ctypes.c_int32, vp, i64]
    lib.skr_recycle_set.restype = i32
    if path is None:
        _lib = lib
    return lib


def _ptr(buf) -> int:
    if buf is None:
        return 0
    if isinstance(buf, int):
        return buf
    return int(buf.data_ptr())


def _check(rc: int) -> int:
    if rc < 0:
        raise SkrError(rc, load_library().skr_last_error().decode())
    return rc


# ----------------------------------------------------------------------------------- operators
@dataclass
class Operator:
    """An skr_op plus references that keep its device buffers alive."""
    c: skr_op
    keep: tuple


def csr_op(rowptr, colind, values, n: int) -> Operator:
    """CSR operator from device buffers (int32 rowptr[n+1], int32 colind[nnz], float64 values[nnz])."""
    nnz = int(values.numel()) if hasattr(values, "numel") else 0
    c = skr_op(kind=SKR_OP_CSR, n=n, nnz=nnz, rowptr=_ptr(rowptr), colind=_ptr(colind), values=_ptr(values))
    return Operator(c, (rowptr, colind, values))


def stencil_op(ax, ay, nx: int, ny: int, inv_h2: float) -> Operator:
    """Matrix-free 5-point operator from face coefficients ax[ny*(nx+1)], ay[(ny+1)*nx] (float64)."""
    c = skr_op(kind=SKR_OP_STENCIL5, n=nx * ny, nx=nx, ny=ny, inv_h2=inv_h2, ax=_ptr(ax), ay=_ptr(ay))
    return Operator(c, (ax, ay))


def stencil7_op(ax, ay, az, nx: int, ny: int, nz: int, inv_h2: float) -> Operator:
    """Matrix-free 3-D 7-point operator from face coefficients ax[nz*ny*(nx+1)], ay[nz*(ny+1)*nx],
    az[(nz+1)*ny*nx] (float64, layouts as in skr.h)."""
    c = skr_op(kind=SKR_OP_STENCIL7, n=nx * ny * nz, nx=nx, ny=ny, nz=nz, inv_h2=inv_h2, ax=_ptr(ax),
               ay=_ptr(ay), az=_ptr(az))
    return Operator(c, (ax, ay, az))


# ----------------------------------------------------------------------------------- entry points
def skr_version() -> str:
    return load_library().skr_version().decode()


def skr_ctx_create(device: int = 0, stream=None, arena=None, arena_bytes: int = 0) -> int:
    """Create a context on ``device`` enqueuing on ``stream`` (a hipStream_t address, or None). ``arena``:
    optional caller-owned device buffer (a tensor or an address) the context sub-allocates all its device
    memory from; ``arena_bytes`` defaults to the tensor's size in bytes. The caller keeps it alive."""
    out = ctypes.c_void_p()
    s = stream if isinstance(stream, int) or stream is None else int(stream)
    ap = None
    if arena is not None:
        ap = _ptr(arena)
        if not arena_bytes and hasattr(arena, "numel"):
            arena_bytes = arena.numel() * arena.element_size()
    _check(load_library().skr_ctx_create(device, s, ap, int(arena_bytes), ctypes.byref(out)))
    return out.value


def skr_ctx_destroy(ctx: int) -> None:
    _check(load_library().skr_ctx_destroy(ctx))


def _sort_call(fn, ctx, params, N, p, start, want_dist):
    order = np.zeros(max(N, 1), dtype=np.int64)
    dist = np.zeros(max(N, 1), dtype=np.float64) if want_dist else None
    dptr = dist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_dist else None
    _check(fn(ctx, _ptr(params), N, p, start, order.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), dptr))
    return order[:N], (dist[:N] if want_dist else None)


def skr_sort(ctx: int, params, N: int, p: int, start: int = 0, want_dist: bool = True):
    """Alg. 1 on device parameters (N x p float64, row-major). Returns (order int64, step d2 or None)."""
    return _sort_call(load_library().skr_sort, ctx, params, N, p, start, want_dist)


def skr_sort_noalloc(ctx: int, params, N: int, p: int, start: int = 0, want_dist: bool = True):
    """skr_sort without device allocations (N <= 512; library-owned static scratch per GPU)."""
    return _sort_call(load_library().skr_sort_noalloc, ctx, params, N, p, start, want_dist)


def skr_solve_sequence(ctx: int, ops, bs, xs, order=None, m: int = 30, k: int = 10, rtol: float = 1e-8,
                       maxit: int = 10000, flags: int = 0):
    """Solve the systems in ``order`` with GCRO-DR(m, k) (k = 0: GMRES(m)).

    ``ops``: list of Operator; ``bs``/``xs``: device buffers. Returns (return code, list of result dicts
    at the original indices).
    """
    N = len(ops)
    arr = (skr_op * max(N, 1))(*[o.c for o in ops])
    bp = (ctypes.c_void_p * max(N, 1))(*[_ptr(b) for b in bs])
    xp = (ctypes.c_void_p * max(N, 1))(*[_ptr(x) for x in xs])
    if order is not None:
        ordarr = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
        optr = ordarr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    else:
        optr = None
    opts = skr_opts(m=m, k=k, rtol=rtol, maxit=maxit, flags=flags)
    res = (skr_result * max(N, 1))()
    rc = _check(load_library().skr_solve_sequence(ctx, arr, bp, xp, N, optr, ctypes.byref(opts), res))
    return rc, [_result_dict(r) for r in list(res)[:N]]


def skr_solve_chains(ctx: int, chain_start, ops, bs, xs, order=None, m: int = 30, k: int = 10, rtol: float = 1e-8,
                     maxit: int = 10000, flags: int = 0):
    """Solve the sorted order cut into chains (chain c: positions chain_start[c] .. chain_start[c+1]-1 of
    ``order``), all chains advanced together, each as ``skr_solve_sequence`` would solve it alone.

    Returns (return code, list of result dicts at the original indices).
    """
    N = len(ops)
    cs = np.ascontiguousarray(np.asarray(chain_start, dtype=np.int64))
    C = len(cs) - 1
    arr = (skr_op * max(N, 1))(*[o.c for o in ops])
    bp = (ctypes.c_void_p * max(N, 1))(*[_ptr(b) for b in bs])
    xp = (ctypes.c_void_p * max(N, 1))(*[_ptr(x) for x in xs])
    if order is not None:
        ordarr = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
        optr = ordarr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    else:
        optr = None
    opts = skr_opts(m=m, k=k, rtol=rtol, maxit=maxit, flags=flags)
    res = (skr_result * max(N, 1))()
    rc = _check(load_library().skr_solve_chains(ctx, C, cs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), arr, bp,
                                                xp, N, optr, ctypes.byref(opts), res))
    return rc, [_result_dict(r) for r in list(res)[:N]]


def skr_workspace_bytes(n: int, m: int, k: int, flags: int = 0) -> int:
    """Device bytes a context allocates for solves of size n with GCRO-DR(m, k); 0 for invalid sizes."""
    return int(load_library().skr_workspace_bytes(n, m, k, flags))


def skr_recycle_get(ctx: int, U=None, ld: int = 0) -> int:
    """Number of recycled columns the context carries; with ``U`` (device float64, column j in row j of a
    (k, n) tensor, i.e. n x k column-major with leading dimension ``ld``, default the row stride) also
    copies them."""
    k = ctypes.c_int32()
    if U is not None and not ld:
        ld = U.stride(0) if U.dim() == 2 else U.numel()
    _check(load_library().skr_recycle_get(ctx, ctypes.byref(k), _ptr(U) if U is not None else None, ld))
    return k.value


def skr_recycle_set(ctx: int, U, n: int, kcols: int, m: int, k: int, ld: int = 0, rtol: float = 1e-8,
                    maxit: int = 10000, flags: int = 0) -> None:
    """Make ``U`` (device float64, n x kcols column-major, leading dimension ``ld``, default n) the
    recycle space the next skr_solve_sequence with SKR_FLAG_CONTINUE and the same m, k, flags starts from."""
    opts = skr_opts(m=m, k=k, rtol=rtol, maxit=maxit, flags=flags)
    _check(load_library().skr_recycle_set(ctx, ctypes.byref(opts), n, kcols,
                                          _ptr(U) if U is not None else None, ld or n))


def _result_dict(r: skr_result) -> dict:
    return dict(status=r.status, cycles=r.cycles, k_start=r.k_start, rank_dropped=r.rank_dropped,
                iters=r.iters, spmv=r.spmv, relres_true=r.relres_true, relres_est=r.relres_est, seconds=r.seconds)


def skr_spmv(ctx: int, op: Operator, x, y) -> None:
    """y = A x on the device."""
    _check(load_library().skr_spmv(ctx, ctypes.byref(op.c), _ptr(x), _ptr(y)))


def skr_spmv_repeat(ctx: int, op: Operator, x, y, repeats: int) -> float:
    """Mean device time (ms) of one SpMV launch over ``repeats`` back-to-back launches."""
    ms = ctypes.c_double()
    _check(load_library().skr_spmv_repeat(ctx, ctypes.byref(op.c), _ptr(x), _ptr(y), repeats, ctypes.byref(ms)))
    return ms.value


def skr_profile_get(ctx: int) -> dict:
    """Kernel statistics of solves run with SKR_FLAG_PROFILE since the last reset, and the cycle ends
    of every solve by the eigen stage that formed their recycle space."""
    p = skr_profile()
    _check(load_library().skr_profile_get(ctx, ctypes.byref(p)))
    ks = {name: dict(launches=getattr(p, name).launches, ms=getattr(p, name).ms, bytes=getattr(p, name).bytes)
          for name in ("step_a", "step_b", "step_c")}
    return dict(kernels=ks, steps=p.steps, cycles=p.cycles, step_bytes=p.step_bytes,
                eig_symmetric=p.eig_symmetric, eig_general=p.eig_general)


def skr_profile_reset(ctx: int) -> None:
    _check(load_library().skr_profile_reset(ctx))


# ----------------------------------------------------------------------------------- serving
def skr_serve_start(ctx: int, max_chains: int = 8, workers: int = 4, arena_bytes: int = 0,
                    split_d2_rel: float = float("inf"), max_chain_systems: int = 0) -> None:
    """Start the serving runtime on ``ctx`` (skr.h: nearest-chain admission, one stream per chain)."""
    o = skr_serve_opts(max_chains=max_chains, workers=workers, arena_bytes=arena_bytes, split_d2_rel=split_d2_rel,
                       max_chain_systems=max_chain_systems)
    _check(load_library().skr_serve_start(ctx, ctypes.byref(o)))


def skr_submit(ctx: int, op: Operator, params, p: int, b, x, m: int = 30, k: int = 10, rtol: float = 1e-8,
               maxit: int = 10000, flags: int = 0) -> int:
    """Submit one system; returns its ticket. ``op``, ``b`` and ``x`` must stay alive until it is done."""
    t = ctypes.c_uint64()
    opts = skr_opts(m=m, k=k, rtol=rtol, maxit=maxit, flags=flags)
    _check(load_library().skr_submit(ctx, ctypes.byref(op.c), _ptr(params), p, _ptr(b), _ptr(x),
                                     ctypes.byref(opts), ctypes.byref(t)))
    return t.value


def skr_poll(ctx: int, ticket: int):
    """The result dict when the ticket is done (it is then collected), None while pending."""
    r = skr_result()
    rc = _check(load_library().skr_poll(ctx, ticket, ctypes.byref(r)))
    return None if rc == SKR_PENDING else _result_dict(r)


def skr_wait(ctx: int, ticket: int) -> dict:
    """Block until the ticket is done; returns (and collects) its result dict."""
    r = skr_result()
    _check(load_library().skr_wait(ctx, ticket, ctypes.byref(r)))
    return _result_dict(r)


def skr_ticket_chain(ctx: int, ticket: int):
    """(chain id, position in the chain) of a ticket not yet collected; (-1, -1) while deferred."""
    c, pos = ctypes.c_int32(), ctypes.c_int64()
    _check(load_library().skr_ticket_chain(ctx, ticket, ctypes.byref(c), ctypes.byref(pos)))
    return c.value, pos.value


def skr_serve_stats_get(ctx: int) -> dict:
    st = skr_serve_stats()
    _check(load_library().skr_serve_stats_get(ctx, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in skr_serve_stats._fields_}


def skr_serve_stop(ctx: int) -> None:
    _check(load_library().skr_serve_stop(ctx))
