"""The C ABI library loads and exports every function declared in include/*.h, and the ctypes
structures of the binding match the C layouts (checked with a gcc-compiled probe). No GPU needed."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

from paper_2401_09516_amd import skr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(skr_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_declared_symbols():
    if not os.path.exists(skr.LIB_PATH):
        pytest.fail("libskr.so is not built (run __graft_entry__.build())")
    lib = skr.load_library()
    names = declared_functions()
    assert set(skr.EXPORTED) <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.skr_version().decode().startswith("skr-gfx950")
    assert lib.skr_last_error() is not None


def test_struct_layouts_match_header(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "skr.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("skr_op %zu\nskr_opts %zu\nskr_result %zu\n", sizeof(skr_op), sizeof(skr_opts), sizeof(skr_result));
  F(skr_op, kind); F(skr_op, n); F(skr_op, nnz); F(skr_op, rowptr); F(skr_op, colind); F(skr_op, values);
  F(skr_op, nx); F(skr_op, ny); F(skr_op, inv_h2); F(skr_op, ax); F(skr_op, ay); F(skr_op, nz); F(skr_op, az);
  F(skr_opts, m); F(skr_opts, k); F(skr_opts, rtol); F(skr_opts, maxit); F(skr_opts, flags);
  F(skr_result, status); F(skr_result, cycles); F(skr_result, k_start); F(skr_result, rank_dropped);
  F(skr_result, iters); F(skr_result, spmv); F(skr_result, relres_true); F(skr_result, relres_est);
  F(skr_result, seconds);
  printf("skr_kernel_stat %zu\nskr_profile %zu\n", sizeof(skr_kernel_stat), sizeof(skr_profile));
  F(skr_kernel_stat, launches); F(skr_kernel_stat, ms); F(skr_kernel_stat, bytes);
  F(skr_profile, step_a); F(skr_profile, step_b); F(skr_profile, step_c); F(skr_profile, steps);
  F(skr_profile, cycles); F(skr_profile, step_bytes); F(skr_profile, eig_symmetric); F(skr_profile, eig_general);
  printf("skr_serve_opts %zu\nskr_serve_stats %zu\n", sizeof(skr_serve_opts), sizeof(skr_serve_stats));
  F(skr_serve_opts, max_chains); F(skr_serve_opts, workers); F(skr_serve_opts, arena_bytes);
  F(skr_serve_opts, split_d2_rel); F(skr_serve_opts, max_chain_systems); F(skr_serve_opts, pad0);
  F(skr_serve_stats, submitted); F(skr_serve_stats, completed); F(skr_serve_stats, chains_live);
  F(skr_serve_stats, chains_created); F(skr_serve_stats, chains_retired); F(skr_serve_stats, deferred);
  F(skr_serve_stats, bytes_in_use);
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)], check=True)
    out = dict(ln.rsplit(" ", 1) for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    for cname, ct in (("skr_op", skr.skr_op), ("skr_opts", skr.skr_opts), ("skr_result", skr.skr_result),
                      ("skr_kernel_stat", skr.skr_kernel_stat), ("skr_profile", skr.skr_profile),
                      ("skr_serve_opts", skr.skr_serve_opts), ("skr_serve_stats", skr.skr_serve_stats)):
        assert int(out[cname]) == ctypes.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(ct, f).offset, (cname, f)


def test_binding_rejects_missing_library(tmp_path):
    with pytest.raises(ImportError):
        skr.load_library(str(tmp_path / "nope.so"))


def test_workspace_bytes_query():
    """skr_workspace_bytes is host arithmetic (no device): positive for valid sizes, at least the
    basis [C V] and U in FP64, growing with n and m, 0 for sizes a solve rejects."""
    n, m, k = 65536, 60, 20
    b = skr.skr_workspace_bytes(n, m, k)
    assert b >= (k + m + 1 + k) * n * 8
    assert skr.skr_workspace_bytes(2 * n, m, k) > b and skr.skr_workspace_bytes(n, 80, k) > b
    assert skr.skr_workspace_bytes(n, m, k, skr.SKR_FLAG_MIXED) == b
    for args in ((0, m, k), (n, 87, 20), (n, 20, 20), (n, 60, 33), (n, 60, -1), (2 ** 31, m, k)):
        assert skr.skr_workspace_bytes(*args) == 0, args
