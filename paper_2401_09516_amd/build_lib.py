"""Build libskr.so for gfx950 with hipcc (in-tree, next to this file).

Each source is compiled to its own object in parallel (no cross-unit device code: every kernel is
launched from the unit that defines it), then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
# (source, object, extra flags): skr_solver.hip is compiled twice, its single-chain kernels and its
# batched (one grid row per chain) kernels, which share the device bodies
UNITS = [("skr_solver.hip", "skr_solver.o", []),
         ("skr_solver.hip", "skr_solver_chains.o", ["-DSKR_CHAINS_UNIT"]),
         ("skr_dense.hip", "skr_dense.o", []),
         ("skr_sort.hip", "skr_sort.o", []),
         ("skr_api.hip", "skr_api.o", []),
         ("skr_serve.hip", "skr_serve.o", []),
         ("skr_state.hip", "skr_state.o", []),
         ("skr_batch.hip", "skr_batch.o", [])]
SOURCES = sorted({u[0] for u in UNITS})
OUTPUT = os.path.join(HERE, "libskr.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # packed FP32 instructions off (see the build notes of this project)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (proc.stdout + proc.stderr).splitlines() if "packed-fp32-ops" not in ln]
    return proc.returncode, msgs


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libskr.so; returns the library path. Raises on failure."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for src, o, extra in UNITS:
        obj = os.path.join(OBJDIR, o)
        jobs.append((obj, [HIPCC, *FLAGS, *extra, "-c", os.path.join(HERE, "csrc", src), "-o", obj]))
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    msgs = []
    for (obj, cmd), (rc, out) in zip(jobs, results):
        msgs += out
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(cmd[-3])}:\n" + "\n".join(out))
    tmp = OUTPUT + ".tmp"
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[j[0] for j in jobs], "-o", tmp])
    msgs += out
    if rc != 0:
        raise RuntimeError("link failed:\n" + "\n".join(out))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, OUTPUT)
    return OUTPUT


if __name__ == "__main__":
    print(build(verbose=True))
