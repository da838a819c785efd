"""Build libskr.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["skr_solver.hip", "skr_dense.hip", "skr_sort.hip", "skr_api.hip", "skr_serve.hip", "skr_state.hip"]
OUTPUT = os.path.join(HERE, "libskr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # packed FP32 instructions off (see the build notes of this project)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libskr.so; returns the library path. Raises on failure."""
    src = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = OUTPUT + ".tmp"
    cmd = [HIPCC, *FLAGS, *src, "-o", tmp]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (proc.stdout + proc.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, OUTPUT)
    return OUTPUT


if __name__ == "__main__":
    print(build(verbose=True))
