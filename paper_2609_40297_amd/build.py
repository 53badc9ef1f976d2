"""Builds the HIP library ``libmg.so`` for gfx950 in this package directory.

hipcc cross-compiles on a machine without a GPU. Flags: -ffp-contract=off and
no fast-math (every decision is taken in IEEE binary32 in the order written),
packed FP32 instructions disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmg.so")
SOURCES = ["mg_api.hip", "mg_kernels.hip", "mg_batch.hip", "mg_serve.hip", "mg_interval.hip", "mg_map.hip", "mg_exact.hip",
           "mg_noalloc.hip"]
ARCH = os.environ.get("MG_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
