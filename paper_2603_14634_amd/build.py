"""Builds libpbdr.so (the HIP gfx950 solver behind include/pbdr.h) in this package directory.

Usage: ``python -m paper_2603_14634_amd.build`` or ``build()`` from Python.
Compiles every source with hipcc for gfx950 only; packed FP32 instructions are
disabled (``-packed-fp32-ops``) and the host pass warns that it does not know
that feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpbdr.so")
SOURCES = ["pbdr_kernels.hip", "pbdr_pool_kernels.hip", "pbdr_state.hip", "pbdr_abi.cpp", "pbdr_pool.cpp",
           "pbdr_batch.cpp", "pbdr_static.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Contraction only within one source expression keeps the rounding of the same
# arithmetic identical wherever it is instantiated: the pool kernel in its
# several launch shapes, the solver iteration in its per-iteration, multi-scene
# and one-launch kernels.
EXTRA_FLAGS = {"pbdr_pool_kernels.hip": ["-ffp-contract=on"], "pbdr_kernels.hip": ["-ffp-contract=on"]}

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS + EXTRA_FLAGS.get(src, [])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
