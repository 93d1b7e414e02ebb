"""Build libpot3d.so (the gfx950 HIP solver library) in-tree with hipcc.

    python -m paper_1709_01126_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpot3d.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["kernels.hip", "api.hip", "server.hip", "noalloc.hip"]
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # identical rounding for the two recomputations of A p: contraction only
    # where the code asks for fma explicitly
    "-ffp-contract=off",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


LIB_CHECKED = os.path.join(PKG, "libpot3d_checked.so")


def _build_one(lib: str, extra, tag: str, verbose: bool) -> str:
    objs = []
    os.makedirs(os.path.join(PKG, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(PKG, "_build", src.replace(".hip", f"{tag}.o"))
        cmd = [HIPCC, *FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """The production library, and a checked twin in which every global index of
    the kernels is range-tested (used to try new kernels before the real one)."""
    _build_one(LIB_CHECKED, ["-DPOT3D_CHECKED"], "_checked", verbose)
    return _build_one(LIB, [], "", verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
