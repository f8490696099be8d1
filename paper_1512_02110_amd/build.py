"""Builds libmcrt.so (the HIP kernels and the C ABI) for gfx950 in-tree.

    python -m paper_1512_02110_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmcrt.so")
SOURCES = ["mcrt_api.hip", "mcrt_kernels.hip", "mcrt_voxel.hip"]
MICRO_LIB = os.path.join(PKG, "libmcrt_micro.so")
MICRO_SOURCES = ["mcrt_micro.hip"]
ARCH = os.environ.get("MCRT_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware floating-point atomics on coarse-grained device memory
    "-munsafe-fp-atomics",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _link(sources, lib, verbose):
    objs = []
    odir = os.path.join(PKG, "_build")
    os.makedirs(odir, exist_ok=True)
    for src in sources:
        obj = os.path.join(odir, src.replace(".hip", ".o"))
        cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + HIP_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Builds libmcrt.so and the micro-benchmark library libmcrt_micro.so."""
    _link(SOURCES, LIB, verbose)
    _link(MICRO_SOURCES, MICRO_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
