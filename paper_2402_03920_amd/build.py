"""Build the HIP library libqsg.so for gfx950, in-tree.

hipcc compiles the kernels and the C ABI; g++ compiles the binary128 table
builder (GNU quadmath).  Packed FP32 instructions are disabled for all device
code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libqsg.so")
ARCH = os.environ.get("QSG_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in ("qsg_kernels.hip", "qsg_overlaps.hip", "qsg_transfer.hip", "qsg_corr_mix.hip",
                "qsg_mlp.hip", "qsg_api.cpp", "qsg_transfer_api.cpp"):
        obj = os.path.join(BUILD, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run(["hipcc", *HIP_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tobj = os.path.join(BUILD, "qsg_tables.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c",
          os.path.join(CSRC, "qsg_tables.cpp"), "-o", tobj], verbose)
    objs.append(tobj)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
          "-lquadmath"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
