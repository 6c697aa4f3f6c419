"""Build ``libkl.so`` (HIP, gfx950) and the instruction-rate calibration
library ``libkl_calib.so`` in the package directory.

The libraries are compiled in place so that they travel with the source tree:
    python -m paper_1709_08018_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkl.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "decode.hip", "cayley.hip", "surrogate.hip", "walk.hip", "abi.cpp")]
CALIB_LIB = os.path.join(PKG, "libkl_calib.so")
CALIB_SOURCES = [os.path.join(CSRC, "calib.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every floating-point step is written out; no contraction behind our back
    "-ffp-contract=off",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


OBJ_DIR = os.path.join(PKG, "_build")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c", "-o", obj, "-x", "hip", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def _link(lib: str, objs: list[str], verbose: bool) -> None:
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one hipcc per file), then link."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJ_DIR, exist_ok=True)
    sources = SOURCES + CALIB_SOURCES
    jobs = max(1, min(len(sources), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, verbose), sources))
    _link(LIB, objs[:len(SOURCES)], verbose)
    _link(CALIB_LIB, objs[len(SOURCES):], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
