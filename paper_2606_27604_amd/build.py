"""Build the gfx950 shared library librw.so in-tree with hipcc.

    python -m paper_2606_27604_amd.build

Compiles the HIP kernels and the host runtime for gfx950 only, with packed FP32
instructions disabled (they are not used by hand and the compiler is told not
to form them), and links them into paper_2606_27604_amd/librw.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librw.so")
MICRO_LIB = os.path.join(PKG, "librw_micro.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["rw_kernels.hip", "rw_lut.hip", "rw_hero.hip", "rw_dwivedi.hip", "rw_runtime.hip"]
MICRO_SOURCES = ["rw_micro.hip"]
HEADERS = ["rw_device.hpp", "rw_internal.hpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wshadow",
    "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # tally atomics come from one or two lanes at a time: plain atomics, not
    # the compiler's lane-serialising reduction loop around each of them
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return exe


def _link(sources, lib, verbose):
    objs = []
    for src in sources:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, cwd=BUILD_DIR, stderr=subprocess.PIPE if not verbose else None)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=BUILD_DIR)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile every source and link librw.so and the micro-benchmark library
    librw_micro.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    _link(SOURCES, LIB, verbose)
    _link(MICRO_SOURCES, MICRO_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
