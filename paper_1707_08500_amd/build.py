"""Builds libpsatd.so (HIP, gfx950 only) in-tree next to this file.

    python -m paper_1707_08500_amd.build

The library is the whole product path; the Python binding only marshals
arguments into it.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpsatd.so")

SOURCES = ["psatd_api.hip", "psatd_kernels.hip"]
HEADERS = ["fft_engine.hpp", "psatd_device.hpp", "psatd_launch.hpp", "plan_host.hpp", "dft_consts.h",
           "mfma_dft.hpp", "reg_fft.hpp", "zreg.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # hand-written code only: keep the compiler from forming packed FP32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
]


def build(verbose: bool = True) -> str:
    """Compiles every HIP source into libpsatd.so; returns its path."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp] + \
        [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpsatd.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
