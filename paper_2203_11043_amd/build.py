"""Builds libgccd.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3; -ffp-contract=off so the FP64 update rounds exactly as written
(the FP32 pair loop uses explicit fused multiply-adds); packed FP32 VALU
instructions disabled.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgccd.so")
SOURCES = [os.path.join(HERE, "csrc", "gccd_api.hip"),
           os.path.join(HERE, "csrc", "gccd_sort.hip"),
           os.path.join(HERE, "csrc", "gccd_closure.hip"),
           os.path.join(HERE, "csrc", "gccd_kernels.hip")]
ARCH = os.environ.get("GCCD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
]


def build_library(verbose: bool = False, extra=None) -> str:
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + list(extra or []) + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
