"""Builds libgccd.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3; -ffp-contract=off so the FP64 update rounds exactly as written
(the FP32 pair loop uses explicit fused multiply-adds); packed FP32 VALU
instructions disabled.

build_sanitized() builds libgccd_san.so, the same sources with the host code
instrumented by AddressSanitizer and UndefinedBehaviorSanitizer (device code
is compiled as usual).  It is loaded in place of libgccd.so by setting
GCCD_LIB, with the ASan runtime preloaded (asan_runtime()).
"""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgccd.so")
SAN_LIB = os.path.join(HERE, "libgccd_san.so")
SOURCES = [os.path.join(HERE, "csrc", "gccd_api.hip"),
           os.path.join(HERE, "csrc", "gccd_sort.hip"),
           os.path.join(HERE, "csrc", "gccd_closure.hip"),
           os.path.join(HERE, "csrc", "gccd_kernels.hip")]
ARCH = os.environ.get("GCCD_OFFLOAD_ARCH", "gfx950")

COMMON = [
    f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
]
FLAGS = ["-O3"] + COMMON
# host code only: each sanitizer flag applies to the host compilation
SAN_FLAGS = ["-O1", "-g"] + COMMON + [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all",
    "-Xarch_host", "-fno-omit-frame-pointer",
]


def _build(flags, out, verbose, extra):
    tmp = out + ".tmp"
    cmd = ["hipcc"] + flags + list(extra or []) + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_library(verbose: bool = False, extra=None) -> str:
    return _build(FLAGS, LIB, verbose, extra)


def build_sanitized(verbose: bool = False) -> str:
    return _build(SAN_FLAGS, SAN_LIB, verbose, None)


def asan_runtime() -> str:
    """Path of the compiler's shared ASan runtime (to LD_PRELOAD into a
    process that loads libgccd_san.so)."""
    out = subprocess.run(["hipcc", "--print-resource-dir"], capture_output=True, text=True)
    dirs = [out.stdout.strip()] if out.returncode == 0 else []
    dirs += glob.glob("/opt/rocm*/lib/llvm/lib/clang/*")
    for d in dirs:
        p = os.path.join(d, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise FileNotFoundError("libclang_rt.asan-x86_64.so not found")


if __name__ == "__main__":
    import sys
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose=True))
    else:
        print(build_library(verbose=True))
