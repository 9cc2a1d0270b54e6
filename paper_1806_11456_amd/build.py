"""Build the gfx950 HIP library (libpmg.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpmg.so")
SRC = os.path.join(HERE, "csrc", "pmg.hip")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# The same library with the host code under AddressSanitizer (device code unchanged), for the CPU checks of
# its host-side logic (order selection, functionals' host parts, argument checking); it is never loaded by the
# GPU tests or the benchmark.
ASAN_LIB = os.path.join(HERE, "libpmg_asan_host.so")
ASAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_asan_host(verbose: bool = False) -> str:
    tmp = ASAN_LIB + ".tmp"
    flags = [f for f in FLAGS if f != "-O3"] + ASAN_FLAGS
    cmd = [HIPCC, *flags, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
