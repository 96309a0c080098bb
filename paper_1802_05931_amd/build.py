"""Compile the HIP library ``libddqmc.so`` for gfx950 (in-tree, next to this file).

Flags: -O3, -ffp-contract=off (no fused multiply-add anywhere, so fp64 sampling
arithmetic rounds exactly as written), packed fp32 ops disabled, C++17.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddqmc.so")
SOURCES = [os.path.join(CSRC, "ddqmc.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "model.hpp", "sampling.hpp")] + [
    os.path.join(os.path.dirname(HERE), "include", "ddqmc.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(force=True, verbose=False):
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= t for s in SOURCES + HEADERS):
            return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
