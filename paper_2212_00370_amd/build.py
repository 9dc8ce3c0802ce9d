"""Build the gfx950 HIP library ``librrmhd.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "rrmhd_api.hip")
LIB = os.path.join(PKG, "librrmhd.so")
ARCH = os.environ.get("RRMHD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17",
    # Evaluation order is part of the numerics (see rrmhd_device.hpp): no
    # contraction into FMA, no fast-math.
    "-ffp-contract=off", "-fno-fast-math",
    # FP32 division and sqrt (mixed-precision flux arithmetic only) use the
    # hardware reciprocal / square-root instructions; binary64 operations are
    # unaffected and stay IEEE correctly rounded.
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    # No packed FP32 instructions in any kernel.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fPIC", "-shared",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
