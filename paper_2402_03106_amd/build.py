"""Build libdarts.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "darts.hip")
LIB = os.path.join(PKG, "libdarts.so")
ARCH = os.environ.get("DARTS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # contract a * b + c into an fma only within one source expression, so a
    # path's arithmetic is the same in every kernel that inlines it (the
    # render, batch and adjoint kernels give the same per-path values)
    "-ffp-contract=on",
    # keep hand-written and compiler-made code off the packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the machine scheduler's maximum-ILP strategy: the path loops are bound
    # by VALU issue at their register budget, and this order issues them
    # about 1% faster (same registers, no scratch in the image kernels)
    "-mllvm", "-amdgpu-sched-strategy=max-ilp",
]


def build_library(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), SRC, "-o", tmp]
    res = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
