"""Build libksvd2.so (HIP, gfx950) in-tree with hipcc.

Floating-point flags matter for the method's bit-exactness: no contraction
(every fused multiply-add is an explicit fma), correctly rounded binary32
division and square root, binary32 denormals kept (gradual underflow), no
fast-math, and no packed-FP32 instruction selection.  Matrix-core instructions
take their accumulators in ordinary vector registers (the compiler otherwise
copies them between the accumulator and vector register files on every trip
of the sigma-gradient's loop); only the kernels that use them change.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libksvd2.so")
SOURCES = ["ksvd2_kernels.hip", "kog_sweep.hip", "ksvd2c.hip", "kog_rect.hip"]
ARCH = os.environ.get("KSVD2_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
