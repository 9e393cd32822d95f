"""Build libmdwf.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmdwf.so")
SOURCES = ["api.hip", "dslash.hip", "blas.hip", "solver.hip", "serve.hip", "flow.hip", "source.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # keep hipcc from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP16 dot products in the three-operand v_dot2_f32_f16 only: without the
    # accumulating v_dot2c form the compiler starts each product chain with an
    # inline zero instead of clearing a register (one VALU instruction less
    # per chain, 96 per FP16 hop kernel), and still sees every instruction
    "-Xclang", "-target-feature", "-Xclang", "-dot5-insts",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(HERE, "..", "include")] + \
        [os.path.join(SRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
