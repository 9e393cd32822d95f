"""Build libmdwf.so (HIP, gfx950) in-tree with hipcc.

Each translation unit is compiled to its own object in parallel (no device
code crosses translation units), then hipcc links the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmdwf.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "dslash.hip", "dslash_plane.hip", "blas.hip", "solver.hip", "serve.hip", "flow.hip", "source.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
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
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]

    def compile_one(src):
        obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + HIPCC_FLAGS + inc + ["-c", os.path.join(SRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return src, obj, r.returncode, r.stdout

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [r for r in results if r[2] != 0]
    for src, _, rc, out in results:
        # hipcc's host pass does not know the device-only target features
        lines = [l for l in out.splitlines() if "is not a recognized feature for this target" not in l]
        if lines and (verbose or rc != 0):
            print("\n".join(lines), file=sys.stderr)
    if failed:
        raise subprocess.CalledProcessError(failed[0][2], "hipcc -c " + failed[0][0])
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + [r[1] for r in results] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
