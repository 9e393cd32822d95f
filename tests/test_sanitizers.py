"""AddressSanitizer and UBSan on the host code (no GPU needed).

* The FP64 oracle, built with gcc -fsanitize=address,undefined, runs every
  entry point on small lattices (tests/sanitize/oracle_run.c).
* The library's host code (the C ABI, solver driver and server), built
  host-only with the sanitizers, runs every entry point's argument and state
  errors and, without a device, the HIP error path of context and server
  creation (tests/sanitize/abi_errors.cpp).  No kernel is launched.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1701_07559_amd", "csrc")
SOURCES = ["api.hip", "dslash.hip", "blas.hip", "solver.hip", "serve.hip", "flow.hip", "source.hip"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_run")
    _run([gcc, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "mdwf_oracle.c"),
          os.path.join(HERE, "sanitize", "oracle_run.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "oracle sanitizer run: ok" in r.stdout


def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    # host code sanitized (-Xarch_host); the device code is built as usual,
    # one source per process
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Xclang", "-target-feature", "-Xclang", "-dot5-insts", "-Wno-unused-result", "-Xarch_host", "-O1", "-Xarch_host", "-g"] + san
    objs, procs = [], []
    for src in SOURCES:
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, "-c"] + flags + ["-I", os.path.join(ROOT, "include"),
                                      os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for pr in procs:
        out, _ = pr.communicate(timeout=900)
        assert pr.returncode == 0, out[-3000:]
    lib = str(tmp_path / "libmdwf_san.so")
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950"] + san + objs + ["-o", lib])
    # the driver is plain host C++: ROCm's clang++, the compiler whose
    # sanitizer runtime the library was built against
    clangxx = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/lib/llvm/bin/clang++"
    exe = str(tmp_path / "abi_errors")
    _run([clangxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
          os.path.join(HERE, "sanitize", "abi_errors.cpp"), lib, "-Wl,-rpath," + str(tmp_path), "-o", exe])
    r = _run([exe], env=ENV)
    assert "abi sanitizer run: ok" in r.stdout
