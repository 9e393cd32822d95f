"""FP64 CPU oracle for the Moebius domain-wall solve -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  The product library never does, and
this package imports nothing from it.

The arithmetic lives in ``mdwf_oracle.c`` (plain C99, ``double complex``,
full-lattice loops with parity masks); this module only loads the shared
library built from it and marshals numpy arrays.  Field layouts are the host
canonical ones of ``paper_1701_07559_amd.inputs``:

* links ``U[t, z, y, x, mu, a, b]`` complex128
* 4D spinors ``[t, z, y, x, spin, colour]``, 5D spinors ``[s, t, z, y, x, spin, colour]``

Parity pins for each routine live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdwf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with OpenMP over lattice sites, used only to time the
# oracle on all host cores.  Only site loops without reductions run in
# parallel, so it returns the same values as the single-threaded build.
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared"] + extra + ["-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single thread, no vector intrinsics),
    and its OpenMP timing build."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, [])
    if force or not os.path.exists(_LIB_OMP):
        _compile(_LIB_OMP, ["-fopenmp"])
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("X", C.c_int), ("Y", C.c_int), ("Z", C.c_int), ("T", C.c_int), ("L5", C.c_int),
        ("antiperiodic_t", C.c_int),
        ("M5", C.c_double), ("b5", C.c_double), ("c5", C.c_double), ("mq", C.c_double),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("restarts", C.c_int),
        ("true_resid", C.c_double), ("schur_resid", C.c_double),
    ]


_libs = {}
_variant = "serial"


def use_threads(n: int) -> int:
    """Route every call of this module to the OpenMP timing build with n
    threads (n >= 2), or back to the single-threaded oracle (n <= 1).
    Returns the thread count now in use."""
    global _variant
    if n <= 1:
        _variant = "serial"
        return 1
    _variant = "omp"
    return int(_load().oracle_set_threads(int(n)))


def _load():
    lib = _libs.get(_variant)
    if lib is None:
        path = _LIB_OMP if _variant == "omp" else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(path)
        P = C.POINTER(Params)
        d = C.c_void_p
        for name, args, res in [
            ("oracle_gamma", [C.c_int, d], None),
            ("oracle_dslash4", [P, d, d, d, C.c_int], None),
            ("oracle_dw4", [P, d, d, d, C.c_int], None),
            ("oracle_C", [P, d, d, C.c_int], None),
            ("oracle_B", [P, d, d, C.c_int], None),
            ("oracle_K5", [P, d, d, C.c_int], None),
            ("oracle_K5inv", [P, d, d, C.c_int], None),
            ("oracle_hop", [P, d, d, d, C.c_int, C.c_int], None),
            ("oracle_D5", [P, d, d, d, C.c_int], None),
            ("oracle_schur", [P, d, d, d, C.c_int], None),
            ("oracle_schur_sym", [P, d, d, d, C.c_int], None),
            ("oracle_schur_rp", [P, d, d, d, C.c_int], None),
            ("oracle_Binv", [P, d, d, C.c_int], None),
            ("oracle_prep_source", [P, d, d, d], None),
            ("oracle_reconstruct", [P, d, d, d], None),
            ("oracle_true_residual", [P, d, d, d], C.c_double),
            ("oracle_solve", [P, d, d, d, C.c_double, C.c_int, C.POINTER(SolveInfo)], C.c_int),
            ("oracle_cgls_step", [P, d, d, d, d, d, d, C.POINTER(C.c_double)], C.c_double),
            ("oracle_D5_sites", [P, d, d, d, C.c_int, d], None),
            ("oracle_schur_sites", [P, d, d, d, C.c_int, C.c_int, d], None),
            ("oracle_schur_rp_sites", [P, d, d, d, C.c_int, C.c_int, d], None),
            ("oracle_set_threads", [C.c_int], C.c_int),
        ]:
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _libs[_variant] = lib
    return lib


class Action:
    """Lattice geometry plus the action parameters (M5, b5, c5, L5, m_q)."""

    def __init__(self, dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05, antiperiodic_t=True):
        self.dims = tuple(int(d) for d in dims)
        self.L5 = int(L5)
        self.M5, self.b5, self.c5, self.mq = float(M5), float(b5), float(c5), float(mq)
        self.antiperiodic_t = bool(antiperiodic_t)

    def params(self) -> Params:
        X, Y, Z, T = self.dims
        return Params(X, Y, Z, T, self.L5, int(self.antiperiodic_t),
                      self.M5, self.b5, self.c5, self.mq)

    def with_mass(self, mq):
        return Action(self.dims, self.L5, self.M5, self.b5, self.c5, mq, self.antiperiodic_t)

    @property
    def shape5(self):
        X, Y, Z, T = self.dims
        return (self.L5, T, Z, Y, X, 4, 3)

    @property
    def shape4(self):
        X, Y, Z, T = self.dims
        return (T, Z, Y, X, 4, 3)


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data


def gamma(mu: int) -> np.ndarray:
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().oracle_gamma(mu, out.ctypes.data)
    return out


def dslash4(act: Action, U, psi4, dag=False):
    U, pu = _c(U)
    psi4, pi = _c(psi4)
    out = np.empty_like(psi4)
    _load().oracle_dslash4(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag))
    return out


def dw4(act: Action, U, psi4, dag=False):
    U, pu = _c(U)
    psi4, pi = _c(psi4)
    out = np.empty_like(psi4)
    _load().oracle_dw4(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag))
    return out


def _site5(name):
    def f(act: Action, psi, dag=False):
        psi, pi = _c(psi)
        out = np.empty_like(psi)
        getattr(_load(), name)(C.byref(act.params()), pi, out.ctypes.data, int(dag))
        return out
    f.__name__ = name
    return f


apply_C = _site5("oracle_C")
apply_B = _site5("oracle_B")
apply_K5 = _site5("oracle_K5")
apply_K5inv = _site5("oracle_K5inv")
apply_Binv = _site5("oracle_Binv")


def hop(act: Action, U, psi, out_parity: int, dag=False):
    """Bare Dslash between 4D parities on every slice (no -1/2 factor)."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    out = np.empty_like(psi)
    _load().oracle_hop(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag), int(out_parity))
    return out


def D5(act: Action, U, psi, dag=False):
    U, pu = _c(U)
    psi, pi = _c(psi)
    out = np.empty_like(psi)
    _load().oracle_D5(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag))
    return out


def schur(act: Action, U, psi, dag=False):
    """Asymmetric Schur complement on the even sites of a full-size field."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    out = np.empty_like(psi)
    _load().oracle_schur(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag))
    return out


def schur_sym(act: Action, U, psi, dag=False):
    """Symmetric even-odd operator K5^-1 S (or S^+ K5^-+) on the even sites."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    out = np.empty_like(psi)
    _load().oracle_schur_sym(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag))
    return out


def schur_rp(act: Action, U, psi, dag=False):
    """S B^-1 (or B^-+ S^+) on the even sites: the Schur operator with right
    preconditioning by B = b5 + c5 C."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    out = np.empty_like(psi)
    _load().oracle_schur_rp(C.byref(act.params()), pu, pi, out.ctypes.data, int(dag))
    return out


def prep_source(act: Action, U, b):
    U, pu = _c(U)
    b, pb = _c(b)
    out = np.empty_like(b)
    _load().oracle_prep_source(C.byref(act.params()), pu, pb, out.ctypes.data)
    return out


def reconstruct(act: Action, U, b, xe):
    U, pu = _c(U)
    b, pb = _c(b)
    x = np.array(xe, dtype=np.complex128, copy=True, order="C")
    _load().oracle_reconstruct(C.byref(act.params()), pu, pb, x.ctypes.data)
    return x


def true_residual(act: Action, U, b, x) -> float:
    U, pu = _c(U)
    b, pb = _c(b)
    x, px = _c(x)
    return float(_load().oracle_true_residual(C.byref(act.params()), pu, pb, px))


def solve(act: Action, U, b, tol=1e-10, max_iter=100000):
    """Full solve of D5 x = b; returns (x, info dict)."""
    U, pu = _c(U)
    b, pb = _c(b)
    x = np.zeros_like(b)
    info = SolveInfo()
    st = _load().oracle_solve(C.byref(act.params()), pu, pb, x.ctypes.data,
                              float(tol), int(max_iter), C.byref(info))
    return x, dict(status=int(st), iters=info.iters, restarts=info.restarts,
                   true_resid=info.true_resid, schur_resid=info.schur_resid)


def cgls_step(act: Action, U, x, r, p, s, q, gam):
    """One CGLS iteration in place on the given full-size vectors."""
    U, pu = _c(U)
    g = C.c_double(gam)
    rr = _load().oracle_cgls_step(C.byref(act.params()), pu, x.ctypes.data, r.ctypes.data,
                                  p.ctypes.data, s.ctypes.data, q.ctypes.data, C.byref(g))
    return float(rr), float(g.value)


def D5_sites(act: Action, U, psi, sites):
    """(D5 psi) at the listed 4D lexicographic sites, all slices: [n, L5, 4, 3]."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(s), act.L5, 4, 3), np.complex128)
    _load().oracle_D5_sites(C.byref(act.params()), pu, pi, s.ctypes.data, len(s), out.ctypes.data)
    return out


def schur_sites(act: Action, U, psi, sites, dag=False):
    """(S psi) or (S^+ psi) at the listed even 4D sites, all slices: [n, L5, 4, 3]."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(s), act.L5, 4, 3), np.complex128)
    _load().oracle_schur_sites(C.byref(act.params()), pu, pi, s.ctypes.data, len(s), int(dag), out.ctypes.data)
    return out


def schur_rp_sites(act: Action, U, psi, sites, dag=False):
    """(S B^-1 psi) or (B^-+ S^+ psi) at the listed even 4D sites, all slices:
    [n, L5, 4, 3]."""
    U, pu = _c(U)
    psi, pi = _c(psi)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(s), act.L5, 4, 3), np.complex128)
    _load().oracle_schur_rp_sites(C.byref(act.params()), pu, pi, s.ctypes.data, len(s), int(dag), out.ctypes.data)
    return out


def even_mask(dims) -> np.ndarray:
    """Boolean [t, z, y, x] mask of even 4D sites."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return ((x + y + z + t) % 2) == 0
