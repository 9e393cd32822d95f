"""ctypes binding of libmdwf (include/mdwf.h), argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: all work runs in the HIP library.  Device pointers are
plain integers (e.g. ``torch.Tensor.data_ptr()``), streams are HIP stream
handles as integers (``torch.cuda.current_stream().cuda_stream``) or None.

Importing this module loads ``libmdwf.so`` from the package directory and
raises if it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdwf.so")

MDWF_OK, MDWF_ERR_ARG, MDWF_ERR_STATE, MDWF_ERR_OOM, MDWF_ERR_HIP, MDWF_ERR_NOCONV, MDWF_ERR_NUMERIC = range(7)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_STATE", "ERR_OOM", "ERR_HIP", "ERR_NOCONV", "ERR_NUMERIC"]
MDWF_F64, MDWF_F32, MDWF_F16 = 0, 1, 2
MDWF_FULL, MDWF_HALF_EVEN, MDWF_HALF_ODD = 0, 1, 2
MDWF_STATIC_SCRATCH_BYTES = 256 << 20   # the static scratch of mdwf_apply_dev_noalloc
(MDWF_OP_D5, MDWF_OP_D5_DAG, MDWF_OP_SCHUR, MDWF_OP_SCHUR_DAG, MDWF_OP_HOP_EO, MDWF_OP_HOP_OE,
 MDWF_OP_K5, MDWF_OP_K5INV, MDWF_OP_HOP_EO_DAG, MDWF_OP_HOP_OE_DAG, MDWF_OP_K5_DAG, MDWF_OP_K5INV_DAG,
 MDWF_OP_B, MDWF_OP_B_DAG, MDWF_OP_SCHUR_SYM, MDWF_OP_SCHUR_SYM_DAG, MDWF_OP_SCHUR_RP, MDWF_OP_SCHUR_RP_DAG,
 MDWF_OP_BINV, MDWF_OP_BINV_DAG) = range(20)

# field kinds (in, out) of each operator
OP_KINDS = {
    MDWF_OP_D5: (MDWF_FULL, MDWF_FULL), MDWF_OP_D5_DAG: (MDWF_FULL, MDWF_FULL),
    MDWF_OP_SCHUR: (MDWF_HALF_EVEN, MDWF_HALF_EVEN), MDWF_OP_SCHUR_DAG: (MDWF_HALF_EVEN, MDWF_HALF_EVEN),
    MDWF_OP_HOP_EO: (MDWF_HALF_ODD, MDWF_HALF_EVEN), MDWF_OP_HOP_OE: (MDWF_HALF_EVEN, MDWF_HALF_ODD),
    MDWF_OP_HOP_EO_DAG: (MDWF_HALF_ODD, MDWF_HALF_EVEN), MDWF_OP_HOP_OE_DAG: (MDWF_HALF_EVEN, MDWF_HALF_ODD),
    MDWF_OP_K5: (MDWF_FULL, MDWF_FULL), MDWF_OP_K5INV: (MDWF_FULL, MDWF_FULL),
    MDWF_OP_K5_DAG: (MDWF_FULL, MDWF_FULL), MDWF_OP_K5INV_DAG: (MDWF_FULL, MDWF_FULL),
    MDWF_OP_B: (MDWF_FULL, MDWF_FULL), MDWF_OP_B_DAG: (MDWF_FULL, MDWF_FULL),
    MDWF_OP_SCHUR_SYM: (MDWF_HALF_EVEN, MDWF_HALF_EVEN), MDWF_OP_SCHUR_SYM_DAG: (MDWF_HALF_EVEN, MDWF_HALF_EVEN),
    MDWF_OP_SCHUR_RP: (MDWF_HALF_EVEN, MDWF_HALF_EVEN), MDWF_OP_SCHUR_RP_DAG: (MDWF_HALF_EVEN, MDWF_HALF_EVEN),
    MDWF_OP_BINV: (MDWF_FULL, MDWF_FULL), MDWF_OP_BINV_DAG: (MDWF_FULL, MDWF_FULL),
}


class mdwf_geometry(C.Structure):
    _fields_ = [("X", C.c_int), ("Y", C.c_int), ("Z", C.c_int), ("T", C.c_int), ("antiperiodic_t", C.c_int)]


class mdwf_action(C.Structure):
    _fields_ = [("M5", C.c_double), ("b5", C.c_double), ("c5", C.c_double), ("mq", C.c_double), ("L5", C.c_int)]


class mdwf_solver_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("inner", C.c_int), ("delta", C.c_double),
                ("check_every", C.c_int), ("use_graph", C.c_int), ("profile_iters", C.c_int),
                ("schur_form", C.c_int), ("max_seconds", C.c_double), ("x_ref", C.c_void_p),
                ("profile_every", C.c_int)]


class mdwf_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("restarts", C.c_int),
                ("true_resid", C.c_double), ("seconds", C.c_double), ("model_flops", C.c_double),
                ("model_bytes", C.c_double), ("hop_us", C.c_double * 4), ("hop_rhs", C.c_int),
                ("hop_samples", C.c_int), ("err_vs_ref", C.c_double), ("launch_rhs", C.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["hop_us"] = list(self.hop_us)
        return d


class mdwf_launch_tune(C.Structure):
    _fields_ = [("tile", C.c_int * 4), ("xcd_remap", C.c_int), ("nt_store", C.c_int), ("link_mode", C.c_int),
                ("rhs_group", C.c_int), ("us", C.c_double), ("plane_bt", C.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["tile"] = list(self.tile)
        return d


class MdwfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES[status] if 0 <= status < 7 else status, msg))
        self.status = status


def _share_hip_runtime_with_torch():
    """Load torch's HIP runtime first, when torch is installed.

    torch ships its own libamdhip64 (same SONAME as the system one, but
    torch's extensions name it without the version suffix, so the loader would
    otherwise map a second copy).  Two HIP runtimes in one process do not
    share devices, streams or allocations; with torch loaded first, libmdwf's
    dependency resolves to torch's already-loaded runtime.
    """
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def _load():
    _share_hip_runtime_with_torch()
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmdwf.so is not built (run __graft_entry__.build() or "
                          "python paper_1701_07559_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.c_int, C.c_double
    sig = {
        "mdwf_create": ([C.POINTER(mdwf_geometry), ip, vp, C.POINTER(vp)], ip),
        "mdwf_destroy": ([vp], None),
        "mdwf_last_error": ([vp], C.c_char_p),
        "mdwf_load_gauge": ([vp, vp], ip),
        "mdwf_load_gauge_dev": ([vp, vp], ip),
        "mdwf_set_action": ([vp, C.POINTER(mdwf_action)], ip),
        "mdwf_field_bytes": ([vp, ip, ip, C.POINTER(C.c_size_t)], ip),
        "mdwf_pack_dev": ([vp, ip, ip, vp, vp, vp], ip),
        "mdwf_unpack_dev": ([vp, ip, ip, vp, vp, vp], ip),
        "mdwf_apply": ([vp, ip, ip, vp, vp], ip),
        "mdwf_apply_dev": ([vp, ip, ip, vp, vp, vp], ip),
        "mdwf_apply_dev_noalloc": ([vp, ip, ip, vp, vp, vp], ip),
        "mdwf_apply_batch_dev": ([vp, ip, ip, ip, vp, vp, C.c_size_t, C.POINTER(dp), vp], ip),
        "mdwf_solve_footprint": ([C.POINTER(mdwf_geometry), ip, ip, ip, ip, C.POINTER(C.c_size_t)], ip),
        "mdwf_solve": ([vp, ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(dp), C.POINTER(mdwf_solver_opts),
                        C.POINTER(mdwf_solve_info)], ip),
        "mdwf_solve_dev": ([vp, ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(dp), C.POINTER(mdwf_solver_opts),
                            C.POINTER(mdwf_solve_info), vp], ip),
        "mdwf_solve_point": ([vp, C.POINTER(ip), ip, C.POINTER(ip), C.POINTER(dp), C.POINTER(mdwf_solver_opts),
                              C.POINTER(vp), C.POINTER(mdwf_solve_info)], ip),
        "mdwf_default_opts": ([C.POINTER(mdwf_solver_opts)], None),
        "mdwf_op_model": ([vp, ip, ip, C.POINTER(dp), C.POINTER(dp)], ip),
        "mdwf_autotune": ([vp, C.POINTER(mdwf_launch_tune)], ip),
        "mdwf_autotune_solve": ([vp, C.POINTER(mdwf_solver_opts), ip, C.POINTER(mdwf_launch_tune)], ip),
        "mdwf_get_tune": ([vp, ip, C.POINTER(mdwf_launch_tune)], ip),
        "mdwf_set_tune": ([vp, ip, C.POINTER(mdwf_launch_tune)], ip),
        "mdwf_wilson_flow": ([C.POINTER(mdwf_geometry), ip, vp, dp, ip, C.POINTER(dp)], ip),
        "mdwf_wilson_flow_dev": ([C.POINTER(mdwf_geometry), vp, dp, ip, vp, C.POINTER(dp)], ip),
        "mdwf_plaquette_dev": ([C.POINTER(mdwf_geometry), vp, vp, C.POINTER(dp)], ip),
        "mdwf_gauss_smear_dev": ([C.POINTER(mdwf_geometry), vp, ip, vp, vp, dp, ip, vp], ip),
        "mdwf_wall_source_dev": ([C.POINTER(mdwf_geometry), C.POINTER(mdwf_action), vp, ip, vp, vp, vp], ip),
        "mdwf_project_4d_dev": ([C.POINTER(mdwf_geometry), ip, ip, vp, vp, vp, vp], ip),
        "mdwf_mres_correlators_dev": ([C.POINTER(mdwf_geometry), ip, ip, vp, vp, C.POINTER(dp), C.POINTER(dp),
                                       C.POINTER(dp)], ip),
        "mdwf_pion_correlator_dev": ([C.POINTER(mdwf_geometry), ip, vp, vp, C.POINTER(dp)], ip),
        "mdwf_server_create": ([ip, C.c_size_t, ip, C.POINTER(vp)], ip),
        "mdwf_server_destroy": ([vp], None),
        "mdwf_server_last_error": ([vp], C.c_char_p),
        "mdwf_server_add_field": ([vp, C.POINTER(mdwf_geometry), vp, C.POINTER(ip)], ip),
        "mdwf_server_submit": ([vp, ip, C.POINTER(mdwf_action), ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(dp),
                                C.POINTER(mdwf_solver_opts), C.POINTER(ip)], ip),
        "mdwf_server_submit_point": ([vp, ip, C.POINTER(mdwf_action), C.POINTER(ip), ip, C.POINTER(ip),
                                      C.POINTER(dp), C.POINTER(mdwf_solver_opts), C.POINTER(vp), C.POINTER(ip)], ip),
        "mdwf_server_wait": ([vp, ip, C.POINTER(mdwf_solve_info), C.POINTER(dp)], ip),
        "mdwf_server_stats": ([vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(ip)], ip),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def mdwf_last_error(ctx) -> str:
    s = lib.mdwf_last_error(ctx)
    return s.decode() if s else ""


def _check(ctx, st, allow=()):
    if st != MDWF_OK and st not in allow:
        raise MdwfError(st, mdwf_last_error(ctx))
    return st


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def mdwf_create(dims, antiperiodic_t=True, hip_device=0, hip_stream=None):
    g = mdwf_geometry(*[int(d) for d in dims], int(bool(antiperiodic_t)))
    out = C.c_void_p()
    _check(None, lib.mdwf_create(C.byref(g), int(hip_device), hip_stream, C.byref(out)))
    return out


def mdwf_destroy(ctx):
    lib.mdwf_destroy(ctx)


def mdwf_load_gauge(ctx, U):
    U = _c128(U)
    _check(ctx, lib.mdwf_load_gauge(ctx, U.ctypes.data))


def mdwf_load_gauge_dev(ctx, U_ptr):
    _check(ctx, lib.mdwf_load_gauge_dev(ctx, int(U_ptr)))


def mdwf_set_action(ctx, M5, b5, c5, mq, L5):
    a = mdwf_action(float(M5), float(b5), float(c5), float(mq), int(L5))
    _check(ctx, lib.mdwf_set_action(ctx, C.byref(a)))


def mdwf_field_bytes(ctx, prec, kind) -> int:
    n = C.c_size_t()
    _check(ctx, lib.mdwf_field_bytes(ctx, int(prec), int(kind), C.byref(n)))
    return int(n.value)


def mdwf_pack_dev(ctx, prec, kind, canon_ptr, native_ptr, stream=None):
    _check(ctx, lib.mdwf_pack_dev(ctx, int(prec), int(kind), int(canon_ptr), int(native_ptr), stream))


def mdwf_unpack_dev(ctx, prec, kind, native_ptr, canon_ptr, stream=None):
    _check(ctx, lib.mdwf_unpack_dev(ctx, int(prec), int(kind), int(native_ptr), int(canon_ptr), stream))


def mdwf_apply(ctx, op, prec, inp, out):
    """Host canonical complex128 arrays; `out` is written in place."""
    inp = _c128(inp)
    if not (out.flags.c_contiguous and out.dtype == np.complex128):
        raise ValueError("out must be a C-contiguous complex128 array")
    _check(ctx, lib.mdwf_apply(ctx, int(op), int(prec), inp.ctypes.data, out.ctypes.data))
    return out


def mdwf_apply_dev(ctx, op, prec, in_ptr, out_ptr, stream=None):
    _check(ctx, lib.mdwf_apply_dev(ctx, int(op), int(prec), int(in_ptr), int(out_ptr), stream))


def mdwf_apply_dev_noalloc(ctx, op, prec, in_ptr, out_ptr, stream=None):
    """mdwf_apply_dev without any device allocation (static scratch)."""
    _check(ctx, lib.mdwf_apply_dev_noalloc(ctx, int(op), int(prec), int(in_ptr), int(out_ptr), stream))


def mdwf_apply_batch_dev(ctx, op, prec, nrhs, in_ptr, out_ptr, stride, mq=None, stream=None):
    """Apply op to nrhs device native fields `stride` bytes apart, RHS k with
    mass mq[k] (None = the action's), all in one launch set."""
    m = (C.c_double * int(nrhs))(*mq) if mq is not None else None
    _check(ctx, lib.mdwf_apply_batch_dev(ctx, int(op), int(prec), int(nrhs), int(in_ptr), int(out_ptr),
                                         int(stride), m, stream))


def mdwf_solve_footprint(dims, L5, inner, nrhs, host_io=1):
    """Device bytes a solve of nrhs RHS would allocate (no device needed);
    host_io 0 device fields, 1 host fields, 2 point sources / wall fields."""
    g = mdwf_geometry(*[int(d) for d in dims], 1)
    n = C.c_size_t()
    st = lib.mdwf_solve_footprint(C.byref(g), int(L5), int(inner), int(nrhs), int(host_io), C.byref(n))
    if st != MDWF_OK:
        raise MdwfError(st, "bad footprint arguments")
    return int(n.value)


def mdwf_default_opts() -> mdwf_solver_opts:
    o = mdwf_solver_opts()
    lib.mdwf_default_opts(C.byref(o))
    return o


def _opts(opts):
    """Options struct from a dict; x_ref (a list of canonical FP64 fields:
    device pointers for *_dev calls, host complex128 arrays otherwise) is
    kept alive on the returned struct."""
    o = mdwf_default_opts()
    if isinstance(opts, mdwf_solver_opts):
        return opts
    for k, v in (opts or {}).items():
        if k == "x_ref":
            if v is None:
                continue
            keep = [_c128(a) if isinstance(a, np.ndarray) else a for a in v]
            ptrs = [a.ctypes.data if isinstance(a, np.ndarray) else int(a) for a in keep]
            arr = (C.c_void_p * len(ptrs))(*ptrs)
            o._x_ref_keep = (keep, arr)
            o.x_ref = C.cast(arr, C.c_void_p).value
            continue
        setattr(o, k, v)
    return o


def mdwf_solve(ctx, b_list, x_list, mq=None, opts=None):
    """Host canonical complex128 fields; returns (status, [info dicts])."""
    n = len(b_list)
    bs = [_c128(b) for b in b_list]
    for x in x_list:
        if not (x.flags.c_contiguous and x.dtype == np.complex128):
            raise ValueError("x must be C-contiguous complex128 arrays")
    bp = (C.c_void_p * n)(*[b.ctypes.data for b in bs])
    xp = (C.c_void_p * n)(*[x.ctypes.data for x in x_list])
    m = (C.c_double * n)(*mq) if mq is not None else None
    infos = (mdwf_solve_info * n)()
    o = _opts(opts)
    st = lib.mdwf_solve(ctx, n, bp, xp, m, C.byref(o), infos)
    _check(ctx, st, allow=(MDWF_ERR_NOCONV, MDWF_ERR_NUMERIC))
    return st, [i.as_dict() for i in infos]


def mdwf_solve_dev(ctx, b_ptrs, x_ptrs, mq=None, opts=None, stream=None):
    """Canonical FP64 device fields (integer pointers); returns (status, [info dicts])."""
    n = len(b_ptrs)
    bp = (C.c_void_p * n)(*[int(p) for p in b_ptrs])
    xp = (C.c_void_p * n)(*[int(p) for p in x_ptrs])
    m = (C.c_double * n)(*mq) if mq is not None else None
    infos = (mdwf_solve_info * n)()
    o = _opts(opts)
    st = lib.mdwf_solve_dev(ctx, n, bp, xp, m, C.byref(o), infos, stream)
    _check(ctx, st, allow=(MDWF_ERR_NOCONV, MDWF_ERR_NUMERIC))
    return st, [i.as_dict() for i in infos]


def mdwf_solve_point(ctx, site, cols, q_list, mq=None, opts=None):
    """Point-source propagator solves: q_list[k] (host complex128 4D canonical
    [T, Z, Y, X, 4, 3], written in place) receives the wall field of the
    solution for spin-colour column cols[k]; returns (status, [info dicts])."""
    n = len(cols)
    for q in q_list:
        if not (q.flags.c_contiguous and q.dtype == np.complex128):
            raise ValueError("q must be C-contiguous complex128 arrays")
    s = (C.c_int * 4)(*[int(v) for v in site])
    cl = (C.c_int * n)(*[int(c) for c in cols])
    qp = (C.c_void_p * n)(*[q.ctypes.data for q in q_list])
    m = (C.c_double * n)(*mq) if mq is not None else None
    infos = (mdwf_solve_info * n)()
    o = _opts(opts)
    st = lib.mdwf_solve_point(ctx, s, n, cl, m, C.byref(o), qp, infos)
    _check(ctx, st, allow=(MDWF_ERR_NOCONV, MDWF_ERR_NUMERIC))
    return st, [i.as_dict() for i in infos]


def mdwf_op_model(ctx, op, prec):
    f, b = C.c_double(), C.c_double()
    _check(ctx, lib.mdwf_op_model(ctx, int(op), int(prec), C.byref(f), C.byref(b)))
    return f.value, b.value


def mdwf_autotune(ctx):
    """Autotune the hop kernels' launch shape per precision; returns 3 dicts."""
    out = (mdwf_launch_tune * 3)()
    _check(ctx, lib.mdwf_autotune(ctx, out))
    return [o.as_dict() for o in out]


def mdwf_autotune_solve(ctx, nrhs, opts=None):
    """Autotune for one solve shape (inner precision and Schur form of opts,
    nrhs RHS per launch); returns 3 dicts."""
    out = (mdwf_launch_tune * 3)()
    o = _opts(opts)
    _check(ctx, lib.mdwf_autotune_solve(ctx, C.byref(o), int(nrhs), out))
    return [t.as_dict() for t in out]


def mdwf_get_tune(ctx, prec):
    t = mdwf_launch_tune()
    _check(ctx, lib.mdwf_get_tune(ctx, int(prec), C.byref(t)))
    return t.as_dict()


def mdwf_set_tune(ctx, prec, tune):
    """Install a launch shape (a dict as mdwf_get_tune returns) for prec."""
    t = mdwf_launch_tune()
    for k, v in tune.items():
        if k == "tile":
            t.tile = (C.c_int * 4)(*v)
        else:
            setattr(t, k, v)
    _check(ctx, lib.mdwf_set_tune(ctx, int(prec), C.byref(t)))


def mdwf_wilson_flow(dims, U, eps, nsteps, hip_device=0):
    """Wilson gradient flow of a host canonical gauge field (a flowed copy is
    returned); returns (U_flowed, (plaquette before, after))."""
    g = mdwf_geometry(*[int(d) for d in dims], 0)
    V = np.array(U, dtype=np.complex128, order="C", copy=True)
    plaq = (C.c_double * 2)()
    st = lib.mdwf_wilson_flow(C.byref(g), int(hip_device), V.ctypes.data, float(eps), int(nsteps), plaq)
    if st != MDWF_OK:
        raise MdwfError(st, mdwf_last_error(None))
    return V, (plaq[0], plaq[1])


def mdwf_wilson_flow_dev(dims, U_ptr, eps, nsteps, stream=None, plaquette=True):
    """Flow a device canonical gauge field in place; returns (plaquette
    before, after), or None with plaquette=False (no reductions launched)."""
    g = mdwf_geometry(*[int(d) for d in dims], 0)
    plaq = (C.c_double * 2)() if plaquette else None
    st = lib.mdwf_wilson_flow_dev(C.byref(g), int(U_ptr), float(eps), int(nsteps), stream, plaq)
    if st != MDWF_OK:
        raise MdwfError(st, mdwf_last_error(None))
    return (plaq[0], plaq[1]) if plaquette else None


def mdwf_plaquette_dev(dims, U_ptr, stream=None):
    g = mdwf_geometry(*[int(d) for d in dims], 0)
    p = C.c_double()
    st = lib.mdwf_plaquette_dev(C.byref(g), int(U_ptr), stream, C.byref(p))
    if st != MDWF_OK:
        raise MdwfError(st, mdwf_last_error(None))
    return p.value


def _geom(dims, antiperiodic_t=True):
    return mdwf_geometry(*[int(d) for d in dims], int(bool(antiperiodic_t)))


def _raise(st):
    if st != MDWF_OK:
        raise MdwfError(st, mdwf_last_error(None))


def mdwf_gauss_smear_dev(dims, U_ptr, nvec, in_ptr, out_ptr, sigma, niter, stream=None):
    """Gaussian-smear nvec consecutive device canonical 4D spinor fields."""
    _raise(lib.mdwf_gauss_smear_dev(C.byref(_geom(dims)), int(U_ptr), int(nvec), int(in_ptr), int(out_ptr),
                                    float(sigma), int(niter), stream))


def mdwf_wall_source_dev(dims, action, U_ptr, nvec, eta_ptr, b_ptr, antiperiodic_t=True, stream=None):
    """5D right-hand sides (1 - c5 D_W) Pbar eta of nvec device 4D sources;
    action = (M5, b5, c5, mq, L5)."""
    M5, b5, c5, mq, L5 = action
    a = mdwf_action(float(M5), float(b5), float(c5), float(mq), int(L5))
    _raise(lib.mdwf_wall_source_dev(C.byref(_geom(dims, antiperiodic_t)), C.byref(a), int(U_ptr), int(nvec),
                                    int(eta_ptr), int(b_ptr), stream))


def mdwf_project_4d_dev(dims, L5, nvec, x_ptr, q_ptr, mid_ptr=None, stream=None):
    """Wall (and optionally midpoint) 4D fields of nvec device 5D fields."""
    _raise(lib.mdwf_project_4d_dev(C.byref(_geom(dims)), int(L5), int(nvec), int(x_ptr), int(q_ptr),
                                   int(mid_ptr) if mid_ptr else None, stream))


def mdwf_mres_correlators_dev(dims, L5, nvec, x_ptr, stream=None):
    """(C_PP, C_mp, m_res) per time slice, summed over nvec device 5D solutions."""
    T = int(dims[3])
    cpp, cmp_, mres = (C.c_double * T)(), (C.c_double * T)(), (C.c_double * T)()
    _raise(lib.mdwf_mres_correlators_dev(C.byref(_geom(dims)), int(L5), int(nvec), int(x_ptr), stream, cpp, cmp_,
                                         mres))
    return np.array(cpp[:]), np.array(cmp_[:]), np.array(mres[:])


def mdwf_pion_correlator_dev(dims, nvec, q_ptr, stream=None):
    """Pseudoscalar correlator per time slice of nvec device 4D fields."""
    T = int(dims[3])
    c = (C.c_double * T)()
    _raise(lib.mdwf_pion_correlator_dev(C.byref(_geom(dims)), int(nvec), int(q_ptr), stream, c))
    return np.array(c[:])


class Server:
    """Request server (mdwf_server_*): resident gauge fields, solves admitted
    by device footprint and run concurrently on worker streams.  Host arrays
    of a request are kept alive here until its wait returns."""

    def __init__(self, hip_device=0, mem_budget=0, max_active=4):
        h = C.c_void_p()
        st = lib.mdwf_server_create(int(hip_device), int(mem_budget), int(max_active), C.byref(h))
        if st != MDWF_OK:
            raise MdwfError(st, "mdwf_server_create failed")
        self.h = h
        self._keep = {}

    def _err(self):
        s = lib.mdwf_server_last_error(self.h)
        return s.decode() if s else ""

    def add_field(self, dims, U, antiperiodic_t=True):
        g = mdwf_geometry(*[int(d) for d in dims], int(bool(antiperiodic_t)))
        U = _c128(U)
        fid = C.c_int()
        st = lib.mdwf_server_add_field(self.h, C.byref(g), U.ctypes.data, C.byref(fid))
        if st != MDWF_OK:
            raise MdwfError(st, self._err())
        return fid.value

    def submit(self, field, M5, b5, c5, mq, L5, b_list, x_list, masses=None, opts=None):
        """Queue a solve; b_list / x_list are host complex128 canonical fields."""
        n = len(b_list)
        bs = [_c128(b) for b in b_list]
        for x in x_list:
            if not (x.flags.c_contiguous and x.dtype == np.complex128):
                raise ValueError("x must be C-contiguous complex128 arrays")
        a = mdwf_action(float(M5), float(b5), float(c5), float(mq), int(L5))
        bp = (C.c_void_p * n)(*[b.ctypes.data for b in bs])
        xp = (C.c_void_p * n)(*[x.ctypes.data for x in x_list])
        m = (C.c_double * n)(*masses) if masses is not None else None
        o = _opts(opts)
        rid = C.c_int()
        st = lib.mdwf_server_submit(self.h, int(field), C.byref(a), n, bp, xp, m, C.byref(o), C.byref(rid))
        if st != MDWF_OK:
            raise MdwfError(st, self._err())
        self._keep[rid.value] = (bs, list(x_list), bp, xp, m, n)
        return rid.value

    def submit_point(self, field, M5, b5, c5, mq, L5, site, cols, q_list, masses=None, opts=None):
        """Queue point-source propagator solves; q_list are host complex128 4D
        canonical fields written in place (kept alive until wait)."""
        n = len(cols)
        for q in q_list:
            if not (q.flags.c_contiguous and q.dtype == np.complex128):
                raise ValueError("q must be C-contiguous complex128 arrays")
        a = mdwf_action(float(M5), float(b5), float(c5), float(mq), int(L5))
        s = (C.c_int * 4)(*[int(v) for v in site])
        cl = (C.c_int * n)(*[int(c) for c in cols])
        qp = (C.c_void_p * n)(*[q.ctypes.data for q in q_list])
        m = (C.c_double * n)(*masses) if masses is not None else None
        o = _opts(opts)
        rid = C.c_int()
        st = lib.mdwf_server_submit_point(self.h, int(field), C.byref(a), s, n, cl, m, C.byref(o), qp, C.byref(rid))
        if st != MDWF_OK:
            raise MdwfError(st, self._err())
        self._keep[rid.value] = (list(q_list), qp, cl, s, m, n)
        return rid.value

    def wait(self, rid):
        """(status, [info dicts], (queued s, running s, latency s))."""
        n = self._keep[rid][5]
        infos = (mdwf_solve_info * n)()
        t = (C.c_double * 3)()
        st = lib.mdwf_server_wait(self.h, int(rid), infos, t)
        del self._keep[rid]
        if st not in (MDWF_OK, MDWF_ERR_NOCONV, MDWF_ERR_NUMERIC):
            raise MdwfError(st, self._err())
        return st, [i.as_dict() for i in infos], tuple(t)

    def stats(self):
        b, p, q = C.c_size_t(), C.c_size_t(), C.c_int()
        lib.mdwf_server_stats(self.h, C.byref(b), C.byref(p), C.byref(q))
        return dict(budget=b.value, peak_reserved=p.value, queued=q.value)

    def close(self):
        if self.h:
            lib.mdwf_server_destroy(self.h)
            self.h = None


def exported_symbols():
    """Names of the C entry points declared in include/mdwf.h."""
    return ["mdwf_create", "mdwf_destroy", "mdwf_last_error", "mdwf_load_gauge", "mdwf_load_gauge_dev",
            "mdwf_set_action", "mdwf_field_bytes", "mdwf_pack_dev", "mdwf_unpack_dev", "mdwf_apply",
            "mdwf_apply_dev", "mdwf_apply_dev_noalloc", "mdwf_apply_batch_dev", "mdwf_solve_footprint", "mdwf_solve",
            "mdwf_solve_point", "mdwf_server_submit_point", "mdwf_solve_dev", "mdwf_default_opts", "mdwf_op_model",
            "mdwf_autotune", "mdwf_autotune_solve", "mdwf_get_tune", "mdwf_set_tune", "mdwf_wilson_flow", "mdwf_wilson_flow_dev",
            "mdwf_plaquette_dev", "mdwf_gauss_smear_dev", "mdwf_wall_source_dev", "mdwf_project_4d_dev",
            "mdwf_mres_correlators_dev", "mdwf_pion_correlator_dev", "mdwf_server_create", "mdwf_server_destroy",
            "mdwf_server_last_error", "mdwf_server_add_field", "mdwf_server_submit", "mdwf_server_wait",
            "mdwf_server_stats"]
