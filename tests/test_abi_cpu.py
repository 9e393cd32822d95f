"""CPU-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdwf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdwf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["mdwf_create", "mdwf_destroy", "mdwf_load_gauge", "mdwf_set_action", "mdwf_apply",
                 "mdwf_apply_dev", "mdwf_solve", "mdwf_solve_dev", "mdwf_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1701_07559_amd import mdwf
    lib = C.CDLL(mdwf.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(mdwf.exported_symbols()) == declared_functions()


def test_create_rejects_odd_extents_without_device():
    from paper_1701_07559_amd import mdwf
    g = mdwf.mdwf_geometry(3, 4, 4, 4, 1)
    out = C.c_void_p()
    st = mdwf.lib.mdwf_create(C.byref(g), 0, None, C.byref(out))
    assert st == mdwf.MDWF_ERR_ARG
    assert "even" in mdwf.mdwf_last_error(None)
    g = mdwf.mdwf_geometry(4, 4, 0, 4, 1)
    assert mdwf.lib.mdwf_create(C.byref(g), 0, None, C.byref(out)) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_create(None, 0, None, C.byref(out)) == mdwf.MDWF_ERR_ARG


def test_null_context_calls_return_arg_errors():
    from paper_1701_07559_amd import mdwf
    a = mdwf.mdwf_action(1.3, 1.5, 0.5, 0.05, 8)
    assert mdwf.lib.mdwf_set_action(None, C.byref(a)) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_load_gauge(None, None) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_apply(None, 0, 0, None, None) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_autotune(None, None) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_autotune_solve(None, None, 1, None) == mdwf.MDWF_ERR_ARG
    o = mdwf.mdwf_default_opts()
    assert o.tol == 1e-10 and o.inner == mdwf.MDWF_F64 and abs(o.delta - 0.1) < 1e-15
    assert o.schur_form == 0 and o.profile_iters == 0 and o.use_graph == 0 and o.max_seconds == 0.0
    mdwf.lib.mdwf_destroy(None)   # ignored


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import importlib.util
    src = os.path.join(ROOT, "paper_1701_07559_amd", "mdwf.py")
    spec = importlib.util.spec_from_file_location("mdwf_copy", str(tmp_path / "mdwf.py"))
    (tmp_path / "mdwf.py").write_text(open(src).read())
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_server_null_and_argument_errors_without_device():
    from paper_1701_07559_amd import mdwf
    out = C.c_void_p()
    assert mdwf.lib.mdwf_server_create(0, 0, 0, C.byref(out)) == mdwf.MDWF_ERR_ARG   # max_active < 1
    assert mdwf.lib.mdwf_server_create(0, 0, 2, None) == mdwf.MDWF_ERR_ARG
    a = mdwf.mdwf_action(1.3, 1.5, 0.5, 0.05, 8)
    rid = C.c_int()
    assert mdwf.lib.mdwf_server_submit(None, 0, C.byref(a), 1, None, None, None, None,
                                       C.byref(rid)) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_server_wait(None, 1, None, None) == mdwf.MDWF_ERR_ARG
    assert mdwf.lib.mdwf_server_add_field(None, None, None, None) == mdwf.MDWF_ERR_ARG
    mdwf.lib.mdwf_server_destroy(None)   # ignored


def test_source_flow_entry_points_reject_bad_arguments_without_device():
    """The source/sink and flow entry points validate every argument before
    any HIP call, so these run without a GPU."""
    from paper_1701_07559_amd import mdwf
    L = mdwf.lib
    ARG = mdwf.MDWF_ERR_ARG
    g = mdwf.mdwf_geometry(4, 4, 4, 8, 1)
    bad = mdwf.mdwf_geometry(4, 0, 4, 8, 1)
    buf = (C.c_double * 64)()
    p = C.cast(buf, C.c_void_p)
    q = C.c_void_p(C.addressof(buf) + (1 << 20))   # a distinct address, never dereferenced
    a = mdwf.mdwf_action(1.3, 1.5, 0.5, 0.05, 8)
    # smearing: geometry, nulls, counts, width, overlap
    assert L.mdwf_gauss_smear_dev(None, p, 1, p, q, 2.0, 3, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(bad), p, 1, p, q, 2.0, 3, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(g), None, 1, p, q, 2.0, 3, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(g), p, 0, p, q, 2.0, 3, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(g), p, 1, p, q, -1.0, 3, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(g), p, 1, p, q, float("inf"), 3, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(g), p, 1, p, q, 2.0, -1, None) == ARG
    assert L.mdwf_gauss_smear_dev(C.byref(g), p, 1, p, p, 2.0, 3, None) == ARG
    assert "overlap" in mdwf.mdwf_last_error(None)
    # wall source
    assert L.mdwf_wall_source_dev(C.byref(g), None, p, 1, p, q, None) == ARG
    assert L.mdwf_wall_source_dev(C.byref(g), C.byref(a), p, 0, p, q, None) == ARG
    a0 = mdwf.mdwf_action(1.3, 1.5, 0.5, 0.05, 0)
    assert L.mdwf_wall_source_dev(C.byref(g), C.byref(a0), p, 1, p, q, None) == ARG
    # projections and correlators: odd L5 has no midpoint
    assert L.mdwf_project_4d_dev(C.byref(g), 5, 1, p, q, q, None) == ARG
    assert L.mdwf_project_4d_dev(C.byref(g), 8, 0, p, q, None, None) == ARG
    d = (C.c_double * 8)()
    assert L.mdwf_mres_correlators_dev(C.byref(g), 5, 1, p, None, d, d, d) == ARG
    assert L.mdwf_mres_correlators_dev(C.byref(g), 8, 1, p, None, None, d, d) == ARG
    big_t = mdwf.mdwf_geometry(1, 1, 1, 70000, 1)
    assert L.mdwf_mres_correlators_dev(C.byref(big_t), 8, 1, p, None, d, d, d) == ARG
    assert L.mdwf_pion_correlator_dev(C.byref(g), 0, p, None, d) == ARG
    assert L.mdwf_pion_correlator_dev(C.byref(g), 1, None, None, d) == ARG
    assert L.mdwf_pion_correlator_dev(C.byref(big_t), 1, p, None, d) == ARG
    # flow
    assert L.mdwf_wilson_flow_dev(C.byref(g), p, 0.0, 3, None, None) == ARG
    assert L.mdwf_wilson_flow_dev(C.byref(g), p, 0.01, -1, None, None) == ARG
    assert L.mdwf_wilson_flow_dev(C.byref(mdwf.mdwf_geometry(4, 1, 4, 4, 0)), p, 0.01, 1, None, None) == ARG
    assert L.mdwf_plaquette_dev(C.byref(g), None, None, d) == ARG


def test_solve_footprint_counts_every_solver_vector():
    """The memory plan (no device needed): per RHS x_hi and b' in FP64 and five
    inner vectors r, p, p', s, q (plus the FP32 x_lo when mixed), the hop
    temporary per RHS, six shared FP64 half fields, the canonical staging
    field with host I/O, and a 64 MiB margin."""
    from paper_1701_07559_amd import mdwf

    def a256(n):
        return (n + 255) // 256 * 256

    for dims, L5 in [((24, 24, 24, 64), 8), ((16, 16, 16, 48), 12), ((4, 4, 4, 8), 5)]:
        Vh = int(np.prod(dims)) // 2 * L5
        H = {0: a256(192 * Vh), 1: a256(96 * Vh), 2: a256(48 * Vh) + a256(4 * Vh)}
        for inner in (0, 1, 2):
            for n in (1, 3, 12):
                for host_io in (0, 1, 2):
                    mixed = inner != 0
                    per = 2 * H[0] + (5 * H[inner] + H[1] if mixed else 5 * H[0])
                    # staging: none, a 5D canonical field, a 4D canonical field
                    stage = (0, 2 * Vh * 24 * 8, int(np.prod(dims)) * 24 * 8)[host_io]
                    shared = 6 * H[0] + stage
                    want = per * n + shared + n * H[inner] + (64 << 20)
                    assert mdwf.mdwf_solve_footprint(dims, L5, inner, n, host_io) == want
    with pytest.raises(mdwf.MdwfError):
        mdwf.mdwf_solve_footprint((3, 4, 4, 4), 8, 0, 1)
    with pytest.raises(mdwf.MdwfError):
        mdwf.mdwf_solve_footprint((4, 4, 4, 4), 0, 0, 1)
    with pytest.raises(mdwf.MdwfError):
        mdwf.mdwf_solve_footprint((4, 4, 4, 4), 8, 0, 0)
    with pytest.raises(mdwf.MdwfError):
        mdwf.mdwf_solve_footprint((4, 4, 4, 4), 8, 0, 1, host_io=3)
