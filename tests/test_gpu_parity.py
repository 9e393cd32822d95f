"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Operator parity: relative 2-norm error of every operator against the oracle,
at most 1e-13 in FP64, 1e-6 in FP32 and 5e-3 in FP16 (the dslash tolerances of
the solver's specification), on lattices that span several workgroup tiles
with a ragged tail, on the degenerate 2^4 lattice (forward and backward
neighbours coincide), with L5 = 1 and with periodic time.

Solver parity: every solve's true FP64 residual ||b - D5 x|| / ||b||, computed
by the oracle's operator on the returned x, is at most 1e-10; where the oracle
solves the same system its solution is compared as well.
"""
import numpy as np
import pytest

import oracle
from paper_1701_07559_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3}
PREC_NAME = {0: "f64", 1: "f32", 2: "f16"}


@pytest.fixture(scope="module")
def M():
    from paper_1701_07559_amd import mdwf
    try:
        ctx = mdwf.mdwf_create((2, 2, 2, 2))
    except mdwf.MdwfError as e:
        pytest.skip("no HIP device: %s" % e)
    mdwf.mdwf_destroy(ctx)
    return mdwf


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def half(psi, dims, parity):
    """Parity-compressed canonical half field of a full canonical field."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    mask = ((x + y + z + t) % 2) == parity
    return np.ascontiguousarray(psi[:, mask])


def expand(h, dims, parity):
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    mask = ((x + y + z + t) % 2) == parity
    out = np.zeros((h.shape[0], T, Z, Y, X, 4, 3), complex)
    out[:, mask] = h
    return out


def make_ctx(M, act, U):
    ctx = M.mdwf_create(act.dims, antiperiodic_t=act.antiperiodic_t)
    M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, act.L5)
    M.mdwf_load_gauge(ctx, U)
    return ctx


def oracle_op(M, op, act, U, psi):
    """Oracle result of `op` on the full canonical field psi, as the kind the op returns."""
    d = act.dims
    if op == M.MDWF_OP_D5:
        return oracle.D5(act, U, psi)
    if op == M.MDWF_OP_D5_DAG:
        return oracle.D5(act, U, psi, dag=True)
    if op in (M.MDWF_OP_SCHUR, M.MDWF_OP_SCHUR_DAG):
        return half(oracle.schur(act, U, psi, dag=(op == M.MDWF_OP_SCHUR_DAG)), d, 0)
    if op in (M.MDWF_OP_SCHUR_SYM, M.MDWF_OP_SCHUR_SYM_DAG):
        return half(oracle.schur_sym(act, U, psi, dag=(op == M.MDWF_OP_SCHUR_SYM_DAG)), d, 0)
    if op in (M.MDWF_OP_SCHUR_RP, M.MDWF_OP_SCHUR_RP_DAG):
        return half(oracle.schur_rp(act, U, psi, dag=(op == M.MDWF_OP_SCHUR_RP_DAG)), d, 0)
    if op in (M.MDWF_OP_HOP_EO, M.MDWF_OP_HOP_EO_DAG):
        return half(oracle.hop(act, U, psi, 0, dag=(op == M.MDWF_OP_HOP_EO_DAG)), d, 0)
    if op in (M.MDWF_OP_HOP_OE, M.MDWF_OP_HOP_OE_DAG):
        return half(oracle.hop(act, U, psi, 1, dag=(op == M.MDWF_OP_HOP_OE_DAG)), d, 1)
    f = {M.MDWF_OP_K5: oracle.apply_K5, M.MDWF_OP_K5_DAG: oracle.apply_K5,
         M.MDWF_OP_K5INV: oracle.apply_K5inv, M.MDWF_OP_K5INV_DAG: oracle.apply_K5inv,
         M.MDWF_OP_B: oracle.apply_B, M.MDWF_OP_B_DAG: oracle.apply_B,
         M.MDWF_OP_BINV: oracle.apply_Binv, M.MDWF_OP_BINV_DAG: oracle.apply_Binv}[op]
    dag = op in (M.MDWF_OP_K5_DAG, M.MDWF_OP_K5INV_DAG, M.MDWF_OP_B_DAG, M.MDWF_OP_BINV_DAG)
    return f(act, psi, dag=dag)


def gpu_op(M, ctx, op, prec, act, psi):
    kin, kout = M.OP_KINDS[op]
    d = act.dims
    if kin == M.MDWF_FULL:
        inp = psi
    else:
        inp = half(psi, d, 0 if kin == M.MDWF_HALF_EVEN else 1)
    if kout == M.MDWF_FULL:
        out = np.zeros(act.shape5, complex)
    else:
        X, Y, Z, T = d
        out = np.zeros((act.L5, X * Y * Z * T // 2, 4, 3), complex)
    M.mdwf_apply(ctx, op, prec, inp, out)
    return out


GEOMS = [
    # dims, L5, antiperiodic -- tiles of 32 (L5=8), 20 (L5=12), 64 (L5=1) sites with ragged tails
    ((6, 4, 2, 6), 8, True),
    ((4, 6, 6, 4), 12, True),
    ((2, 2, 2, 2), 4, True),
    ((4, 2, 4, 6), 1, False),
    ((2, 4, 2, 4), 5, True),
    # long fifth dimensions: 4 sites per wavefront at L5 = 16, 2 at the
    # largest extent the library takes (32)
    ((2, 2, 4, 6), 16, True),
    ((2, 2, 2, 4), 32, False),
]
ALL_OPS = list(range(20))


@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: "x".join(map(str, g[0])) + "_L%d" % g[1])
@pytest.mark.parametrize("prec", [0, 1, 2], ids=lambda p: PREC_NAME[p])
def test_operator_parity(M, geom, prec):
    dims, L5, ap = geom
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05, antiperiodic_t=ap)
    U = I.random_links(dims, 0.3, 41)
    psi = I.gaussian_source(dims, L5, 42)
    ctx = make_ctx(M, act, U)
    try:
        for op in ALL_OPS:
            ref = oracle_op(M, op, act, U, psi)
            out = gpu_op(M, ctx, op, prec, act, psi)
            err = rel(out, ref)
            assert err <= TOL[prec], "op %d prec %s: rel err %.3e" % (op, PREC_NAME[prec], err)
    finally:
        M.mdwf_destroy(ctx)


LAUNCH_VARIANTS = [
    {"MDWF_LINK_MODE": "1"},
    {"MDWF_LINK_MODE": "1", "MDWF_NT_STORE": "1", "MDWF_XCD_REMAP": "0"},
    {"MDWF_LINK_MODE": "2"},
    {"MDWF_LINK_MODE": "2", "MDWF_NT_STORE": "1", "MDWF_XCD_REMAP": "0"},
    {"MDWF_TILE": "zblock1", "MDWF_NT_STORE": "1"},
    {"MDWF_TILE": "zblock2", "MDWF_XCD_REMAP": "0"},
    {"MDWF_TILE": "compact"},
    {"MDWF_TILE": "compact", "MDWF_LINK_MODE": "2", "MDWF_XCD_REMAP": "0"},
]


def tile_for(kind, dims):
    """Traversal tile (parity-compressed x, y, z, t) of the named kind."""
    X, Y, Z, T = dims
    Xh = X // 2
    if kind.startswith("zblock"):
        return (Xh, Y, int(kind[6:]), 1)
    # compact 4D tile: halves of the extents where they are even
    return tuple(e // 2 if e % 2 == 0 else e for e in (Xh, Y, Z, T))


@pytest.mark.parametrize("env", LAUNCH_VARIANTS, ids=lambda e: "-".join("%s%s" % (k[5:], v) for k, v in e.items()))
def test_operator_parity_launch_shapes(M, env, monkeypatch):
    """Every launch shape the autotuner can pick computes the same operators
    (traversal order, XCD numbering, non-temporal stores, link modes; L5 = 4
    is the smallest group the FP32 lane gather accepts, L5 = 12 leaves idle
    lanes in every wave)."""
    for k, v in env.items():
        if k != "MDWF_TILE":
            monkeypatch.setenv(k, v)
    for dims, L5 in (((6, 4, 2, 6), 8), ((4, 6, 6, 4), 12), ((4, 4, 2, 4), 4)):
        tile = tile_for(env["MDWF_TILE"], dims) if "MDWF_TILE" in env else None
        if tile:
            monkeypatch.setenv("MDWF_TILE", ",".join(map(str, tile)))
        act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
        U = I.random_links(dims, 0.3, 49)
        psi = I.gaussian_source(dims, L5, 50)
        ctx = make_ctx(M, act, U)
        try:
            for prec in (0, 1, 2):
                t = M.mdwf_get_tune(ctx, prec)
                if "MDWF_LINK_MODE" in env:
                    assert t["link_mode"] == int(env["MDWF_LINK_MODE"])
                if tile:
                    assert tuple(t["tile"]) == tile
                for op in (M.MDWF_OP_D5, M.MDWF_OP_D5_DAG, M.MDWF_OP_SCHUR, M.MDWF_OP_SCHUR_DAG,
                           M.MDWF_OP_HOP_EO, M.MDWF_OP_HOP_OE_DAG):
                    err = rel(gpu_op(M, ctx, op, prec, act, psi), oracle_op(M, op, act, U, psi))
                    assert err <= TOL[prec], (env, dims, L5, prec, op, err)
        finally:
            M.mdwf_destroy(ctx)


def test_autotune_keeps_parity(M):
    dims, L5 = (6, 4, 2, 6), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 51)
    psi = I.gaussian_source(dims, L5, 52)
    ctx = make_ctx(M, act, U)
    try:
        tunes = M.mdwf_autotune(ctx)
        assert len(tunes) == 3 and all(t["us"] > 0 for t in tunes)
        for prec in (0, 1, 2):
            assert M.mdwf_get_tune(ctx, prec)["tile"] == tunes[prec]["tile"]
            for op in (M.MDWF_OP_SCHUR, M.MDWF_OP_SCHUR_DAG, M.MDWF_OP_D5):
                assert rel(gpu_op(M, ctx, op, prec, act, psi), oracle_op(M, op, act, U, psi)) <= TOL[prec]
    finally:
        M.mdwf_destroy(ctx)


@pytest.mark.parametrize("form", [0, 1, 2], ids=["asym", "sym", "rp"])
def test_solve_shaped_autotune_keeps_parity_and_solves(M, form):
    """mdwf_autotune_solve tunes the FP16 CG operator of the form with 5 RHS
    per launch (RHS grouping among the candidates) and FP64 with one; every
    operator still matches the oracle and a 5-RHS solve still converges."""
    dims, L5 = (6, 4, 2, 6), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 53)
    psi = I.gaussian_source(dims, L5, 54)
    ctx = make_ctx(M, act, U)
    try:
        before = M.mdwf_get_tune(ctx, 1)
        opts = dict(inner=2, schur_form=form)
        tunes = M.mdwf_autotune_solve(ctx, 5, opts)
        assert len(tunes) == 3 and tunes[2]["us"] > 0 and tunes[0]["us"] > 0
        assert M.mdwf_get_tune(ctx, 2)["tile"] == tunes[2]["tile"]
        assert M.mdwf_get_tune(ctx, 2)["rhs_group"] == tunes[2]["rhs_group"]
        assert M.mdwf_get_tune(ctx, 1) == before     # FP32 is not used by this solve
        for prec in (0, 2):
            for op in ALL_OPS:
                assert rel(gpu_op(M, ctx, op, prec, act, psi), oracle_op(M, op, act, U, psi)) <= TOL[prec]
        bs = [I.gaussian_source(dims, L5, 60 + k) for k in range(5)]
        xs = [np.zeros_like(b) for b in bs]
        st, info = M.mdwf_solve(ctx, bs, xs, opts=opts)
        assert st == M.MDWF_OK
        for b, x in zip(bs, xs):
            assert oracle.true_residual(act, U, b, x) <= 1e-10
        with pytest.raises(M.MdwfError):
            M.mdwf_autotune_solve(ctx, 0, opts)
    finally:
        M.mdwf_destroy(ctx)


def test_operator_parity_other_action(M):
    """Shamir-like and heavy-mass corner: b5 = 1, c5 = 0, m_q = 1, M5 = 1.8."""
    dims, L5 = (4, 4, 2, 2), 6
    act = oracle.Action(dims, L5, M5=1.8, b5=1.0, c5=0.0, mq=1.0)
    U = I.random_links(dims, 0.5, 43)
    psi = I.gaussian_source(dims, L5, 44)
    ctx = make_ctx(M, act, U)
    try:
        for op in ALL_OPS:
            assert rel(gpu_op(M, ctx, op, 0, act, psi), oracle_op(M, op, act, U, psi)) <= 1e-13
    finally:
        M.mdwf_destroy(ctx)


def test_dev_entry_points_roundtrip(M):
    """pack -> apply_dev -> unpack on device buffers equals the host path."""
    import torch
    dims, L5 = (6, 4, 2, 6), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 45)
    psi = I.gaussian_source(dims, L5, 46)
    ctx = make_ctx(M, act, U)
    try:
        dev = torch.device("cuda:0")
        side = torch.cuda.Stream(device=dev)
        torch.cuda.set_stream(side)
        for prec in (0, 1, 2):
            nb = M.mdwf_field_bytes(ctx, prec, M.MDWF_FULL)
            a = torch.empty(nb, dtype=torch.uint8, device=dev)
            b = torch.empty(nb, dtype=torch.uint8, device=dev)
            canon = torch.from_numpy(psi.view(np.float64).copy()).to(dev)
            outc = torch.empty_like(canon)
            stream = torch.cuda.current_stream().cuda_stream
            M.mdwf_pack_dev(ctx, prec, M.MDWF_FULL, canon.data_ptr(), a.data_ptr(), stream)
            M.mdwf_apply_dev(ctx, M.MDWF_OP_D5, prec, a.data_ptr(), b.data_ptr(), stream)
            M.mdwf_unpack_dev(ctx, prec, M.MDWF_FULL, b.data_ptr(), outc.data_ptr(), stream)
            torch.cuda.synchronize()
            got = outc.cpu().numpy().view(np.complex128).reshape(psi.shape)
            assert rel(got, oracle.D5(act, U, psi)) <= TOL[prec]
    finally:
        torch.cuda.set_stream(torch.cuda.default_stream())
        M.mdwf_destroy(ctx)


def test_fp16_store_of_sites_below_float_range(M):
    """A 5D site whose largest component is below the smallest normal float
    is stored as zero in FP16 (its norm's reciprocal would overflow and turn
    zero components into NaN); ordinary sites keep their per-site precision."""
    import torch
    dims, L5 = (4, 2, 2, 2), 4
    act = oracle.Action(dims, L5)
    ctx = make_ctx(M, act, I.unit_links(dims))
    try:
        psi = I.gaussian_source(dims, L5, 48)
        psi[1, 0, 0, 0, 0] *= 1e-40      # denormal in FP32
        psi[2, 1, 1, 1, 3] = 0.0          # an all-zero site
        psi[2, 1, 1, 1, 3, 0, 0] = 3e-39  # one denormal component
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            canon = torch.from_numpy(psi.view(np.float64).copy()).cuda()
            nat = torch.empty(M.mdwf_field_bytes(ctx, 2, M.MDWF_FULL), dtype=torch.uint8, device="cuda")
            back = torch.empty_like(canon)
            M.mdwf_pack_dev(ctx, 2, M.MDWF_FULL, canon.data_ptr(), nat.data_ptr(), side.cuda_stream)
            M.mdwf_unpack_dev(ctx, 2, M.MDWF_FULL, nat.data_ptr(), back.data_ptr(), side.cuda_stream)
        torch.cuda.synchronize()
        got = back.cpu().numpy().view(np.complex128).reshape(psi.shape)
        assert np.all(np.isfinite(got))
        assert np.all(got[1, 0, 0, 0, 0] == 0) and np.all(got[2, 1, 1, 1, 3] == 0)
        mask = np.ones(psi.shape[:5], bool)
        mask[1, 0, 0, 0, 0] = mask[2, 1, 1, 1, 3] = False
        site_max = np.abs(np.stack([psi.real, psi.imag])).max(axis=(0, 6, 7))
        err = np.abs(got - psi).max(axis=(5, 6))
        assert np.all(err[mask] <= 2 ** -11 * site_max[mask] * 1.0001)
    finally:
        M.mdwf_destroy(ctx)


@pytest.mark.parametrize("op", ["D5", "SCHUR"])
def test_fp16_prehop_wall_coupling_of_tiny_slice(M, op):
    """FP16 kernels that apply B before the hop rescale the three slices they
    combine by S = max(b5 n_s, c5 |f| n_s-1, c5 |f| n_s+1).  A site whose only
    non-zero slice is s = L5-1 with norm 8e-36 makes S = c5 m_q n = 2e-39 on
    slice 0 (wall coupling f = -m_q), whose reciprocal overflows FP32; the
    result must stay finite and match.  (Outputs below the smallest normal
    float are stored as zero; at this scale they are 3e-4 of the largest.)"""
    dims, L5 = (4, 4, 2, 4), 8
    act = oracle.Action(dims, L5, mq=0.0005)
    U = I.random_links(dims, 0.3, 51)
    psi = np.zeros(act.shape5, complex)
    rng = np.random.default_rng(52)
    for x in ((0, 0, 0, 0), (1, 0, 0, 0)):   # one site of each parity (x fastest)
        v = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi[L5 - 1, x[3], x[2], x[1], x[0]] = 8e-36 * v / np.abs(np.stack([v.real, v.imag])).max()
    code = getattr(M, "MDWF_OP_" + op)
    ctx = make_ctx(M, act, U)
    try:
        out = gpu_op(M, ctx, code, 2, act, psi)
        ref = oracle_op(M, code, act, U, psi)
        assert np.all(np.isfinite(out))
        assert rel(out, ref) <= TOL[2]
    finally:
        M.mdwf_destroy(ctx)


# ---------------------------------------------------------------- solver

CFG1 = dict(dims=(4, 4, 4, 8), L5=8, M5=1.3, b5=1.5, c5=0.5, mq=0.05, eps=0.3, gseed=101, sseed=301)


@pytest.fixture(scope="module")
def cfg1():
    c = CFG1
    act = oracle.Action(c["dims"], c["L5"], M5=c["M5"], b5=c["b5"], c5=c["c5"], mq=c["mq"])
    U = I.random_links(c["dims"], c["eps"], c["gseed"])
    b = I.gaussian_source(c["dims"], c["L5"], c["sseed"])
    x_ref, info = oracle.solve(act, U, b, tol=1e-12)
    assert info["status"] == 0
    return act, U, b, x_ref


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "f32_inner", "f16_inner"])
def test_solve_matches_oracle(M, cfg1, inner):
    act, U, b, x_ref = cfg1
    ctx = make_ctx(M, act, U)
    try:
        x = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(tol=1e-10, inner=inner, max_iter=20000))
        assert st == M.MDWF_OK, info
        tr = oracle.true_residual(act, U, b, x)
        assert tr <= 1e-10, (tr, info)
        assert abs(tr - info[0]["true_resid"]) <= 1e-11
        assert rel(x, x_ref) <= 1e-7
        if inner:
            assert info[0]["reliable_updates"] >= 1
    finally:
        M.mdwf_destroy(ctx)


@pytest.mark.parametrize("inner,form", [(0, 0), (2, 2)], ids=["f64_asym", "f16_inner_rp"])
def test_solve_with_long_fifth_dimension(M, inner, form):
    """L5 = 16 on 4^4 (four sites per wavefront, dense L5 x L5 polynomials of
    sixteen terms): the solution's true residual by the oracle's operator
    is at most 1e-10."""
    dims, L5 = (4, 4, 4, 4), 16
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 61)
    b = I.gaussian_source(dims, L5, 62)
    ctx = make_ctx(M, act, U)
    try:
        x = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(tol=1e-10, inner=inner, max_iter=20000, schur_form=form))
        assert st == M.MDWF_OK, info
        tr = oracle.true_residual(act, U, b, x)
        assert tr <= 1e-10, (tr, info)
        assert abs(tr - info[0]["true_resid"]) <= 1e-11
    finally:
        M.mdwf_destroy(ctx)


@pytest.mark.parametrize("inner", [0, 1, 2], ids=["f64", "f32_inner", "f16_inner"])
@pytest.mark.parametrize("form", [1, 2], ids=["sym", "rp"])
def test_other_schur_forms_solve_matches_oracle(M, cfg1, inner, form):
    """CG on K5^-1 S x_e = K5^-1 b'_e (Sec. VII's symmetric form) or on
    S B^-1 y = b'_e (right preconditioning by B) reaches the same solution:
    true residual by the oracle's operator at most 1e-10."""
    act, U, b, x_ref = cfg1
    ctx = make_ctx(M, act, U)
    try:
        x = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(tol=1e-10, inner=inner, max_iter=20000, schur_form=form))
        assert st == M.MDWF_OK, info
        tr = oracle.true_residual(act, U, b, x)
        assert tr <= 1e-10, (tr, info)
        assert abs(tr - info[0]["true_resid"]) <= 1e-11
        assert rel(x, x_ref) <= 1e-7
    finally:
        M.mdwf_destroy(ctx)


def test_schur_forms_with_graph_and_shamir_action(M):
    """Shamir action (b5 = 1, c5 = 0), where K5 is far from a multiple of 1:
    every Schur form solves to 1e-10 with the graph-replayed iteration and
    the results match the asymmetric solve's."""
    dims, L5 = (4, 4, 4, 8), 8
    act = oracle.Action(dims, L5, M5=1.5, b5=1.0, c5=0.0, mq=0.02)
    U = I.random_links(dims, 0.3, 48)
    b = I.gaussian_source(dims, L5, 49)
    ctx = make_ctx(M, act, U)
    try:
        xs = {}
        for form in (0, 1, 2):
            x = np.zeros_like(b)
            st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(inner=2, use_graph=1, schur_form=form))
            assert st == M.MDWF_OK, info
            assert oracle.true_residual(act, U, b, x) <= 1e-10
            xs[form] = x
        assert rel(xs[1], xs[0]) <= 1e-7 and rel(xs[2], xs[0]) <= 1e-7
        with pytest.raises(M.MdwfError):
            M.mdwf_solve(ctx, [b], [np.zeros_like(b)], opts=dict(schur_form=3))
    finally:
        M.mdwf_destroy(ctx)


def _free_d5(p, L5, M5, b5, c5, mq):
    """D5(p) = D_W(p)(b5 + c5 C) + 1 - C on C^{4 L5} for unit links, with
    D_W(p) = 4 - M5 - sum cos p_mu + i sum gamma_mu sin p_mu (colour trivial)."""
    import kron_ref as KR
    g = KR.gammas()
    dw = (4 - M5 - np.cos(p).sum()) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
    Sp, Sm = KR.c5_matrix(L5, mq)
    Cm = np.kron(Sp, KR.PPLUS) + np.kron(Sm, KR.PMINUS)
    Id = np.eye(4 * L5)
    return np.kron(np.eye(L5), dw) @ (b5 * Id + c5 * Cm) + Id - Cm


@pytest.mark.parametrize("form", [0, 1, 2], ids=["asym", "sym", "rp"])
def test_free_field_plane_wave_solve_closed_form(M, form):
    """Unit links, b = e^{ipx} chi on 8^3 x 16, L5 = 8, m = 0.0102, FP16
    inner: the solution equals e^{ipx} D5(p)^-1 chi to within the condition
    number of D5 (exact over every momentum of the lattice) times 1e-10."""
    dims, L5 = (8, 8, 8, 16), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.0102)
    X, Y, Z, T = dims
    n = (1, 3, 0, 2)
    p = np.array([2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z, (2 * n[3] + 1) * np.pi / T])
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(17)
    chi = rng.standard_normal((L5, 4, 3)) + 1j * rng.standard_normal((L5, 4, 3))
    b = np.ascontiguousarray(ph[None, ..., None, None] * chi[:, None, None, None, None])
    Dp = _free_d5(p, L5, 1.3, 1.5, 0.5, 0.0102)
    xc = np.linalg.solve(Dp, chi.reshape(L5 * 4, 3)).reshape(L5, 4, 3)
    ref = ph[None, ..., None, None] * xc[:, None, None, None, None]
    # condition number of D5 on this lattice: extreme singular values over all momenta
    smax, smin = 0.0, np.inf
    for nt in range(T):
        for nz in range(Z):
            for ny in range(Y):
                ps = np.stack(np.meshgrid(2 * np.pi * np.arange(X) / X, [2 * np.pi * ny / Y], [2 * np.pi * nz / Z],
                                          [(2 * nt + 1) * np.pi / T], indexing="ij"), -1).reshape(-1, 4)
                sv = np.linalg.svd(np.array([_free_d5(q, L5, 1.3, 1.5, 0.5, 0.0102) for q in ps]), compute_uv=False)
                smax, smin = max(smax, sv.max()), min(smin, sv.min())
    kappa = smax / smin
    ctx = make_ctx(M, act, I.unit_links(dims))
    try:
        xg = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b], [xg], opts=dict(inner=2, schur_form=form))
        assert st == M.MDWF_OK, info
        assert oracle.true_residual(act, I.unit_links(dims), b, xg) <= 1e-10
        assert rel(xg, ref) <= kappa * 1e-10, (rel(xg, ref), kappa)
    finally:
        M.mdwf_destroy(ctx)


def test_solve_graph_replay_matches_eager(M, cfg1):
    act, U, b, _ = cfg1
    ctx = make_ctx(M, act, U)
    try:
        xs = []
        for g in (0, 1, 1):
            x = np.zeros_like(b)
            st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(inner=1, use_graph=g))
            assert st == M.MDWF_OK
            xs.append((x, info[0]["iters"]))
        for x, it in xs[1:]:
            assert it == xs[0][1]
            assert np.array_equal(x, xs[0][0])
    finally:
        M.mdwf_destroy(ctx)


def test_solve_launch_timing_changes_nothing(M, cfg1):
    """profile_iters records HIP events around the batched hop launches of a
    few iterations: positive durations, and the solution is bit-identical."""
    act, U, b, _ = cfg1
    bs = [b, 0.5 * b]
    ctx = make_ctx(M, act, U)
    try:
        out = []
        for prof in (0, 3):
            xs = [np.zeros_like(v) for v in bs]
            st, info = M.mdwf_solve(ctx, bs, xs, opts=dict(inner=2, profile_iters=prof))
            assert st == M.MDWF_OK
            out.append((xs, info))
        (x0, i0), (x1, i1) = out
        assert all(np.array_equal(a, c) for a, c in zip(x0, x1))
        assert i0[0]["hop_samples"] == 0 and i0[0]["hop_us"] == [0.0] * 4
        assert i1[0]["hop_samples"] == 3 and i1[0]["hop_rhs"] == 2
        assert all(u > 0.0 for u in i1[0]["hop_us"])
    finally:
        M.mdwf_destroy(ctx)


@pytest.mark.parametrize("form", [0, 1, 2], ids=["asym", "sym", "rp"])
def test_multi_rhs_multi_mass_equals_single(M, form):
    """Point-source columns at three masses in one launch; each equals its solo solve."""
    dims, L5 = (4, 4, 4, 8), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 47)
    site = I.random_point_site(dims, 404)
    cols = I.point_source_columns(dims, L5, site)
    bs = [cols[0], cols[7], cols[11], cols[4]]
    masses = [0.05, 0.02, 0.1, 0.04]
    ctx = make_ctx(M, act, U)
    try:
        for inner in (0, 2):
            xs = [np.zeros_like(b) for b in bs]
            st, info = M.mdwf_solve(ctx, bs, xs, mq=masses, opts=dict(inner=inner, schur_form=form))
            assert st == M.MDWF_OK
            for k, b in enumerate(bs):
                a_k = act.with_mass(masses[k])
                assert oracle.true_residual(a_k, U, b, xs[k]) <= 1e-10
                x1 = np.zeros_like(b)
                st1, info1 = M.mdwf_solve(ctx, [b], [x1], mq=[masses[k]], opts=dict(inner=inner, schur_form=form))
                assert st1 == M.MDWF_OK
                assert info1[0]["iters"] == info[k]["iters"]
                assert np.array_equal(x1, xs[k]), "RHS %d differs alone vs batched" % k
    finally:
        M.mdwf_destroy(ctx)


def test_multi_rhs_chunked_schur_is_bitwise_identical(M, monkeypatch):
    """Splitting the RHS into chunks that share the hop temporary, or the
    batch into sub-batches solved in turn, changes no bit."""
    dims, L5 = (4, 4, 4, 8), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 53)
    bs = [I.gaussian_source(dims, L5, 60 + k) for k in range(5)]
    masses = [0.05, 0.03, 0.08, 0.05, 0.2]
    ctx = make_ctx(M, act, U)
    try:
        res = []
        for chunk, batch in ((None, None), ("2", None), ("1", None), (None, "2")):
            monkeypatch.delenv("MDWF_SOLVE_CHUNK", raising=False)
            if chunk:
                monkeypatch.setenv("MDWF_SOLVE_CHUNK", chunk)
            if batch:   # sub-batches of 2, 2, 1 RHS solved in turn
                monkeypatch.setenv("MDWF_SOLVE_BATCH", batch)
            xs = [np.zeros_like(b) for b in bs]
            st, info = M.mdwf_solve(ctx, bs, xs, mq=masses, opts=dict(inner=2))
            assert st == M.MDWF_OK
            res.append((xs, [i["iters"] for i in info]))
        for xs, its in res[1:]:
            assert its == res[0][1]
            for a, b in zip(xs, res[0][0]):
                assert np.array_equal(a, b)
        for k, b in enumerate(bs):
            assert oracle.true_residual(act.with_mass(masses[k]), U, b, res[0][0][k]) <= 1e-10
    finally:
        M.mdwf_destroy(ctx)


def test_multi_rhs_group_order_is_bitwise_identical(M, monkeypatch):
    """The order in which RHS groups sweep the tiles (rhs_group) changes no bit."""
    dims, L5 = (4, 4, 4, 8), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 54)
    bs = [I.gaussian_source(dims, L5, 70 + k) for k in range(5)]
    masses = [0.05, 0.03, 0.08, 0.05, 0.2]
    res = []
    for rg in ("0", "1", "2", "3"):
        monkeypatch.setenv("MDWF_RHS_GROUP", rg)
        ctx = make_ctx(M, act, U)
        try:
            assert M.mdwf_get_tune(ctx, 2)["rhs_group"] == int(rg)
            xs = [np.zeros_like(b) for b in bs]
            st, info = M.mdwf_solve(ctx, bs, xs, mq=masses, opts=dict(inner=2))
            assert st == M.MDWF_OK
            res.append((xs, [i["iters"] for i in info]))
        finally:
            M.mdwf_destroy(ctx)
    for xs, its in res[1:]:
        assert its == res[0][1]
        assert all(np.array_equal(a, b) for a, b in zip(xs, res[0][0]))


def test_solve_dev_with_torch_buffers(M, cfg1):
    import torch
    act, U, b, x_ref = cfg1
    ctx = make_ctx(M, act, U)
    try:
        dev = torch.device("cuda:0")
        side = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(side):
            bt = torch.from_numpy(b.view(np.float64).copy()).to(dev)
            xt = torch.zeros_like(bt)
            st, info = M.mdwf_solve_dev(ctx, [bt.data_ptr()], [xt.data_ptr()], opts=dict(inner=2),
                                        stream=side.cuda_stream)
        torch.cuda.synchronize()
        assert st == M.MDWF_OK
        x = xt.cpu().numpy().view(np.complex128).reshape(b.shape)
        assert oracle.true_residual(act, U, b, x) <= 1e-10
    finally:
        M.mdwf_destroy(ctx)


def test_solve_is_deterministic(M, cfg1):
    """The same solve twice (and the same operator twice) gives bitwise the
    same result: every reduction runs in a fixed order."""
    act, U, b, _ = cfg1
    ctx = make_ctx(M, act, U)
    try:
        xs = []
        for _ in range(2):
            x = np.zeros_like(b)
            st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(inner=2, schur_form=2))
            assert st == M.MDWF_OK
            xs.append((x, info[0]["iters"], info[0]["true_resid"]))
        assert np.array_equal(xs[0][0], xs[1][0]) and xs[0][1:] == xs[1][1:]
        for prec in (0, 1, 2):
            outs = [gpu_op(M, ctx, M.MDWF_OP_SCHUR_RP, prec, act, b) for _ in range(2)]
            assert np.array_equal(outs[0], outs[1])
    finally:
        M.mdwf_destroy(ctx)


def test_solve_time_limit(M, cfg1):
    """max_seconds stops an unconverged solve as max_iter does: ERR_NOCONV,
    the best x written, its true residual reported."""
    act, U, b, _ = cfg1
    ctx = make_ctx(M, act, U)
    try:
        x = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b, b], [x, np.zeros_like(b)], opts=dict(inner=2, max_seconds=1e-4))
        assert st == M.MDWF_ERR_NOCONV
        assert info[0]["true_resid"] > 1e-10 and np.all(np.isfinite(x)) and np.any(x != 0)
        assert abs(oracle.true_residual(act, U, b, x) - info[0]["true_resid"]) <= 1e-9
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(inner=2, max_seconds=60.0))
        assert st == M.MDWF_OK and info[0]["true_resid"] <= 1e-10
        with pytest.raises(M.MdwfError) as e:
            M.mdwf_solve(ctx, [b], [x], opts=dict(max_seconds=-1.0))
        assert e.value.status == M.MDWF_ERR_ARG
    finally:
        M.mdwf_destroy(ctx)


def test_solver_failure_paths(M, cfg1):
    act, U, b, _ = cfg1
    ctx = M.mdwf_create(act.dims)
    try:
        x = np.zeros_like(b)
        with pytest.raises(M.MdwfError) as e:
            M.mdwf_solve(ctx, [b], [x])
        assert e.value.status == M.MDWF_ERR_STATE
        M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, act.L5)
        with pytest.raises(M.MdwfError) as e:
            M.mdwf_apply(ctx, M.MDWF_OP_D5, 0, b, x)
        assert e.value.status == M.MDWF_ERR_STATE
        M.mdwf_load_gauge(ctx, U)
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(max_iter=3))
        assert st == M.MDWF_ERR_NOCONV and info[0]["iters"] >= 3
        assert info[0]["true_resid"] > 1e-10
        bad = b.copy()
        bad[0, 0, 0, 0, 0, 0, 0] = np.nan
        st, info = M.mdwf_solve(ctx, [bad], [x])
        assert st == M.MDWF_ERR_NUMERIC
        zero = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [zero], [x])
        assert st == M.MDWF_OK and np.all(x == 0)
        with pytest.raises(M.MdwfError) as e:
            M.mdwf_solve(ctx, [b], [x], opts=dict(tol=-1.0))
        assert e.value.status == M.MDWF_ERR_ARG
        with pytest.raises(M.MdwfError) as e:
            M.mdwf_set_action(ctx, 1.3, 0.5, 0.5, 0.05, 8)
        assert e.value.status == M.MDWF_ERR_ARG
    finally:
        M.mdwf_destroy(ctx)


def test_action_rejects_fields_beyond_32bit_offsets(M):
    """The kernels address a field block with 32-bit byte offsets, so an
    action whose L5 x V/2 reaches 2^28 is refused (48^3 x 160 holds
    V/2 = 8847360 sites: L5 = 32 is over, L5 = 30 under)."""
    ctx = M.mdwf_create((48, 48, 48, 160))
    try:
        with pytest.raises(M.MdwfError) as e:
            M.mdwf_set_action(ctx, 1.3, 1.5, 0.5, 0.05, 32)
        assert e.value.status == M.MDWF_ERR_ARG and "32-bit" in str(e.value)
        M.mdwf_set_action(ctx, 1.3, 1.5, 0.5, 0.05, 30)
    finally:
        M.mdwf_destroy(ctx)
