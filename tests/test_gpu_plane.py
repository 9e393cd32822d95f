"""Parity of the plane-staged bare hop (launch option plane_bt) with the FP64
oracle and with the lane-per-site kernel, through the C ABI: the hop
between the 4D parities on every slice and its adjoint, FP32 and FP16, on
lattices where 4x4x4 blocks wrap onto themselves (extent 4), with several
time-plane runs and L5 from 4 to 12 (workgroups of 128 to 448 threads).
Where a plane's buffer does not fit in LDS the launch falls back to the
lane-per-site kernel, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1701_07559_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = {1: 1e-6, 2: 5e-3}
# dims, L5, plane_bt, antiperiodic t
CASES = [
    ((8, 8, 8, 8), 8, 4, True),
    ((4, 8, 4, 6), 8, 3, True),
    ((8, 4, 12, 4), 4, 4, False),
    ((8, 4, 4, 8), 12, 8, True),
    ((4, 4, 4, 2), 6, 2, True),
]


def plane_applies(prec, L5, lds_limit=160 * 1024):
    """Whether the plane-staged kernel runs for this precision and L5: a
    workgroup of 128..512 threads and a plane's LDS buffer that fits."""
    spw = 64 // L5
    nthreads = 64 * -(-32 // spw)
    site, link = (96, 72) if prec == 1 else (52, 36)
    lds = 80 * site * L5 + 256 * link + 2 * 80 * 4
    return 128 <= nthreads <= 512 and L5 <= 16 and lds <= lds_limit


@pytest.fixture(scope="module")
def M():
    from paper_1701_07559_amd import mdwf
    try:
        ctx = mdwf.mdwf_create((2, 2, 2, 2))
    except mdwf.MdwfError as e:
        pytest.skip("no HIP device: %s" % e)
    mdwf.mdwf_destroy(ctx)
    return mdwf


def half(psi, dims, parity):
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return np.ascontiguousarray(psi[:, ((x + y + z + t) % 2) == parity])


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])) + "_L%d_bt%d" % (c[1], c[2]))
@pytest.mark.parametrize("prec", [1, 2], ids=["f32", "f16"])
def test_plane_staged_hop_parity(M, case, prec):
    dims, L5, bt, ap = case
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05, antiperiodic_t=ap)
    U = I.random_links(dims, 0.3, 51)
    psi = I.gaussian_source(dims, L5, 52)
    ctx = M.mdwf_create(dims, antiperiodic_t=ap)
    try:
        M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, L5)
        M.mdwf_load_gauge(ctx, U)
        base = M.mdwf_get_tune(ctx, prec)
        assert base["plane_bt"] == 0
        V = int(np.prod(dims))
        for op, out_par, dag in ((M.MDWF_OP_HOP_EO, 0, False), (M.MDWF_OP_HOP_OE, 1, False),
                                 (M.MDWF_OP_HOP_EO_DAG, 0, True), (M.MDWF_OP_HOP_OE_DAG, 1, True)):
            inp = half(psi, dims, 1 - out_par)
            ref = half(oracle.hop(act, U, psi, out_par, dag=dag), dims, out_par)
            lane = np.zeros((L5, V // 2, 4, 3), complex)
            M.mdwf_set_tune(ctx, prec, dict(base, plane_bt=0))
            M.mdwf_apply(ctx, op, prec, inp, lane)
            plane = np.zeros_like(lane)
            M.mdwf_set_tune(ctx, prec, dict(base, plane_bt=bt))
            print("[plane] %s L5 %d bt %d prec %d op %d" % (dims, L5, bt, prec, op), flush=True)
            M.mdwf_apply(ctx, op, prec, inp, plane)
            assert M.mdwf_get_tune(ctx, prec)["plane_bt"] == bt
            e_plane = np.linalg.norm(plane - ref) / np.linalg.norm(ref)
            e_lane = np.linalg.norm(lane - ref) / np.linalg.norm(ref)
            assert e_plane <= TOL[prec], "op %d: plane-staged %.3e (lane-per-site %.3e)" % (op, e_plane, e_lane)
            # both kernels round the same terms; only the summation order
            # differs (so the plane-staged kernel did run: not bitwise equal)
            assert np.linalg.norm(plane - lane) / np.linalg.norm(ref) <= 2 * TOL[prec]
            # where it does not fit, the lane-per-site kernel runs instead
            assert np.array_equal(plane, lane) != plane_applies(prec, L5)
    finally:
        M.mdwf_destroy(ctx)


def test_set_tune_rejects_bad_shapes(M):
    ctx = M.mdwf_create((4, 4, 4, 6))
    try:
        M.mdwf_set_action(ctx, 1.3, 1.5, 0.5, 0.05, 4)
        t = M.mdwf_get_tune(ctx, 1)
        with pytest.raises(M.MdwfError):
            M.mdwf_set_tune(ctx, 1, dict(t, plane_bt=4))     # does not divide T = 6
        with pytest.raises(M.MdwfError):
            M.mdwf_set_tune(ctx, 1, dict(t, tile=[2, 4, 4, 4]))  # 4 does not divide T = 6
        M.mdwf_set_tune(ctx, 1, dict(t, plane_bt=3))
        assert M.mdwf_get_tune(ctx, 1)["plane_bt"] == 3
    finally:
        M.mdwf_destroy(ctx)
