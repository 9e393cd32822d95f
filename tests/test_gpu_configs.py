"""Parity at the other two one-GPU configurations the benchmark runs, at
their full sizes and in the launch configurations bench.py uses.

* The a15m310 shape (16^3 x 48, L5 = 12, m = 0.0158; `bench.py --workload
  fp64`): the plain FP64 CG on S, and the FP16-inner S B^-1 solve of the
  same Gaussian source, each after the solve-shaped autotuner.  The oracle's
  own D5 gives each solution's true residual, at most 1e-10.
* The a12m220 volume (32^3 x 64, L5 = 10; `bench.py --workload batched`):
  the batched FP16 S B^-1 and its adjoint on 12 RHS of three masses in one
  launch set (one source field), after the solve-shaped autotuner for 12
  RHS, against the oracle's site-by-site S B^-1 at sampled sites (both time
  boundaries, the x wrap, random sites), as a per-site relative error.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1701_07559_amd import inputs as I

pytestmark = pytest.mark.gpu

WORKERS = min(16, os.cpu_count() or 1)
ACT = dict(M5=1.3, b5=1.5, c5=0.5)


def _device_or_skip():
    from paper_1701_07559_amd import mdwf as M
    try:
        ctx = M.mdwf_create((2, 2, 2, 2))
    except M.MdwfError as e:
        pytest.skip("no HIP device: %s" % e)
    M.mdwf_destroy(ctx)
    return M


def sample_sites(dims, n_random=8, seed=13):
    X, Y, Z, T = dims
    pts = [(0, 0, 0, 0), (X - 1, Y - 1, Z - 1, T - 1), (0, 5, 3, T - 1), (X - 1, 0, 4, 0),
           (3, Y - 1, 7, T // 2), (1, 1, Z // 2, T - 1)]
    rng = np.random.default_rng(seed)
    pts += [tuple(int(rng.integers(0, d)) for d in dims) for _ in range(n_random)]
    out = []
    for x, y, z, t in pts:
        if (x + y + z + t) % 2:
            x = (x + 1) % X
        out.append(x + X * (y + Y * (z + Z * t)))
    return np.array(sorted(set(out)), dtype=np.int64)


@pytest.mark.parametrize("inner,form", [(0, 0), (2, 2)], ids=["f64_S", "f16_inner_SBinv"])
def test_a15m310_shape_solve_certified_by_oracle(inner, form):
    M = _device_or_skip()
    dims, L5 = (16, 16, 16, 48), 12
    act = oracle.Action(dims, L5, mq=0.0158, **ACT)
    print("[configs] a15m310 shape, inner %d form %d" % (inner, form), flush=True)
    U = I.random_links(dims, 0.25, 102, workers=WORKERS)
    b = I.gaussian_source(dims, L5, 302)
    ctx = M.mdwf_create(dims)
    try:
        M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, L5)
        M.mdwf_load_gauge(ctx, U)
        M.mdwf_autotune_solve(ctx, 1, dict(inner=inner, schur_form=form))
        x = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(tol=1e-10, inner=inner, schur_form=form))
        assert st == M.MDWF_OK, info
    finally:
        M.mdwf_destroy(ctx)
    oracle.use_threads(WORKERS)
    try:
        tr = oracle.true_residual(act, U, b, x)
    finally:
        oracle.use_threads(1)
    assert tr <= 1e-10, tr
    assert abs(tr - info[0]["true_resid"]) <= 1e-3 * tr, (tr, info[0]["true_resid"])


@pytest.fixture(scope="module")
def batched_ctx():
    import torch
    M = _device_or_skip()
    dims, L5 = (32, 32, 32, 64), 10
    act = oracle.Action(dims, L5, mq=0.0074, **ACT)
    print("[configs] links 32^3x64 seed 104", flush=True)
    U = I.random_links(dims, 0.25, 104, workers=WORKERS)
    dev = torch.device("cuda:0")
    work = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(work)
    ctx = M.mdwf_create(dims, hip_stream=work.cuda_stream)
    M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, L5)
    M.mdwf_load_gauge(ctx, U)
    print("[configs] autotune_solve nrhs 12 f16 rp", flush=True)
    M.mdwf_autotune_solve(ctx, 12, dict(inner=M.MDWF_F16, schur_form=2))
    fields = [I.gaussian_source(dims, L5, 404)]
    yield M, torch, ctx, act, U, work, fields
    torch.cuda.synchronize()
    M.mdwf_destroy(ctx)
    torch.cuda.set_stream(torch.cuda.default_stream(dev))


@pytest.mark.parametrize("dag", [False, True], ids=["SBinv", "BinvdagSdag"])
def test_a12m220_volume_batched_operator_sampled_sites(batched_ctx, dag):
    M, torch, ctx, act, U, work, fields = batched_ctx
    dims, L5, nrhs, prec = act.dims, act.L5, 12, M.MDWF_F16
    masses = (0.0074, 0.02, 0.04)
    dev = torch.device("cuda:0")
    op = M.MDWF_OP_SCHUR_RP_DAG if dag else M.MDWF_OP_SCHUR_RP
    st = work.cuda_stream
    even = oracle.even_mask(dims)
    hb = M.mdwf_field_bytes(ctx, prec, M.MDWF_HALF_EVEN)
    stride = (hb + 255) // 256 * 256
    nat_in = torch.zeros(nrhs * stride, dtype=torch.uint8, device=dev)
    nat_out = torch.zeros(nrhs * stride, dtype=torch.uint8, device=dev)
    canon = [torch.from_numpy(np.ascontiguousarray(f[:, even]).view(np.float64).ravel()).to(dev) for f in fields]
    rhs_field = [0] * nrhs
    rhs_mass = [masses[k % 3] for k in range(nrhs)]
    for k in range(nrhs):
        M.mdwf_pack_dev(ctx, prec, M.MDWF_HALF_EVEN, canon[rhs_field[k]].data_ptr(),
                        nat_in.data_ptr() + k * stride, st)
    print("[configs] batched op %d, 12 RHS" % op, flush=True)
    M.mdwf_apply_batch_dev(ctx, op, prec, nrhs, nat_in.data_ptr(), nat_out.data_ptr(), stride, mq=rhs_mass,
                           stream=st)
    sites = sample_sites(dims)
    hidx = torch.from_numpy(sites // 2).to(dev)
    out_c = torch.empty_like(canon[0])
    oracle.use_threads(WORKERS)
    try:
        # each mass once, and the last RHS of the launch
        for k in (0, 1, 2, 11):
            M.mdwf_unpack_dev(ctx, prec, M.MDWF_HALF_EVEN, nat_out.data_ptr() + k * stride, out_c.data_ptr(), st)
            got = out_c.view(L5, -1, 24)[:, hidx].cpu().numpy()
            got = got.view(np.complex128).reshape(L5, len(sites), 4, 3).transpose(1, 0, 2, 3)
            print("[configs] oracle S B^-1 at %d sites, RHS %d" % (len(sites), k), flush=True)
            ref = oracle.schur_rp_sites(act.with_mass(rhs_mass[k]), U, fields[rhs_field[k]], sites, dag=dag)
            num = np.linalg.norm((got - ref).reshape(len(sites), L5, -1), axis=2)
            den = np.linalg.norm(ref.reshape(len(sites), L5, -1), axis=2)
            e = float(np.max(num / den))
            assert e <= 5e-3, "RHS %d (field %d, m %g): worst per-site error %.3e" % (
                k, rhs_field[k], rhs_mass[k], e)
    finally:
        oracle.use_threads(1)
