"""The benchmark's own operator and solve at full size (24^3 x 64, L5 = 8),
in the launch configuration the benchmark times.

* The CG operator of the benchmark's mixed solve, S B^-1, and its adjoint
  B^-+ S^+, on 12 right-hand sides in one batched launch set (each with its
  own field and mass), in FP16 and FP32, after the solve-shaped autotuner has
  installed the launch shape the solve uses.  At sampled sites (both time
  boundaries, the x wrap, tile edges, random sites) every 5D site must agree
  with the oracle's site-by-site evaluation to the dslash tolerance, as a
  per-site relative error (not a norm over the sample).
* The benchmark's solve itself (12 point-source columns, FP16 inner, S B^-1)
  is certified by the oracle: the oracle's own D5 gives the true residual of
  four of the returned columns, which must be at most 1e-10.
* The per-solve error against the FP64 solution (err_vs_ref) equals the
  norm the test computes from both solutions.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1701_07559_amd import inputs as I

pytestmark = pytest.mark.gpu

DIMS, L5 = (24, 24, 24, 64), 8
ACT = dict(M5=1.3, b5=1.5, c5=0.5, mq=0.0102)
NRHS = 12
MASSES = (0.0102, 0.02, 0.04, 0.0048)
TOL = {1: 1e-6, 2: 5e-3}
WORKERS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def bench_ctx():
    import torch
    from paper_1701_07559_amd import mdwf as M
    try:
        ctx = M.mdwf_create((2, 2, 2, 2))
    except M.MdwfError as e:
        pytest.skip("no HIP device: %s" % e)
    M.mdwf_destroy(ctx)
    act = oracle.Action(DIMS, L5, **ACT)
    print("[bench-operator] links 24^3x64 seed 103", flush=True)
    U = I.random_links(DIMS, 0.25, 103, workers=WORKERS)
    dev = torch.device("cuda:0")
    work = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(work)
    ctx = M.mdwf_create(DIMS, hip_stream=work.cuda_stream)
    M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, L5)
    M.mdwf_load_gauge(ctx, U)
    # the benchmark's launch shapes: the FP16 CG operator of S B^-1 with 12
    # RHS per launch (and FP64 with one), as bench.py tunes before its solve
    print("[bench-operator] autotune_solve nrhs 12 f16 rp", flush=True)
    tune = M.mdwf_autotune_solve(ctx, NRHS, dict(inner=M.MDWF_F16, schur_form=2))
    fields = [I.gaussian_source(DIMS, L5, 303 + j) for j in range(3)]
    yield M, torch, ctx, act, U, work, tune, fields
    torch.cuda.synchronize()
    M.mdwf_destroy(ctx)
    torch.cuda.set_stream(torch.cuda.default_stream(dev))


def sample_sites(n_random=12, seed=11):
    """Even 4D sites (lexicographic) at the boundaries, tile edges and random places."""
    X, Y, Z, T = DIMS
    pts = [(0, 0, 0, 0), (X - 1, Y - 1, Z - 1, T - 1), (0, 5, 3, T - 1), (X - 1, 0, 4, 0),
           (3, Y - 1, 7, 31), (12, 11, 5, 32), (11, 12, 6, 33), (7, 2, 23, 1), (1, 1, 12, 63)]
    rng = np.random.default_rng(seed)
    pts += [tuple(int(rng.integers(0, d)) for d in DIMS) for _ in range(n_random)]
    out = []
    for x, y, z, t in pts:
        if (x + y + z + t) % 2:
            x = (x + 1) % X
        out.append(x + X * (y + Y * (z + Z * t)))
    return np.array(sorted(set(out)), dtype=np.int64)


@pytest.mark.parametrize("prec", [2, 1], ids=["f16", "f32"])
@pytest.mark.parametrize("dag", [False, True], ids=["SBinv", "BinvdagSdag"])
def test_benchmark_operator_batched_sampled_sites(bench_ctx, prec, dag):
    M, torch, ctx, act, U, work, tune, fields = bench_ctx
    dev = torch.device("cuda:0")
    op = M.MDWF_OP_SCHUR_RP_DAG if dag else M.MDWF_OP_SCHUR_RP
    st = work.cuda_stream
    print("[bench-operator] op %d prec %d, 12 RHS, tile %s" % (op, prec, tune[prec]["tile"]), flush=True)
    even = oracle.even_mask(DIMS)
    hb = M.mdwf_field_bytes(ctx, prec, M.MDWF_HALF_EVEN)
    stride = (hb + 255) // 256 * 256
    nat_in = torch.zeros(NRHS * stride, dtype=torch.uint8, device=dev)
    nat_out = torch.zeros(NRHS * stride, dtype=torch.uint8, device=dev)
    canon = [torch.from_numpy(np.ascontiguousarray(f[:, even]).view(np.float64).ravel()).to(dev) for f in fields]
    rhs_field = [k % 3 for k in range(NRHS)]
    rhs_mass = [MASSES[k % 4] for k in range(NRHS)]
    for k in range(NRHS):
        M.mdwf_pack_dev(ctx, prec, M.MDWF_HALF_EVEN, canon[rhs_field[k]].data_ptr(),
                        nat_in.data_ptr() + k * stride, st)
    M.mdwf_apply_batch_dev(ctx, op, prec, NRHS, nat_in.data_ptr(), nat_out.data_ptr(), stride, mq=rhs_mass,
                           stream=st)
    sites = sample_sites()
    hidx = torch.from_numpy(sites // 2).to(dev)
    out_c = torch.empty_like(canon[0])
    worst = 0.0
    oracle.use_threads(WORKERS)   # the site oracle's full-lattice B^-1 / K5 passes, same values
    for k in range(NRHS):
        M.mdwf_unpack_dev(ctx, prec, M.MDWF_HALF_EVEN, nat_out.data_ptr() + k * stride, out_c.data_ptr(), st)
        got = out_c.view(L5, -1, 24)[:, hidx].cpu().numpy()                 # [L5, n, 24] doubles
        got = got.view(np.complex128).reshape(L5, len(sites), 4, 3).transpose(1, 0, 2, 3)
        ref = oracle.schur_rp_sites(act.with_mass(rhs_mass[k]), U, fields[rhs_field[k]], sites, dag=dag)
        num = np.linalg.norm((got - ref).reshape(len(sites), L5, -1), axis=2)
        den = np.linalg.norm(ref.reshape(len(sites), L5, -1), axis=2)
        e = float(np.max(num / den))
        worst = max(worst, e)
        assert e <= TOL[prec], "RHS %d (field %d, m %g): worst per-site error %.3e" % (
            k, rhs_field[k], rhs_mass[k], e)
    oracle.use_threads(1)
    print("[bench-operator] worst per-site relative error %.3e" % worst, flush=True)


def test_benchmark_solve_certified_by_oracle(bench_ctx):
    """The 12-column FP16-inner S B^-1 solve of the benchmark; the oracle's
    D5 gives the true residual of columns 0, 4, 8 and 11."""
    M, torch, ctx, act, U, work, tune, _ = bench_ctx
    dev = torch.device("cuda:0")
    X, Y, Z, T = DIMS
    V = X * Y * Z * T
    site = I.random_point_site(DIMS, 403)
    ncan = L5 * V * 24
    b = torch.zeros((NRHS, ncan), dtype=torch.float64, device=dev)
    xs, ys, zs, ts = site
    for k in range(NRHS):
        spin, colour = k // 3, k % 3
        s = L5 - 1 if spin < 2 else 0
        idx = ((((s * T + ts) * Z + zs) * Y + ys) * X + xs) * 12 + spin * 3 + colour
        b[k, 2 * idx] = 1.0
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    print("[bench-operator] 12-column f16 solve", flush=True)
    opts = dict(tol=1e-10, inner=M.MDWF_F16, schur_form=2)
    st, info = M.mdwf_solve_dev(ctx, [b[k].data_ptr() for k in range(NRHS)], [x[k].data_ptr() for k in range(NRHS)],
                                opts=opts, stream=work.cuda_stream)
    torch.cuda.synchronize()
    assert st == M.MDWF_OK, [i["true_resid"] for i in info]
    assert all(i["true_resid"] <= 1e-10 for i in info)
    assert all(i["err_vs_ref"] == -1.0 for i in info)
    oracle.use_threads(WORKERS)
    try:
        for k in (0, 4, 8, 11):
            bk = b[k].cpu().numpy().view(np.complex128).reshape(act.shape5)
            xk = x[k].cpu().numpy().view(np.complex128).reshape(act.shape5)
            print("[bench-operator] oracle true residual of column %d" % k, flush=True)
            tr = oracle.true_residual(act, U, bk, xk)
            assert tr <= 1e-10, "column %d: oracle true residual %.3e" % (k, tr)
            assert abs(tr - info[k]["true_resid"]) <= 1e-3 * tr, (tr, info[k]["true_resid"])
    finally:
        oracle.use_threads(1)


def test_err_vs_ref_full_size(bench_ctx):
    """err_vs_ref of the mixed solve against the plain FP64 CG solution of
    the same column equals ||x_mixed - x_fp64|| / ||x_fp64|| computed here."""
    M, torch, ctx, act, U, work, tune, _ = bench_ctx
    dev = torch.device("cuda:0")
    ncan = L5 * int(np.prod(DIMS)) * 24
    g = torch.Generator(device=dev)
    g.manual_seed(305)
    b = torch.randn(ncan, dtype=torch.float64, device=dev, generator=g)
    x64 = torch.zeros_like(b)
    xm = torch.zeros_like(b)
    st = work.cuda_stream
    s64, i64 = M.mdwf_solve_dev(ctx, [b.data_ptr()], [x64.data_ptr()], opts=dict(tol=1e-10), stream=st)
    assert s64 == M.MDWF_OK and i64[0]["true_resid"] <= 1e-10
    sm, im = M.mdwf_solve_dev(ctx, [b.data_ptr()], [xm.data_ptr()],
                              opts=dict(tol=1e-10, inner=M.MDWF_F16, schur_form=2, x_ref=[x64.data_ptr()]),
                              stream=st)
    torch.cuda.synchronize()
    assert sm == M.MDWF_OK and im[0]["true_resid"] <= 1e-10
    ref = float(torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64))
    print("[bench-operator] err_vs_ref %.3e (recomputed %.3e)" % (im[0]["err_vs_ref"], ref), flush=True)
    assert im[0]["err_vs_ref"] >= 0.0
    assert abs(im[0]["err_vs_ref"] - ref) <= 1e-9 * ref + 1e-18
