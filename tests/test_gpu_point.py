"""Point-source propagator solves: the sources generated on the device and
only the 4D wall fields q = P- x_0 + P+ x_{L5-1} returned (mdwf_solve_point,
mdwf_server_submit_point).

* Bitwise the wall fields of the same columns solved as 5D fields by
  mdwf_solve (the inputs' point_source builds them) and projected here.
* The oracle's own solution of a column, projected, agrees to the accuracy
  both solves reach (true residual 1e-10).
* Served point requests that share one solve return bitwise the wall
  fields of the request solved alone.
"""
import numpy as np
import pytest

import oracle
from paper_1701_07559_amd import inputs as I

pytestmark = pytest.mark.gpu

DIMS, L5 = (4, 4, 4, 8), 8


@pytest.fixture(scope="module")
def M():
    from paper_1701_07559_amd import mdwf
    try:
        ctx = mdwf.mdwf_create((2, 2, 2, 2))
    except mdwf.MdwfError as e:
        pytest.skip("no HIP device: %s" % e)
    mdwf.mdwf_destroy(ctx)
    return mdwf


def wall(x):
    """q = P- x_0 + P+ x_{L5-1} of a canonical 5D field (spins 0, 1 are P+)."""
    q = np.empty(x.shape[1:], complex)
    q[..., 0:2, :] = x[-1][..., 0:2, :]
    q[..., 2:4, :] = x[0][..., 2:4, :]
    return q


def q_fields(n, dims):
    X, Y, Z, T = dims
    return [np.zeros((T, Z, Y, X, 4, 3), complex) for _ in range(n)]


@pytest.mark.parametrize("inner", [0, 2], ids=["f64", "f16"])
def test_point_solve_equals_projected_5d_solve(M, inner):
    act = oracle.Action(DIMS, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(DIMS, 0.3, 101)
    site = (1, 2, 3, 5)
    cols = [0, 4, 7, 11]
    masses = [0.05, 0.1, 0.02, 0.05]
    ctx = M.mdwf_create(DIMS)
    try:
        M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, L5)
        M.mdwf_load_gauge(ctx, U)
        opts = dict(tol=1e-10, inner=inner, schur_form=2 if inner else 0)
        qs = q_fields(len(cols), DIMS)
        st, info = M.mdwf_solve_point(ctx, site, cols, qs, mq=masses, opts=opts)
        assert st == M.MDWF_OK and all(i["true_resid"] <= 1e-10 for i in info)
        bs = [I.point_source(DIMS, L5, site, c // 3, c % 3) for c in cols]
        xs = [np.zeros_like(b) for b in bs]
        st, info5 = M.mdwf_solve(ctx, bs, xs, mq=masses, opts=opts)
        assert st == M.MDWF_OK
        assert [i["iters"] for i in info] == [i["iters"] for i in info5]
        for q, x in zip(qs, xs):
            assert np.array_equal(q, wall(x))
        # the oracle's solution of the first column, projected
        xo, oi = oracle.solve(act.with_mass(masses[0]), U, bs[0], tol=1e-12)
        assert oi["status"] == 0
        assert np.linalg.norm(qs[0] - wall(xo)) / np.linalg.norm(wall(xo)) <= 1e-7
        with pytest.raises(M.MdwfError):
            M.mdwf_solve_point(ctx, (4, 0, 0, 0), [0], q_fields(1, DIMS))   # site outside the lattice
        with pytest.raises(M.MdwfError):
            M.mdwf_solve_point(ctx, site, [12], q_fields(1, DIMS))          # no such column
    finally:
        M.mdwf_destroy(ctx)


def test_served_point_requests_share_one_solve(M):
    dims = (8, 8, 8, 8)
    U = I.random_links(dims, 0.3, 111)
    big = (16, 16, 16, 16)
    Ub = I.random_links(big, 0.3, 112)
    reqs = [((0, 1, 2, 3), [0, 1, 2], [0.05, 0.1, 0.02]), ((5, 6, 7, 0), [3, 9], [0.05, 0.05]),
            ((2, 2, 2, 2), list(range(12)), None)]
    srv = M.Server(mem_budget=0, max_active=1)
    try:
        fid = srv.add_field(dims, U)
        fbig = srv.add_field(big, Ub)
        # keep the one worker busy so the point requests queue and then share a solve
        bb = I.gaussian_source(big, L5, 113)
        xb = np.zeros_like(bb)
        r0 = srv.submit(fbig, 1.3, 1.5, 0.5, 0.01, L5, [bb], [xb], opts=dict(tol=1e-11))
        jobs = []
        for site, cols, masses in reqs:
            qs = q_fields(len(cols), dims)
            rid = srv.submit_point(fid, 1.3, 1.5, 0.5, 0.05, L5, site, cols, qs, masses=masses,
                                   opts=dict(inner=2, schur_form=2))
            jobs.append((rid, site, cols, masses, qs))
        st0, _, _ = srv.wait(r0)
        assert st0 == M.MDWF_OK
        total = sum(len(c) for _, c, _ in reqs)
        ctx = M.mdwf_create(dims)
        try:
            M.mdwf_set_action(ctx, 1.3, 1.5, 0.5, 0.05, L5)
            M.mdwf_load_gauge(ctx, U)
            for rid, site, cols, masses, qs in jobs:
                st, info, _ = srv.wait(rid)
                assert st == M.MDWF_OK and all(i["true_resid"] <= 1e-10 for i in info)
                assert all(i["launch_rhs"] == total for i in info)
                ref = q_fields(len(cols), dims)
                M.mdwf_solve_point(ctx, site, cols, ref, mq=masses, opts=dict(inner=2, schur_form=2))
                for a, b in zip(qs, ref):
                    assert np.array_equal(a, b), "a served point request differs from the request alone"
        finally:
            M.mdwf_destroy(ctx)
    finally:
        srv.close()
