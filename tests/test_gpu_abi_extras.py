"""C-ABI behaviour around the solve (through the library, on the GPU).

* err_vs_ref: the per-solve error of a mixed solve against a reference
  solution (host and device paths), checked against the norm computed here
  from the oracle's own FP64 solution.
* mdwf_set_action replaces the coefficient table that an operator launch
  already enqueued on the context's stream reads: that launch must still see
  the old action.
* A batched apply that needs larger context temporaries than the launches
  still queued on its stream (a coefficient table and an odd intermediate
  for more RHS) replaces them only after those launches are done: both the
  queued and the new results match the oracle.
* The solver's memory plan (mdwf_solve_footprint) matches what a solve
  actually allocates.
* A gauge field added to a server while a request is queued shrinks the
  budget: a queued request that no longer fits ends with ERR_OOM instead of
  waiting forever, and the server still shuts down.
"""
import numpy as np
import pytest

import oracle
from paper_1701_07559_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_1701_07559_amd import mdwf
    try:
        ctx = mdwf.mdwf_create((2, 2, 2, 2))
    except mdwf.MdwfError as e:
        pytest.skip("no HIP device: %s" % e)
    mdwf.mdwf_destroy(ctx)
    return mdwf


def make_ctx(M, act, U):
    ctx = M.mdwf_create(act.dims, antiperiodic_t=act.antiperiodic_t)
    M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, act.mq, act.L5)
    M.mdwf_load_gauge(ctx, U)
    return ctx


def test_err_vs_ref_against_oracle_solution(M):
    import torch
    dims, L5 = (4, 4, 4, 8), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 101)
    b = I.gaussian_source(dims, L5, 301)
    xo, oi = oracle.solve(act, U, b, tol=1e-12)
    assert oi["status"] == 0 and oi["true_resid"] <= 1e-12
    ctx = make_ctx(M, act, U)
    try:
        # host path: reference on the host
        x = np.zeros_like(b)
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(inner=M.MDWF_F16, schur_form=2, x_ref=[xo]))
        assert st == M.MDWF_OK
        ref = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        assert 0.0 < info[0]["err_vs_ref"] <= 1e-6
        assert abs(info[0]["err_vs_ref"] - ref) <= 1e-9 * ref
        # no reference: -1
        st, info = M.mdwf_solve(ctx, [b], [x], opts=dict(inner=M.MDWF_F32))
        assert info[0]["err_vs_ref"] == -1.0
        # device path, two RHS with sub-batching: the reference of each RHS follows it
        dev = torch.device("cuda:0")
        bd = torch.from_numpy(b.view(np.float64).ravel()).to(dev)
        b2 = I.gaussian_source(dims, L5, 302)
        xo2, _ = oracle.solve(act, U, b2, tol=1e-12)
        bd2 = torch.from_numpy(b2.view(np.float64).ravel()).to(dev)
        refs = [torch.from_numpy(v.view(np.float64).ravel()).to(dev) for v in (xo, xo2)]
        xd = [torch.zeros_like(bd), torch.zeros_like(bd)]
        torch.cuda.synchronize()
        import os
        os.environ["MDWF_SOLVE_BATCH"] = "1"
        try:
            st, info = M.mdwf_solve_dev(ctx, [bd.data_ptr(), bd2.data_ptr()], [v.data_ptr() for v in xd],
                                        opts=dict(inner=M.MDWF_F32, x_ref=[r.data_ptr() for r in refs]))
        finally:
            del os.environ["MDWF_SOLVE_BATCH"]
        torch.cuda.synchronize()
        assert st == M.MDWF_OK
        for k in range(2):
            e = float(torch.linalg.vector_norm(xd[k] - refs[k]) / torch.linalg.vector_norm(refs[k]))
            assert abs(info[k]["err_vs_ref"] - e) <= 1e-9 * e, (k, info[k]["err_vs_ref"], e)
    finally:
        M.mdwf_destroy(ctx)


def test_set_action_waits_for_enqueued_apply(M):
    import torch
    dims, L5 = (12, 12, 12, 16), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 111)
    psi = I.gaussian_source(dims, L5, 112)
    even = oracle.even_mask(dims)
    ctx = make_ctx(M, act, U)   # the library's own stream
    try:
        dev = torch.device("cuda:0")
        canon = torch.from_numpy(np.ascontiguousarray(psi[:, even]).view(np.float64).ravel()).to(dev)
        nb = M.mdwf_field_bytes(ctx, M.MDWF_F64, M.MDWF_HALF_EVEN)
        nin = torch.empty(nb, dtype=torch.uint8, device=dev)
        nout = torch.empty(nb, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        M.mdwf_pack_dev(ctx, M.MDWF_F64, M.MDWF_HALF_EVEN, canon.data_ptr(), nin.data_ptr())
        for _ in range(3):   # a queue of launches ahead of the action change
            M.mdwf_apply_dev(ctx, M.MDWF_OP_SCHUR, M.MDWF_F64, nin.data_ptr(), nout.data_ptr())
        M.mdwf_set_action(ctx, act.M5, act.b5, act.c5, 0.5, L5)   # no synchronisation before it
        out = torch.empty_like(canon)
        M.mdwf_unpack_dev(ctx, M.MDWF_F64, M.MDWF_HALF_EVEN, nout.data_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.complex128).reshape(L5, -1, 4, 3)
        ref = oracle.schur(act, U, psi)[:, even]
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13
    finally:
        M.mdwf_destroy(ctx)


def test_batched_apply_grows_temporaries_behind_queued_launches(M):
    import torch
    dims, L5 = (12, 12, 12, 16), 8
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
    U = I.random_links(dims, 0.3, 113)
    fields = [I.gaussian_source(dims, L5, 114 + k) for k in range(3)]
    even = oracle.even_mask(dims)
    masses = (0.05, 0.1, 0.2)
    ctx = make_ctx(M, act, U)
    dev = torch.device("cuda:0")
    work = torch.cuda.Stream(device=dev)   # a caller's stream, not the context's
    try:
        prec, kind = M.MDWF_F64, M.MDWF_HALF_EVEN
        stride = (M.mdwf_field_bytes(ctx, prec, kind) + 255) // 256 * 256
        canon = [torch.from_numpy(np.ascontiguousarray(f[:, even]).view(np.float64).ravel()).to(dev)
                 for f in fields]
        nin = torch.zeros(3 * stride, dtype=torch.uint8, device=dev)
        one = torch.zeros(stride, dtype=torch.uint8, device=dev)
        three = torch.zeros(3 * stride, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        st = work.cuda_stream
        for k in range(3):
            M.mdwf_pack_dev(ctx, prec, kind, canon[k].data_ptr(), nin.data_ptr() + k * stride, st)
        # first use of the batched temporaries: sized for one RHS
        for _ in range(3):
            M.mdwf_apply_batch_dev(ctx, M.MDWF_OP_SCHUR_RP, prec, 1, nin.data_ptr(), one.data_ptr(), stride,
                                   mq=[masses[0]], stream=st)
        # no synchronisation: three RHS need larger ones
        M.mdwf_apply_batch_dev(ctx, M.MDWF_OP_SCHUR_RP, prec, 3, nin.data_ptr(), three.data_ptr(), stride,
                               mq=list(masses), stream=st)
        outs = [(one, 0, 0)] + [(three, k, k) for k in range(3)]
        got = []
        for buf, slot, _ in outs:
            o = torch.empty_like(canon[0])
            M.mdwf_unpack_dev(ctx, prec, kind, buf.data_ptr() + slot * stride, o.data_ptr(), st)
            got.append(o)
        torch.cuda.synchronize()
        for (buf, slot, k), o in zip(outs, got):
            g = o.cpu().numpy().view(np.complex128).reshape(L5, -1, 4, 3)
            ref = oracle.schur_rp(act.with_mass(masses[k]), U, fields[k])[:, even]
            e = np.linalg.norm(g - ref) / np.linalg.norm(ref)
            assert e <= 1e-13, "RHS %d of the %d-RHS launch: %.3e" % (k, 1 if buf is one else 3, e)
    finally:
        torch.cuda.synchronize()
        M.mdwf_destroy(ctx)


def test_solve_footprint_matches_allocation(M):
    import torch
    dims, L5, nrhs = (16, 16, 16, 32), 8, 4
    act = oracle.Action(dims, L5, M5=1.3, b5=1.5, c5=0.5, mq=0.1)
    U = I.random_links(dims, 0.25, 121)
    bs = [I.gaussian_source(dims, L5, 122 + k) for k in range(nrhs)]
    xs = [np.zeros_like(b) for b in bs]
    ctx = make_ctx(M, act, U)
    try:
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        st, info = M.mdwf_solve(ctx, bs, xs, opts=dict(inner=M.MDWF_F32, tol=1e-8))
        assert st == M.MDWF_OK
        free1, _ = torch.cuda.mem_get_info()
        used = free0 - free1   # the context keeps its solver buffers until destroyed
        fp = M.mdwf_solve_footprint(dims, L5, M.MDWF_F32, nrhs, host_io=True)
        margin = 64 << 20
        print("[footprint] planned %.1f MB (+ %d MB margin), allocated %.1f MB" %
              ((fp - margin) / 1e6, margin >> 20, used / 1e6), flush=True)
        # the plan counts every solver vector; the margin covers the small tables
        assert fp - margin - (32 << 20) <= used <= fp
    finally:
        M.mdwf_destroy(ctx)


def test_server_add_field_rebudgets_queued_request(M):
    dims, L5 = (8, 8, 8, 16), 8
    U = I.random_links(dims, 0.3, 131)
    b = I.gaussian_source(dims, L5, 132)
    big_dims = (16, 16, 16, 16)
    fp1 = M.mdwf_solve_footprint(dims, L5, M.MDWF_F64, 1, host_io=True)
    V_big = int(np.prod(big_dims))
    gauge_big = V_big * 4 * (144 + 72 + 36)   # resident links of the added field, all precisions
    # room for one request of the first field; after adding the big field,
    # not even one
    budget = fp1 + gauge_big // 2
    assert budget - gauge_big < fp1
    U_big = I.random_links(big_dims, 0.3, 133)
    srv = M.Server(mem_budget=budget, max_active=1)
    try:
        fid = srv.add_field(dims, U)
        x1, x2 = np.zeros_like(b), np.zeros_like(b)
        # the first request runs for about two seconds (its residual target is
        # out of reach; the time limit stops it), the second one queues behind it
        r1 = srv.submit(fid, 1.3, 1.5, 0.5, 0.05, L5, [b], [x1], opts=dict(tol=1e-18, max_seconds=2.0))
        r2 = srv.submit(fid, 1.3, 1.5, 0.5, 0.05, L5, [b], [x2])
        srv.add_field(big_dims, U_big)
        with pytest.raises(M.MdwfError) as ei:
            srv.wait(r2)
        assert ei.value.status == M.MDWF_ERR_OOM
        # the first one stops at its time limit (NOCONV) or when its recursion
        # breaks down below the reachable residual (NUMERIC); either way it ends
        st1, _, _ = srv.wait(r1)
        assert st1 in (M.MDWF_ERR_NOCONV, M.MDWF_ERR_NUMERIC)
    finally:
        srv.close()   # must return: no request is left waiting on the budget
