"""mdwf_apply_dev_noalloc: the operator entry point for callers that cannot
allocate device memory.  Through the C ABI its output must equal
mdwf_apply_dev's bit for bit (the same kernels on the same inputs), on two
calls in a row that share the static scratch, the second on a smaller
lattice; the first call on a fresh context must not change the device's free
memory; an intermediate larger than the scratch is refused."""
import numpy as np
import pytest

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


def _ctx(M, dims, L5, seed):
    ctx = M.mdwf_create(dims)
    M.mdwf_set_action(ctx, 1.3, 1.5, 0.5, 0.02, L5)
    M.mdwf_load_gauge(ctx, I.random_links(dims, 0.3, seed))
    return ctx


def _fields(M, torch, ctx, op, prec, dims, L5, seed):
    """A packed input of op's kind and two zeroed outputs."""
    dev = torch.device("cuda:0")
    kin, kout = M.OP_KINDS[op]
    V = int(np.prod(dims))
    nsites = V * L5 // (1 if kin == M.MDWF_FULL else 2)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    canon = torch.randn(nsites * 24, dtype=torch.float64, device=dev, generator=g)
    nin = torch.zeros(M.mdwf_field_bytes(ctx, prec, kin), dtype=torch.uint8, device=dev)
    M.mdwf_pack_dev(ctx, prec, kin, canon.data_ptr(), nin.data_ptr())
    nb = M.mdwf_field_bytes(ctx, prec, kout)
    return nin, torch.zeros(nb, dtype=torch.uint8, device=dev), torch.zeros(nb, dtype=torch.uint8, device=dev)


def _noalloc(M, ctx, op, prec, a, b, stream=None):
    """Status of one mdwf_apply_dev_noalloc call through the C ABI."""
    return M.lib.mdwf_apply_dev_noalloc(ctx, int(op), int(prec), a.data_ptr(), b.data_ptr(), stream)


OPS = ["MDWF_OP_SCHUR_RP", "MDWF_OP_SCHUR_RP_DAG", "MDWF_OP_SCHUR", "MDWF_OP_SCHUR_SYM_DAG", "MDWF_OP_D5",
       "MDWF_OP_HOP_EO"]


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "f16"])
def test_noalloc_equals_apply_dev_two_calls(M, prec):
    import torch
    big, small = ((8, 8, 8, 16), 8, 201), ((4, 4, 4, 4), 4, 202)
    ctxs = [_ctx(M, d, l5, s) for d, l5, s in (big, small)]
    try:
        for name in OPS:
            op = getattr(M, name)
            # first the larger lattice, then the smaller one: the second call
            # reuses the scratch the first one left behind
            for ctx, (dims, L5, seed) in zip(ctxs, (big, small)):
                print("[noalloc] %s prec %d lattice %s L5 %d" % (name, prec, dims, L5), flush=True)
                a, ref, out = _fields(M, torch, ctx, op, prec, dims, L5, seed + op)
                M.mdwf_apply_dev(ctx, op, prec, a.data_ptr(), ref.data_ptr())
                assert _noalloc(M, ctx, op, prec, a, out) == M.MDWF_OK, M.mdwf_last_error(ctx)
                torch.cuda.synchronize()
                assert torch.equal(out, ref), "%s prec %d on %s differs from mdwf_apply_dev" % (name, prec, dims)
    finally:
        for c in ctxs:
            M.mdwf_destroy(c)


def test_noalloc_allocates_nothing(M):
    import torch
    dims, L5 = (8, 8, 8, 16), 8
    warm = _ctx(M, dims, L5, 211)   # loads the kernels' code objects first
    ctx = _ctx(M, dims, L5, 212)
    s = torch.cuda.Stream()         # one stream for every launch, used before the measurement
    try:
        op, prec = M.MDWF_OP_SCHUR_RP, M.MDWF_F32
        a, ref, out = _fields(M, torch, warm, op, prec, dims, L5, 213)
        M.mdwf_apply_dev(warm, op, prec, a.data_ptr(), ref.data_ptr(), s.cuda_stream)
        assert _noalloc(M, warm, op, prec, a, out, s.cuda_stream) == M.MDWF_OK
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        for _ in range(3):   # a fresh context: mdwf_apply_dev would allocate its intermediate here
            assert _noalloc(M, ctx, op, prec, a, out, s.cuda_stream) == M.MDWF_OK, M.mdwf_last_error(ctx)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0, (free0, free1)
        M.mdwf_apply_dev(ctx, op, prec, a.data_ptr(), ref.data_ptr(), s.cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        M.mdwf_destroy(ctx)
        M.mdwf_destroy(warm)


def test_noalloc_refuses_an_intermediate_larger_than_the_scratch(M):
    import torch
    dims, L5 = (16, 16, 16, 32), 16   # FP64 half field: 201 MB; two of them exceed 256 MiB
    ctx = M.mdwf_create(dims)
    try:
        M.mdwf_set_action(ctx, 1.3, 1.5, 0.5, 0.02, L5)
        M.mdwf_load_gauge(ctx, I.unit_links(dims))
        hb = M.mdwf_field_bytes(ctx, M.MDWF_F64, M.MDWF_HALF_EVEN)
        assert hb <= M.MDWF_STATIC_SCRATCH_BYTES < 2 * hb
        dev = torch.device("cuda:0")
        a = torch.zeros(hb, dtype=torch.uint8, device=dev)
        b = torch.zeros(hb, dtype=torch.uint8, device=dev)
        st = _noalloc(M, ctx, M.MDWF_OP_SCHUR_SYM_DAG, M.MDWF_F64, a, b)
        assert st == M.MDWF_ERR_ARG and "static scratch" in M.mdwf_last_error(ctx)
        # one intermediate fits
        assert _noalloc(M, ctx, M.MDWF_OP_SCHUR, M.MDWF_F64, a, b) == M.MDWF_OK
        torch.cuda.synchronize()
    finally:
        M.mdwf_destroy(ctx)
