"""mttkrp_noalloc (the entry point that allocates nothing) against mttkrp,
through the C ABI: two calls in a row on one context, the second with a
smaller input, each equal to mttkrp's result bit for bit (same plan and
kernels) and within the oracle bar; a shape whose plan needs more scratch
than the static buffer is refused before anything is enqueued."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_04785_amd.mttkrp import Context
    c = Context(0)
    yield c
    c.close()


def _case(dims, R, seed):
    w = synth.Workload("na", tuple(dims), min(R, 8), R, 1e-4, seed)
    return synth.tensor(w, threads=4), synth.init_factors(w)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6", "fp8"])
def test_noalloc_matches_mttkrp_twice(ctx, prec):
    import torch
    from gpu_util import dev, host, rel
    # First a larger call, then a smaller one: the second must not see the
    # first one's partial slices in the shared scratch.
    for dims, R, seed in (((96, 80, 200), 40, 1), ((37, 50, 29), 5, 2)):
        X, facs = _case(dims, R, seed)
        fd = [dev(f) for f in facs]
        Xd = dev(X)
        kw = {}
        if prec == "fp8":
            q, e, qt = ctx.quantize_fp8(Xd, transposed=True)
            Xd, kw = q, {"slice_exp": e, "X_t": qt}
            qo, eo = oracle.quantize_slices_e4m3(X)
            Xref = oracle.dequantize_slices_e4m3(qo, eo)
            bar = 5e-3            # only the factor's two-term e4m3 rounding remains
        else:
            Xref, bar = X, 1e-5
        for mode in range(3):
            _say("noalloc", prec, dims, R, mode)
            ref = host(ctx.mttkrp(Xd, fd, mode, prec, **kw))
            out = torch.full((dims[mode], R), float("nan"), dtype=torch.float32, device="cuda")
            got = host(ctx.mttkrp_noalloc(Xd, fd, mode, out, prec, **kw))
            ctx.check()
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (prec, dims, mode)
            assert rel(got, oracle.mttkrp(Xref, facs, mode)) <= bar


def test_noalloc_refuses_oversized_plan(ctx):
    # 2048 x 2048 x 2048 at R = 128, FP32 mode 2, needs far more than 64 MiB
    # of partial slices: refused with MTK_EUNSUPPORTED; the output is left
    # untouched.  Only descriptors are built: the (unread) tensor is a 4-byte
    # buffer.
    import ctypes
    import torch
    from paper_2411_04785_amd.mttkrp import MtkError, MTK_EUNSUPPORTED, Tensor, _dims, _stream
    buf = torch.zeros(1, dtype=torch.float32, device="cuda")
    f = torch.zeros((2048, 128), dtype=torch.float32, device="cuda")
    out = torch.full((2048, 128), 7.0, dtype=torch.float32, device="cuda")
    d = Tensor(buf.data_ptr(), None, _dims((2048, 2048, 2048)), 0, None)
    fp = (ctypes.c_void_p * 3)(f.data_ptr(), f.data_ptr(), f.data_ptr())
    st = ctx._L.mttkrp_noalloc(ctx.h, ctypes.byref(d), fp, 128, 2, 0, out.data_ptr(), _stream())
    assert st == MTK_EUNSUPPORTED
    assert b"static" in ctx._L.mtk_last_error(ctx.h)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
