"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (device-resident tensors, the library's own plans): sampled output
rows of every mode against the FP64 oracle computed row by row, plus one
CP-ALS sweep at 512^3 against the oracle's sweep.

Rows: the first, the last and six seeded random rows of each mode.  Bars as
in the other tests: FP32 and bf16x3 1e-5 on the sampled rows; FP8 3e-2 per
mode (all rows, the oracle's full MTTKRP) against the unquantised tensor, and
the FP8 codes and exponents of sampled slices (including the smallest and
largest) bit-exact.  (The comparison with the dequantised tensor is made at
the smaller sizes of the other FP8 tests: dequantising all of this tensor on
the host takes most of a minute.)"""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_04785_amd.mttkrp import Context
    c = Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rows(n, seed, extra=()):
    r = np.random.default_rng(seed).integers(0, n, 6)
    return np.unique(np.concatenate([[0, n - 1], list(extra), r])).astype(np.int64)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _workload(name):
    w = synth.WORKLOADS[name]
    _say("generating", name)
    return w, synth.tensor(w, threads=16), synth.init_factors(w)


def test_full_512_r32_fp32(ctx):
    import torch
    from gpu_util import dev, host
    w, X, facs = _workload("cp512_r32")
    Xd = dev(X)
    fd = [dev(f) for f in facs]
    for prec in ("fp32", "bf16x3"):
        for mode in range(3):
            rows = _rows(w.dims[mode], 100 + mode)
            ref = oracle.mttkrp_rows(X, facs, mode, rows)
            got = host(ctx.mttkrp(Xd, fd, mode, prec))[rows]
            _say("512^3", prec, "mode", mode, _rel(got, ref))
            assert _rel(got, ref) <= 1e-5
            if mode < 2:
                got = host(ctx.mttkrp_dimtree(Xd, fd, mode, prec))[rows]
                _say("512^3 tree", prec, "mode", mode, _rel(got, ref))
                assert _rel(got, ref) <= 1e-5
    # One sweep (the dimension-tree path at this shape) against the oracle's.
    lam = dev(np.ones(w.R))
    ctx.als_sweep(Xd, fd, lam, 1, "fp32")
    of, ol, _ = oracle.cp_als(X, facs, 1, fit_every_sweep=False)
    _say("512^3 sweep lambda", _rel(host(lam), ol))
    assert _rel(host(lam), ol) <= 1e-4
    for a, b in zip(fd, of):
        assert _rel(host(a), b) <= 1e-4
    del Xd
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def cp1024():
    import torch
    from gpu_util import dev
    w, X, facs = _workload("cp1024_r64")
    yield w, X, facs, dev(X), [dev(f) for f in facs]
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_full_1024_r64(ctx, cp1024, prec):
    from gpu_util import host
    w, X, facs, Xd, fd = cp1024
    for mode in range(3):
        rows = _rows(w.dims[mode], 200 + mode)
        ref = oracle.mttkrp_rows(X, facs, mode, rows)
        got = host(ctx.mttkrp(Xd, fd, mode, prec))[rows]
        _say("1024^3", prec, "mode", mode, _rel(got, ref))
        assert _rel(got, ref) <= 1e-5
        if mode < 2:
            got = host(ctx.mttkrp_dimtree(Xd, fd, mode, prec))[rows]
            assert _rel(got, ref) <= 1e-5


def test_full_768_r128_fp8(ctx):
    import torch
    from gpu_util import dev, host
    w, X, facs = _workload("cp768_r128_sliced")
    mags = synth.slice_magnitudes(w)
    q, ex, qt = ctx.quantize_fp8(dev(X), transposed=True)
    torch.cuda.synchronize()
    # Codes and exponents of the sampled slices are the oracle's, bit for bit.
    si = _rows(w.dims[0], 300, (int(np.argmin(mags)), int(np.argmax(mags))))
    qo, eo = oracle.quantize_slices_e4m3(X[si])
    assert np.array_equal(host(q)[si], qo) and np.array_equal(host(ex)[si], eo)
    fd = [dev(f) for f in facs]
    for mode in range(3):
        got = host(ctx.mttkrp(q, fd, mode, "fp8", slice_exp=ex, X_t=qt))
        e = _rel(got, oracle.mttkrp(X, facs, mode))
        _say("768^3 fp8 mode", mode, e)
        assert e <= 3e-2
    del q, qt
    torch.cuda.empty_cache()
