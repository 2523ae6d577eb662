"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (device-resident tensors, the library's own plans): every output row
of every mode against the FP64 oracle's full MTTKRP, plus CP-ALS sweeps at
512^3 against the oracle's.

Bars: FP32 and bf16x3 <= 1e-5 relative Frobenius error per mode (the stated
bar), and a worst-row bar (relative 2-norm error of one output row of R
values): 1e-5 for FP32 (whose rows sit near 3e-7) and 4e-5 for bf16x3.  A
row's error fluctuates about the per-mode figure (bf16x3: about 4.6e-6 at
1024^3, from the 2^-16 representation error of each two-term operand);
with 512 or 1024 rows of 32 or 64 values the largest of them stays within a
small multiple of it, while a systematic fault in a row (a dropped, doubled
or misplaced slice of one sum) shows as 1e-3 or more.  FP8: 3e-2 per mode
(all rows) against the unquantised tensor, and the FP8 codes and exponents
of sampled slices (including the smallest and largest) bit-exact.  (The
comparison with the dequantised tensor is made at the smaller sizes of the
other FP8 tests: dequantising all of this tensor on the host takes most of a
minute.)"""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu

MODE_BAR = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16x6": 2e-6}
ROW_BAR = {"fp32": 1e-5, "bf16x3": 4e-5, "bf16x6": 1e-5}


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


def _worst_row(a, b):
    d = np.linalg.norm(np.asarray(a, np.float64) - b, axis=1)
    return float(np.max(d / np.linalg.norm(b, axis=1)))


def _check_all_rows(tag, got, ref, prec):
    e, wr = _rel(got, ref), _worst_row(got, ref)
    _say(tag, prec, f"mode err {e:.3e} worst row {wr:.3e}")
    assert e <= MODE_BAR[prec], (tag, prec, e)
    assert wr <= ROW_BAR[prec], (tag, prec, wr)


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
    for mode in range(3):
        ref = oracle.mttkrp(X, facs, mode)
        for prec in ("fp32", "bf16x3", "bf16x6"):
            _check_all_rows(f"512^3 mode {mode}", host(ctx.mttkrp(Xd, fd, mode, prec)), ref, prec)
            if mode < 2:
                _check_all_rows(f"512^3 tree mode {mode}", host(ctx.mttkrp_dimtree(Xd, fd, mode, prec)), ref, prec)
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


@pytest.fixture(scope="module")
def cp1024_ref(cp1024):
    w, X, facs, Xd, fd = cp1024
    _say("oracle 1024^3 (three full modes)")
    return [oracle.mttkrp(X, facs, mode) for mode in range(3)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_full_1024_r64(ctx, cp1024, cp1024_ref, prec):
    from gpu_util import host
    w, X, facs, Xd, fd = cp1024
    for mode in range(3):
        ref = cp1024_ref[mode]
        _check_all_rows(f"1024^3 mode {mode}", host(ctx.mttkrp(Xd, fd, mode, prec)), ref, prec)
        if mode < 2:
            _check_all_rows(f"1024^3 tree mode {mode}", host(ctx.mttkrp_dimtree(Xd, fd, mode, prec)), ref, prec)


def test_cp512_r32_ten_sweeps(ctx):
    # The 512^3 workload's 10 CP-ALS sweeps (dimension tree, FP32) against
    # the oracle's 10 sweeps from the same start: the direct-residual fit and
    # the model on sampled slices.  After 10 sweeps ALS is still leaving its
    # initial plateau (fit about 0.71), where FP32 and FP64 trajectories
    # separate by the rounding of the MTTKRP (about 1e-7) amplified by the
    # conditioning of the normal equations; the bars are the transient-fit
    # and model bars of the smaller sweep tests.
    import torch
    from gpu_util import dev, host
    w, X, facs = _workload("cp512_r32")
    Xd = dev(X)
    fd = [dev(f) for f in facs]
    lam = dev(np.ones(w.R))
    ctx.als_sweep(Xd, fd, lam, w.als_sweeps, "fp32")
    fit = ctx.fit(Xd, fd, lam)
    _say("oracle: 10 sweeps at 512^3")
    of, ol, _ = oracle.cp_als(X, facs, w.als_sweeps, fit_every_sweep=False)
    ofit = oracle.fit(X, of, ol)
    gf = [host(f) for f in fd]
    gl = host(lam)
    si = _rows(w.dims[0], 400)
    me = max(_rel(oracle.reconstruct_slices(gf, gl, int(i), int(i) + 1),
                  oracle.reconstruct_slices(of, ol, int(i), int(i) + 1)) for i in si)
    _say(f"512^3 10 sweeps: fit {fit:.9f} oracle {ofit:.9f} |d| {abs(fit - ofit):.2e} model (worst sampled slice) {me:.2e}")
    assert abs(fit - ofit) <= 1e-4
    assert me <= 1e-3
    del Xd
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def cp768():
    return _workload("cp768_r128_sliced")


def test_full_768_r128_fp8(ctx, cp768):
    import torch
    from gpu_util import dev, host
    w, X, facs = cp768
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


def test_cp768_r128_fp8_twenty_sweeps(ctx, cp768):
    # The 768^3 workload's 20 CP-ALS sweeps on the FP8 tensor (per-slice
    # scales, e4m3 MFMA, FP64 solves) against the oracle's 20 sweeps on the
    # FP32 tensor (summary in tests/golden/cp768_r128_als.json, written by
    # tests/golden/make_cp768_r128_als.py from the oracle alone).  This is a
    # reported comparison, not a parity bar: the e4m3 tensor differs from
    # the FP32 one by about 2.65% per element, so the two iterations solve
    # different least-squares problems.  The figures are printed; the
    # bounds only catch a broken iteration (a fit far from the oracle's, or
    # a model unrelated to it).
    import json
    import os
    import torch
    from gpu_util import dev, host
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cp768_r128_als.json")
    g = json.load(open(path))
    w, X, facs = cp768
    assert g["dims"] == list(w.dims) and g["R"] == w.R and g["sweeps"] == w.als_sweeps
    Xd = dev(X)
    q, ex, qt = ctx.quantize_fp8(Xd, transposed=True)
    fd = [dev(f) for f in facs]
    lam = dev(np.ones(w.R))
    ctx.als_sweep(q, fd, lam, w.als_sweeps, "fp8", slice_exp=ex, X_t=qt)
    fit = ctx.fit(Xd, fd, lam)                  # direct residual against the FP32 tensor
    A, B, C = (host(f).astype(np.float64) for f in fd)
    lv = host(lam)
    got, ref = [], []
    for s, i in enumerate(g["sample_slices"]):
        for (j, k), v in zip(g["sample_jk"][s], g["model_at_samples"][s]):
            got.append(float(np.sum(lv * A[i] * B[j] * C[k])))
            ref.append(v)
    me = _rel(got, np.array(ref))
    _say(f"768^3 FP8 20 sweeps: fit {fit:.6f} oracle (FP64, FP32 tensor) {g['fit']:.6f} "
         f"|d| {abs(fit - g['fit']):.3e}; model at {len(ref)} samples rel err {me:.3e}")
    assert abs(fit - g["fit"]) <= 0.05
    assert me <= 0.5
    del q, qt, Xd
    torch.cuda.empty_cache()
