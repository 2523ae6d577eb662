"""GPU parity of the HIP MTTKRP (through the C ABI) against the FP64 oracle.

Bars (relative Frobenius error per result against the FP64 oracle on the same
FP32 input bytes): FP32 <= 1e-5, bf16x3 <= 1e-5, bf16x6 <= 2e-6, FP8 e4m3 <= 3e-2 against the
*unquantised* tensor.  The FP8 tensor codes and slice exponents must match the
oracle's quantiser bit for bit.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16x6": 2e-6}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2411_04785_amd.mttkrp import Context
    c = Context(0)
    yield c
    c.close()


def _case(dims, R, seed, noise=1e-4):
    w = synth.Workload("t", tuple(dims), max(1, min(R, 8)), R, noise, seed)
    return synth.tensor(w, threads=4), synth.init_factors(w)


def _run(ctx, X, facs, mode, prec):
    from gpu_util import dev, host
    out = ctx.mttkrp(dev(X), [dev(f) for f in facs], mode, prec)
    ctx.check()
    return host(out)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_cp64_r8_all_modes(ctx, prec, mode):
    from gpu_util import rel
    w = synth.WORKLOADS["cp64_r8"]
    X = synth.tensor(w)
    facs = synth.init_factors(w)
    _say("cp64_r8", prec, mode)
    got = _run(ctx, X, facs, mode, prec)
    ref = oracle.mttkrp(X, facs, mode)
    assert rel(got, ref) <= TOL[prec]


RAGGED = [
    ((37, 50, 29), 5),
    ((1, 1, 1), 1),
    ((3, 200, 7), 20),
    ((130, 17, 300), 37),
    ((33, 65, 129), 64),
    ((20, 24, 260), 128),
    ((17, 300, 18), 96),
    ((64, 96, 128), 16),
    ((5, 7, 1000), 33),
    ((70, 300, 132), 48),
    ((300, 130, 68), 24),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("dims,R", RAGGED)
def test_ragged_shapes_and_ranks(ctx, prec, dims, R):
    from gpu_util import rel
    X, facs = _case(dims, R, seed=hash((dims, R)) % 1000)
    for mode in range(3):
        _say("ragged", dims, R, prec, mode)
        got = _run(ctx, X, facs, mode, prec)
        ref = oracle.mttkrp(X, facs, mode)
        assert rel(got, ref) <= TOL[prec], (mode, rel(got, ref))


def test_unaligned_tensor_pointer(ctx):
    # A view starting one element in: 4-byte aligned only, so no 16-byte loads.
    import torch
    from gpu_util import dev, host, rel
    from paper_2411_04785_amd.mttkrp import Context
    X, facs = _case((9, 10, 12), 8, seed=5)
    flat = np.concatenate([[0.0], X.ravel()]).astype(np.float32)
    d = dev(flat)[1:]
    for mode in range(3):
        out = ctx.mttkrp(d, [dev(f) for f in facs], mode, "fp32", desc=Context.tensor_desc(d, dims=X.shape))
        assert rel(host(out), oracle.mttkrp(X, facs, mode)) <= 1e-5


def test_deterministic_bitwise(ctx):
    from gpu_util import dev, host
    X, facs = _case((96, 80, 200), 32, seed=7)
    Xd, fd = dev(X), [dev(f) for f in facs]
    for prec in ("fp32", "bf16x3", "bf16x6"):
        for mode in range(3):
            a = host(ctx.mttkrp(Xd, fd, mode, prec))
            b = host(ctx.mttkrp(Xd, fd, mode, prec))
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_closed_form_noise_free(ctx):
    # X = [[A, B, C]] exactly (up to FP32 rounding of X): M_1 = A (B^T B * C^T C).
    from gpu_util import dev, host, rel
    w = synth.Workload("cf", (48, 40, 56), 6, 6, 0.0, 77)
    X = synth.tensor(w)
    A, B, C = synth.true_factors(w)
    facs = [f.astype(np.float32) for f in (A, B, C)]
    got = host(ctx.mttkrp(dev(X), [dev(f) for f in facs], 0, "bf16x3"))
    F = [f.astype(np.float64) for f in facs]
    closed = F[0] @ ((F[1].T @ F[1]) * (F[2].T @ F[2]))
    assert rel(got, closed) <= 1e-5


# ------------------------------------------------------------------ FP8 ---

def _sliced_case(dims, R, seed):
    w = synth.Workload("s", tuple(dims), R, R, 0.0, seed, slice_log10=(-3.0, 3.0))
    return synth.tensor(w, threads=4), synth.init_factors(w)


def test_fp8_quantize_bit_exact(ctx):
    from gpu_util import dev, host
    X, _ = _sliced_case((40, 33, 50), 16, seed=3)
    X[0, 0, :5] = [0.0, -0.0, 1e-30, -1e-30, 448.0]
    X[1] = 0.0
    q, e = ctx.quantize_fp8(dev(X))
    qo, eo = oracle.quantize_slices_e4m3(X)
    assert np.array_equal(host(e), eo)
    assert np.array_equal(host(q), qo)


# Lanes hold 32, 64 or 128 values as 16-byte pieces; the cases with long
# reductions (608: 16-byte loads, 600: byte loads; 528 in mode 3, also
# strided) exercise 64- and 128-value lanes (R <= 32) and a ragged last
# window.  Ranks above 64 run one wave of up to eight column tiles: R = 100
# (seven tiles, the last one partial) on rows of 70 bytes (byte-wise loads
# in every mode) and R = 72 (five tiles) with a ragged third window.
@pytest.mark.parametrize("dims,R", [((40, 33, 50), 16), ((64, 64, 160), 128), ((31, 70, 130), 40),
                                    ((20, 24, 608), 16), ((20, 24, 608), 32), ((18, 22, 600), 32),
                                    ((12, 528, 20), 16), ((33, 40, 70), 100), ((48, 40, 272), 72)])
def test_fp8_mttkrp(ctx, dims, R):
    from gpu_util import dev, host, rel
    X, facs = _sliced_case(dims, R, seed=11)
    Xd = dev(X)
    q, e, qt = ctx.quantize_fp8(Xd, transposed=True)
    qo, eo = oracle.quantize_slices_e4m3(X)
    assert np.array_equal(host(qt), np.ascontiguousarray(np.transpose(qo, (0, 2, 1))))
    Xq = oracle.dequantize_slices_e4m3(qo, eo)
    fd = [dev(f) for f in facs]
    for mode in range(3):
        _say("fp8", dims, R, mode)
        got = host(ctx.mttkrp(q, fd, mode, "fp8", slice_exp=e, X_t=qt))
        if mode == 2:
            # The strided path (no transposed copy) gives the same bits while
            # the reduction over j is one window (32 values per lane, J <=
            # 128); with more windows the two plans add the windows in a
            # different order (in-workgroup vs split-K), so the results agree
            # to FP32 rounding and each meets the oracle bar below.
            plain = host(ctx.mttkrp(q, fd, mode, "fp8", slice_exp=e))
            _say("fp8 strided vs transposed", rel(plain, got))
            if dims[1] <= 128:
                assert np.array_equal(plain, got)
            else:
                assert rel(plain, got) <= 1e-6
                assert rel(plain, oracle.mttkrp(Xq, facs, mode)) <= 5e-3
        ref = oracle.mttkrp(X, facs, mode)
        refq = oracle.mttkrp(Xq, facs, mode)
        # Against the dequantised tensor only the factor's two-term e4m3
        # rounding (about 2^-8 relative per entry) remains.  (The stated 3e-2
        # against the unquantised tensor is test_fp8_stated_bar below.)
        assert rel(got, refq) <= 5e-3
        # Worst output row: per-slice scaling keeps the 1e-3 slices as accurate
        # as the 1e3 ones (an underflowed slice would show an error near 1).
        if mode == 0:
            rr = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
            assert rr.max() <= 0.1


# The stated FP8 bar, 3e-2 relative Frobenius error per mode against the
# FP64 oracle on the *unquantised* tensor, asserted as stated.  Where the
# e4m3 rounding of the tensor alone (the oracle on the dequantised tensor
# against the oracle on the original) already exceeds 3e-2 the case cannot
# meet the bar whatever the kernel does; those are expected failures, with
# the measured floor as the reason.  (Per-slice scales leave a relative
# rounding of about 2.65% rms per element; on small tensors whose slice
# magnitudes span 10^6, a few slices dominate and the figure fluctuates
# around it.)
FP8_FLOOR_OVER_BAR = {
    ((20, 24, 608), 32, 0): 3.035e-2,
    ((12, 528, 20), 16, 2): 3.067e-2,
}
FP8_CASES = [(d, r, m) for d, r in [((40, 33, 50), 16), ((64, 64, 160), 128), ((31, 70, 130), 40),
                                     ((20, 24, 608), 16), ((20, 24, 608), 32), ((18, 22, 600), 32),
                                     ((12, 528, 20), 16)] for m in range(3)]


@pytest.mark.parametrize("dims,R,mode", [
    pytest.param(d, r, m, marks=pytest.mark.xfail(
        strict=True, reason=f"e4m3 rounding of this tensor alone gives {FP8_FLOOR_OVER_BAR[(d, r, m)]:.3e} > 3e-2"))
    if (d, r, m) in FP8_FLOOR_OVER_BAR else (d, r, m) for d, r, m in FP8_CASES])
def test_fp8_stated_bar(ctx, dims, R, mode):
    from gpu_util import dev, host, rel
    X, facs = _sliced_case(dims, R, seed=11)
    q, e, qt = ctx.quantize_fp8(dev(X), transposed=True)
    got = host(ctx.mttkrp(q, [dev(f) for f in facs], mode, "fp8", slice_exp=e, X_t=qt))
    err = rel(got, oracle.mttkrp(X, facs, mode))
    _say("fp8 stated bar", dims, R, mode, f"{err:.4e}")
    assert err <= 3e-2


# --------------------------------------------------------- ABI errors ---

def test_abi_errors(ctx):
    import torch
    from gpu_util import dev
    from paper_2411_04785_amd.mttkrp import MtkError, MTK_EINVAL
    X, facs = _case((8, 9, 10), 4, seed=1)
    Xd, fd = dev(X), [dev(f) for f in facs]
    with pytest.raises(MtkError) as ei:
        ctx.mttkrp(Xd, fd, 3, "fp32")
    assert ei.value.status == MTK_EINVAL
    with pytest.raises(MtkError):
        ctx.mttkrp(Xd, fd, 0, "fp32", R=129)
    with pytest.raises(MtkError):
        ctx.mttkrp(Xd, fd, 0, "fp8")             # FP32 tensor with FP8 precision
    with pytest.raises(MtkError):
        ctx.mttkrp(Xd, [fd[0], None, fd[2]], 0, "fp32")
    ok = ctx.mttkrp(Xd, [None, fd[1], fd[2]], 0, "fp32")   # factors[mode] may be NULL
    assert ok.shape == (8, 4)


DIMTREE = [
    ((1, 1, 1), 1),
    ((37, 50, 29), 5),
    ((3, 200, 7), 20),
    ((130, 17, 300), 37),
    ((33, 65, 129), 64),
    ((20, 24, 260), 128),
    ((64, 96, 128), 16),
    ((5, 7, 1000), 33),
    ((70, 30, 131), 32),
    ((9, 11, 66), 8),
    ((16, 16, 64), 80),
    # J a multiple of the Y kernel's rows per workgroup (256; 128 above R =
    # 64): mode 0's sum is formed inside the Y kernel, in J/256 (J/128) slices.
    ((6, 256, 48), 8),
    ((4, 512, 40), 40),
    ((3, 256, 30), 72),
    ((2, 768, 20), 128),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("dims,R", DIMTREE)
def test_dimtree_matches_oracle(ctx, prec, dims, R):
    # Y = X x3 C (row tiles x LDS chunks of C, ragged in both), then the
    # sums over Y for modes 0 and 1.
    from gpu_util import dev, host, rel
    X, facs = _case(dims, R, seed=sum(dims) + R)
    Xd, fd = dev(X), [dev(f) for f in facs]
    for mode in (1, 0):            # each call forms its own Y
        _say("dimtree", prec, dims, R, mode)
        got = host(ctx.mttkrp_dimtree(Xd, fd, mode, prec))
        ctx.check()
        ref = oracle.mttkrp(X, facs, mode)
        assert rel(got, ref) <= TOL[prec], (mode, rel(got, ref))


# Mode 0 (the paper's mode 1) of an FP32 tensor in bf16x3 with J a multiple
# of the Y kernel's rows per workgroup, K >= 512 and J*K >= 65536: mttkrp
# takes the Y kernel's row sums with Y not stored.  The same kernel and
# summation as mttkrp_dimtree's mode 0 (which also stores Y), so the two
# agree bit for bit, as does mttkrp_noalloc; against the oracle the usual
# bar.  R = 100 and 128 take 128-row workgroups (two or six J slices); the
# unaligned K = 513 takes the byte-wise loads; (5, 256, 511) falls just
# below the K threshold and keeps the contraction.
M1_ROUTE = [((4, 256, 512), 16), ((3, 512, 520), 64), ((3, 256, 513), 32), ((2, 256, 600), 100),
            ((2, 768, 512), 128), ((5, 256, 511), 48)]


@pytest.mark.parametrize("prec", ["bf16x3"])
@pytest.mark.parametrize("dims,R", M1_ROUTE)
def test_mode1_row_sum_route(ctx, prec, dims, R):
    import torch
    from gpu_util import dev, host, rel
    X, facs = _case(dims, R, seed=sum(dims) + 3 * R)
    Xd, fd = dev(X), [dev(f) for f in facs]
    _say("mode-1 row-sum route", prec, dims, R)
    got = host(ctx.mttkrp(Xd, fd, 0, prec))
    ref = oracle.mttkrp(X, facs, 0)
    assert rel(got, ref) <= TOL[prec], rel(got, ref)
    rows = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert rows.max() <= 4 * TOL[prec], rows.max()
    out = torch.empty((dims[0], R), dtype=torch.float32, device=Xd.device)
    ctx.mttkrp_noalloc(Xd, fd, 0, out, prec)
    assert np.array_equal(host(out), got)
    if dims[1] * dims[2] >= 65536 and dims[2] >= 512:
        assert np.array_equal(host(ctx.mttkrp_dimtree(Xd, fd, 0, prec)), got)


def test_dimtree_deterministic_and_rejects(ctx):
    from gpu_util import dev, host
    from paper_2411_04785_amd.mttkrp import MtkError
    X, facs = _case((45, 38, 150), 24, seed=3)
    Xd, fd = dev(X), [dev(f) for f in facs]
    a = host(ctx.mttkrp_dimtree(Xd, fd, 1, "fp32"))
    b = host(ctx.mttkrp_dimtree(Xd, fd, 1, "fp32"))
    assert np.array_equal(a, b)
    with pytest.raises(MtkError):
        ctx.mttkrp_dimtree(Xd, fd, 2, "fp32")


def test_skewed_slices_beyond_grid_y(ctx):
    # I = 70000 slices: more than a y or z grid dimension holds.  The fit and
    # the transposed FP8 copy stride over (slice, tile) items in one grid
    # dimension; every path must still match the oracle.
    from gpu_util import dev, host, rel
    g = np.random.default_rng(70)
    X = (g.standard_normal((70000, 8, 8)) * np.power(10.0, g.uniform(-2, 2, (70000, 1, 1)))).astype(np.float32)
    facs = [g.standard_normal((d, 8)).astype(np.float32) for d in X.shape]
    Xd, fd = dev(X), [dev(f) for f in facs]
    for mode in range(3):
        for prec in ("fp32", "bf16x3", "bf16x6"):
            _say("skewed 70000x8x8", prec, mode)
            got = host(ctx.mttkrp(Xd, fd, mode, prec))
            assert rel(got, oracle.mttkrp(X, facs, mode)) <= TOL[prec], (prec, mode)
    q, e, qt = ctx.quantize_fp8(Xd, transposed=True)
    qo, eo = oracle.quantize_slices_e4m3(X)
    assert np.array_equal(host(e), eo) and np.array_equal(host(q), qo)
    assert np.array_equal(host(qt), np.ascontiguousarray(np.transpose(qo, (0, 2, 1))))
    Xq = oracle.dequantize_slices_e4m3(qo, eo)
    for mode in range(3):
        got = host(ctx.mttkrp(q, fd, mode, "fp8", slice_exp=e, X_t=qt))
        assert rel(got, oracle.mttkrp(Xq, facs, mode)) <= 5e-3, mode
    lam = np.array([1.0, -0.5, 2.0, 0.25, 1.5, 0.75, -1.25, 0.5])
    got = ctx.fit(Xd, fd, dev(lam))
    assert abs(got - oracle.fit(X, facs, lam, slices_per_chunk=4096)) <= 1e-10
    got = ctx.fit(q, fd, dev(lam), slice_exp=e)
    assert abs(got - oracle.fit(Xq, facs, lam, slices_per_chunk=4096)) <= 1e-10
