"""Sparse MTTKRP (mtk_coo_create / mttkrp_coo through the C ABI) against
the oracle's sum over stored entries.  Integer-valued inputs make every
product and partial sum exact in FP32, so those cases must agree bit for
bit whatever the summation order; Gaussian inputs are held to the rounding
bound of an FP32 sum of the row's terms, entry by entry."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_04785_amd.mttkrp import Context
    c = Context(0)
    yield c
    c.close()


def _dev(idx, vals, facs):
    import torch
    di = [torch.from_numpy(np.ascontiguousarray(i)).cuda() for i in idx]
    dv = torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float32)).cuda()
    df = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda() for f in facs]
    return di, dv, df


def _run(ctx, dims, idx, vals, facs, modes=(0, 1, 2), garbage=True):
    import torch
    di, dv, df = _dev(idx, vals, facs)
    t = ctx.coo_create(dims, di, dv)
    outs = []
    for mode in modes:
        out = torch.full((dims[mode], facs[0].shape[1]), float("nan"), device="cuda") if garbage else None
        outs.append(ctx.mttkrp_coo(t, df, mode, out=out).cpu().numpy().astype(np.float64))
    t.close()
    return outs


def _bound(idx, vals, dims, facs, mode):
    """(n_r + 3) u sum |terms| per output entry: an FP32 sum of the row's
    n_r products, each product rounded twice."""
    s = oracle.mttkrp_coo(idx, np.abs(vals.astype(np.float64)), dims, [np.abs(f.astype(np.float64)) for f in facs],
                          mode)
    n = np.bincount(idx[mode], minlength=dims[mode]).astype(np.float64)
    return (n[:, None] + 3.0) * U24 * s


@pytest.mark.parametrize("R", [1, 8, 13, 16, 24, 64, 100, 128])
def test_integer_inputs_exact(ctx, R):
    # Ragged nnz (not a multiple of the 64-entry segment), empty rows in
    # every mode, repeated coordinates; exact arithmetic, so bit for bit.
    dims = (300, 77, 129)
    idx, vals = synth.coo(dims, 70001, seed=100 + R, integer=True)
    for m in range(3):
        idx[m][-5:] = idx[m][:5]
    facs = synth.integer_factors(200 + R, dims, R)
    outs = _run(ctx, dims, idx, vals, facs)
    for mode, got in enumerate(outs):
        ref = oracle.mttkrp_coo(idx, vals, dims, facs, mode)
        assert np.array_equal(got, ref), (R, mode, np.abs(got - ref).max())


def test_power_law_rows_exact(ctx):
    # Zipf-distributed mode-0 rows: heavy rows cross many segments and their
    # carry slots are added by the fix-up; light and empty rows around them.
    dims = (5000, 200, 300)
    idx, vals = synth.coo(dims, 300000, seed=5, skew=1.2, integer=True)
    facs = synth.integer_factors(6, dims, 32)
    _say("heaviest row", np.bincount(idx[0]).max(), "of", len(vals))
    outs = _run(ctx, dims, idx, vals, facs)
    for mode, got in enumerate(outs):
        assert np.array_equal(got, oracle.mttkrp_coo(idx, vals, dims, facs, mode)), mode


def test_single_row_spanning_every_segment(ctx):
    dims = (9, 40, 50)
    idx, vals = synth.coo(dims, 200000, seed=8, integer=True)
    idx[0][:] = 5
    facs = synth.integer_factors(9, dims, 64)
    got = _run(ctx, dims, idx, vals, facs, modes=(0,))[0]
    ref = oracle.mttkrp_coo(idx, vals, dims, facs, 0)
    assert np.array_equal(got, ref)
    assert not got[np.arange(9) != 5].any()


@pytest.mark.parametrize("R", [16, 64, 128])
def test_gaussian_within_fp32_sum_bound(ctx, R):
    dims = (400, 350, 90)
    idx, vals = synth.coo(dims, 250007, seed=40 + R, skew=1.5)
    facs = synth.gaussian_factors(41 + R, synth.STREAM_INIT, dims, R)
    outs = _run(ctx, dims, idx, vals, facs)
    for mode, got in enumerate(outs):
        ref = oracle.mttkrp_coo(idx, vals, dims, facs, mode)
        err = np.abs(got - ref)
        b = _bound(idx, vals, dims, facs, mode)
        _say(R, mode, "max err / bound", float((err / np.maximum(b, 1e-300)).max()))
        assert (err <= b).all()


def test_deterministic_and_overwrites(ctx):
    import torch
    dims = (120, 130, 140)
    idx, vals = synth.coo(dims, 100000, seed=11)
    facs = synth.gaussian_factors(12, synth.STREAM_INIT, dims, 48)
    di, dv, df = _dev(idx, vals, facs)
    t = ctx.coo_create(dims, di, dv)
    for mode in range(3):
        a = ctx.mttkrp_coo(t, df, mode, out=torch.full((dims[mode], 48), 7.0, device="cuda")).cpu()
        b = ctx.mttkrp_coo(t, df, mode, out=torch.full((dims[mode], 48), -3.0, device="cuda")).cpu()
        assert torch.equal(a, b)
    t.close()


def test_degenerate_tensors(ctx):
    import torch
    from paper_2411_04785_amd.mttkrp import MtkError, MTK_EINVAL
    # No entries: every mode's MTTKRP is zero.
    facs = synth.gaussian_factors(1, synth.STREAM_INIT, (5, 6, 7), 8)
    di = [torch.zeros(0, dtype=torch.int32, device="cuda") for _ in range(3)]
    t = ctx.coo_create((5, 6, 7), di, torch.zeros(0, device="cuda"))
    df = [torch.from_numpy(f.astype(np.float32)).cuda() for f in facs]
    for mode in range(3):
        out = torch.full(((5, 6, 7)[mode], 8), float("nan"), device="cuda")
        assert not ctx.mttkrp_coo(t, df, mode, out=out).cpu().numpy().any()
    t.close()
    # One entry; a size-1 mode; a mode with far more rows than entries.
    for dims, nnz in (((4, 5, 6), 1), ((1, 70, 3), 999), ((100000, 3, 4), 500)):
        idx, vals = synth.coo(dims, nnz, seed=nnz, integer=True)
        facs = synth.integer_factors(nnz, dims, 5)
        for mode, got in enumerate(_run(ctx, dims, idx, vals, facs)):
            assert np.array_equal(got, oracle.mttkrp_coo(idx, vals, dims, facs, mode)), (dims, mode)
    # An index outside dims is refused when the tensor is made.
    idx, vals = synth.coo((10, 10, 10), 1000, seed=3)
    idx[2][700] = 10
    di, dv, _ = _dev(idx, vals, [])
    with pytest.raises(MtkError) as ei:
        ctx.coo_create((10, 10, 10), di, dv)
    assert ei.value.status == MTK_EINVAL
    idx[2][700] = -1
    di, dv, _ = _dev(idx, vals, [])
    with pytest.raises(MtkError):
        ctx.coo_create((10, 10, 10), di, dv)
    # Bad arguments to the contraction.
    idx[2][700] = 0
    di, dv, df = _dev(idx, vals, synth.gaussian_factors(2, synth.STREAM_INIT, (10, 10, 10), 4))
    t = ctx.coo_create((10, 10, 10), di, dv)
    for mode, R in ((3, 4), (0, 0), (0, 129)):
        with pytest.raises(MtkError) as ei:
            ctx.mttkrp_coo(t, df, mode, R=R, out=torch.empty(10, max(R, 1), device="cuda"))
        assert ei.value.status == MTK_EINVAL
    t.close()


def test_large_sampled_rows(ctx):
    # 2^24 entries over 2^14 x 2^14 x 2^14, R = 64: sampled output rows of
    # each mode against the oracle over those rows' entries.
    dims = (1 << 14, 1 << 14, 1 << 14)
    nnz = 1 << 24
    idx, vals = synth.coo(dims, nnz, seed=77)
    facs = synth.gaussian_factors(78, synth.STREAM_INIT, dims, 64)
    outs = _run(ctx, dims, idx, vals, facs, garbage=False)
    g = np.random.default_rng(79)
    for mode, got in enumerate(outs):
        rows = np.unique(g.integers(0, dims[mode], 64))
        sel = np.isin(idx[mode], rows)
        sub = [i[sel] for i in idx]
        ref = oracle.mttkrp_coo(sub, vals[sel], dims, facs, mode)[rows]
        b = _bound(sub, vals[sel], dims, facs, mode)[rows]
        assert (np.abs(got[rows] - ref) <= b).all(), mode


def test_sparse_cp_als_matches_oracle(ctx):
    # Entries observed at random positions of a rank-6 CP tensor (repeats
    # add); five sparse CP-ALS sweeps on the device against the oracle's
    # CP-ALS on the densified tensor from the same start.
    import torch
    dims, R = (40, 50, 60), 6
    Xfull, _, init = synth.small_cp(dims, R, seed=17, noise_var=1e-4)
    idx, _ = synth.coo(dims, 30000, seed=18)
    vals = Xfull[idx[0], idx[1], idx[2]].astype(np.float32)
    Xs = np.zeros(dims)
    np.add.at(Xs, tuple(idx), vals.astype(np.float64))
    of, ol, ofits = oracle.cp_als(Xs, init, 5)
    di, dv, df = _dev(idx, vals, init)
    t = ctx.coo_create(dims, di, dv)
    lam = torch.ones(R, dtype=torch.float64, device="cuda")
    ctx.als_sweep_coo(t, df, lam, 5)
    t.close()
    gf = [f.cpu().numpy() for f in df]
    gl = lam.cpu().numpy()
    gfit = oracle.fit(Xs, gf, gl)
    model = oracle.reconstruct_slices(gf, gl, 0, dims[0])
    ref = oracle.reconstruct_slices(of, ol, 0, dims[0])
    me = float(np.linalg.norm(model - ref) / np.linalg.norm(ref))
    _say(f"fit {gfit:.9f} oracle {ofits[-1]:.9f} model {me:.2e}")
    assert abs(gfit - ofits[-1]) <= 1e-4
    assert me <= 1e-3


@pytest.mark.parametrize("R", [8, 64, 100])
def test_partitioned_modes_exact(ctx, R):
    # A large second mode makes mode 0 partitioned (entries ordered by which
    # eighth of B's rows they gather, one partial output per part, added in
    # part order); integer inputs, so bit for bit, with power-law rows too.
    # (20000, 200, 9000) with a power-law mode-0 index: mode 1 partitions by
    # the mode-2 index, which spreads its entries evenly, not by the skewed one.
    for dims, skew in (((200, 10000, 9000), None), ((200, 10000, 9000), 1.3), ((20000, 200, 9000), 1.3)):
        idx, vals = synth.coo(dims, 120001, seed=300 + R, skew=skew, integer=True)
        facs = synth.integer_factors(301 + R, dims, R)
        outs = _run(ctx, dims, idx, vals, facs)
        for mode, got in enumerate(outs):
            assert np.array_equal(got, oracle.mttkrp_coo(idx, vals, dims, facs, mode)), (dims, R, skew, mode)
