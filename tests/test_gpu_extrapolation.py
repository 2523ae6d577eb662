"""CP-ALS with extrapolation (als_run_extrapolated through the C ABI) against
the oracle's cp_als_extrapolated: the candidate, its acceptance and the kept
fits, on a well-posed CP tensor and on a collinear 'swamp' where the step
pays.  The GPU decides acceptance from its FP64 <F, M> fit and the oracle
from the explicit residual, so decisions are compared only where the
oracle's margin is clear.  The device's per-sweep fit is the <F, M>
expansion, good to a few 1e-7 near convergence in FP32 and to ~1e-4 in
bf16x3, so the kept fits are monotone only to within that (the final fit
is the direct residual)."""

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
    from paper_2411_04785_amd.mttkrp import Context
    c = Context(0)
    yield c
    c.close()


def _swamp(dims, R, corr, seed, noise=0.01):
    g = np.random.default_rng(seed)
    facs = []
    for d in dims:
        base = g.standard_normal(d)
        facs.append(np.stack([corr * base + np.sqrt(1 - corr ** 2) * g.standard_normal(d) for _ in range(R)], 1))
    X = np.einsum("ir,jr,kr->ijk", *facs)
    X += noise * np.linalg.norm(X) / np.sqrt(X.size) * g.standard_normal(X.shape)
    return X.astype(np.float32), [g.standard_normal((d, R)).astype(np.float32) for d in dims]


def _dev(X, init):
    import torch
    return torch.from_numpy(X).cuda(), [torch.from_numpy(f.copy()).cuda() for f in init]


def test_off_equals_als_run(ctx):
    import torch
    X, _, init = synth.small_cp((40, 36, 30), 5, seed=3, noise_var=1e-4)
    Xd, f1 = _dev(X, init)
    _, f2 = _dev(X, init)
    l1 = torch.ones(5, dtype=torch.float64, device="cuda")
    l2 = l1.clone()
    fits1, n1, _ = ctx.als_run(Xd, f1, l1, 6, final_fit=False)
    fits2, acc, n2, _ = ctx.als_run_extrapolated(Xd, f2, l2, 6, ls_start=7, final_fit=False)
    assert n1 == n2 == 6 and not acc.any()
    assert np.array_equal(fits1, fits2)
    assert all(torch.equal(a, b) for a, b in zip(f1, f2)) and torch.equal(l1, l2)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_kept_fits_follow_the_oracle(ctx, prec):
    import torch
    X, _, init = synth.small_cp((48, 40, 36), 6, seed=11, noise_var=1e-3)
    Xd, fd = _dev(X, init)
    lam = torch.ones(6, dtype=torch.float64, device="cuda")
    fits, acc, n, ffin = ctx.als_run_extrapolated(Xd, fd, lam, 10, ls_start=2, prec=prec)
    of, ol, ofits, oacc, ocand = oracle.cp_als_extrapolated(X.astype(np.float64), init, 10)
    _say(prec, "gpu", np.round(fits, 9).tolist(), acc.astype(int).tolist())
    _say(prec, "oracle", np.round(ofits, 9).tolist(), [int(a) for a in oacc])
    # The <F, M> fit carries the MTTKRP's error magnified by ||X|| / ||X - Xhat||
    # (about 75 here): a few 1e-7 for FP32, up to ~1e-4 for bf16x3's 4.5e-6.
    tol = 1e-5 if prec == "fp32" else 1e-4
    mono = 1e-6 if prec == "fp32" else 1e-4
    assert n == 10
    assert np.abs(fits - np.array(ofits)).max() <= tol
    for s in range(1, 10):
        if not oacc[s] and ofits[s] - ocand[s] > tol:
            assert not acc[s], s              # a clearly worse candidate is dropped on the device too
        if oacc[s]:
            assert fits[s] >= ocand[s] - tol, s
    gf = [f.cpu().numpy() for f in fd]
    assert abs(ffin - oracle.fit(X.astype(np.float64), gf, lam.cpu().numpy())) <= 1e-10
    assert abs(ffin - oracle.fit(X.astype(np.float64), of, ol)) <= tol
    assert all(b >= a - mono for a, b in zip(fits, fits[1:]))


def test_swamp_needs_fewer_sweeps_on_the_device(ctx):
    # The collinear problem of the oracle's pin: the device run with
    # extrapolation reaches plain ALS's 150-sweep fit (the oracle's, less
    # 1e-4) in at most 0.6 as many sweeps as plain ALS on the device.
    import torch
    X, init = _swamp((20, 18, 16), 3, 0.9, 0)
    _, _, plain = oracle.cp_als(X.astype(np.float64), init, 150)
    target = plain[-1] - 1e-4
    Xd, f1 = _dev(X, init)
    _, f2 = _dev(X, init)
    l1 = torch.ones(3, dtype=torch.float64, device="cuda")
    l2 = l1.clone()
    gp, _, _ = ctx.als_run(Xd, f1, l1, 150, final_fit=False)
    ge, acc, _, _ = ctx.als_run_extrapolated(Xd, f2, l2, 150, ls_start=2, final_fit=False)
    n0 = next(i + 1 for i, f in enumerate(gp) if f >= target)
    n1 = next((i + 1 for i, f in enumerate(ge) if f >= target), 10 ** 6)
    _say("plain", n0, "extrapolated", n1, "accepted", int(acc.sum()))
    assert n1 <= 0.6 * n0
    # Residual ~1% of ||X||: the <F, M> fit's FP32 noise is ~1e-5 here.
    drop = max(a - b for a, b in zip(ge, ge[1:]))
    _say("largest drop of the kept fit", drop)
    assert drop <= 3e-5


def test_arguments(ctx):
    import torch
    from paper_2411_04785_amd.mttkrp import MtkError, MTK_EINVAL
    X, _, init = synth.small_cp((10, 9, 8), 2, seed=1)
    Xd, fd = _dev(X, init)
    lam = torch.ones(2, dtype=torch.float64, device="cuda")
    with pytest.raises(MtkError) as ei:
        ctx.als_run_extrapolated(Xd, fd, lam, 3, ls_start=0)
    assert ei.value.status == MTK_EINVAL
