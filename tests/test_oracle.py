"""Pins of the FP64 oracle against facts it does not compute itself.

Every check compares the oracle with an independent route: brute-force
loops, closed forms that hold for exact CP tensors, special cases that reduce
to library routines, invariants, or library casts.  The cases are chosen so
that a plausible slip (swapped Khatri-Rao order, transposed operand, dropped
term, wrong sign, wrong tie rule) fails at least one of them; the
``test_pins_catch_*`` tests plant such slips in copies of the oracle and
check that a pin fires.
"""

import numpy as np
import pytest
import scipy.linalg
import torch

import oracle

from oracle import formats as ofm

from paper_2411_04785_amd import synth


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rand_case(dims, R, seed):
    g = np.random.default_rng(seed)
    X = g.standard_normal(dims)
    facs = [g.standard_normal((d, R)) for d in dims]
    return X, facs


def exact_cp(dims, R, seed):
    g = np.random.default_rng(seed)
    facs = [g.standard_normal((d, R)) for d in dims]
    A, B, C = facs
    X = np.zeros(dims)
    for r in range(R):
        X += np.multiply.outer(np.multiply.outer(A[:, r], B[:, r]), C[:, r])
    return X, facs


# ---------------------------------------------------------------- MTTKRP ---

@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("dims,R", [((3, 4, 5), 3), ((5, 2, 6), 2), ((1, 6, 4), 1)])
def test_mttkrp_matches_brute_force(mode, dims, R):
    X, facs = rand_case(dims, R, seed=11 + mode)
    assert rel(oracle.mttkrp(X, facs, mode), oracle.mttkrp_brute(X, facs, mode)) < 1e-13


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_closed_form_exact_cp(mode):
    # X = [[A, B, C]] gives M_1 = A (B^T B * C^T C) and its analogues.
    dims = (7, 9, 11)
    X, facs = exact_cp(dims, 4, seed=5)
    G = [f.T @ f for f in facs]
    others = [m for m in range(3) if m != mode]
    closed = facs[mode] @ (G[others[0]] * G[others[1]])
    assert rel(oracle.mttkrp(X, facs, mode), closed) < 1e-12


def test_mttkrp_rank1_tensor():
    # X = a o b o c: M_1 = a * ((b^T B) * (c^T C)) row-wise.
    g = np.random.default_rng(3)
    a, b, c = g.standard_normal(6), g.standard_normal(5), g.standard_normal(4)
    X = np.einsum("i,j,k->ijk", a, b, c)
    facs = [g.standard_normal((n, 3)) for n in (6, 5, 4)]
    want = np.outer(a, (b @ facs[1]) * (c @ facs[2]))
    assert rel(oracle.mttkrp(X, facs, 0), want) < 1e-13


def test_mttkrp_rank_one_factors_is_ttv_chain():
    # R = 1: M_1 = X x_2 b x_3 c (tensor-times-vector chain via tensordot).
    X, facs = rand_case((6, 7, 8), 1, seed=9)
    for mode in range(3):
        t = X
        for m in (2, 1, 0):
            if m != mode:
                t = np.tensordot(t, facs[m][:, 0], axes=([m], [0]))
        assert rel(oracle.mttkrp(X, facs, mode)[:, 0], t) < 1e-13


def test_mttkrp_all_ones_tensor():
    g = np.random.default_rng(4)
    facs = [g.standard_normal((n, 5)) for n in (4, 6, 3)]
    X = np.ones((4, 6, 3))
    want = np.tile(facs[1].sum(0) * facs[2].sum(0), (4, 1))
    assert rel(oracle.mttkrp(X, facs, 0), want) < 1e-13


def test_mttkrp_mode_permutation_invariance():
    X, (A, B, C) = rand_case((5, 6, 7), 3, seed=21)
    m2 = oracle.mttkrp(X, [A, B, C], 1)
    assert rel(m2, oracle.mttkrp(np.transpose(X, (1, 0, 2)), [B, A, C], 0)) < 1e-13
    m3 = oracle.mttkrp(X, [A, B, C], 2)
    assert rel(m3, oracle.mttkrp(np.transpose(X, (2, 0, 1)), [C, A, B], 0)) < 1e-13


def test_mttkrp_linearity_and_slice_scaling():
    X, facs = rand_case((5, 4, 6), 3, seed=31)
    Y, _ = rand_case((5, 4, 6), 3, seed=32)
    for mode in range(3):
        lhs = oracle.mttkrp(2.0 * X - 3.0 * Y, facs, mode)
        rhs = 2.0 * oracle.mttkrp(X, facs, mode) - 3.0 * oracle.mttkrp(Y, facs, mode)
        assert rel(lhs, rhs) < 1e-13
    s = np.array([1e-3, 1.0, 10.0, 1e3, 0.5])
    Xs = X * s[:, None, None]
    assert rel(oracle.mttkrp(Xs, facs, 0), s[:, None] * oracle.mttkrp(X, facs, 0)) < 1e-13


def test_mttkrp_rows_matches_full():
    X, facs = rand_case((9, 8, 7), 4, seed=41)
    for mode in range(3):
        rows = [0, X.shape[mode] - 1, 3]
        assert rel(oracle.mttkrp_rows(X, facs, mode, rows, rows_per_chunk=2),
                   oracle.mttkrp(X, facs, mode)[rows]) < 1e-14


def test_mttkrp_fp32_input_promoted_exactly():
    X, facs = rand_case((4, 5, 6), 2, seed=42)
    X32 = X.astype(np.float32)
    assert rel(oracle.mttkrp(X32, facs, 1), oracle.mttkrp_brute(X32.astype(np.float64), facs, 1)) < 1e-13


# ------------------------------------------------------- Gram and solve ---

def test_gram_hadamard_is_khatri_rao_gram():
    # (P kr Q)^T (P kr Q) = P^T P * Q^T Q, formed here from the explicit product.
    _, facs = rand_case((5, 6, 7), 4, seed=51)
    for mode in range(3):
        others = [m for m in range(3) if m != mode]
        P, Q = facs[others[0]], facs[others[1]]
        W = np.stack([np.kron(P[:, r], Q[:, r]) for r in range(4)], axis=1)
        assert rel(oracle.gram_hadamard(facs, mode), W.T @ W) < 1e-13


def test_gram_solve_recovers_true_factor():
    # For exact X = [[A, B, C]], M_1 = A V, so solving returns A (up to column norms).
    X, facs = exact_cp((8, 9, 10), 3, seed=61)
    for mode in range(3):
        M = oracle.mttkrp(X, facs, mode)
        An, lam = oracle.gram_solve(facs, M, mode)
        assert rel(An * lam, facs[mode]) < 1e-11
        assert np.allclose(np.linalg.norm(An, axis=0), 1.0, atol=1e-14)


def test_gram_solve_normal_equations_and_cholesky_library():
    X, facs = rand_case((6, 7, 8), 4, seed=62)
    for mode in range(3):
        M = oracle.mttkrp(X, facs, mode)
        raw, _ = oracle.gram_solve(facs, M, mode, normalize=False)
        V = oracle.gram_hadamard(facs, mode)
        assert rel(raw @ V, M) < 1e-12
        cho = scipy.linalg.cho_solve(scipy.linalg.cho_factor(V), M.T).T
        assert rel(raw, cho) < 1e-11
        An, lam = oracle.gram_solve(facs, M, mode)
        assert rel(An * lam, raw) < 1e-14


# ---------------------------------------------------------------- CP-ALS ---

def test_fit_values():
    X, facs = exact_cp((5, 6, 7), 3, seed=71)
    assert abs(oracle.fit(X, facs, np.ones(3)) - 1.0) < 1e-13
    assert abs(oracle.fit(X, facs, np.zeros(3)) - 0.0) < 1e-15
    # half the model: residual = X/2 exactly -> fit 0.5
    assert abs(oracle.fit(X, facs, 0.5 * np.ones(3)) - 0.5) < 1e-13


def test_fit_matches_expansion_when_well_conditioned():
    X, facs = rand_case((5, 6, 7), 3, seed=72)
    lam = np.array([0.5, 2.0, -1.0])
    A, B, C = facs
    Xhat = np.einsum("r,ir,jr,kr->ijk", lam, A, B, C)
    res = np.sqrt((X * X).sum() - 2 * (X * Xhat).sum() + (Xhat * Xhat).sum())
    assert abs(oracle.fit(X, facs, lam) - (1 - res / np.linalg.norm(X))) < 1e-12


def test_fit_from_last_update_inner_product():
    # After a least-squares update of the last factor, F = M V^{-1} (before
    # normalising) satisfies ||Xhat||^2 = <X, Xhat> = <F, M>, so the squared
    # residual is ||X||^2 - <F, M> (the per-sweep fit the sweep kernels form).
    X, facs = rand_case((7, 8, 9), 4, seed=73)
    X = X + np.einsum("ir,jr,kr->ijk", *facs)
    facs = [f + 0.2 * np.random.default_rng(9 + m).standard_normal(f.shape) for m, f in enumerate(facs)]
    M = oracle.mttkrp(X, facs, 2)
    V = oracle.gram_hadamard(facs, 2)
    F = np.linalg.solve(V, M.T).T
    C, lam = oracle.normalize_columns(F)
    direct = oracle.fit(X, [facs[0], facs[1], C], lam)
    nx2 = float((X * X).sum())
    expansion = 1.0 - np.sqrt(nx2 - float((F * M).sum())) / np.sqrt(nx2)
    assert abs(direct - expansion) < 1e-12
    # It is not an identity away from the solution (a wrong update fails it).
    F2 = 1.01 * F
    C2, lam2 = oracle.normalize_columns(F2)
    assert abs(oracle.fit(X, [facs[0], facs[1], C2], lam2)
               - (1.0 - np.sqrt(nx2 - float((F2 * M).sum())) / np.sqrt(nx2))) > 1e-6


def test_als_fixed_point_exact_cp():
    X, facs = exact_cp((6, 7, 8), 3, seed=81)
    f, lam, fits = oracle.cp_als(X, facs, sweeps=1)
    assert abs(fits[-1] - 1.0) < 1e-12
    Xhat = np.einsum("r,ir,jr,kr->ijk", lam, *f)
    assert rel(Xhat, X) < 1e-12


def test_als_fit_never_decreases():
    X, facs = exact_cp((8, 9, 10), 3, seed=82)
    X = X + 0.3 * np.random.default_rng(1).standard_normal(X.shape)
    init = [np.random.default_rng(2 + m).standard_normal((d, 3)) for m, d in enumerate(X.shape)]
    _, _, fits = oracle.cp_als(X, init, sweeps=6, record_mode_fits=True)
    assert all(b >= a - 1e-12 for a, b in zip(fits, fits[1:]))
    assert fits[-1] > 0.8


def test_als_noise_floor():
    # Exact rank-4 CP + small noise: ALS converges to fit ~ 1 - ||E|| / ||X||.
    X, facs = exact_cp((12, 13, 14), 4, seed=83)
    E = 1e-3 * np.random.default_rng(3).standard_normal(X.shape)
    init = [f + 0.1 * np.random.default_rng(4 + m).standard_normal(f.shape) for m, f in enumerate(facs)]
    _, _, fits = oracle.cp_als(X + E, init, sweeps=25)
    floor = 1.0 - np.linalg.norm(E) / np.linalg.norm(X + E)
    assert fits[-1] >= floor - 1e-6
    assert fits[-1] <= 1.0 - 0.9 * np.linalg.norm(E) / np.linalg.norm(X + E)


# --------------------------------------------------------------- formats ---

def test_bf16_round_every_code_and_every_midpoint():
    codes = np.arange(0, 1 << 16, dtype=np.uint32)
    vals = (codes << 16).view(np.float32)
    fin = np.isfinite(vals)
    # each bf16 value is a fixed point
    assert np.array_equal(ofm.bf16_round(vals[fin]).view(np.uint32), (codes << 16)[fin])
    # midpoints between a code and the next one (same sign) round to the even code
    mids = ((codes << 16) | np.uint32(0x8000)).view(np.float32)
    ok = np.isfinite(mids)
    got = ofm.bf16_round(mids[ok]).view(np.uint32) >> 16
    lo = codes[ok]
    want = np.where(lo % 2 == 0, lo, lo + 1)
    assert np.array_equal(got, want)


def test_bf16_round_matches_torch_cast():
    g = np.random.default_rng(5)
    bits = g.integers(0, 2**32, size=2_000_000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    ours = ofm.bf16_round(x).view(np.uint32) >> 16
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours.astype(np.uint16), ref)
    big = np.array([3.3895e38, -3.3895e38, 3.4e38], dtype=np.float32)
    ref = torch.from_numpy(big).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ofm.bf16_round(big), ref)


def test_bf16x2_split_error_bound():
    g = np.random.default_rng(6)
    x = (g.standard_normal(100000) * np.exp(g.uniform(-20, 20, 100000))).astype(np.float32)
    hi, lo = ofm.bf16x2_split(x)
    assert np.array_equal(ofm.bf16_round(hi), hi) and np.array_equal(ofm.bf16_round(lo), lo)
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert np.all(err <= 2.0 ** -17 * np.abs(x.astype(np.float64)))


def test_e4m3_decode_matches_torch_for_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    ours = ofm.e4m3_decode(codes)
    assert np.array_equal(np.isnan(ours), np.isnan(ref))
    assert np.array_equal(ours[~np.isnan(ours)], ref[~np.isnan(ref)])
    assert ofm.e4m3_decode(np.uint8(0x7E)) == 448.0
    assert ofm.e4m3_decode(np.uint8(0x01)) == 2.0 ** -9


def test_e4m3_encode_matches_torch_in_range():
    pos = ofm.e4m3_values()[:0x7F]
    mids = (pos[:-1] + pos[1:]) / 2
    g = np.random.default_rng(7)
    rnd = g.uniform(-448, 448, 200000) * np.exp(g.uniform(-12, 0, 200000))
    x = np.concatenate([pos, -pos, mids, -mids, rnd, np.nextafter(mids, 0), np.nextafter(mids, 1e9)])
    x = x.astype(np.float32).astype(np.float64)      # values the GPU sees are binary32
    ours = ofm.e4m3_encode(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_encode_saturates_and_handles_nan():
    x = np.array([448.0, 449.0, 464.0, 1e6, -1e30, np.inf, -np.inf, np.nan, -0.0, -1e-30])
    got = ofm.e4m3_encode(x)
    assert list(got) == [0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0x7E, 0xFE, 0x7F, 0x80, 0x80]


def test_slice_scale_exponent_definition():
    for amax, e in [(448.0, 0), (448.00003, 1), (224.0, -1), (224.0001, 0), (1.0, -8),
                    (0.0, 0), (1e5, 8), (1e-3, -18)]:
        got = ofm.slice_scale_exponent(np.float32(amax))
        assert got == e, (amax, got, e)
    g = np.random.default_rng(8)
    for a in np.exp(g.uniform(-30, 30, 5000)).astype(np.float32):
        e = ofm.slice_scale_exponent(a)
        assert float(a) <= 448.0 * 2.0 ** e and float(a) > 448.0 * 2.0 ** (e - 1)


def test_quantize_slices_roundtrip_error():
    g = np.random.default_rng(9)
    X = (g.standard_normal((6, 20, 30)) * np.power(10.0, g.uniform(-3, 3, 6))[:, None, None]).astype(np.float32)
    q, e = ofm.quantize_slices_e4m3(X)
    D = ofm.dequantize_slices_e4m3(q, e)
    amax = np.abs(X).max(axis=(1, 2))
    assert np.all(np.abs(D).max(axis=(1, 2)) <= 448.0 * 2.0 ** e)
    # normal-range values: relative error <= 2^-4 (half an ulp of a 3-bit mantissa)
    big = np.abs(X) >= (2.0 ** -6 * 2.0 ** e)[:, None, None]
    relerr = np.abs(D - X)[big] / np.abs(X)[big]
    assert relerr.max() <= 2.0 ** -4 + 1e-12
    assert np.all(amax > 448.0 * 2.0 ** (e - 1))


# ----------------------------------------------------------- generators ---

def test_generators_deterministic_and_slice_addressable():
    w = synth.Workload("t", (6, 5, 4), 3, 3, 1e-4, 1234)
    X1 = synth.tensor(w, threads=1)
    X2 = synth.tensor(w, threads=4)
    assert X1.dtype == np.float32 and np.array_equal(X1, X2)
    assert np.array_equal(synth.tensor_slices(w, 2, 4), X1[2:4])
    f1, f2 = synth.init_factors(w), synth.init_factors(w)
    assert all(np.array_equal(a, b) and a.dtype == np.float32 for a, b in zip(f1, f2))


def test_generator_cp_structure():
    # Noise-free workload: the FP32 tensor is the exact CP model rounded to FP32.
    w = synth.Workload("t", (7, 6, 5), 3, 3, 0.0, 99)
    X = synth.tensor(w)
    A, B, C = synth.true_factors(w)
    ref = np.einsum("ir,jr,kr->ijk", A, B, C)
    assert np.max(np.abs(X - ref)) <= 2.0 ** -23 * np.max(np.abs(ref)) * 2


def test_generator_slice_magnitudes():
    w = synth.WORKLOADS["cp768_r128_sliced"]
    s = synth.slice_magnitudes(w)
    assert s.shape == (768,) and s.min() >= 1e-3 and s.max() <= 1e3
    assert s.min() < 2e-3 and s.max() > 5e2


def test_request_stream():
    reqs = synth.make_requests(200)
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    assert 0.5 < (len(reqs) - 1) / t[-1] / 200.0 < 1.5
    assert all(32 <= d <= 384 for r in reqs for d in r.dims)
    assert set(r.R for r in reqs) <= {8, 16, 32, 64}


# ---------------------------------------- the pins catch planted slips ---

def _planted_mttkrp(kind):
    def f(X, facs, mode):
        facs = [np.asarray(x, np.float64) for x in facs]
        others = [m for m in range(3) if m != mode]
        P, Q = facs[others[0]], facs[others[1]]
        if kind == "swapped_kr":
            W = oracle.khatri_rao(Q, P)
        elif kind == "dropped_factor":
            W = oracle.khatri_rao(P, np.ones_like(Q))
        else:
            W = oracle.khatri_rao(P, Q)
        U = oracle.unfold(X, mode)
        if kind == "sign":
            U = U.copy()
            U[:, -1] *= -1
        return U @ W
    return f


@pytest.mark.parametrize("kind", ["swapped_kr", "dropped_factor", "sign"])
def test_pins_catch_planted_mttkrp_slips(kind):
    bad = _planted_mttkrp(kind)
    X, facs = rand_case((3, 4, 5), 3, seed=12)
    caught = any(rel(bad(X, facs, m), oracle.mttkrp_brute(X, facs, m)) > 1e-6 for m in range(3))
    assert caught


def test_pins_catch_wrong_tie_rule():
    pos = ofm.e4m3_values()[:0x7F]
    mids = (pos[:-1] + pos[1:]) / 2
    away = np.searchsorted(pos, mids, side="right")      # ties away from zero
    ref = torch.from_numpy(mids.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert not np.array_equal(away.astype(np.uint8), ref)


# ----------------------------------------------------------- N-way MTTKRP ---

@pytest.mark.parametrize("dims", [(3, 2, 4, 2), (2, 3, 2, 2, 3), (4, 1, 3, 2)])
def test_mttkrp_nway_matches_brute_force(dims):
    g = np.random.default_rng(len(dims))
    X = g.standard_normal(dims)
    facs = [g.standard_normal((d, 3)) for d in dims]
    for mode in range(len(dims)):
        assert rel(oracle.mttkrp_nway(X, facs, mode), oracle.mttkrp_nway_brute(X, facs, mode)) < 1e-13


def test_mttkrp_nway_three_way_is_the_three_way_definition():
    X, facs = rand_case((5, 4, 6), 3, seed=21)
    for mode in range(3):
        assert rel(oracle.mttkrp_nway(X, facs, mode), oracle.mttkrp_brute(X, facs, mode)) < 1e-13


def test_mttkrp_nway_closed_form_exact_cp():
    # X = [[A_1, ..., A_4]] gives M_n = A_n (*_{m != n} A_m^T A_m).
    g = np.random.default_rng(8)
    dims, R = (5, 6, 4, 7), 3
    facs = [g.standard_normal((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr,lr->ijkl", *facs)
    for mode in range(4):
        V = np.ones((R, R))
        for m in range(4):
            if m != mode:
                V *= facs[m].T @ facs[m]
        assert rel(oracle.mttkrp_nway(X, facs, mode), facs[mode] @ V) < 1e-12


def test_mttkrp_nway_unit_mode_reduces_order():
    # A mode of size 1 with factor row a: the 4-way MTTKRP equals the 3-way
    # one of the squeezed tensor with the other factors' rows scaled by a.
    g = np.random.default_rng(9)
    X3 = g.standard_normal((4, 5, 6))
    facs3 = [g.standard_normal((d, 2)) for d in X3.shape]
    a = g.standard_normal((1, 2))
    X4 = X3[:, :, None, :]
    facs4 = [facs3[0], facs3[1], a, facs3[2]]
    for m4, m3 in ((0, 0), (1, 1), (3, 2)):
        assert rel(oracle.mttkrp_nway(X4, facs4, m4), oracle.mttkrp(X3, facs3, m3) * a) < 1e-13


def test_pins_catch_reversed_nway_khatri_rao():
    # The Khatri-Rao order must follow the unfolding's column order.
    g = np.random.default_rng(10)
    X = g.standard_normal((3, 2, 4, 2))
    facs = [g.standard_normal((d, 2)) for d in X.shape]
    others = [facs[m] for m in range(4) if m != 1]
    wrong = oracle.unfold_nway(X, 1) @ oracle.khatri_rao_many(others[::-1])
    assert rel(wrong, oracle.mttkrp_nway_brute(X, facs, 1)) > 1e-3


# ---------------------------------------------------------- sparse MTTKRP ---

def _coo_case(dims, nnz, R, seed, dup=True):
    g = np.random.default_rng(seed)
    idx = [g.integers(0, d, nnz) for d in dims]
    if dup:                                   # a repeated coordinate adds
        for m in range(3):
            idx[m][-1] = idx[m][0]
    vals = g.standard_normal(nnz)
    facs = [g.standard_normal((d, R)) for d in dims]
    return idx, vals, facs


def _densify(idx, vals, dims):
    X = np.zeros(dims)
    np.add.at(X, tuple(idx), vals)
    return X


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_mttkrp_coo_equals_dense_definition(mode):
    dims = (9, 7, 11)
    idx, vals, facs = _coo_case(dims, 120, 4, seed=30 + mode)
    X = _densify(idx, vals, dims)
    assert rel(oracle.mttkrp_coo(idx, vals, dims, facs, mode), oracle.mttkrp_brute(X, facs, mode)) < 1e-13


def test_mttkrp_coo_single_entry_closed_form():
    # One nonzero v at (i, j, k): row i of M_1 is v * B(j,:) * C(k,:), all else 0.
    g = np.random.default_rng(31)
    facs = [g.standard_normal((d, 3)) for d in (4, 5, 6)]
    M = oracle.mttkrp_coo([np.array([2]), np.array([3]), np.array([1])], np.array([1.5]), (4, 5, 6), facs, 0)
    want = np.zeros((4, 3))
    want[2] = 1.5 * facs[1][3] * facs[2][1]
    assert np.array_equal(M, want)


def test_pins_catch_coo_factor_swap():
    dims = (6, 8, 5)
    idx, vals, facs = _coo_case(dims, 60, 3, seed=32)
    X = _densify(idx, vals, dims)
    wrong = oracle.mttkrp_coo([idx[0], idx[2], idx[1]], vals, (6, 5, 8), [facs[0], facs[2], facs[1]], 0)
    assert rel(wrong, oracle.mttkrp_brute(X, facs, 0)) < 1e-13      # a consistent relabelling is harmless
    bad = vals[:, None] * facs[1][idx[2] % 8] * facs[2][idx[1] % 5]
    out = np.zeros((6, 3))
    np.add.at(out, idx[0], bad)
    assert rel(out, oracle.mttkrp_brute(X, facs, 0)) > 1e-3         # crossed indices are caught


# ------------------------------------------------- CP-ALS with extrapolation ---

def _swamp(dims, R, corr, seed, noise=0.01):
    """A rank-R CP tensor whose factor columns share a common direction with
    correlation `corr` in every mode (a 'swamp': plain ALS crawls), plus noise."""
    g = np.random.default_rng(seed)
    facs = []
    for d in dims:
        base = g.standard_normal(d)
        facs.append(np.stack([corr * base + np.sqrt(1 - corr ** 2) * g.standard_normal(d) for _ in range(R)], 1))
    X = np.einsum("ir,jr,kr->ijk", *facs)
    X += noise * np.linalg.norm(X) / np.sqrt(X.size) * g.standard_normal(X.shape)
    return X, [g.standard_normal((d, R)) for d in dims]


def test_extrapolation_off_is_plain_als():
    X, init = _swamp((12, 10, 9), 3, 0.8, 0)
    f0, l0, fits0 = oracle.cp_als(X, init, 6)
    f1, l1, fits1, acc, cand = oracle.cp_als_extrapolated(X, init, 6, start=7)
    assert fits0 == fits1 and not any(acc) and all(c is None for c in cand)
    assert all(np.array_equal(a, b) for a, b in zip(f0, f1)) and np.array_equal(l0, l1)


def test_extrapolation_unit_step_reproduces_the_sweep():
    # d = 1: A_E, B_E are the sweep's own (unit-column) factors, so the
    # candidate's third factor is the sweep's and its fit the sweep's.
    X, init = _swamp((12, 10, 9), 3, 0.9, 1)
    _, _, fits0 = oracle.cp_als(X, init, 8)
    _, _, fits1, acc, cand = oracle.cp_als_extrapolated(X, init, 8, start=2, step=1.0)
    assert all(abs(c - f) < 1e-12 for c, f in zip(cand[1:], fits0[1:]))
    assert np.allclose(fits1, fits0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("corr,seed", [(0.0, 3), (0.9, 2)])
def test_extrapolation_fits_never_decrease(corr, seed):
    X, init = _swamp((14, 12, 10), 3, corr, seed)
    _, _, fits, acc, cand = oracle.cp_als_extrapolated(X, init, 40)
    assert all(b >= a - 1e-12 for a, b in zip(fits, fits[1:]))
    assert all(f >= c for f, c in zip(fits, cand) if c is not None)   # the kept fit is the better one


def _sweeps_to(fits, target):
    return next((i + 1 for i, f in enumerate(fits) if f >= target), 10 ** 6)


@pytest.mark.parametrize("seed", [0, 2])
def test_extrapolation_cuts_sweeps_in_a_swamp(seed):
    # Plain ALS on a collinear problem needs 50-110 sweeps to come within
    # 1e-4 of its 150-sweep fit; with extrapolation from sweep 2 on (d =
    # s^(1/3)) the same fit comes in at most 0.6 as many (measured 0.44-0.5).
    X, init = _swamp((20, 18, 16), 3, 0.9, seed)
    _, _, plain = oracle.cp_als(X, init, 150)
    target = plain[-1] - 1e-4
    _, _, ext, acc, _ = oracle.cp_als_extrapolated(X, init, 150)
    n0, n1 = _sweeps_to(plain, target), _sweeps_to(ext, target)
    assert n1 <= 0.6 * n0, (n0, n1)
    assert sum(acc) > 10


def test_pins_catch_a_backward_extrapolation():
    # Stepping back along the last change (d = -1) is a plausible sign slip:
    # its candidates are almost never better, and the swamp pin fails.
    X, init = _swamp((20, 18, 16), 3, 0.9, 0)
    _, _, plain = oracle.cp_als(X, init, 150)
    target = plain[-1] - 1e-4
    _, _, ext, acc, _ = oracle.cp_als_extrapolated(X, init, 150, step=-1.0)
    assert _sweeps_to(ext, target) > 0.6 * _sweeps_to(plain, target)


# ------------------------------------------------------------ N-way CP-ALS ---

def _cp_nway(dims, R, seed, noise=0.0):
    g = np.random.default_rng(seed)
    facs = [g.standard_normal((d, R)) for d in dims]
    X = np.einsum(",".join(f"{chr(97 + m)}r" for m in range(len(dims))) + "->" +
                  "".join(chr(97 + m) for m in range(len(dims))), *facs)
    X = X + noise * np.linalg.norm(X) / np.sqrt(X.size) * g.standard_normal(X.shape)
    return X, facs, [g.standard_normal((d, R)) for d in dims]


def test_nway_als_at_three_ways_is_cp_als():
    X, _, init = _cp_nway((9, 8, 7), 3, 1, noise=0.05)
    f0, l0, fits0 = oracle.cp_als(X, init, 5)
    f1, l1, fits1 = oracle.cp_als_nway(X, init, 5)
    assert np.allclose(fits0, fits1, rtol=0, atol=1e-12)
    assert all(np.allclose(a, b, rtol=0, atol=1e-10) for a, b in zip(f0, f1))


def test_nway_fit_matches_brute_reconstruction():
    g = np.random.default_rng(4)
    dims, R = (3, 4, 2, 5), 2
    X = g.standard_normal(dims)
    F = [g.standard_normal((d, R)) for d in dims]
    lam = np.array([0.7, -1.3])
    Xh = np.zeros(dims)
    for idx in np.ndindex(*dims):
        Xh[idx] = sum(lam[r] * np.prod([F[m][idx[m], r] for m in range(4)]) for r in range(R))
    assert abs(oracle.fit_nway(X, F, lam) - (1 - np.linalg.norm(X - Xh) / np.linalg.norm(X))) < 1e-13


@pytest.mark.parametrize("dims,R,seed", [((6, 5, 4, 7), 3, 2), ((4, 3, 5, 3, 4), 2, 3)])
def test_nway_als_recovers_an_exact_cp_tensor(dims, R, seed):
    X, _, init = _cp_nway(dims, R, seed)
    _, _, fits = oracle.cp_als_nway(X, init, 60)
    assert fits[-1] > 1 - 1e-6
    assert all(b >= a - 1e-12 for a, b in zip(fits, fits[1:]))


def test_pins_catch_nway_gram_of_the_wrong_modes():
    # Taking every Gram (the updated mode's too) into V is a plausible slip:
    # the updates then stop solving the normal equations and the exact
    # tensor is not recovered.
    # (here the iteration even runs into a singular V).
    X, _, init = _cp_nway((6, 5, 4, 7), 3, 2)
    F = [np.asarray(f, np.float64).copy() for f in init]
    try:
        for _ in range(60):
            for n in range(4):
                M = oracle.mttkrp_nway(X, F, n)
                V = oracle.gram_hadamard_nway(F, -1)
                F[n], lam = oracle.normalize_columns(np.linalg.solve(V, M.T).T)
        recovered = oracle.fit_nway(X, F, lam) > 1 - 1e-6
    except np.linalg.LinAlgError:
        recovered = False
    assert not recovered
