"""FP64 CP-ALS pieces written out from their definitions -- test infrastructure only.

CP model: ``X ~ [[lambda; A, B, C]] = sum_r lambda_r a_r o b_r o c_r``.
Alternating least squares fixes two factors and solves the third from the
normal equations of ``min || X_(n) - A_n diag(lambda) KR^T ||_F``:

    A_n V = M_n,   V = *_{m != n} (A_m^T A_m),   M_n = mode-n MTTKRP,

then rescales the columns of A_n to unit 2-norm and keeps the norms as
lambda.  Modes are updated in the order 1, 2, 3 within a sweep, each update
using the factors already updated in that sweep.  The paper has no passage
on this method; these are the standard definitions.

The oracle solves the normal equations with a general LU solve
(``numpy.linalg.solve``), deliberately a different factorisation from the
symmetric (LDL^T) elimination the GPU uses.
"""

from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from .mttkrp import mttkrp


def gram_hadamard(factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """V = elementwise product of A_m^T A_m over the two modes m != mode (FP64)."""
    R = np.asarray(factors[0]).shape[1]
    V = np.ones((R, R))
    for m in range(3):
        if m != mode:
            F = np.asarray(factors[m], dtype=np.float64)
            V = V * (F.T @ F)
    return V


def normalize_columns(F: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Return (F scaled to unit column 2-norms, the norms).  A zero column is
    left as is with norm 0."""
    F = np.asarray(F, dtype=np.float64)
    lam = np.sqrt((F * F).sum(axis=0))
    safe = np.where(lam > 0.0, lam, 1.0)
    return F / safe, lam


def gram_solve(factors: Sequence[np.ndarray], M: np.ndarray, mode: int,
               normalize: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    """Solve A_n V = M_n for A_n (FP64), then normalise its columns.

    Returns (A_n, lambda).  With ``normalize=False`` returns the raw solution
    and a lambda of ones.
    """
    V = gram_hadamard(factors, mode)
    M = np.asarray(M, dtype=np.float64)
    # V is symmetric, so A_n = M V^{-1} = (V^{-1} M^T)^T.
    An = np.linalg.solve(V, M.T).T
    if not normalize:
        return An, np.ones(An.shape[1])
    return normalize_columns(An)


def reconstruct_slices(factors: Sequence[np.ndarray], lam: np.ndarray, i0: int, i1: int) -> np.ndarray:
    """Slices [i0, i1) of [[lambda; A, B, C]] in FP64, built from outer products:
    Xhat(i, j, k) = sum_r lambda_r A(i,r) B(j,r) C(k,r)."""
    A, B, C = (np.asarray(f, dtype=np.float64) for f in factors)
    lam = np.asarray(lam, dtype=np.float64)
    out = np.empty((i1 - i0, B.shape[0], C.shape[0]))
    for i in range(i0, i1):
        out[i - i0] = np.einsum("r,jr,kr->jk", lam * A[i], B, C, optimize=True)
    return out


def fit(X: np.ndarray, factors: Sequence[np.ndarray], lam: np.ndarray,
        slices_per_chunk: int = 16) -> float:
    """fit = 1 - ||X - Xhat||_F / ||X||_F, with Xhat formed explicitly (FP64).

    The residual is accumulated from the explicit difference, never from the
    expansion ||X||^2 - 2<X, Xhat> + ||Xhat||^2, which cancels badly when
    the fit is close to 1.
    """
    X = np.asarray(X)
    res2 = 0.0
    nrm2 = 0.0
    for i0 in range(0, X.shape[0], slices_per_chunk):
        i1 = min(X.shape[0], i0 + slices_per_chunk)
        xs = X[i0:i1].astype(np.float64)
        d = xs - reconstruct_slices(factors, lam, i0, i1)
        res2 += float((d * d).sum())
        nrm2 += float((xs * xs).sum())
    return 1.0 - np.sqrt(res2) / np.sqrt(nrm2)


def cp_als(X: np.ndarray, init: Sequence[np.ndarray], sweeps: int,
           fit_every_sweep: bool = True, record_mode_fits: bool = False):
    """Fixed-count CP-ALS in FP64 (no early stop).

    Returns (factors, lambda, fits) where fits[s] is the fit after sweep s
    (or, with ``record_mode_fits``, a list of the fit after every single mode
    update).  ``init`` is used as given (not normalised); lambda starts at 1.
    """
    factors: List[np.ndarray] = [np.asarray(f, dtype=np.float64).copy() for f in init]
    lam = np.ones(factors[0].shape[1])
    fits: List[float] = []
    for _ in range(sweeps):
        for n in range(3):
            M = mttkrp(X, factors, n)
            factors[n], lam = gram_solve(factors, M, n)
            if record_mode_fits:
                fits.append(fit(X, factors, lam))
        if fit_every_sweep and not record_mode_fits:
            fits.append(fit(X, factors, lam))
    return factors, lam, fits


def cp_als_extrapolated(X: np.ndarray, init: Sequence[np.ndarray], sweeps: int, start: int = 2,
                        step: Optional[float] = None):
    """CP-ALS with an extrapolation step after every sweep s >= start
    (sweeps counted from 1), in FP64.

    After sweep s has produced A_s, B_s, C_s from the factors A_p, B_p it
    started with, a candidate moves the first two factors further along
    their last change,
        A_E = normalise(A_p + d (A_s - A_p)),  B_E = normalise(B_p + d (B_s - B_p)),
    with d = s^(1/3) (or the fixed ``step``), and solves the third factor
    exactly from them: C_E, lambda_E = the mode-3 update from A_E and B_E.
    The candidate replaces the sweep's result when its fit (explicit
    residual) is higher.

    Returns (factors, lambda, fits, accepted, cand_fits): fits[s] is the fit
    kept after sweep s, accepted[s] whether the candidate was kept, and
    cand_fits[s] the candidate's fit (None before ``start``).
    """
    factors: List[np.ndarray] = [np.asarray(f, dtype=np.float64).copy() for f in init]
    lam = np.ones(factors[0].shape[1])
    fits: List[float] = []
    accepted: List[bool] = []
    cand_fits: List[Optional[float]] = []
    for s in range(1, sweeps + 1):
        A_p, B_p = factors[0].copy(), factors[1].copy()
        for n in range(3):
            factors[n], lam = gram_solve(factors, mttkrp(X, factors, n), n)
        f = fit(X, factors, lam)
        took, fc = False, None
        if s >= start:
            d = float(step) if step is not None else s ** (1.0 / 3.0)
            A_E, _ = normalize_columns(A_p + d * (factors[0] - A_p))
            B_E, _ = normalize_columns(B_p + d * (factors[1] - B_p))
            cand = [A_E, B_E, factors[2]]
            cand[2], lam_E = gram_solve(cand, mttkrp(X, cand, 2), 2)
            fc = fit(X, cand, lam_E)
            if fc > f:
                factors, lam, f, took = cand, lam_E, fc, True
        fits.append(f)
        accepted.append(took)
        cand_fits.append(fc)
    return factors, lam, fits, accepted, cand_fits


def gram_hadamard_nway(factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """V = elementwise product of A_m^T A_m over every mode m != mode (FP64),
    for any number of factors."""
    R = np.asarray(factors[0]).shape[1]
    V = np.ones((R, R))
    for m, F in enumerate(factors):
        if m != mode:
            F = np.asarray(F, dtype=np.float64)
            V = V * (F.T @ F)
    return V


def fit_nway(X: np.ndarray, factors: Sequence[np.ndarray], lam: np.ndarray) -> float:
    """fit = 1 - ||X - Xhat||_F / ||X||_F for an N-way CP model, Xhat formed
    explicitly in FP64 through its mode-1 unfolding A_1 diag(lambda) (Khatri-
    Rao product of the other factors)^T."""
    from .mttkrp import khatri_rao_many
    X = np.asarray(X, dtype=np.float64)
    F = [np.asarray(f, dtype=np.float64) for f in factors]
    Xh = (F[0] * np.asarray(lam, dtype=np.float64)) @ khatri_rao_many(F[1:]).T
    return float(1.0 - np.linalg.norm(X.reshape(X.shape[0], -1) - Xh) / np.linalg.norm(X))


def cp_als_nway(X: np.ndarray, init: Sequence[np.ndarray], sweeps: int):
    """Fixed-count CP-ALS of an N-way tensor in FP64: each sweep updates the
    factors in mode order, A_n = M_n V^{-1} with M_n the mode-n MTTKRP and V
    the Hadamard product of the other factors' Gram matrices, then normalises
    its columns (the norms become lambda).  ``init`` is used as given.
    Returns (factors, lambda, fits) with fits[s] the fit after sweep s."""
    from .mttkrp import mttkrp_nway
    factors: List[np.ndarray] = [np.asarray(f, dtype=np.float64).copy() for f in init]
    lam = np.ones(factors[0].shape[1])
    fits: List[float] = []
    for _ in range(sweeps):
        for n in range(len(factors)):
            M = mttkrp_nway(X, factors, n)
            V = gram_hadamard_nway(factors, n)
            factors[n], lam = normalize_columns(np.linalg.solve(V, M.T).T)
        fits.append(fit_nway(X, factors, lam))
    return factors, lam, fits
