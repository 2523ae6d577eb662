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
