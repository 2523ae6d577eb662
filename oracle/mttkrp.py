"""FP64 MTTKRP written out from its definition -- test infrastructure only.

Mode numbering: mode 0, 1, 2 here are the mathematical modes 1, 2, 3.
Tensor X has shape (I, J, K); factors are A (I x R), B (J x R), C (K x R).

Definition (standard; the paper has no passage on it):

    M_1 = X_(1) (B kr C),   M_1(i, r) = sum_{j,k} X(i,j,k) B(j,r) C(k,r)
    M_2 = X_(2) (A kr C),   M_2(j, r) = sum_{i,k} X(i,j,k) A(i,r) C(k,r)
    M_3 = X_(3) (A kr B),   M_3(k, r) = sum_{i,j} X(i,j,k) A(i,r) B(j,r)

``X_(n)`` is the mode-n unfolding whose columns run over the two remaining
indices in their natural (row-major) order, and ``kr`` is the column-wise
Khatri-Rao product whose rows run over the same index pairs in the same
order.  The pairing of unfolding column and Khatri-Rao row is what makes the
matrix product equal the entrywise sum; the brute-force loops below check it.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np


def khatri_rao(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Column-wise Khatri-Rao product: row (p, q) -> P(p, :) * Q(q, :), p slow."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    return (P[:, None, :] * Q[None, :, :]).reshape(P.shape[0] * Q.shape[0], P.shape[1])


def unfold(X: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n unfolding in FP64: rows = index of ``mode``, columns = the other
    two indices in increasing mode order, the earlier one slow."""
    X = np.asarray(X, dtype=np.float64)
    order = [mode] + [m for m in range(3) if m != mode]
    return np.transpose(X, order).reshape(X.shape[mode], -1)


def _kr_for_mode(factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    others = [m for m in range(3) if m != mode]
    return khatri_rao(factors[others[0]], factors[others[1]])


def mttkrp(X: np.ndarray, factors: Sequence[np.ndarray], mode: int,
           rows_per_chunk: int = 0) -> np.ndarray:
    """FP64 mode-n MTTKRP ``X_(n) @ KhatriRao(other two factors)``.

    The input values are promoted to FP64 exactly.  ``rows_per_chunk`` only
    bounds memory: output rows are independent dot products, so computing
    them in groups changes nothing about any single row's sum.
    """
    if mode not in (0, 1, 2):
        raise ValueError("mode must be 0, 1 or 2")
    X = np.asarray(X)
    n_out = X.shape[mode]
    if rows_per_chunk <= 0:
        rows_per_chunk = max(1, int(2**26 // max(1, X.size // n_out)))
    return mttkrp_rows(X, factors, mode, np.arange(n_out), rows_per_chunk)


def mttkrp_rows(X: np.ndarray, factors: Sequence[np.ndarray], mode: int,
                rows, rows_per_chunk: int = 64) -> np.ndarray:
    """Selected output rows of the mode-n MTTKRP, same definition as
    :func:`mttkrp` restricted to ``rows`` (used to sample full-size runs)."""
    rows = np.asarray(rows, dtype=np.int64)
    W = _kr_for_mode(factors, mode)
    out = np.empty((rows.size, W.shape[1]), dtype=np.float64)
    X = np.asarray(X)
    for s in range(0, rows.size, rows_per_chunk):
        idx = rows[s:s + rows_per_chunk]
        sub = np.take(X, idx, axis=mode)              # mode-n fibres of these rows
        out[s:s + idx.size] = unfold(sub, mode) @ W
    return out


def mttkrp_brute(X: np.ndarray, factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """Plain nested loops over (i, j, k, r) of the entrywise definition.
    Pure Python, for tiny inputs only."""
    A, B, C = (np.asarray(f, dtype=np.float64) for f in factors)
    X = np.asarray(X, dtype=np.float64)
    I, J, K = X.shape
    R = A.shape[1]
    out = np.zeros((X.shape[mode], R))
    for i in range(I):
        for j in range(J):
            for k in range(K):
                x = float(X[i, j, k])
                for r in range(R):
                    if mode == 0:
                        out[i, r] += x * B[j, r] * C[k, r]
                    elif mode == 1:
                        out[j, r] += x * A[i, r] * C[k, r]
                    else:
                        out[k, r] += x * A[i, r] * B[j, r]
    return out


def khatri_rao_many(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Column-wise Khatri-Rao product of several matrices, the first one's row
    index slowest: row (p, q, ..., z) -> P(p, :) * Q(q, :) * ... * Z(z, :)."""
    out = np.asarray(mats[0], dtype=np.float64)
    for M in mats[1:]:
        out = khatri_rao(out, M)
    return out


def unfold_nway(X: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n unfolding of an N-way tensor in FP64: rows = index of ``mode``,
    columns = the other indices in increasing mode order, the earliest
    slowest (the same convention as :func:`unfold`)."""
    X = np.asarray(X, dtype=np.float64)
    order = [mode] + [m for m in range(X.ndim) if m != mode]
    return np.transpose(X, order).reshape(X.shape[mode], -1)


def mttkrp_nway(X: np.ndarray, factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """FP64 mode-n MTTKRP of an N-way tensor (N >= 2):
    M_n(i_n, r) = sum over all other indices of X(i_1, ..., i_N) prod_{m != n} A_m(i_m, r),
    computed as the unfolding times the Khatri-Rao product of the other factors
    (same pairing of unfolding column and Khatri-Rao row as for three ways)."""
    X = np.asarray(X)
    if not 0 <= mode < X.ndim:
        raise ValueError("mode out of range")
    others = [factors[m] for m in range(X.ndim) if m != mode]
    return unfold_nway(X, mode) @ khatri_rao_many(others)


def mttkrp_nway_brute(X: np.ndarray, factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """Plain loops over every element of X and every column r of the N-way
    definition.  Pure Python, for tiny inputs only."""
    X = np.asarray(X, dtype=np.float64)
    F = [np.asarray(f, dtype=np.float64) for f in factors]
    R = F[0].shape[1]
    out = np.zeros((X.shape[mode], R))
    for idx in np.ndindex(*X.shape):
        x = float(X[idx])
        for r in range(R):
            p = x
            for m, i in enumerate(idx):
                if m != mode:
                    p *= F[m][i, r]
            out[idx[mode], r] += p
    return out


def mttkrp_coo(idx: Sequence[np.ndarray], vals: np.ndarray, dims: Sequence[int],
               factors: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """FP64 mode-n MTTKRP of a sparse 3-way tensor given as coordinates
    (idx[0][e], idx[1][e], idx[2][e]) and values vals[e]; repeated
    coordinates add.  Each nonzero contributes vals[e] times the product of
    the other two factors' rows to output row idx[mode][e] -- the dense
    definition restricted to the stored entries."""
    F = [np.asarray(f, dtype=np.float64) for f in factors]
    R = F[0].shape[1]
    v = np.asarray(vals, dtype=np.float64)
    others = [m for m in range(3) if m != mode]
    contrib = v[:, None] * F[others[0]][np.asarray(idx[others[0]])] * F[others[1]][np.asarray(idx[others[1]])]
    out = np.zeros((int(dims[mode]), R))
    np.add.at(out, np.asarray(idx[mode]), contrib)
    return out
