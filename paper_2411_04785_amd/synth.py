"""Seeded synthetic inputs for dense (and sparse) 3-way CP workloads.

This module only *draws* inputs: Gaussian factor matrices, CP-structured
tensors (a sum of R outer products plus Gaussian noise), log-uniform slice
magnitudes and open-loop request streams.  It holds none of the arithmetic
being tested (no MTTKRP, Gram matrix, solve, normalisation or fit), so both
the GPU path and the FP64 oracle may consume what it produces.

Determinism: every array is a pure function of (workload seed, stream,
index).  Tensor slices are drawn from a per-slice stream, so any mode-1
slice X[i] can be regenerated on its own, which lets tests check sampled
output rows of full-size runs without holding the whole tensor twice.

Noise convention: ``noise_var`` is the *variance* of the additive
N(0, var) noise (standard deviation sqrt(var)).
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 20241107

# Independent random streams per workload.
STREAM_FACTORS = 0   # true CP factors of the synthetic tensor
STREAM_NOISE = 1     # additive Gaussian noise (one sub-stream per slice)
STREAM_INIT = 2      # query / initial factors given to MTTKRP and CP-ALS
STREAM_SCALES = 3    # per-slice magnitudes
STREAM_REQUESTS = 4  # serving request stream
STREAM_SPARSE = 5    # coordinates and values of sparse tensors


@dataclass(frozen=True)
class Workload:
    """A dense 3-way CP workload.

    dims:        (I, J, K) tensor shape, row-major with k fastest.
    rank_true:   rank of the CP model the tensor is built from.
    R:           number of columns of the factor matrices used by MTTKRP/ALS.
    noise_var:   variance of the iid Gaussian noise added to every entry.
    slice_log10: if set, (lo, hi): mode-1 slice i is multiplied by 10**u_i,
                 u_i ~ U(lo, hi) (log-uniform magnitudes); no noise is added
                 to such workloads unless noise_var > 0.
    seed:        base seed; stream s uses seed + s.
    """

    name: str
    dims: Tuple[int, int, int]
    rank_true: int
    R: int
    noise_var: float
    seed: int
    slice_log10: Optional[Tuple[float, float]] = None
    als_sweeps: int = 0


# The workloads used by tests and the benchmark.  Seeds follow
# BASE_SEED + 100 * n for the n-th workload (n = 1..5).
WORKLOADS = {
    "cp64_r8": Workload("cp64_r8", (64, 64, 64), 8, 8, 1e-6, BASE_SEED + 100),
    "cp512_r32": Workload("cp512_r32", (512, 512, 512), 32, 32, 1e-4, BASE_SEED + 200,
                          als_sweeps=10),
    "cp1024_r64": Workload("cp1024_r64", (1024, 1024, 1024), 64, 64, 1e-3, BASE_SEED + 300),
    "cp768_r128_sliced": Workload("cp768_r128_sliced", (768, 768, 768), 128, 128, 0.0,
                                  BASE_SEED + 400, slice_log10=(-3.0, 3.0), als_sweeps=20),
}


def rng(seed: int, stream: int, *extra: int) -> np.random.Generator:
    """PCG64 generator for (seed + stream, *extra)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed + stream, *extra])))


def gaussian_factors(seed: int, stream: int, dims: Sequence[int], R: int,
                     dtype=np.float64) -> List[np.ndarray]:
    """Three iid N(0,1) factor matrices of shape (dims[n], R), row-major."""
    g = rng(seed, stream)
    return [g.standard_normal((int(d), R)).astype(dtype) for d in dims]


def true_factors(w: Workload) -> List[np.ndarray]:
    """FP64 factors A, B, C the workload's tensor is built from."""
    return gaussian_factors(w.seed, STREAM_FACTORS, w.dims, w.rank_true, np.float64)


def init_factors(w: Workload, R: Optional[int] = None) -> List[np.ndarray]:
    """FP32 N(0,1) factors used as MTTKRP operands and as the CP-ALS start."""
    return gaussian_factors(w.seed, STREAM_INIT, w.dims, R or w.R, np.float32)


def slice_magnitudes(w: Workload) -> Optional[np.ndarray]:
    """FP64 per-slice multipliers 10**u_i, u_i ~ U(lo, hi); None if unscaled."""
    if w.slice_log10 is None:
        return None
    lo, hi = w.slice_log10
    u = rng(w.seed, STREAM_SCALES).uniform(lo, hi, size=w.dims[0])
    return np.power(10.0, u)


def _slice(w: Workload, facs: List[np.ndarray], mags: Optional[np.ndarray], i: int) -> np.ndarray:
    A, B, C = facs
    a = A[i].copy()
    if mags is not None:
        a *= mags[i]
    s = (B * a) @ C.T                      # sum_r a_r B(:,r) C(:,r)^T in FP64
    if w.noise_var > 0.0:
        noise = rng(w.seed, STREAM_NOISE, i).standard_normal(s.shape)
        s += math.sqrt(w.noise_var) * noise
    return s.astype(np.float32)


def tensor_slices(w: Workload, i0: int, i1: int, out: Optional[np.ndarray] = None,
                  threads: Optional[int] = None) -> np.ndarray:
    """FP32 slices X[i0:i1] of the workload tensor, shape (i1-i0, J, K).

    Each slice is built in FP64 from the true factors (times its magnitude,
    if any) plus its own noise stream, then rounded to FP32.
    """
    facs = true_factors(w)
    mags = slice_magnitudes(w)
    _, J, K = w.dims
    if out is None:
        out = np.empty((i1 - i0, J, K), dtype=np.float32)

    def work(i):
        out[i - i0] = _slice(w, facs, mags, i)

    nthr = threads or min(16, os.cpu_count() or 1)
    if nthr <= 1 or i1 - i0 <= 1:
        for i in range(i0, i1):
            work(i)
    else:
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, range(i0, i1)))
    return out


def tensor(w: Workload, threads: Optional[int] = None) -> np.ndarray:
    """The whole FP32 tensor of the workload, shape dims."""
    return tensor_slices(w, 0, w.dims[0], threads=threads)


def small_cp(dims: Sequence[int], rank: int, seed: int, noise_var: float = 0.0,
             R: Optional[int] = None):
    """A small ad-hoc CP tensor: returns (X fp32, true factors fp64, query factors fp32)."""
    w = Workload("adhoc", tuple(int(d) for d in dims), rank, R or rank, noise_var, seed)
    return tensor(w, threads=1), true_factors(w), init_factors(w)


# --------------------------------------------------------------------------
# Serving request stream
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Request:
    """One decomposition request of the serving workload."""

    rid: int
    arrival_s: float                 # scheduled arrival time from stream start
    dims: Tuple[int, int, int]
    R: int
    sweeps: int
    workload: Workload               # tensor recipe (rank-R CP + noise)


def make_requests(n: int = 2000, rate_per_s: float = 200.0, dim_lo: int = 32,
                  dim_hi: int = 384, ranks=(8, 16, 32, 64), noise_var: float = 1e-4,
                  sweeps: int = 10, seed: int = BASE_SEED + 500) -> List[Request]:
    """Open-loop Poisson request stream: exponential gaps at ``rate_per_s``,
    dims iid uniform on [dim_lo, dim_hi] per mode, R uniform over ``ranks``."""
    g = rng(seed, STREAM_REQUESTS)
    gaps = g.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps) - gaps[0]
    dims = g.integers(dim_lo, dim_hi + 1, size=(n, 3))
    rs = g.choice(np.asarray(ranks), size=n)
    out = []
    for q in range(n):
        d = tuple(int(x) for x in dims[q])
        R = int(rs[q])
        wl = Workload(f"req{q}", d, R, R, noise_var, seed + 1000 * (q + 1))
        out.append(Request(q, float(t[q]), d, R, sweeps, wl))
    return out


# --------------------------------------------------------------------------
# Fast per-request tensors for the serving benchmark
# --------------------------------------------------------------------------

class NoisePool:
    """A fixed, seeded pool of iid N(0,1) FP32 values.  A request takes a
    window at a seeded offset, so its noise is iid within the request while
    building it costs a copy instead of fresh Gaussian draws."""

    def __init__(self, n: int = 1 << 26, seed: int = BASE_SEED + 900):
        self.values = rng(seed, 0).standard_normal(n, dtype=np.float32)

    def window(self, count: int, seed: int) -> np.ndarray:
        if count > self.values.size:
            raise ValueError("request larger than the noise pool")
        off = int(rng(seed, 7).integers(0, self.values.size - count + 1))
        return self.values[off:off + count]


def request_tensor(req: Request, pool: NoisePool):
    """(X fp32, initial factors fp32) of a serving request: an exact rank-R CP
    model (FP32 products of N(0,1) factors) plus sqrt(noise_var) times a
    window of the noise pool."""
    w = req.workload
    I, J, K = w.dims
    g = rng(w.seed, STREAM_FACTORS)
    A = g.standard_normal((I, w.rank_true), dtype=np.float32)
    B = g.standard_normal((J, w.rank_true), dtype=np.float32)
    C = g.standard_normal((K, w.rank_true), dtype=np.float32)
    # X(i,j,k) = sum_r A(i,r) B(j,r) C(k,r), built as A times the stacked
    # outer-product rows (input synthesis only; FP32).
    BC = (B[:, None, :] * C[None, :, :]).reshape(J * K, w.rank_true)
    X = (A @ BC.T).reshape(I, J, K)
    if w.noise_var > 0.0:
        X += np.float32(math.sqrt(w.noise_var)) * pool.window(X.size, w.seed).reshape(X.shape)
    return np.ascontiguousarray(X, dtype=np.float32), init_factors(w)


def coo(dims: Sequence[int], nnz: int, seed: int, skew: Optional[float] = None,
        integer: bool = False) -> Tuple[List[np.ndarray], np.ndarray]:
    """A sparse 3-way tensor in coordinates: three int32 index arrays and
    float32 values, nnz entries (repeats allowed: they add).

    Indices are uniform over each mode, except that with ``skew`` (a Zipf
    exponent > 1) the mode-0 index follows a power law -- index rank q drawn
    with probability ~ q^-skew, ranks above dims[0] folded back -- mapped
    through a seeded permutation so that the heavy rows are scattered.
    Values are N(0, 1); with ``integer`` they are integers in [-3, 3] (all
    products and sums of such values and integer factors stay exact in
    FP32 for moderate sizes)."""
    idx = []
    for m, d in enumerate(dims):
        g = rng(seed, STREAM_SPARSE, m)
        if m == 0 and skew is not None:
            q = (g.zipf(skew, nnz) - 1) % int(d)
            perm = g.permutation(int(d))
            idx.append(perm[q].astype(np.int32))
        else:
            idx.append(g.integers(0, int(d), nnz, dtype=np.int32))
    g = rng(seed, STREAM_SPARSE, 3)
    if integer:
        vals = g.integers(-3, 4, nnz).astype(np.float32)
    else:
        vals = g.standard_normal(nnz, dtype=np.float32)
    return idx, vals


def integer_factors(seed: int, dims: Sequence[int], R: int, lo: int = -4, hi: int = 4) -> List[np.ndarray]:
    """Factor matrices with integer entries in [lo, hi] (float32)."""
    return [rng(seed, STREAM_INIT, m).integers(lo, hi + 1, (int(d), R)).astype(np.float32)
            for m, d in enumerate(dims)]


def cp_nway(dims: Sequence[int], rank: int, R: int, seed: int, noise_var: float = 0.0):
    """An N-way CP tensor of the given rank plus N(0, noise_var) noise, FP32,
    and N(0,1) starting factors (FP32) of rank R.  Built through its mode-1
    unfolding: X_(1) = A (Khatri-Rao product of the other true factors)^T, the
    first remaining mode's index slowest (row-major order of X)."""
    g = rng(seed, STREAM_FACTORS)
    facs = [g.standard_normal((int(d), rank)) for d in dims]
    kr = facs[1]
    for F in facs[2:]:
        kr = (kr[:, None, :] * F[None, :, :]).reshape(-1, rank)
    X = (facs[0] @ kr.T).reshape([int(d) for d in dims])
    if noise_var > 0:
        X += math.sqrt(noise_var) * rng(seed, STREAM_NOISE).standard_normal(X.shape)
    gi = rng(seed, STREAM_INIT)
    init = [gi.standard_normal((int(d), R)).astype(np.float32) for d in dims]
    return X.astype(np.float32), init
