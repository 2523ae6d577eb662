"""Reduced-precision number formats written out from their definitions --
test infrastructure only.

bf16: 1 sign, 8 exponent, 7 stored mantissa bits; the upper half of an
IEEE binary32.  Rounding from binary32 is to the nearest bf16 value, ties to
the value whose code is even.

OCP FP8 E4M3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits; no
infinities; codes 0x7F / 0xFF are NaN; the largest finite magnitude is
448 = 1.75 * 2**8; subnormals are m * 2**-9.  Encoding here rounds to the
nearest finite value, ties to the even code, and saturates magnitudes above
448 to 448 (saturate-finite).  The sign bit is always the input's sign (a
negative value that rounds to zero gives 0x80).  NaN encodes to 0x7F.

Per-slice power-of-two scaling (the FP8 tensor format): slice i of the
tensor (the mode-1 slice X[i, :, :]) gets the exponent
``e_i = min { e integer : amax_i <= 448 * 2**e }`` (e_i = 0 for an all-zero
slice), and is stored as ``q = e4m3(X[i] * 2**-e_i)``; its value is
``decode(q) * 2**e_i``.  Multiplying by a power of two is exact, so the only
rounding is the e4m3 rounding itself.

bf16x2 split of a binary32 value x: ``hi = bf16(x)``, ``lo = bf16(x - hi)``
(x - hi is exact in binary32).

The paper has no passage on these formats; they are the published format
definitions.
"""

from __future__ import annotations

import math

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """Round binary32 values to the nearest bf16 value (ties to even code),
    returned as binary32.  NaN stays NaN, infinities stay infinite."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32)
    trunc = (u & np.uint32(0xFFFF0000))                 # bf16 toward zero
    up = trunc + np.uint32(0x10000)                       # next bf16 away from zero
    lo_v = trunc.view(np.float32).astype(np.float64)
    hi_v = up.view(np.float32).astype(np.float64)
    # Past the largest finite bf16 the next step is infinity; for rounding
    # purposes it sits where the next binade would start (2**128), as IEEE
    # rounding with an unbounded exponent prescribes.
    overflow = (up & np.uint32(0x7FFFFFFF)) == np.uint32(0x7F800000)
    hi_v = np.where(overflow, np.copysign(2.0 ** 128, lo_v), hi_v)
    xv = x.astype(np.float64)
    d_lo = np.abs(xv - lo_v)
    d_hi = np.abs(hi_v - xv)
    lo_even = ((trunc >> np.uint32(16)) & np.uint32(1)) == 0
    pick_up = (d_hi < d_lo) | ((d_hi == d_lo) & ~lo_even)
    with np.errstate(invalid="ignore"):
        res = np.where(pick_up, up, trunc)
    special = ~np.isfinite(x)                             # inf / nan: keep (quiet nan)
    res = np.where(special, u | np.where(np.isnan(x), np.uint32(0x00400000), np.uint32(0)), res)
    return res.astype(np.uint32).view(np.float32)


def bf16x2_split(x):
    """(hi, lo) with hi = bf16(x), lo = bf16(x - hi), both as binary32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x.astype(np.float64) - hi.astype(np.float64)).astype(np.float32))
    return hi, lo


def e4m3_values() -> np.ndarray:
    """Value of every e4m3 code 0..255 (NaN for 0x7F and 0xFF), FP64."""
    v = np.empty(256)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e = (c >> 3) & 0xF
        m = c & 0x7
        if e == 0xF and m == 0x7:
            v[c] = np.nan
        elif e == 0:
            v[c] = s * m * 2.0 ** -9
        else:
            v[c] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return v


_POS = e4m3_values()[:0x7F]          # codes 0x00..0x7E: 0 .. 448, increasing


def e4m3_encode(x) -> np.ndarray:
    """Nearest e4m3 code (ties to even code), saturating to +-448; NaN -> 0x7F."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.clip(np.searchsorted(_POS, a, side="left"), 0, _POS.size - 1)
    lo = np.clip(hi - 1, 0, _POS.size - 1)
    d_lo = a - _POS[lo]
    d_hi = _POS[hi] - a
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (lo % 2 == 1))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    # The sign is kept even when the magnitude rounds to zero (-0 -> 0x80).
    code = code | np.where(np.signbit(x), np.uint8(0x80), np.uint8(0))
    code = np.where(np.isnan(x), np.uint8(0x7F), code)
    return code.astype(np.uint8)


def e4m3_decode(q) -> np.ndarray:
    """FP64 value of e4m3 codes."""
    return e4m3_values()[np.asarray(q, dtype=np.uint8)]


def slice_scale_exponent(amax: float) -> int:
    """Smallest integer e with amax <= 448 * 2**e (0 for amax == 0)."""
    amax = float(amax)
    if amax == 0.0 or not math.isfinite(amax):
        return 0
    e = math.ceil(math.log2(amax / E4M3_MAX))
    while amax > E4M3_MAX * 2.0 ** e:
        e += 1
    while amax <= E4M3_MAX * 2.0 ** (e - 1):
        e -= 1
    return e


def quantize_slices_e4m3(X):
    """Per mode-1 slice power-of-two scaled e4m3 quantisation.

    Returns (codes uint8 of X's shape, exponents int32 of length X.shape[0]).
    """
    X = np.asarray(X, dtype=np.float32)
    codes = np.empty(X.shape, dtype=np.uint8)
    exps = np.empty(X.shape[0], dtype=np.int32)
    for i in range(X.shape[0]):
        xi = X[i].astype(np.float64)
        e = slice_scale_exponent(np.max(np.abs(xi)) if xi.size else 0.0)
        exps[i] = e
        codes[i] = e4m3_encode(xi * 2.0 ** (-e))
    return codes, exps


def dequantize_slices_e4m3(codes, exps) -> np.ndarray:
    """FP64 values decode(q) * 2**e_i of a per-slice scaled e4m3 tensor."""
    codes = np.asarray(codes, dtype=np.uint8)
    exps = np.asarray(exps, dtype=np.int64)
    scale = np.ldexp(1.0, exps).reshape((-1,) + (1,) * (codes.ndim - 1))
    return e4m3_decode(codes) * scale
