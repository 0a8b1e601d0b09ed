"""Oracle: BF16 and FP8 (OCP E4M3FN) rounding with per-column scales.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written from the formats' definitions, by nearest-value selection:
  * BF16: 1 sign, 8 exponent, 7 mantissa bits (the top half of an IEEE
    binary32); round to nearest, ties to the even mantissa.
  * FP8 E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits; exponent 0 is
    subnormal (m * 2^-9); exponent 15 with mantissa 7 is NaN; no infinities;
    largest finite value 448.  Encoding saturates to +-448, rounds to
    nearest, ties to the even code.
  * Per-column scale (FP32): c_r = amax_r / 448, or 1 for an all-zero column;
    codes are fp8(x / c_r) with the division in FP32.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# BF16
# ----------------------------------------------------------------------------


def bf16_round(x) -> np.ndarray:
    """FP32 -> nearest BF16 value (returned as float32), ties to even."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32)
    lo_bits = bits & np.uint32(0xFFFF0000)                  # toward zero
    lo = lo_bits.view(np.float32).astype(np.float64)
    # next BF16 value away from zero: add one unit in the 16th bit
    hi_bits = (lo_bits.astype(np.uint64) + 0x10000).astype(np.uint32)
    hi = hi_bits.view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dlo = np.abs(xd - lo)
    dhi = np.abs(hi - xd)
    lo_even = ((lo_bits >> np.uint32(16)) & np.uint32(1)) == 0
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ~lo_even)
    out = np.where(pick_hi, hi_bits, lo_bits).astype(np.uint32)
    out = np.where(np.isnan(x), np.uint32(0x7FC00000), out)
    out = np.where(np.isinf(x), bits, out)
    return out.view(np.float32)


def bf16_bits(x) -> np.ndarray:
    """Raw 16-bit codes of bf16_round(x)."""
    return (bf16_round(x).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_decode(codes) -> np.ndarray:
    return (np.asarray(codes, dtype=np.uint32) << np.uint32(16)).view(np.float32)


# ----------------------------------------------------------------------------
# FP8 E4M3FN
# ----------------------------------------------------------------------------

FP8_MAX = 448.0


def fp8_decode(codes) -> np.ndarray:
    """Value of each 8-bit E4M3FN code (float64; NaN codes give NaN)."""
    c = np.asarray(codes, dtype=np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    val = np.where((e == 15) & (m == 7), np.nan, val)
    return sign * val


_POS = fp8_decode(np.arange(0, 127))      # codes 0..126: finite non-negative, increasing


def fp8_encode(x) -> np.ndarray:
    """Nearest E4M3FN code (uint8), saturating, ties to even code."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), FP8_MAX)
    j = np.searchsorted(_POS, a, side="left")        # _POS[j-1] < a <= _POS[j]
    j = np.clip(j, 1, 126)
    lo = j - 1
    dlo = a - _POS[lo]
    dhi = _POS[j] - a
    pick = np.where(dhi < dlo, j, np.where(dlo < dhi, lo, np.where(j % 2 == 0, j, lo)))
    pick = np.where(a == 0.0, 0, pick)
    code = pick.astype(np.int64) | np.where(np.signbit(x), 0x80, 0)
    code = np.where(np.isnan(x), 0x7F, code)
    return code.astype(np.uint8)


def column_scales(X) -> np.ndarray:
    """FP32 per-column scale amax / 448 (1 for an all-zero column)."""
    X = np.asarray(X, dtype=np.float32)
    amax = np.max(np.abs(X), axis=0).astype(np.float32)
    sc = (amax / np.float32(FP8_MAX)).astype(np.float32)
    return np.where(amax > 0, sc, np.float32(1.0)).astype(np.float32)


def fp8_quantize(X):
    """Codes [rows][R] uint8 and scales [R] float32 for an FP32 matrix."""
    X = np.asarray(X, dtype=np.float32)
    sc = column_scales(X)
    y = (X / sc[None, :]).astype(np.float32)          # FP32 division
    return fp8_encode(y), sc


def fp8_dequantize(codes, sc) -> np.ndarray:
    return fp8_decode(codes) * np.asarray(sc, dtype=np.float64)[None, :]
