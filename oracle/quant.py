"""Reference quantisers for the reduced-precision dictionary copies.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The precision form of the decoder stores the dictionary as BF16, or as
OCP FP8 E4M3 ("e4m3fn": bias 7, no infinities, 0x7F/0xFF are NaN, largest
finite value 448) with one FP32 scale per column.  These functions define the
codes bit by bit from the formats' definitions, in numpy integer arithmetic:

* BF16: the top 16 bits of the FP32 pattern after round-to-nearest-even on
  the 16 dropped bits.
* FP8 scale: s_m = fp32(amax_m / 448), computed as one correctly rounded FP32
  division; an all-zero column gets s_m = 1.
* FP8 code: v = fp32(psi_nm / s_m) (one correctly rounded FP32 division),
  then round-to-nearest-even to e4m3fn, saturating to +-448.
"""
from __future__ import annotations

import numpy as np

FP8_MAX = 448.0


def bf16_codes(a: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest even."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    rounded = (u + 0x7FFF + lsb) >> 16
    return (rounded & 0xFFFF).astype(np.uint16)


def bf16_decode(codes: np.ndarray) -> np.ndarray:
    """BF16 bit patterns -> FP32 values (exact)."""
    return (np.asarray(codes, dtype=np.uint32) << 16).view(np.float32)


def fp8_decode(codes: np.ndarray) -> np.ndarray:
    """e4m3fn bit patterns -> FP32 values (exact; 0x7F/0xFF -> NaN)."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    f = c & 0x7
    mag = np.where(e == 0, f * 2.0 ** -9, (1.0 + f / 8.0) * np.exp2(e - 7.0))
    mag = np.where((c & 0x7F) == 0x7F, np.nan, mag)
    return (sign * mag).astype(np.float32)


# every finite non-negative e4m3fn value, ascending, with its code
_POS_CODES = np.arange(0, 0x7F, dtype=np.uint8)
_POS_VALS = fp8_decode(_POS_CODES).astype(np.float64)


def fp8_codes(v: np.ndarray) -> np.ndarray:
    """FP32 values -> e4m3fn codes: round to nearest even, saturate at 448.

    Works on magnitudes: finds the two neighbouring representable values and
    picks the nearer, the one with an even code (even mantissa) on a tie.
    """
    v = np.asarray(v, dtype=np.float32).astype(np.float64)
    if np.isnan(v).any():
        raise ValueError("NaN input")
    mag = np.minimum(np.abs(v), FP8_MAX)
    hi = np.searchsorted(_POS_VALS, mag, side="left")      # first value >= mag
    hi = np.minimum(hi, len(_POS_VALS) - 1)
    lo = np.maximum(hi - 1, 0)
    exact = _POS_VALS[hi] == mag
    dlo = mag - _POS_VALS[lo]
    dhi = _POS_VALS[hi] - mag
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((_POS_CODES[hi] & 1) == 0))
    code = np.where(exact, hi, np.where(pick_hi, hi, lo)).astype(np.uint8)
    neg = np.signbit(v)
    return np.where(neg, code | 0x80, code).astype(np.uint8)


def fp8_column_scales(psi: np.ndarray) -> np.ndarray:
    """Per-column FP32 scale s_m = fp32(max_n |psi_nm| / 448), 1 for zero columns."""
    amax = np.max(np.abs(np.asarray(psi, dtype=np.float32)), axis=0)
    s = (amax / np.float32(FP8_MAX)).astype(np.float32)
    return np.where(amax == 0, np.float32(1.0), s).astype(np.float32)


def fp8_quantise(psi: np.ndarray):
    """(codes uint8 (N, M) Fortran, scales float32 (M,)) for a dictionary."""
    psi = np.asarray(psi, dtype=np.float32)
    s = fp8_column_scales(psi)
    q = (psi / s[None, :]).astype(np.float32)
    return np.asfortranarray(fp8_codes(q).reshape(psi.shape)), s
