"""Oracle rounding to the reduced-precision input formats (test infrastructure).

The paper covers FP32/FP64 real and complex GEMM only (Table 1); the reduced
precision modes are an extension, so these follow the format definitions
rather than the paper:

* bfloat16: sign, 8 exponent bits (bias 127, as binary32), 7 fraction bits.
* binary16 (IEEE 754): sign, 5 exponent bits (bias 15), 10 fraction bits,
  largest finite 65504, subnormal quantum 2^-24, overflow rounds to inf.
* FP8 E4M3 (OCP 8-bit floating point, the "FN" variant): sign, 4 exponent
  bits (bias 7), 3 fraction bits, no infinities, one NaN code per sign
  (S.1111.111), largest finite 448, subnormal quantum 2^-9.  Here rounding
  saturates to +-448 (the power-of-two absmax scale keeps inputs in range).

All rounding is round-to-nearest-even, done as exact FP64 arithmetic: for a
value x with binade exponent e = floor(log2|x|) (clamped to the format's
minimum normal exponent), the quantum is 2^(e - fraction_bits) and
``rint(x / quantum) * quantum`` is the rounded value (``np.rint`` rounds ties
to even; division by a power of two is exact).
"""
from __future__ import annotations

import numpy as np


def _round_to_format(x, frac_bits: int, emin: int):
    """RNE of FP64 values to a binary format with ``frac_bits`` fraction bits
    and minimum normal exponent ``emin`` (no overflow handling)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    fin = np.isfinite(x) & (x != 0)
    ax = np.abs(x[fin])
    e = np.floor(np.log2(ax))
    # log2 can be off by one ulp near binade edges: correct e so 2^e <= ax < 2^(e+1)
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > ax, e - 1, e)
    e = np.where(np.ldexp(1.0, (e + 1).astype(np.int64)) <= ax, e + 1, e)
    e = np.maximum(e, emin).astype(np.int64)
    q = np.ldexp(1.0, e - frac_bits)
    out[fin] = np.rint(x[fin] / q) * q
    return out


def bf16_round(x):
    """FP32 (or FP64) values -> nearest bfloat16 values (as float64).  NaN stays
    NaN; values past the largest bfloat16 round to +-inf."""
    r = _round_to_format(x, 7, -126)
    big = np.ldexp(1.0, 128)
    return np.where(np.isfinite(r) & (np.abs(r) >= big), np.copysign(np.inf, r), r)


def f16_round(x):
    """Values -> nearest IEEE binary16 values (as float64); overflow -> +-inf."""
    r = _round_to_format(x, 10, -14)
    return np.where(np.isfinite(r) & (np.abs(r) > 65504.0), np.copysign(np.inf, r), r)


E4M3_MAX = 448.0


def e4m3_round(x):
    """Values -> nearest E4M3 values (as float64), saturating at +-448."""
    r = _round_to_format(x, 3, -6)
    return np.where(np.isfinite(r) & (np.abs(r) > E4M3_MAX), np.copysign(E4M3_MAX, r), r)


def e4m3_decode(code):
    """8-bit E4M3 code(s) -> float64 values (NaN for S.1111.111)."""
    c = np.asarray(code, dtype=np.int64) & 0xFF
    s = np.where(c & 0x80, -1.0, 1.0)
    ef = (c >> 3) & 0xF
    mf = c & 0x7
    val = np.where(ef == 0, np.ldexp(mf.astype(np.float64), -9),
                   np.ldexp((8 + mf).astype(np.float64), (ef - 10).astype(np.int64)))
    val = s * val
    return np.where((ef == 15) & (mf == 7), np.nan, val)


def bf16_decode(code):
    """16-bit bfloat16 code(s) -> float64 values (the code is the top half of
    the binary32 pattern)."""
    c = np.asarray(code, dtype=np.uint32) & 0xFFFF
    return (c << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def f16_decode(code):
    """16-bit binary16 code(s) -> float64 values, decoded field by field."""
    c = np.asarray(code, dtype=np.int64) & 0xFFFF
    s = np.where(c & 0x8000, -1.0, 1.0)
    ef = (c >> 10) & 0x1F
    mf = c & 0x3FF
    val = np.where(ef == 0, np.ldexp(mf.astype(np.float64), -24),
                   np.ldexp((1024 + mf).astype(np.float64), (ef - 25).astype(np.int64)))
    val = np.where(ef == 31, np.where(mf == 0, np.inf, np.nan), val)
    return s * val


def fp8_scale(absmax: float) -> float:
    """Per-matrix power-of-two scale s = 2^floor(log2(448 / absmax)) so that
    |x*s| <= 448 and scaling is exact; 1 for an all-zero matrix."""
    if not np.isfinite(absmax) or absmax <= 0.0:
        return 1.0
    e = int(np.floor(np.log2(E4M3_MAX / absmax)))
    # guard the floor against log2 rounding
    while np.ldexp(absmax, e) > E4M3_MAX:
        e -= 1
    while np.ldexp(absmax, e + 1) <= E4M3_MAX:
        e += 1
    return float(np.ldexp(1.0, e))


def split_bf16(x):
    """FP32 x -> (hi, lo) with hi = bf16(x), lo = bf16(x - hi); x - hi is exact
    in FP32 (the split used by three-product bf16 compensation, Henry, Tang
    and Heinecke, ARITH 2019)."""
    x32 = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi = bf16_round(x32)
    lo = bf16_round(x32 - hi)
    return hi, lo
