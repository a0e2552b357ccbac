"""Parity oracle of the reduced-precision modes (test infrastructure).

A and B are rounded from their FP32 masters by the format definitions in
``quant.py``; the product is then the plain FP64 GEMM of ``oracle.gemm_dequant``
on the dequantised values (every product of two such values is exact in
FP32, so a correct FP32-accumulating kernel meets the FP32 gate against
this).  Split-bfloat16 multiplies three term pairs, hi*hi + hi*lo + lo*hi
(the lo*lo term is dropped by the method: Henry, Tang and Heinecke, ARITH
2019), each an FP64 GEMM, summed in FP64.

Modes are named "bf16", "f16", "e4m3" and "bf16x3".
"""
from __future__ import annotations

import numpy as np

from . import gemm_dequant, quant

MODES = ("bf16", "f16", "e4m3", "bf16x3")


def dequant_terms(mode: str, x):
    """(list of dequantised FP64 term arrays, scale) of an FP32 master array:
    one term, or [hi, lo] for split-bfloat16.  The scale is the FP8
    per-matrix power of two (1 otherwise); the terms already include 1/s."""
    x64 = np.asarray(x, np.float32).astype(np.float64)
    if mode == "bf16":
        return [quant.bf16_round(x64)], 1.0
    if mode == "f16":
        return [quant.f16_round(x64)], 1.0
    if mode == "e4m3":
        amax = float(np.max(np.abs(x64))) if x64.size else 0.0
        s = quant.fp8_scale(amax)
        return [quant.e4m3_round(x64 * s) / s], s
    if mode == "bf16x3":
        hi, lo = quant.split_bf16(x64)
        return [hi, lo], 1.0
    raise ValueError(mode)


def gemm_lowp(mode, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc):
    """C* of one problem in a reduced-precision mode from FP32 masters A, B
    (C0 and the scalars stay FP32).  Returns (m x n FP64, scale_a, scale_b)."""
    a_terms, sa = dequant_terms(mode, A)
    b_terms, sb = dequant_terms(mode, B)
    args = (ta, tb, m, n, k, alpha)
    if mode != "bf16x3":
        return gemm_dequant(*args, a_terms[0], lda, b_terms[0], ldb, beta, C0, ldc), sa, sb
    (ah, al), (bh, bl) = a_terms, b_terms
    r = gemm_dequant(*args, ah, lda, bh, ldb, beta, C0, ldc)
    r = r + gemm_dequant(*args, ah, lda, bl, ldb, 0.0, None, ldc)
    r = r + gemm_dequant(*args, al, lda, bh, ldb, 0.0, None, ldc)
    return r, sa, sb


def abs_terms(mode, x):
    """Sum of the magnitudes of the dequantised terms (the operand of the
    scaled error measure)."""
    terms, _ = dequant_terms(mode, x)
    return sum(np.abs(t) for t in terms)
