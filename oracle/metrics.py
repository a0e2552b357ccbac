"""Error measures used by the parity checks (test infrastructure).

The normwise relative error of a computed C-hat against the FP64 result C*
is ||C-hat - C*||_F / ||C*||_F per problem; when C* is identically zero the
computed result must be identically zero too (reported as 0 or inf).

The scaled form divides by |alpha| * || |op(A)| |op(B)| ||_F + |beta| ||C0||_F
instead: any FP32 evaluation order of a K-term dot product plus the
epilogue stays below (K + 2) * 2^-24 in that measure (the standard
gamma_n bound for recursive, pairwise or blocked summation with fused
multiply-adds).
"""
from __future__ import annotations

import numpy as np


def normwise_rel(c_hat, c_star) -> float:
    c_hat = np.asarray(c_hat, dtype=np.float64)
    c_star = np.asarray(c_star, dtype=np.float64)
    den = np.linalg.norm(c_star.ravel())
    num = np.linalg.norm((c_hat - c_star).ravel())
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)


def abs_product_norm(opA_abs, opB_abs) -> float:
    """|| |op(A)| |op(B)| ||_F from nonnegative FP64 operands."""
    return float(np.linalg.norm((np.asarray(opA_abs) @ np.asarray(opB_abs)).ravel()))


def scaled_rel(c_hat, c_star, alpha, absAB_norm, beta, c0_norm) -> float:
    c_hat = np.asarray(c_hat, dtype=np.float64)
    c_star = np.asarray(c_star, dtype=np.float64)
    den = abs(alpha) * absAB_norm + abs(beta) * c0_norm
    num = np.linalg.norm((c_hat - c_star).ravel())
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)
