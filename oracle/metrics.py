"""Error measures used by the parity checks (test infrastructure).

The normwise relative error of a computed C-hat against the FP64 result C*
is ||C-hat - C*||_F / ||C*||_F per problem; when C* is identically zero the
computed result must be identically zero too (reported as 0 or inf).

The scaled form divides by |alpha| * || |op(A)| |op(B)| ||_F + |beta| ||C0||_F
instead: any FP32 evaluation order of a K-term dot product plus the
epilogue stays below (K + 2) * 2^-24 in that measure (the standard
gamma_n bound for recursive, pairwise or blocked summation with fused
multiply-adds).  It is the gate of the reduced-precision modes, whose
log-uniform inputs make C* cancel far below the size of its terms.
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


def op_abs(arr, ld, rows, cols, trans):
    """|op(X)| in FP64 from a stored column-major matrix of ``rows`` x
    ``cols`` (the stored shape) with leading dimension ``ld``: the absolute
    value of every entry, transposed when ``trans`` (op(X) = X^T)."""
    x = np.abs(np.asarray(arr, np.float64)[:ld * cols].reshape(cols, ld).T[:rows, :])
    return x.T if trans else x


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


def scaled_error(c_hat, c_star, ta, tb, m, n, k, alpha, a_abs, lda, b_abs, ldb, beta, C0, ldc):
    """scaled_rel of one problem from its stored operands.

    ``a_abs`` / ``b_abs`` are the stored A and B magnitudes (FP64, the sum of
    the magnitudes of the terms a mode multiplies, e.g. |hi| + |lo|); ``C0``
    the stored initial C (its m x n part enters the denominator)."""
    ra, ca = (k, m) if ta else (m, k)
    rb, cb = (n, k) if tb else (k, n)
    ab = (abs_product_norm(op_abs(a_abs, lda, ra, ca, ta), op_abs(b_abs, ldb, rb, cb, tb))
          if k > 0 else 0.0)
    c0 = np.asarray(C0, np.float64)[:ldc * n].reshape(n, ldc).T[:m, :] if n > 0 else np.zeros(0)
    return scaled_rel(c_hat, c_star, alpha, ab, beta, float(np.linalg.norm(c0)))
