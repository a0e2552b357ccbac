"""CPU pins of the reduced-precision parity oracle and of the error measures
it is gated with.

* ``oracle.gemm_dequant`` (FP64 operands) against ``oracle.gemm`` (FP32
  operands, pinned in test_oracle.py) bit for bit on FP32-representable
  values, in every layout, with padded leading dimensions and the alpha = 0,
  beta = 0 and K = 0 rules; and against closed forms (identity, rank one) on
  values with more significant bits than FP32 holds.
* ``metrics.op_abs``, ``abs_product_norm``, ``scaled_rel`` and
  ``scaled_error`` against hand-computed 2 x 2 cases chosen so that a missing
  absolute value, a missing |beta| ||C0|| term, an op() not transposed, a
  signed alpha or a padded leading dimension read as data all change the
  value.
* ``lowp.gemm_lowp`` against the definitions: single-term modes equal the FP32
  oracle on the rounded values, split-bfloat16's three products plus the
  dropped lo*lo term equal the full (hi + lo)(hi + lo) product.
"""
import numpy as np
import pytest

import oracle
from oracle import lowp, metrics, quant

LAY = [(0, 0), (1, 0), (0, 1), (1, 1)]


def stored_random(rng, rows, cols, ld, lo=-1.0, hi=1.0):
    """Column-major FP32 storage of a rows x cols matrix at leading dimension
    ld, the padding rows filled with NaN (never read by a correct oracle)."""
    a = np.full((cols, ld), np.nan, np.float32)
    a[:, :rows] = rng.uniform(lo, hi, (cols, rows)).astype(np.float32)
    return a.reshape(-1)


@pytest.mark.parametrize("ta,tb", LAY)
def test_dequant_equals_fp32_oracle_bitwise(ta, tb):
    rng = np.random.default_rng(11)
    for (m, n, k) in [(1, 1, 1), (5, 3, 7), (16, 9, 33), (3, 17, 1), (8, 8, 80)]:
        ra, ca = (k, m) if ta else (m, k)
        rb, cb = (n, k) if tb else (k, n)
        lda, ldb, ldc = ra + 3, rb + 1, m + 2
        A = stored_random(rng, ra, ca, lda)
        B = stored_random(rng, rb, cb, ldb)
        C0 = stored_random(rng, m, n, ldc)
        for alpha, beta in [(1.25, -0.75), (0.0, 2.0), (-1.5, 0.0)]:
            want = oracle.gemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc)
            got = oracle.gemm_dequant(ta, tb, m, n, k, alpha, A.astype(np.float64), lda,
                                      B.astype(np.float64), ldb, beta, C0, ldc)
            assert np.isfinite(want).all()
            assert np.array_equal(got, want), (m, n, k, alpha, beta)


def test_dequant_quick_returns_and_nan_rules():
    m, n, k = 3, 2, 4
    A = np.full(m * k, np.nan)
    B = np.full(k * n, np.nan)
    C0 = np.arange(1, m * n + 1, dtype=np.float32)
    out = oracle.gemm_dequant(0, 0, m, n, k, 0.0, A, m, B, k, -2.0, C0, m)
    assert np.array_equal(out, -2.0 * C0.reshape(n, m).T.astype(np.float64))
    out = oracle.gemm_dequant(0, 0, m, n, 0, 3.0, A, m, B, 1, 0.5, C0, m)
    assert np.array_equal(out, 0.5 * C0.reshape(n, m).T.astype(np.float64))
    A1, B1 = np.ones(m * k), np.ones(k * n)
    C_nan = np.full(m * n, np.nan, np.float32)
    out = oracle.gemm_dequant(0, 0, m, n, k, 2.0, A1, m, B1, k, 0.0, C_nan, m)
    assert np.array_equal(out, np.full((m, n), 2.0 * k))
    assert oracle.gemm_dequant(0, 0, 0, 5, 3, 1.0, A1, 1, B1, 3, 1.0, None, 1).size == 0


@pytest.mark.parametrize("ta,tb", LAY)
def test_dequant_identity_beyond_fp32(ta, tb):
    """A = I: C = alpha*op(B) + beta*C0 for FP64 values FP32 cannot hold."""
    rng = np.random.default_rng(12)
    M, N = 6, 5
    opB = 1.0 + rng.integers(0, 2 ** 40, (M, N)) * 2.0 ** -40  # 41 significant bits
    assert not np.array_equal(opB.astype(np.float32).astype(np.float64), opB)
    Bs = opB.T if tb else opB
    C0 = rng.integers(-4, 5, (M, N)).astype(np.float32)
    out = oracle.gemm_dequant(ta, tb, M, N, M, 1.0, np.eye(M).reshape(-1), M,
                              Bs.T.reshape(-1).copy(), Bs.shape[0], 0.5,
                              C0.T.reshape(-1).copy(), M)
    assert np.array_equal(out, 1.0 * opB + 0.5 * C0.astype(np.float64))


@pytest.mark.parametrize("ta,tb", LAY)
def test_dequant_rank_one_closed_form(ta, tb):
    """op(A) = x 1^T, op(B) = 1 y^T: C = 2 K x y^T exactly (x with 26-bit and
    y with 20-bit significands, so K * x_i * y_j is exact in FP64)."""
    rng = np.random.default_rng(13)
    M, N, K = 7, 4, 80
    x = rng.integers(2 ** 25, 2 ** 26, M) * 2.0 ** -25 * rng.choice([-1, 1], M)
    y = rng.integers(1, 2 ** 20, N) * 2.0 ** -20
    opA = np.outer(x, np.ones(K))
    opB = np.outer(np.ones(K), y)
    As = opA.T if ta else opA
    Bs = opB.T if tb else opB
    out = oracle.gemm_dequant(ta, tb, M, N, K, 2.0, As.T.reshape(-1).copy(), As.shape[0],
                              Bs.T.reshape(-1).copy(), Bs.shape[0], 0.0, None, M)
    assert np.array_equal(out, 2.0 * K * np.outer(x, y))


def test_op_abs_transposes_and_skips_padding():
    # stored 2 x 3 matrix at ld 4: columns [1,-2], [3,4], [-5,6]; padding NaN
    st = np.array([1, -2, np.nan, np.nan, 3, 4, np.nan, np.nan, -5, 6, np.nan, np.nan])
    assert np.array_equal(metrics.op_abs(st, 4, 2, 3, 0), np.array([[1, 3, 5], [2, 4, 6.0]]))
    assert np.array_equal(metrics.op_abs(st, 4, 2, 3, 1), np.array([[1, 2], [3, 4], [5, 6.0]]))


def test_abs_product_norm_hand_computed():
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    b = np.array([[1.0, 0.0], [2.0, 3.0]])
    # |A||B| = [[5, 6], [11, 12]]
    assert metrics.abs_product_norm(a, b) == np.sqrt(326.0)
    assert metrics.abs_product_norm(b, a) == np.sqrt(1 + 4 + 121 + 256.0)  # [[1,2],[11,16]]


def test_scaled_rel_hand_computed_and_degenerate():
    c_star = np.zeros((2, 2))
    c_hat = np.array([[3.0, 0.0], [0.0, 4.0]])
    v = metrics.scaled_rel(c_hat, c_star, -2.0, np.sqrt(326.0), 0.5, np.sqrt(6.0))
    assert v == 5.0 / (2.0 * np.sqrt(326.0) + 0.5 * np.sqrt(6.0))
    assert metrics.scaled_rel(c_star, c_star, 0.0, 1.0, 0.0, 1.0) == 0.0
    assert metrics.scaled_rel(c_hat, c_star, 0.0, 1.0, 0.0, 1.0) == float("inf")


def test_scaled_error_end_to_end_tn():
    """TN, m = n = k = 2, op(A) = [[1,-2],[3,4]] stored transposed at lda 3,
    op(B) = [[-1,0],[2,-3]] at ldb 2, C0 = [[1,-1],[2,0]], alpha = -2,
    beta = 0.5: the denominator is 2 sqrt(326) + 0.5 sqrt(6).  Without the
    absolute values it would use sqrt(230); with op(A) left untransposed,
    sqrt(374); without the C0 term, 2 sqrt(326)."""
    A = np.array([1, -2, 100, 3, 4, 100.0])   # stored K x M = [[1,3],[-2,4]]
    B = np.array([-1, 2, 0, -3.0])
    C0 = np.array([1, 2, -1, 0], np.float32)
    c_star = np.zeros((2, 2))
    c_hat = np.array([[3.0, 0.0], [0.0, 4.0]])
    v = metrics.scaled_error(c_hat, c_star, 1, 0, 2, 2, 2, -2.0, np.abs(A), 3, np.abs(B), 2,
                             0.5, C0, 2)
    assert v == 5.0 / (2.0 * np.sqrt(326.0) + 0.5 * np.sqrt(6.0))
    # the stored operands may carry their signs: op_abs takes magnitudes
    assert metrics.scaled_error(c_hat, c_star, 1, 0, 2, 2, 2, -2.0, A, 3, B, 2, 0.5, C0, 2) == v
    # K = 0: only the C0 term remains
    assert metrics.scaled_error(c_hat, c_star, 1, 0, 2, 2, 0, -2.0, A, 1, B, 1, 0.5, C0, 2) == \
        5.0 / (0.5 * np.sqrt(6.0))


def problem(rng, ta, tb, m, n, k):
    ra, ca = (k, m) if ta else (m, k)
    rb, cb = (n, k) if tb else (k, n)
    mag = lambda s: (10.0 ** rng.uniform(-3, 3, s) * rng.choice([-1, 1], s)).astype(np.float32)
    return mag(ra * ca), ra, mag(rb * cb), rb, mag(m * n)


@pytest.mark.parametrize("mode", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("ta,tb", LAY)
def test_single_term_modes_equal_fp32_oracle_on_rounded_values(mode, ta, tb):
    rng = np.random.default_rng(14)
    m, n, k = 9, 6, 13
    A, lda, B, ldb, C0 = problem(rng, ta, tb, m, n, k)
    got, sa, sb = lowp.gemm_lowp(mode, ta, tb, m, n, k, 1.0, A, lda, B, ldb, 1.0, C0, m)
    rnd = {"bf16": quant.bf16_round, "f16": quant.f16_round,
           "e4m3": lambda v: quant.e4m3_round(v)}[mode]
    if mode == "e4m3":
        sa_w = quant.fp8_scale(float(np.abs(A).max()))
        sb_w = quant.fp8_scale(float(np.abs(B).max()))
        assert (sa, sb) == (sa_w, sb_w)
        Aq = rnd(A.astype(np.float64) * sa) / sa
        Bq = rnd(B.astype(np.float64) * sb) / sb
        assert np.abs(A * sa).max() <= 448.0 and np.abs(A * sa).max() > 224.0
    else:
        assert (sa, sb) == (1.0, 1.0)
        Aq, Bq = rnd(A.astype(np.float64)), rnd(B.astype(np.float64))
    # the rounded values are FP32 numbers: the FP32-input oracle must agree bit for bit
    assert np.array_equal(Aq.astype(np.float32).astype(np.float64), Aq)
    want = oracle.gemm(ta, tb, m, n, k, 1.0, Aq.astype(np.float32), lda, Bq.astype(np.float32),
                       ldb, 1.0, C0, m)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("ta,tb", LAY)
def test_split_bf16_three_products(ta, tb):
    rng = np.random.default_rng(15)
    m, n, k = 7, 5, 11
    A, lda, B, ldb, C0 = problem(rng, ta, tb, m, n, k)
    got, _, _ = lowp.gemm_lowp("bf16x3", ta, tb, m, n, k, 1.0, A, lda, B, ldb, 1.0, C0, m)
    ah, al = quant.split_bf16(A)
    bh, bl = quant.split_bf16(B)
    full = oracle.gemm_dequant(ta, tb, m, n, k, 1.0, ah + al, lda, bh + bl, ldb, 1.0, C0, m)
    lolo = oracle.gemm_dequant(ta, tb, m, n, k, 1.0, al, lda, bl, ldb, 0.0, None, m)
    # hi + lo carries 16 of the master's 24 significant bits
    a64 = A.astype(np.float64)
    assert np.all(np.abs(ah + al - a64) <= 2.0 ** -16 * np.abs(a64))
    scale = metrics.abs_product_norm(metrics.op_abs(np.abs(A), lda, *((k, m) if ta else (m, k)), ta),
                                     metrics.op_abs(np.abs(B), ldb, *((n, k) if tb else (k, n)), tb))
    assert np.abs(got + lolo - full).max() <= 1e-14 * (scale + np.abs(C0).max())
    # the dropped term is not negligible at FP64 resolution: a mode that kept
    # it (or dropped another) would be caught
    assert np.abs(lolo).max() > 1e-10 * scale
