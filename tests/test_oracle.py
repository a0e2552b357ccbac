"""Pins for the FP64 GEMM oracle (CPU only).

Each check compares the oracle with something other than itself: exact
closed forms (identity, permutation, rank-one), special cases, brute force
over tiny integer matrices against the outer-product expansion, numpy's
float64 matmul (a library routine), and layout metamorphic relations.  A
dropped term, a wrong sign, a swapped index or a transposed operand in the
oracle fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2208_09822_amd import inputs

LAY = {"NN": (0, 0), "TN": (1, 0), "NT": (0, 1), "TT": (1, 1)}


def col_major(mat):
    """2-D array -> flat column-major FP32 storage, ld = rows."""
    return np.asarray(mat, dtype=np.float32).T.reshape(-1).copy()


def stored(opmat, trans):
    """The stored matrix whose op() is ``opmat``."""
    return opmat.T if trans else opmat


def run(layout, opA, opB, alpha, beta, C0):
    ta, tb = LAY[layout]
    M, K = opA.shape
    _, N = opB.shape
    As = stored(opA, ta); Bs = stored(opB, tb)
    return oracle.gemm(ta, tb, M, N, K, alpha, col_major(As), max(As.shape[0], 1),
                       col_major(Bs), max(Bs.shape[0], 1), beta,
                       None if C0 is None else col_major(C0), max(M, 1))


@pytest.mark.parametrize("layout", list(LAY))
def test_identity(layout):
    rng = np.random.default_rng(1)
    M, N = 7, 5
    B = rng.integers(-4, 5, (M, N)).astype(np.float32)
    C0 = rng.integers(-4, 5, (M, N)).astype(np.float32)
    out = run(layout, np.eye(M, dtype=np.float32), B, 1.5, -0.5, C0)
    assert np.array_equal(out, 1.5 * B.astype(np.float64) - 0.5 * C0)


@pytest.mark.parametrize("layout", list(LAY))
def test_permutation_rows_and_cols(layout):
    rng = np.random.default_rng(2)
    M, K, N = 6, 6, 9
    perm = rng.permutation(M)
    P = np.zeros((M, K), np.float32)
    P[np.arange(M), perm] = 1.0
    B = rng.uniform(-1, 1, (K, N)).astype(np.float32)
    out = run(layout, P, B, 1.0, 0.0, None)
    assert np.array_equal(out, B[perm].astype(np.float64))
    # permutation on the right permutes columns
    A = rng.uniform(-1, 1, (M, N)).astype(np.float32)
    Q = np.zeros((N, N), np.float32)
    qp = rng.permutation(N)
    Q[qp, np.arange(N)] = 1.0  # column j of A@Q is column qp[j] of A
    out2 = run(layout, A, Q, 1.0, 0.0, None)
    assert np.array_equal(out2, A[:, qp].astype(np.float64))


@pytest.mark.parametrize("layout", list(LAY))
def test_rank_one_closed_form(layout):
    rng = np.random.default_rng(3)
    M, N, K = 9, 4, 13
    x = rng.integers(-4, 5, M).astype(np.float32)
    y = rng.integers(-4, 5, N).astype(np.float32)
    opA = np.repeat(x[:, None], K, axis=1)       # x 1^T
    opB = np.repeat(y[None, :], K, axis=0)       # 1 y^T
    C0 = rng.integers(-4, 5, (M, N)).astype(np.float32)
    out = run(layout, opA, opB, -2.0, 1.5, C0)
    expect = -2.0 * K * np.outer(x, y).astype(np.float64) + 1.5 * C0
    assert np.array_equal(out, expect)


def test_alpha_zero_and_k_zero_do_not_read_ab():
    C0 = np.arange(12, dtype=np.float32).reshape(3, 4)
    # A and B passed as None: the oracle must not touch them
    for alpha, k in ((0.0, 5), (1.0, 0)):
        out = oracle.gemm(0, 0, 3, 4, k, alpha, None, 3, None, max(k, 1), 0.5, col_major(C0), 3)
        assert np.array_equal(out, 0.5 * C0.astype(np.float64))


def test_beta_zero_ignores_nan_c():
    rng = np.random.default_rng(4)
    A = rng.uniform(-1, 1, (4, 3)).astype(np.float32)
    B = rng.uniform(-1, 1, (3, 5)).astype(np.float32)
    C0 = np.full((4, 5), np.nan, np.float32)
    out = run("NN", A, B, 1.0, 0.0, C0)
    assert np.all(np.isfinite(out))
    out_b = run("NN", A, B, 1.0, 1.0, C0)
    assert np.all(np.isnan(out_b))


def test_nan_in_a_propagates_to_its_row_only():
    A = np.ones((3, 2), np.float32); A[1, 0] = np.nan
    B = np.ones((2, 4), np.float32)
    out = run("NN", A, B, 1.0, 0.0, None)
    assert np.all(np.isnan(out[1])) and np.all(np.isfinite(out[[0, 2]]))


def test_empty_shapes():
    assert oracle.gemm(0, 0, 0, 5, 3, 1.0, None, 1, None, 3, 1.0, None, 1).shape == (0, 5)
    assert oracle.gemm(0, 0, 4, 0, 3, 1.0, None, 4, None, 3, 1.0, None, 4).shape == (4, 0)


def test_brute_force_tiny_integer():
    """Every op(A), op(B) over {-1,0,1} for M, N, K <= 2 (all four layouts),
    against the outer-product expansion C = sum_p a_p b_p^T (numpy.outer)."""
    vals = (-1.0, 0.0, 1.0)
    for M, N, K in itertools.product((1, 2), repeat=3):
        mats_a = [np.array(v, np.float32).reshape(M, K) for v in itertools.product(vals, repeat=M * K)]
        mats_b = [np.array(v, np.float32).reshape(K, N) for v in itertools.product(vals, repeat=K * N)]
        if M * K * K * N > 8:  # keep 2x2x2 at a strided sample of pairs
            pairs = [(a, b) for ia, a in enumerate(mats_a) for ib, b in enumerate(mats_b)
                     if (ia * 7 + ib) % 5 == 0]
        else:
            pairs = [(a, b) for a in mats_a for b in mats_b]
        for layout in LAY:
            for a, b in pairs:
                expect = sum(np.outer(a[:, p], b[p, :]) for p in range(K))
                out = run(layout, a, b, 1.0, 0.0, None)
                assert np.array_equal(out, expect), (layout, a, b)


@pytest.mark.parametrize("layout", list(LAY))
def test_against_numpy_matmul(layout):
    rng = np.random.default_rng(5)
    for M, N, K in ((1, 1, 1), (5, 3, 80), (17, 33, 31), (80, 80, 80), (64, 1, 48)):
        opA = rng.uniform(-1, 1, (M, K)).astype(np.float32)
        opB = rng.uniform(-1, 1, (K, N)).astype(np.float32)
        C0 = rng.uniform(-1, 1, (M, N)).astype(np.float32)
        out = run(layout, opA, opB, 0.75, -1.25, C0)
        ref = 0.75 * (opA.astype(np.float64) @ opB.astype(np.float64)) - 1.25 * C0.astype(np.float64)
        bound = (K + 2) * 2.0 ** -53 * (0.75 * (np.abs(opA) @ np.abs(opB)) + 1.25 * np.abs(C0))
        assert np.all(np.abs(out - ref) <= 2 * bound + 1e-300)
        # integer inputs: exact
        ia = rng.integers(-4, 5, (M, K)).astype(np.float32)
        ib = rng.integers(-4, 5, (K, N)).astype(np.float32)
        assert np.array_equal(run(layout, ia, ib, 1.0, 0.0, None),
                              ia.astype(np.float64) @ ib.astype(np.float64))


def test_layout_metamorphic():
    """Same op(A), op(B) in every stored layout gives the same C; and
    op = TT equals (NN with the operands swapped) transposed."""
    rng = np.random.default_rng(6)
    M, N, K = 11, 7, 9
    opA = rng.uniform(-1, 1, (M, K)).astype(np.float32)
    opB = rng.uniform(-1, 1, (K, N)).astype(np.float32)
    outs = [run(l, opA, opB, 1.0, 0.0, None) for l in LAY]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # TT with stored A (K x M) = opA^T, stored B (N x K) = opB^T:
    # C = A_s^T B_s^T = (B_s A_s)^T  -> NN of (B_s, A_s), transposed
    As = opA.T.copy(); Bs = opB.T.copy()
    tt = oracle.gemm(1, 1, M, N, K, 1.0, col_major(As), K, col_major(Bs), N, 0.0, None, M)
    nn = oracle.gemm(0, 0, N, M, K, 1.0, col_major(Bs), N, col_major(As), K, 0.0, None, N)
    assert np.array_equal(tt, nn.T)


def test_leading_dimension_padding_ignored():
    rng = np.random.default_rng(7)
    M, N, K = 5, 6, 7
    A = rng.uniform(-1, 1, (M, K)).astype(np.float32)
    B = rng.uniform(-1, 1, (K, N)).astype(np.float32)
    base = oracle.gemm(0, 0, M, N, K, 1.0, col_major(A), M, col_major(B), K, 0.0, None, M)
    Ap = np.full((M + 3, K), 1e30, np.float32); Ap[:M] = A
    Bp = np.full((K + 2, N), -1e30, np.float32); Bp[:K] = B
    padded = oracle.gemm(0, 0, M, N, K, 1.0, col_major(Ap), M + 3, col_major(Bp), K + 2, 0.0, None, M)
    assert np.array_equal(base, padded)


def test_batch_driver_matches_single_calls():
    ps = inputs.uneven_batch(300, seed=11)
    out, secs, off = oracle.gemm_batch(ps, nthreads=4)
    assert secs >= 0
    for q in range(0, ps.count, 37):
        M, N = int(ps.m[q]), int(ps.n[q])
        single = oracle.gemm(int(ps.trans[q]) & 1, int(ps.trans[q]) >> 1, M, N, int(ps.k[q]),
                             float(ps.alpha[q]), ps.A(q), int(ps.lda[q]), ps.B(q), int(ps.ldb[q]),
                             float(ps.beta[q]), ps.C(q), int(ps.ldc[q]))
        got = out[off[q]:off[q] + M * N].reshape(N, M).T
        assert np.array_equal(single, got)


# ---- DGEMM (FP64 operands): pinned independently of the FP32-input loop

def _rand64(rng, shape):
    return rng.uniform(-1, 1, shape)


def test_dgemm_identity_and_rank_one():
    rng = np.random.Generator(np.random.PCG64(901))
    m, n = 7, 5
    B = _rand64(rng, (m, n))
    C0 = _rand64(rng, (m, n))
    got = oracle.dgemm(0, 0, m, n, m, 1.5, np.eye(m).ravel(order="F"), m, B.ravel(order="F"), m,
                       -0.5, C0.ravel(order="F"), m)
    assert np.array_equal(got, 1.5 * B - 0.5 * C0)
    x = rng.integers(-4, 5, m).astype(np.float64)
    y = rng.integers(-4, 5, n).astype(np.float64)
    K = 9
    A = np.outer(x, np.ones(K))
    Bm = np.outer(np.ones(K), y)
    got = oracle.dgemm(0, 0, m, n, K, 2.0, A.ravel(order="F"), m, Bm.ravel(order="F"), K, 0.0,
                       None, m)
    assert np.array_equal(got, 2.0 * K * np.outer(x, y))


def test_dgemm_quick_returns_and_nan_rules():
    m, n, k = 3, 4, 5
    A = np.full(m * k, np.nan)
    C0 = np.arange(m * n, dtype=np.float64)
    got = oracle.dgemm(0, 0, m, n, k, 0.0, A, m, A, k, 2.0, C0, m)
    assert np.array_equal(got, 2.0 * C0.reshape(n, m).T)
    ones = np.ones(m * k)
    got = oracle.dgemm(0, 0, m, n, k, 1.0, ones, m, np.ones(k * n), k, 0.0, np.full(m * n, np.nan), m)
    assert np.array_equal(got, np.full((m, n), float(k)))


@pytest.mark.parametrize("lay", ["NN", "NT", "TN", "TT"])
def test_dgemm_against_numpy_and_layouts(lay):
    rng = np.random.Generator(np.random.PCG64(902))
    m, n, k = 13, 11, 17
    Aop = _rand64(rng, (m, k))
    Bop = _rand64(rng, (k, n))
    C0 = _rand64(rng, (m, n))
    ta, tb = lay[0] == "T", lay[1] == "T"
    A = (Aop.T if ta else Aop).ravel(order="F")
    B = (Bop.T if tb else Bop).ravel(order="F")
    got = oracle.dgemm(int(ta), int(tb), m, n, k, 0.75, A, k if ta else m, B, n if tb else k,
                       1.25, C0.ravel(order="F"), m)
    ref = 0.75 * (Aop @ Bop) + 1.25 * C0
    assert np.linalg.norm(got - ref) <= (k + 2) * 2.0 ** -52 * np.linalg.norm(
        0.75 * np.abs(Aop) @ np.abs(Bop) + 1.25 * np.abs(C0))


def test_dgemm_brute_force_tiny():
    vals = (-1.0, 0.0, 1.0)
    for m, n, k in [(1, 1, 1), (1, 2, 2), (2, 1, 2), (2, 2, 1)]:
        for a in itertools.product(vals, repeat=m * k):
            b = np.array([1.0, -1.0][:k * n] + [0.0] * max(0, k * n - 2))
            got = oracle.dgemm(0, 0, m, n, k, 1.0, np.array(a), m, b, k, 0.0, None, m)
            for i in range(m):
                for j in range(n):
                    assert got[i, j] == sum(a[i + p * m] * b[p + j * k] for p in range(k))


# ---- CGEMM (complex): pinned independently

def _crand(rng, shape):
    return (rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)).astype(np.complex64)


def test_cgemm_identity_and_scalars():
    rng = np.random.Generator(np.random.PCG64(911))
    m, n = 6, 4
    B = _crand(rng, (m, n))
    C0 = _crand(rng, (m, n))
    al, be = 1.5 - 0.5j, 0.25 + 2j
    got = oracle.cgemm(0, 0, m, n, m, al, np.eye(m, dtype=np.complex64).ravel(order="F"), m,
                       B.ravel(order="F"), m, be, C0.ravel(order="F"), m)
    exp = al * B.astype(np.complex128) + be * C0.astype(np.complex128)
    assert np.array_equal(got, exp)


def test_cgemm_rank_one_gaussian_integers():
    rng = np.random.Generator(np.random.PCG64(912))
    m, n, K = 5, 3, 7
    x = (rng.integers(-3, 4, m) + 1j * rng.integers(-3, 4, m)).astype(np.complex64)
    y = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex64)
    A = np.outer(x, np.ones(K)).astype(np.complex64)
    B = np.outer(np.ones(K), y).astype(np.complex64)
    got = oracle.cgemm(0, 0, m, n, K, 1j, A.ravel(order="F"), m, B.ravel(order="F"), K, 0, None, m)
    assert np.array_equal(got, 1j * K * np.outer(x.astype(np.complex128), y.astype(np.complex128)))


def test_cgemm_quick_return_rules():
    m, n, k = 2, 3, 4
    A = np.full(m * k, np.nan, dtype=np.complex64)
    C0 = (np.arange(m * n) + 1j).astype(np.complex64)
    got = oracle.cgemm(0, 0, m, n, k, 0, A, m, A, k, 2 - 1j, C0, m)
    assert np.array_equal(got, (2 - 1j) * C0.astype(np.complex128).reshape(n, m).T)
    ones = np.ones(m * k, dtype=np.complex64)
    got = oracle.cgemm(0, 0, m, n, k, 1, ones, m, np.ones(k * n, dtype=np.complex64), k, 0,
                       np.full(m * n, np.nan, dtype=np.complex64), m)
    assert np.array_equal(got, np.full((m, n), float(k), dtype=np.complex128))


@pytest.mark.parametrize("lay", ["NN", "NT", "TN", "TT"])
def test_cgemm_against_numpy(lay):
    rng = np.random.Generator(np.random.PCG64(913))
    m, n, k = 9, 7, 11
    Aop, Bop, C0 = _crand(rng, (m, k)), _crand(rng, (k, n)), _crand(rng, (m, n))
    ta, tb = lay[0] == "T", lay[1] == "T"
    A = (Aop.T if ta else Aop).ravel(order="F")
    B = (Bop.T if tb else Bop).ravel(order="F")
    al, be = 0.5 + 0.25j, -1 + 0.5j
    got = oracle.cgemm(int(ta), int(tb), m, n, k, al, A, k if ta else m, B, n if tb else k, be,
                       C0.ravel(order="F"), m)
    ref = al * (Aop.astype(np.complex128) @ Bop.astype(np.complex128)) + be * C0.astype(np.complex128)
    assert np.max(np.abs(got - ref)) <= 1e-12


# ---- ZGEMM (complex, FP64 storage): pinned independently

def _zrand(rng, shape):
    return rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)


def _gauss_int(rng, shape, lo=-3, hi=4):
    return (rng.integers(lo, hi, shape) + 1j * rng.integers(lo, hi, shape)).astype(np.complex128)


def test_zgemm_identity_and_scalars():
    # A = I: C* = alpha*B + beta*C0; dyadic entries keep every step exact
    rng = np.random.Generator(np.random.PCG64(931))
    m, n = 6, 4
    B = _gauss_int(rng, (m, n)) / 2
    C0 = _gauss_int(rng, (m, n)) / 4
    al, be = 1.5 - 0.5j, 0.25 + 2j
    got = oracle.zgemm(0, 0, m, n, m, al, np.eye(m, dtype=np.complex128).ravel(order="F"), m,
                       B.ravel(order="F"), m, be, C0.ravel(order="F"), m)
    assert np.array_equal(got, al * B + be * C0)


def test_zgemm_rank_one_gaussian_integers():
    # (x 1^T)(1 y^T) = K x y^T, exact on Gaussian integers
    rng = np.random.Generator(np.random.PCG64(932))
    m, n, K = 5, 3, 7
    x, y = _gauss_int(rng, m), _gauss_int(rng, n)
    A = np.outer(x, np.ones(K))
    B = np.outer(np.ones(K), y)
    got = oracle.zgemm(0, 0, m, n, K, 1j, A.ravel(order="F"), m, B.ravel(order="F"), K, 0, None, m)
    assert np.array_equal(got, 1j * K * np.outer(x, y))


def test_zgemm_quick_return_rules():
    m, n, k = 2, 3, 4
    A = np.full(m * k, np.nan, dtype=np.complex128)
    C0 = np.arange(m * n) + 1j
    got = oracle.zgemm(0, 0, m, n, k, 0, A, m, A, k, 2 - 1j, C0, m)
    assert np.array_equal(got, (2 - 1j) * C0.reshape(n, m).T)
    ones = np.ones(m * k, dtype=np.complex128)
    got = oracle.zgemm(0, 0, m, n, k, 1, ones, m, np.ones(k * n, dtype=np.complex128), k, 0,
                       np.full(m * n, np.nan, dtype=np.complex128), m)
    assert np.array_equal(got, np.full((m, n), float(k), dtype=np.complex128))


def test_zgemm_brute_force_tiny():
    # every entry from the definition, Python complex arithmetic, parts in {-1, 0, 1}
    rng = np.random.Generator(np.random.PCG64(933))
    for (m, n, k) in [(1, 1, 1), (2, 3, 2), (3, 2, 4)]:
        a = _gauss_int(rng, m * k, -1, 2)
        b = _gauss_int(rng, k * n, -1, 2)
        got = oracle.zgemm(0, 0, m, n, k, 1, a, m, b, k, 0, None, m)
        for i in range(m):
            for j in range(n):
                assert got[i, j] == sum(complex(a[i + p * m]) * complex(b[p + j * k])
                                        for p in range(k))


def test_zgemm_equals_cgemm_on_widened_inputs():
    # FP32 complex inputs widen exactly, and both loops use Eq. 2's expansion
    # in FP64 in the same order, so the two oracles agree bit for bit
    rng = np.random.Generator(np.random.PCG64(934))
    m, n, k = 7, 5, 9
    A = _crand(rng, (k, m)).ravel(order="F")
    B = _crand(rng, (n, k)).ravel(order="F")
    C0 = _crand(rng, (m, n)).ravel(order="F")
    al, be = np.complex64(0.75 - 0.5j), np.complex64(-0.5 + 1j)
    want = oracle.cgemm(1, 1, m, n, k, al, A, k, B, n, be, C0, m)
    got = oracle.zgemm(1, 1, m, n, k, complex(al), A.astype(np.complex128), k,
                       B.astype(np.complex128), n, complex(be), C0.astype(np.complex128), m)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("lay", ["NN", "NT", "TN", "TT"])
def test_zgemm_against_numpy(lay):
    rng = np.random.Generator(np.random.PCG64(935))
    m, n, k = 9, 7, 11
    Aop, Bop, C0 = _zrand(rng, (m, k)), _zrand(rng, (k, n)), _zrand(rng, (m, n))
    ta, tb = lay[0] == "T", lay[1] == "T"
    A = (Aop.T if ta else Aop).ravel(order="F")
    B = (Bop.T if tb else Bop).ravel(order="F")
    al, be = 0.5 + 0.25j, -1 + 0.5j
    got = oracle.zgemm(int(ta), int(tb), m, n, k, al, A, k if ta else m, B, n if tb else k, be,
                       C0.ravel(order="F"), m)
    ref = al * (Aop @ Bop) + be * C0
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_zgemm_padded_leading_dimensions():
    # ld > rows: the padding is never read (NaN there must not leak)
    rng = np.random.Generator(np.random.PCG64(936))
    m, n, k, pad = 4, 3, 5, 3
    Aop, Bop = _gauss_int(rng, (m, k)), _gauss_int(rng, (k, n))
    A = np.full((m + pad, k), np.nan + 0j)
    A[:m] = Aop
    B = np.full((k + pad, n), np.nan + 0j)
    B[:k] = Bop
    got = oracle.zgemm(0, 0, m, n, k, 1, A.ravel(order="F"), m + pad, B.ravel(order="F"), k + pad,
                       0, None, m)
    assert np.array_equal(got, Aop @ Bop)
