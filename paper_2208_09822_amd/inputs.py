"""Seeded synthetic workloads for the small-GEMM path.

This module only draws inputs: shapes, layouts, scalars and matrix entries.
It holds none of the GEMM arithmetic, so both the oracle side and the HIP
side of a check can use it.

A problem set is struct-of-arrays (``ProblemSet``) over one flat FP32 buffer:
problem q has op flags ``trans[q]`` (bit0: A transposed, bit1: B transposed),
sizes m, n, k, leading dimensions lda/ldb/ldc (column-major, each equal to
the stored row count unless padding is asked for) and element offsets
a_off/b_off/c_off into ``buf``.  Offsets are aligned to ``align`` elements
(64 elements = 256 bytes by default).

The small-GEMM domain (Section I): cbrt(MNK) <= 80, or <= 32 when the layout
is TN; tested in integers as MNK <= 512000 / 32768.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

LAYOUTS = ("NN", "NT", "TN", "TT")
LAYOUT_BITS = {"NN": 0, "TN": 1, "NT": 2, "TT": 3}  # bit0 = A^T, bit1 = B^T
BITS_LAYOUT = {v: k for k, v in LAYOUT_BITS.items()}
SEED_BASE = 2208098220
SWEEP_SIZES = (1, 2, 3, 4, 5, 7, 8, 12, 16, 17, 24, 31, 32, 33, 48, 63, 64, 80)


def in_small_domain(layout: str, m: int, n: int, k: int) -> bool:
    lim = 32 ** 3 if layout == "TN" else 80 ** 3
    return m * n * k <= lim


@dataclass
class ProblemSet:
    trans: np.ndarray
    m: np.ndarray
    n: np.ndarray
    k: np.ndarray
    lda: np.ndarray
    ldb: np.ndarray
    ldc: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    a_off: np.ndarray
    b_off: np.ndarray
    c_off: np.ndarray
    buf: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def count(self) -> int:
        return int(self.m.shape[0])

    def layout(self, q: int) -> str:
        return BITS_LAYOUT[int(self.trans[q])]

    def a_span(self, q):
        rows_cols = self.stored_cols_a(q)
        return int(self.lda[q]) * max(rows_cols - 1, 0) + self.stored_rows_a(q)

    def stored_rows_a(self, q):
        return int(self.k[q]) if self.trans[q] & 1 else int(self.m[q])

    def stored_cols_a(self, q):
        return int(self.m[q]) if self.trans[q] & 1 else int(self.k[q])

    def stored_rows_b(self, q):
        return int(self.n[q]) if self.trans[q] & 2 else int(self.k[q])

    def stored_cols_b(self, q):
        return int(self.k[q]) if self.trans[q] & 2 else int(self.n[q])

    def A(self, q):
        """Problem q's stored A (flat, column-major, length lda*cols)."""
        n = int(self.lda[q]) * self.stored_cols_a(q)
        return self.buf[self.a_off[q]:self.a_off[q] + n]

    def B(self, q):
        n = int(self.ldb[q]) * self.stored_cols_b(q)
        return self.buf[self.b_off[q]:self.b_off[q] + n]

    def C(self, q):
        n = int(self.ldc[q]) * int(self.n[q])
        return self.buf[self.c_off[q]:self.c_off[q] + n]

    def flops(self) -> float:
        return float(np.sum(2.0 * self.m.astype(np.float64) * self.n * self.k))

    def algorithmic_bytes(self, elem_bytes_ab: float = 4.0) -> float:
        """A + B read, C read when beta != 0, C written (FP32 C)."""
        m = self.m.astype(np.float64); n = self.n.astype(np.float64); k = self.k.astype(np.float64)
        readc = (self.beta != 0).astype(np.float64)
        return float(np.sum(elem_bytes_ab * (m * k + k * n) + 4.0 * m * n * (1.0 + readc)))

    def subset(self, idx) -> "ProblemSet":
        idx = np.asarray(idx, dtype=np.int64)
        g = lambda a: np.ascontiguousarray(a[idx])
        return ProblemSet(g(self.trans), g(self.m), g(self.n), g(self.k), g(self.lda),
                          g(self.ldb), g(self.ldc), g(self.alpha), g(self.beta),
                          g(self.a_off), g(self.b_off), g(self.c_off), self.buf,
                          name=self.name + "[subset]", meta=dict(self.meta))


def _assemble(trans, m, n, k, alpha, beta, fill, align=64, ld_pad=0, name="", meta=None):
    """Lay problems out in one FP32 buffer; ``fill(rng_slice_len)`` draws
    values.  ``ld_pad`` adds extra rows to every leading dimension."""
    trans = np.asarray(trans, dtype=np.int32)
    m = np.asarray(m, dtype=np.int32); n = np.asarray(n, dtype=np.int32); k = np.asarray(k, dtype=np.int32)
    cnt = m.shape[0]
    at = (trans & 1).astype(bool); bt = (trans & 2).astype(bool)
    rows_a = np.where(at, k, m); cols_a = np.where(at, m, k)
    rows_b = np.where(bt, n, k); cols_b = np.where(bt, k, n)
    lda = np.maximum(rows_a + ld_pad, 1).astype(np.int32)
    ldb = np.maximum(rows_b + ld_pad, 1).astype(np.int32)
    ldc = np.maximum(m + ld_pad, 1).astype(np.int32)
    sa = lda.astype(np.int64) * cols_a
    sb = ldb.astype(np.int64) * cols_b
    sc = ldc.astype(np.int64) * n
    up = lambda x: ((x + align - 1) // align) * align
    sizes = np.stack([up(sa), up(sb), up(sc)], axis=1).reshape(-1)
    offs = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    total = int(offs[-1])
    offs = offs[:-1].reshape(cnt, 3)
    buf = fill(total)
    return ProblemSet(trans, m, n, k, lda, ldb, ldc,
                      np.asarray(alpha, dtype=np.float32), np.asarray(beta, dtype=np.float32),
                      offs[:, 0].copy(), offs[:, 1].copy(), offs[:, 2].copy(), buf,
                      name=name, meta=meta or {})


def _uniform_fill(rng, lo=-1.0, hi=1.0, chunk=1 << 24):
    def fill(total):
        out = np.empty(total, dtype=np.float32)
        for s in range(0, total, chunk):
            e = min(total, s + chunk)
            out[s:e] = rng.uniform(lo, hi, e - s).astype(np.float32)
        return out
    return fill


def _int_fill(rng, lo=-4, hi=4, chunk=1 << 24):
    def fill(total):
        out = np.empty(total, dtype=np.float32)
        for s in range(0, total, chunk):
            e = min(total, s + chunk)
            out[s:e] = rng.integers(lo, hi + 1, e - s).astype(np.float32)
        return out
    return fill


def _loguniform_fill(rng, lo_exp=-3.0, hi_exp=3.0, chunk=1 << 24):
    def fill(total):
        out = np.empty(total, dtype=np.float32)
        for s in range(0, total, chunk):
            e = min(total, s + chunk)
            mag = 10.0 ** rng.uniform(lo_exp, hi_exp, e - s)
            sign = np.where(rng.integers(0, 2, e - s) == 0, -1.0, 1.0)
            out[s:e] = (sign * mag).astype(np.float32)
        return out
    return fill


EXACT_SCALARS = np.array([0.0, 0.5, -0.5, 1.0, -1.0, 1.5, -1.5, 2.0, -2.0], dtype=np.float32)


def uniform_problems(shapes: Sequence[Tuple[str, int, int, int]], seed: int, *,
                     alpha=1.0, beta=1.0, integer=False, ld_pad=0, align=64,
                     name="shapes") -> ProblemSet:
    """Problems of the given (layout, M, N, K) shapes, entries U[-1,1] (or
    integers in [-4,4] with ``integer``), fixed or per-problem scalars."""
    rng = np.random.Generator(np.random.PCG64(seed))
    trans = [LAYOUT_BITS[s[0]] for s in shapes]
    m = [s[1] for s in shapes]; n = [s[2] for s in shapes]; k = [s[3] for s in shapes]
    cnt = len(shapes)
    al = np.broadcast_to(np.asarray(alpha, dtype=np.float32), (cnt,)).copy()
    be = np.broadcast_to(np.asarray(beta, dtype=np.float32), (cnt,)).copy()
    fill = _int_fill(rng) if integer else _uniform_fill(rng)
    return _assemble(trans, m, n, k, al, be, fill, align=align, ld_pad=ld_pad, name=name)


def plain_nn16(seed: int = SEED_BASE + 0, count: int = 1000, integer=False) -> ProblemSet:
    """1,000 independent NN problems M=N=K=16, ld 16, entries U[-1,1],
    alpha 1.5, beta 0.5."""
    return uniform_problems([("NN", 16, 16, 16)] * count, seed, alpha=1.5, beta=0.5,
                            integer=integer, name="plain_nn16")


def sweep_shapes(layouts: Sequence[str] = LAYOUTS) -> List[Tuple[str, int, int, int]]:
    """Every (M, N, K) over the sweep sizes inside the small domain, per layout."""
    out = []
    for lay in layouts:
        for M in SWEEP_SIZES:
            for N in SWEEP_SIZES:
                for K in SWEEP_SIZES:
                    if in_small_domain(lay, M, N, K):
                        out.append((lay, M, N, K))
    return out


def sweep_problems(per_shape: int = 256, seed: int = SEED_BASE + 1, shapes=None,
                   integer=False) -> ProblemSet:
    """The shape sweep: ``per_shape`` problems of every sweep shape, U[-1,1],
    alpha = beta = 1."""
    shapes = sweep_shapes() if shapes is None else shapes
    rep = [s for s in shapes for _ in range(per_shape)]
    return uniform_problems(rep, seed, alpha=1.0, beta=1.0, integer=integer, name="sweep")


def uneven_shapes(count: int, rng, max_dim: int = 80):
    """Layout uniform over NN/NT/TN/TT; M, N, K uniform over [1, max_dim],
    redrawn until inside the small domain."""
    lays = rng.integers(0, 4, count)
    out = []
    for q in range(count):
        lay = LAYOUTS[int(lays[q])]
        while True:
            M, N, K = (int(x) for x in rng.integers(1, max_dim + 1, 3))
            if in_small_domain(lay, M, N, K):
                break
        out.append((lay, M, N, K))
    return out


def uneven_batch(count: int = 65536, seed: int = SEED_BASE + 2, *, integer=False,
                 align=64, ld_pad=0) -> ProblemSet:
    """Uneven batch: shapes from ``uneven_shapes``, entries U[-1,1], alpha and
    beta U[-2,2].  With ``integer``: entries integers in [-4,4], alpha and beta
    drawn from {0, +-1/2, +-1, +-3/2, +-2} (every intermediate exact in FP32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = uneven_shapes(count, rng)
    if integer:
        al = rng.choice(EXACT_SCALARS, count)
        be = rng.choice(EXACT_SCALARS, count)
        fill = _int_fill(rng)
    else:
        al = rng.uniform(-2.0, 2.0, count).astype(np.float32)
        be = rng.uniform(-2.0, 2.0, count).astype(np.float32)
        fill = _uniform_fill(rng)
    trans = [LAYOUT_BITS[s[0]] for s in shapes]
    return _assemble(trans, [s[1] for s in shapes], [s[2] for s in shapes],
                     [s[3] for s in shapes], al, be, fill, align=align, ld_pad=ld_pad,
                     name="uneven%d" % count)


def precision_problems(per_shape: int = 16, seed: int = SEED_BASE + 3, shapes=None) -> ProblemSet:
    """Reduced-precision workload: the sweep grid, ``per_shape`` problems each,
    entries |x| = 10^U(-3,3) with random sign (FP32 masters), alpha = beta = 1."""
    shapes = sweep_shapes() if shapes is None else shapes
    rep = [s for s in shapes for _ in range(per_shape)]
    rng = np.random.Generator(np.random.PCG64(seed))
    trans = [LAYOUT_BITS[s[0]] for s in rep]
    return _assemble(trans, [s[1] for s in rep], [s[2] for s in rep], [s[3] for s in rep],
                     np.ones(len(rep), np.float32), np.ones(len(rep), np.float32),
                     _loguniform_fill(rng), name="precision")


def poisson_trace(rate_per_s: float, duration_s: float, seed: int, max_gemms: int = 256):
    """Open-loop request trace: exponential inter-arrival times at
    ``rate_per_s``; each request holds U{1..max_gemms} GEMMs.  Returns
    (arrival_times_s, gemm_counts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_est = int(rate_per_s * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_per_s, n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = rng.exponential(1.0 / rate_per_s, n_est)
        t = np.concatenate([t, t[-1] + np.cumsum(more)])
    t = t[t < duration_s]
    counts = rng.integers(1, max_gemms + 1, t.shape[0])
    return t, counts


def pool_indices(total: int, pool_size: int, seed: int):
    """Which pool entries a stream of ``total`` GEMMs refers to (uniform)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, pool_size, total)


def serve_pool(size: int = 4096, seed: int = SEED_BASE + 4) -> ProblemSet:
    """Resident GEMM pool of the serving workload: shapes uniform over the
    sweep grid (layouts NN/NT/TN/TT, TN limited to its domain), entries
    U[-1,1], alpha = beta = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = sweep_shapes()
    pick = rng.integers(0, len(grid), size)
    return uniform_problems([grid[int(i)] for i in pick], seed=seed + 1000, alpha=1.0, beta=1.0,
                            name="serve_pool")
