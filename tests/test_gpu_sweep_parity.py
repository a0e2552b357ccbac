"""The plain-method sweep at its stated size, checked problem by problem.

Every (layout, M, N, K) of the sweep grid, 256 problems each (U[-1,1],
alpha = beta = 1, ld = stored rows), through both timed forms -- one
batched launch of the whole chunk, and one iaat_gemm call per problem --
against the FP64 oracle C*.  Bars, per problem:

* scaled error ||C - C*||_F / (|alpha| || |op(A)| |op(B)| ||_F + |beta| ||C0||_F)
  <= 1e-6 * K for every problem;
* normwise relative error ||C - C*||_F / ||C*||_F <= 1e-6 * K for every
  problem whose ||C*||_F is at least half that denominator.  Where C*
  cancels far below its terms (the 1 x 1 x 1 shapes draw a*b close to -c
  now and then among 256 problems) the relative error is not bounded by
  any FP32 evaluation; the scaled form is (its bound is (K + 2) 2^-24).

The problems are generated a chunk of shapes at a time (the full grid
holds about 40 GB of operands)."""
import copy

import numpy as np
import pytest
import torch

import oracle
from paper_2208_09822_amd import iaat, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
PER_SHAPE = 256
CHUNK_SHAPES = 512


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def per_problem_sq(ps, vals, ref_off):
    """Per-problem sum of squares of vals (laid out like the oracle output)."""
    sizes = ps.m.astype(np.int64) * ps.n.astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return np.add.reduceat(vals[:int(sizes.sum())] ** 2, starts)


def gather_c(ps, out, ref_off):
    """Every problem's C (compact: ldc == m) in the oracle's output order."""
    sizes = ps.m.astype(np.int64) * ps.n.astype(np.int64)
    pos = np.repeat(ps.c_off - ref_off, sizes) + np.arange(int(sizes.sum()), dtype=np.int64)
    return out[pos].astype(np.float64)


def scale_terms(ps):
    """|alpha| || |op(A)| |op(B)| ||_F + |beta| ||C0||_F per problem, through
    the oracle on the magnitudes (alpha = 1, beta = 0)."""
    pa = copy.copy(ps)
    pa.buf = np.abs(ps.buf)
    pa.alpha = np.ones_like(ps.alpha)
    pa.beta = np.zeros_like(ps.beta)
    ab, _, off = oracle.gemm_batch(pa, nthreads=16)
    ab_n = np.sqrt(per_problem_sq(ps, ab, off))
    c0_n = np.sqrt(per_problem_sq(ps, gather_c(ps, ps.buf, off), off))
    return np.abs(ps.alpha.astype(np.float64)) * ab_n + np.abs(ps.beta.astype(np.float64)) * c0_n


@pytest.mark.parametrize("lay", ["NN", "NT", "TN", "TT"])
def test_sweep_every_problem(ctx, lay):
    shapes = inputs.sweep_shapes((lay,))
    s = torch.cuda.current_stream(DEV).cuda_stream
    L = iaat.lib()
    checked = 0
    for c0 in range(0, len(shapes), CHUNK_SHAPES):
        chunk = shapes[c0:c0 + CHUNK_SHAPES]
        print("[sweep parity] %s shapes %d..%d of %d" % (lay, c0, c0 + len(chunk), len(shapes)),
              flush=True)
        ps = inputs.sweep_problems(per_shape=PER_SHAPE, shapes=chunk,
                                   seed=inputs.SEED_BASE + 501 + c0 + 100000 * {"NN": 0, "NT": 1, "TN": 2, "TT": 3}[lay])
        assert np.array_equal(ps.ldc, ps.m)
        buf = torch.from_numpy(ps.buf).to(DEV)
        buf2 = buf.clone()
        desc = torch.from_numpy(iaat.descriptors(ps, buf.data_ptr()).view(np.uint8)).to(DEV)
        iaat.iaat_gemm_vbatched_device(ctx, desc.data_ptr(), ps.count, stream=s)
        base = buf2.data_ptr()
        ao = (base + 4 * ps.a_off).tolist(); bo = (base + 4 * ps.b_off).tolist()
        co = (base + 4 * ps.c_off).tolist()
        tr = ps.trans.tolist(); mm = ps.m.tolist(); nn = ps.n.tolist(); kk = ps.k.tolist()
        la = ps.lda.tolist(); lb = ps.ldb.tolist()
        for q in range(ps.count):
            L.iaat_gemm(ctx, tr[q] & 1, tr[q] >> 1, mm[q], nn[q], kk[q], 1.0, ao[q], la[q], bo[q],
                        lb[q], 1.0, co[q], mm[q], s)
        torch.cuda.synchronize(DEV)
        ref, _, ref_off = oracle.gemm_batch(ps, nthreads=16)
        k = ps.k.astype(np.float64)
        den = scale_terms(ps)
        ref_n = np.sqrt(per_problem_sq(ps, ref, ref_off))
        plain = ref_n >= 0.5 * den  # no severe cancellation
        for name, b in (("batched", buf), ("per-call", buf2)):
            d = np.sqrt(per_problem_sq(ps, gather_c(ps, b.cpu().numpy(), ref_off) - ref[:len(ref) - 1],
                                       ref_off))
            for what, err, mask in (("scaled", d / den, np.ones_like(plain)),
                                    ("normwise", d / np.maximum(ref_n, 1e-300), plain)):
                bad = np.nonzero(mask & (err > 1e-6 * k))[0]
                assert bad.size == 0, "%s %s: problem %d (%dx%dx%d) %s error %.3g" % (
                    lay, name, bad[0], ps.m[bad[0]], ps.n[bad[0]], ps.k[bad[0]], what, err[bad[0]])
        checked += ps.count
        del buf, buf2, desc
    assert checked == PER_SHAPE * len(shapes)
