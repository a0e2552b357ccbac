"""Same-size strided batch (one shape, one plan, one launch) through the C ABI:
bitwise equal to one iaat_gemm call per problem, and on the oracle's bar."""
import numpy as np
import pytest
import torch

from paper_2208_09822_amd import iaat, inputs
from _helpers import fp32_equal, normwise
import oracle

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def stored(lay, m, n, k):
    ta, tb = lay[0] == "T", lay[1] == "T"
    ra, ca = (k, m) if ta else (m, k)
    rb, cb = (n, k) if tb else (k, n)
    return ta, tb, ra, ca, rb, cb


def strided_set(ta, tb, m, n, k, ra, rb, sa, sb, sc, batch, al, be, A, B, C):
    """The strided batch as a problem set over one buffer (A, B, C back to
    back), for the oracle's batch driver."""
    z = np.arange(batch, dtype=np.int64)
    na, nb = sa * batch, sb * batch
    full = lambda v, t: np.full(batch, v, dtype=t)
    return inputs.ProblemSet(full(int(ta) | (int(tb) << 1), np.int32), full(m, np.int32),
                             full(n, np.int32), full(k, np.int32), full(ra, np.int32),
                             full(rb, np.int32), full(m, np.int32), full(al, np.float32),
                             full(be, np.float32), z * sa, na + z * sb, na + nb + z * sc,
                             np.concatenate([A, B, C]), name="strided")


@pytest.mark.parametrize("integer", [False, True])
@pytest.mark.parametrize("lay,m,n,k,batch", [
    ("NN", 16, 16, 16, 300), ("TN", 17, 9, 31, 200), ("NT", 80, 48, 33, 64),
    ("TT", 5, 80, 64, 100), ("NN", 3, 2, 7, 70000), ("NN", 81, 90, 40, 3),
    # shapes the library routes to the staged batched kernel
    ("TN", 56, 72, 40, 500), ("TT", 40, 80, 80, 64), ("NN", 80, 80, 80, 100)])
def test_strided_equals_per_call(ctx, lay, m, n, k, batch, integer):
    """Every problem of the batch: bitwise equal to its own iaat_gemm call,
    and against the FP64 oracle bit-exact (integer inputs) or within
    1e-6 * K normwise (U[-1,1])."""
    ta, tb, ra, ca, rb, cb = stored(lay, m, n, k)
    rng = np.random.Generator(np.random.PCG64(inputs.SEED_BASE + 71 + m + n + k))
    pad = 3  # strides larger than the matrices
    sa, sb, sc = ra * ca + pad, rb * cb + pad, m * n + pad
    draw = (lambda c: rng.integers(-4, 5, c).astype(np.float32)) if integer else \
        (lambda c: rng.uniform(-1, 1, c).astype(np.float32))
    A, B, C = draw(sa * batch), draw(sb * batch), draw(sc * batch)
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC1, dC2 = torch.from_numpy(C).to(DEV), torch.from_numpy(C).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    al, be = (1.5, -0.5) if integer else (1.25, -0.75)
    iaat.iaat_gemm_strided_batched(ctx, int(ta), int(tb), m, n, k, al, dA.data_ptr(), ra, sa,
                                   dB.data_ptr(), rb, sb, be, dC1.data_ptr(), m, sc, batch, s)
    L = iaat.lib()
    pa, pb, pc = dA.data_ptr(), dB.data_ptr(), dC2.data_ptr()
    for z in range(batch):
        L.iaat_gemm(ctx, int(ta), int(tb), m, n, k, al, pa + 4 * z * sa, ra, pb + 4 * z * sb, rb,
                    be, pc + 4 * z * sc, m, s)
    torch.cuda.synchronize(DEV)
    c1, c2 = dC1.cpu().numpy(), dC2.cpu().numpy()
    assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32))
    ps = strided_set(ta, tb, m, n, k, ra, rb, sa, sb, sc, batch, al, be, A, B, C)
    ref, _, off = oracle.gemm_batch(ps, nthreads=16)
    got = c1.reshape(batch, sc)[:, :m * n].astype(np.float64)
    want = ref[:batch * m * n].reshape(batch, m * n)
    if integer:
        assert np.array_equal(got, want)
    else:
        err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
        assert err.max() <= 1e-6 * k, float(err.max())
    # padding between problems untouched
    pads = c1.reshape(batch, sc)[:, m * n:]
    assert np.array_equal(pads, C.reshape(batch, sc)[:, m * n:])


def test_strided_quick_return_and_errors(ctx):
    m, n, batch = 7, 5, 10
    C = np.arange(m * n * batch, dtype=np.float32)
    dC = torch.from_numpy(C).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    iaat.iaat_gemm_strided_batched(ctx, 0, 0, m, n, 0, 1.0, 0, m, 0, 0, 1, 0, 2.0, dC.data_ptr(),
                                   m, m * n, batch, s)
    torch.cuda.synchronize(DEV)
    assert fp32_equal(dC.cpu().numpy(), 2.0 * C)
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_gemm_strided_batched(ctx, 0, 0, m, n, 4, 1.0, dC.data_ptr(), m, 0, dC.data_ptr(),
                                       4, 0, 0.0, dC.data_ptr(), m, m * n - 1, batch, s)
    assert e.value.code == -17
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_gemm_strided_batched(ctx, 0, 0, m, n, 4, 1.0, dC.data_ptr(), m, 0, dC.data_ptr(),
                                       3, 0, 0.0, dC.data_ptr(), m, m * n, batch, s)
    assert e.value.code == -12


@pytest.mark.parametrize("lay", ["NN", "TN", "NT", "TT"])
def test_staged_route_padded_leading_dimensions_and_beta_zero(ctx, lay):
    """A shape the library runs on the staged batched kernel (56 x 72 x 40),
    with leading dimensions larger than the matrices and stride 0 for B (one
    B shared by every problem): bitwise equal to per-call iaat_gemm; with
    beta = 0 and NaN in C, C is not read."""
    m, n, k, batch = 56, 72, 40, 257
    ta, tb, ra, ca, rb, cb = stored(lay, m, n, k)
    lda, ldb, ldc = ra + 3, rb + 5, m + 2
    sa, sb, sc = lda * ca, 0, ldc * n
    rng = np.random.Generator(np.random.PCG64(inputs.SEED_BASE + 97))
    A = rng.uniform(-1, 1, sa * batch).astype(np.float32)
    B = rng.uniform(-1, 1, ldb * cb).astype(np.float32)
    s = torch.cuda.current_stream(DEV).cuda_stream
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    for be in (0.5, 0.0):
        print("[staged-route] lay=%s beta=%g" % (lay, be), flush=True)
        C = rng.uniform(-1, 1, sc * batch).astype(np.float32)
        if be == 0.0:
            C[:] = np.nan
        dC1, dC2 = torch.from_numpy(C).to(DEV), torch.from_numpy(C).to(DEV)
        iaat.iaat_gemm_strided_batched(ctx, int(ta), int(tb), m, n, k, 0.75, dA.data_ptr(), lda, sa,
                                       dB.data_ptr(), ldb, sb, be, dC1.data_ptr(), ldc, sc, batch, s)
        L = iaat.lib()
        for z in range(batch):
            L.iaat_gemm(ctx, int(ta), int(tb), m, n, k, 0.75, dA.data_ptr() + 4 * z * sa, lda,
                        dB.data_ptr(), ldb, be, dC2.data_ptr() + 4 * z * sc, ldc, s)
        torch.cuda.synchronize(DEV)
        c1, c2 = dC1.cpu().numpy(), dC2.cpu().numpy()
        assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32))
        got = c1.reshape(batch, n, ldc)[:, :, :m]
        if be == 0.0:
            assert np.isfinite(got).all()
        # rows m..ldc-1 of every column untouched
        assert np.array_equal(c1.reshape(batch, n, ldc)[:, :, m:].view(np.uint32),
                              C.reshape(batch, n, ldc)[:, :, m:].view(np.uint32))
