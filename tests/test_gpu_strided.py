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


@pytest.mark.parametrize("lay,m,n,k,batch", [
    ("NN", 16, 16, 16, 300), ("TN", 17, 9, 31, 200), ("NT", 80, 48, 33, 64),
    ("TT", 5, 80, 64, 100), ("NN", 3, 2, 7, 70000), ("NN", 81, 90, 40, 3)])
def test_strided_equals_per_call(ctx, lay, m, n, k, batch):
    ta, tb, ra, ca, rb, cb = stored(lay, m, n, k)
    rng = np.random.Generator(np.random.PCG64(inputs.SEED_BASE + 71 + m + n + k))
    pad = 3  # strides larger than the matrices
    sa, sb, sc = ra * ca + pad, rb * cb + pad, m * n + pad
    A = rng.uniform(-1, 1, sa * batch).astype(np.float32)
    B = rng.uniform(-1, 1, sb * batch).astype(np.float32)
    C = rng.uniform(-1, 1, sc * batch).astype(np.float32)
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC1, dC2 = torch.from_numpy(C).to(DEV), torch.from_numpy(C).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    al, be = 1.25, -0.75
    iaat.iaat_gemm_strided_batched(ctx, int(ta), int(tb), m, n, k, al, dA.data_ptr(), ra, sa,
                                   dB.data_ptr(), rb, sb, be, dC1.data_ptr(), m, sc, batch, s)
    for z in ([0, 1, batch // 2, batch - 1] if batch > 1000 else range(batch)):
        iaat.iaat_gemm(ctx, int(ta), int(tb), m, n, k, al, dA.data_ptr() + 4 * z * sa, ra,
                       dB.data_ptr() + 4 * z * sb, rb, be, dC2.data_ptr() + 4 * z * sc, m, s)
    torch.cuda.synchronize(DEV)
    c1, c2 = dC1.cpu().numpy(), dC2.cpu().numpy()
    zs = [0, 1, batch // 2, batch - 1] if batch > 1000 else range(batch)
    for z in zs:
        g1 = c1[z * sc:z * sc + m * n]
        assert np.array_equal(g1.view(np.uint32), c2[z * sc:z * sc + m * n].view(np.uint32)), z
        ref = oracle.gemm(int(ta), int(tb), m, n, k, al, A[z * sa:z * sa + ra * ca], ra,
                          B[z * sb:z * sb + rb * cb], rb, be, C[z * sc:z * sc + m * n], m)
        assert normwise(g1.reshape(n, m).T, ref) <= 1e-6 * k
    # padding between problems untouched
    for z in range(min(batch, 50)):
        assert np.array_equal(c1[z * sc + m * n:(z + 1) * sc], C[z * sc + m * n:(z + 1) * sc])


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
