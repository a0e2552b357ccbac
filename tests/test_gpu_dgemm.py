"""DGEMM (FP64) against the FP64 oracle, through the C ABI.

Bar: bit-exact on integer inputs in [-4, 4] with exact scalars (every
product and partial sum is an exact FP64 integer); normwise <= 2e-15 * K on
U[-1, 1] inputs (the FP64 analogue of the FP32 bar: 16 * 2^-53 * K, the
same multiple of the unit roundoff as 1e-6 * K is of 2^-24)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_09822_amd import iaat, inputs
from _helpers import normwise

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SIZES = [(1, 1, 1), (3, 5, 7), (16, 16, 16), (17, 33, 9), (48, 80, 80), (80, 80, 80), (5, 79, 64),
         (64, 2, 33), (100, 90, 20)]


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def run(ctx, lay, m, n, k, alpha, beta, integer, seed):
    ta, tb = lay[0] == "T", lay[1] == "T"
    ra, ca = (k, m) if ta else (m, k)
    rb, cb = (n, k) if tb else (k, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    draw = (lambda s: rng.integers(-4, 5, s).astype(np.float64)) if integer else \
        (lambda s: rng.uniform(-1, 1, s))
    A, B, C = draw(ra * ca), draw(rb * cb), draw(m * n)
    dA, dB, dC = (torch.from_numpy(x).to(DEV) for x in (A, B, C))
    iaat.iaat_dgemm(ctx, int(ta), int(tb), m, n, k, alpha, dA.data_ptr(), ra, dB.data_ptr(), rb,
                    beta, dC.data_ptr(), m, torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize(DEV)
    got = dC.cpu().numpy().reshape(n, m).T
    ref = oracle.dgemm(int(ta), int(tb), m, n, k, alpha, A, ra, B, rb, beta, C, m)
    return got, ref


@pytest.mark.parametrize("lay", ["NN", "TN", "NT", "TT"])
def test_dgemm_integer_bit_exact(ctx, lay):
    for (m, n, k) in SIZES:
        got, ref = run(ctx, lay, m, n, k, 1.5, -0.5, True, 11 + m + n + k)
        assert np.array_equal(got, ref), (lay, m, n, k)


@pytest.mark.parametrize("lay", ["NN", "TN", "NT", "TT"])
def test_dgemm_uniform_normwise(ctx, lay):
    for (m, n, k) in SIZES:
        got, ref = run(ctx, lay, m, n, k, 0.7, 1.3, False, 17 + m + n + k)
        assert normwise(got, ref) <= 2e-15 * k, (lay, m, n, k, normwise(got, ref))


def test_dgemm_quick_returns_and_strided(ctx):
    m, n, k, batch = 9, 7, 13, 50
    rng = np.random.Generator(np.random.PCG64(3))
    A = rng.uniform(-1, 1, m * k * batch)
    B = rng.uniform(-1, 1, k * n * batch)
    C = rng.uniform(-1, 1, m * n * batch)
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC1, dC2 = torch.from_numpy(C).to(DEV), torch.from_numpy(C).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    iaat.iaat_dgemm_strided_batched(ctx, 0, 0, m, n, k, 2.0, dA.data_ptr(), m, m * k, dB.data_ptr(),
                                    k, k * n, -1.0, dC1.data_ptr(), m, m * n, batch, s)
    for z in range(batch):
        iaat.iaat_dgemm(ctx, 0, 0, m, n, k, 2.0, dA.data_ptr() + 8 * z * m * k, m,
                        dB.data_ptr() + 8 * z * k * n, k, -1.0, dC2.data_ptr() + 8 * z * m * n, m, s)
    torch.cuda.synchronize(DEV)
    assert np.array_equal(dC1.cpu().numpy(), dC2.cpu().numpy())
    dC3 = torch.from_numpy(C).to(DEV)
    iaat.iaat_dgemm_strided_batched(ctx, 0, 0, m, n, 0, 2.0, 0, m, 0, 0, 1, 0, 3.0, dC3.data_ptr(),
                                    m, m * n, batch, s)
    torch.cuda.synchronize(DEV)
    assert np.array_equal(dC3.cpu().numpy(), 3.0 * C)
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_dgemm(ctx, 0, 0, m, n, k, 1.0, dA.data_ptr(), m, dB.data_ptr(), k - 1, 0.0,
                        dC3.data_ptr(), m, s)
    assert e.value.code == -11
