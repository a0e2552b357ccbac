"""CGEMM (complex FP32) against the complex FP64 oracle, through the C ABI.

Bar: bit-exact on Gaussian-integer inputs (parts in [-4, 4]) with exact
complex scalars (every product and sum is an exact FP32 integer or half
integer); normwise <= 1e-6 * K on inputs with parts U[-1, 1]."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_09822_amd import iaat


def normwise(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SIZES = [(1, 1, 1), (3, 5, 7), (16, 16, 16), (17, 33, 9), (48, 80, 40), (80, 80, 80), (5, 79, 64)]


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
    if integer:
        draw = lambda s: (rng.integers(-4, 5, s) + 1j * rng.integers(-4, 5, s)).astype(np.complex64)
    else:
        draw = lambda s: (rng.uniform(-1, 1, s) + 1j * rng.uniform(-1, 1, s)).astype(np.complex64)
    A, B, C = draw(ra * ca), draw(rb * cb), draw(m * n)
    dA, dB, dC = (torch.from_numpy(x).to(DEV) for x in (A, B, C))
    iaat.iaat_cgemm(ctx, int(ta), int(tb), m, n, k, alpha, dA.data_ptr(), ra, dB.data_ptr(), rb,
                    beta, dC.data_ptr(), m, torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize(DEV)
    got = dC.cpu().numpy().reshape(n, m).T
    ref = oracle.cgemm(int(ta), int(tb), m, n, k, alpha, A, ra, B, rb, beta, C, m)
    return got, ref


@pytest.mark.parametrize("lay", ["NN", "TN", "NT", "TT"])
def test_cgemm_integer_bit_exact(ctx, lay):
    for (m, n, k) in SIZES:
        got, ref = run(ctx, lay, m, n, k, 1.5 - 0.5j, 0.5 + 1j, True, 21 + m + n + k)
        assert np.array_equal(got, ref.astype(np.complex64)), (lay, m, n, k)


@pytest.mark.parametrize("lay", ["NN", "TN", "NT", "TT"])
def test_cgemm_uniform_normwise(ctx, lay):
    for (m, n, k) in SIZES:
        got, ref = run(ctx, lay, m, n, k, 0.7 + 0.2j, -0.4 + 1.1j, False, 27 + m + n + k)
        assert normwise(got, ref) <= 1e-6 * k, (lay, m, n, k, normwise(got, ref))


def test_cgemm_strided_quick_return_and_errors(ctx):
    m, n, k, batch = 9, 7, 13, 30
    rng = np.random.Generator(np.random.PCG64(4))
    mk = lambda s: (rng.uniform(-1, 1, s) + 1j * rng.uniform(-1, 1, s)).astype(np.complex64)
    A, B, C = mk(m * k * batch), mk(k * n * batch), mk(m * n * batch)
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC1, dC2 = torch.from_numpy(C).to(DEV), torch.from_numpy(C).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    iaat.iaat_cgemm_strided_batched(ctx, 0, 1, m, n, k, 2 - 1j, dA.data_ptr(), m, m * k,
                                    dB.data_ptr(), n, k * n, -1 + 0.5j, dC1.data_ptr(), m, m * n,
                                    batch, s)
    for z in range(batch):
        iaat.iaat_cgemm(ctx, 0, 1, m, n, k, 2 - 1j, dA.data_ptr() + 8 * z * m * k, m,
                        dB.data_ptr() + 8 * z * k * n, n, -1 + 0.5j,
                        dC2.data_ptr() + 8 * z * m * n, m, s)
    torch.cuda.synchronize(DEV)
    assert np.array_equal(dC1.cpu().numpy(), dC2.cpu().numpy())
    dC3 = torch.from_numpy(C).to(DEV)
    iaat.iaat_cgemm_strided_batched(ctx, 0, 0, m, n, k, 0, dA.data_ptr(), m, m * k, dB.data_ptr(),
                                    k, k * n, 2j, dC3.data_ptr(), m, m * n, batch, s)
    torch.cuda.synchronize(DEV)
    exp = (2j * C.astype(np.complex128)).astype(np.complex64)
    assert np.array_equal(dC3.cpu().numpy(), exp)
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_cgemm(ctx, 0, 0, m, n, k, 1, dA.data_ptr(), m - 1, dB.data_ptr(), k, 0,
                        dC3.data_ptr(), m, s)
    assert e.value.code == -9
