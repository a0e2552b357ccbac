"""DGEMM, CGEMM and ZGEMM on the plan-driven path (Table 1 rows D, C, Z),
through the C ABI, against the FP64 oracles.

Bars: bit-exact on integer (real) or Gaussian-integer (complex) inputs with
parts in [-4, 4] and exact scalars -- every product and partial sum is then
exact in the element type; normwise <= 2e-15 * K for FP64 (real and
complex) and <= 1e-6 * K for complex FP32 on inputs with parts U[-1, 1].
The uneven batched form runs the same family members as the per-call form,
so its results must equal per-call results bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2208_09822_amd import iaat

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
LAYS = ["NN", "TN", "NT", "TT"]
# shapes that reach every family: K-split (<= 4 x 4), row / column strips
# (<= 8 rows or columns), matrix-core grids, ragged tiles, super-blocks (> 80)
SIZES = [(1, 1, 1), (3, 4, 70), (2, 50, 9), (6, 64, 33), (45, 7, 20), (80, 3, 5), (16, 16, 16),
         (17, 33, 9), (48, 80, 40), (80, 80, 80), (100, 90, 20), (161, 5, 7)]
DTYPES = {
    "D": (iaat.IAAT_DT_F64, np.float64, 8, 2e-15),
    "C": (iaat.IAAT_DT_C64, np.complex64, 8, 1e-6),
    "Z": (iaat.IAAT_DT_C128, np.complex128, 16, 2e-15),
}


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def normwise(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def draw(rng, dt, size, integer):
    np_t = DTYPES[dt][1]
    if integer:
        x = rng.integers(-4, 5, size).astype(np.float64)
        if dt != "D":
            x = x + 1j * rng.integers(-4, 5, size)
    else:
        x = rng.uniform(-1, 1, size)
        if dt != "D":
            x = x + 1j * rng.uniform(-1, 1, size)
    return x.astype(np_t)


def oracle_call(dt, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc):
    if dt == "D":
        return oracle.dgemm(ta, tb, m, n, k, al.real, A, lda, B, ldb, be.real, C, ldc)
    f = oracle.cgemm if dt == "C" else oracle.zgemm
    return f(ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc)


def gemm_call(ctx, dt, ta, tb, m, n, k, al, pA, lda, pB, ldb, be, pC, ldc, s):
    if dt == "D":
        iaat.iaat_dgemm(ctx, ta, tb, m, n, k, al.real, pA, lda, pB, ldb, be.real, pC, ldc, s)
    elif dt == "C":
        iaat.iaat_cgemm(ctx, ta, tb, m, n, k, al, pA, lda, pB, ldb, be, pC, ldc, s)
    else:
        iaat.iaat_zgemm(ctx, ta, tb, m, n, k, al, pA, lda, pB, ldb, be, pC, ldc, s)


def scalars(dt, integer):
    if dt == "D":
        return (1.5 + 0j, -0.5 + 0j) if integer else (0.7 + 0j, 1.3 + 0j)
    return (1.5 - 0.5j, 0.5 + 1j) if integer else (0.75 + 0.25j, -0.5 + 1j)


def one(ctx, dt, lay, m, n, k, integer, seed, pad=0):
    ta, tb = int(lay[0] == "T"), int(lay[1] == "T")
    ra, ca = (k, m) if ta else (m, k)
    rb, cb = (n, k) if tb else (k, n)
    lda, ldb, ldc = ra + pad, rb + pad, m + pad
    rng = np.random.Generator(np.random.PCG64(seed))
    A = draw(rng, dt, lda * ca, integer)
    B = draw(rng, dt, ldb * cb, integer)
    C = draw(rng, dt, ldc * n, integer)
    al, be = scalars(dt, integer)
    dA, dB, dC = (torch.from_numpy(x).to(DEV) for x in (A, B, C))
    s = torch.cuda.current_stream(DEV).cuda_stream
    gemm_call(ctx, dt, ta, tb, m, n, k, al, dA.data_ptr(), lda, dB.data_ptr(), ldb, be,
              dC.data_ptr(), ldc, s)
    torch.cuda.synchronize(DEV)
    got = dC.cpu().numpy().reshape(n, ldc).T[:m]
    ref = oracle_call(dt, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc)
    return got, ref


@pytest.mark.parametrize("dt", ["D", "C", "Z"])
@pytest.mark.parametrize("lay", LAYS)
def test_integer_bit_exact(ctx, dt, lay):
    for (m, n, k) in SIZES:
        got, ref = one(ctx, dt, lay, m, n, k, True, 101 + m + 3 * n + 7 * k, pad=(m % 3))
        want = ref.astype(DTYPES[dt][1])
        assert np.array_equal(got, want), (dt, lay, m, n, k)


@pytest.mark.parametrize("dt", ["D", "C", "Z"])
@pytest.mark.parametrize("lay", LAYS)
def test_uniform_normwise(ctx, dt, lay):
    tol = DTYPES[dt][3]
    for (m, n, k) in SIZES:
        got, ref = one(ctx, dt, lay, m, n, k, False, 211 + m + 3 * n + 7 * k)
        err = normwise(got, ref)
        assert err <= tol * k, (dt, lay, m, n, k, err)


@pytest.mark.parametrize("dt", ["D", "C", "Z"])
def test_quick_returns(ctx, dt):
    np_t = DTYPES[dt][1]
    m, n, k = 7, 5, 6
    s = torch.cuda.current_stream(DEV).cuda_stream
    C = (np.arange(m * n) + 1).astype(np_t)
    nanA = torch.full((m * k,), float("nan"), dtype=torch.float64 if dt == "D" else
                      (torch.complex64 if dt == "C" else torch.complex128), device=DEV)
    # alpha = 0: C = beta*C, A and B not read
    dC = torch.from_numpy(C.copy()).to(DEV)
    be = 2.0 + (0.5j if dt != "D" else 0j)
    gemm_call(ctx, dt, 0, 0, m, n, k, 0j, nanA.data_ptr(), m, nanA.data_ptr(), k, be,
              dC.data_ptr(), m, s)
    torch.cuda.synchronize(DEV)
    want = (be if dt != "D" else be.real) * C.astype(np.complex128)
    assert np.array_equal(dC.cpu().numpy().astype(np.complex128), want.astype(np_t))
    # beta = 0: C is not read (NaN there does not propagate)
    A = np.ones(m * k, np_t)
    B = np.ones(k * n, np_t)
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC = torch.full((m * n,), float("nan"), dtype=nanA.dtype, device=DEV)
    gemm_call(ctx, dt, 0, 0, m, n, k, 1 + 0j, dA.data_ptr(), m, dB.data_ptr(), k, 0j,
              dC.data_ptr(), m, s)
    torch.cuda.synchronize(DEV)
    assert np.array_equal(dC.cpu().numpy(), np.full(m * n, float(k), np_t))


def test_zgemm_strided_equals_per_call(ctx):
    m, n, k, batch = 19, 23, 13, 40
    rng = np.random.Generator(np.random.PCG64(5))
    A, B, C = (draw(rng, "Z", m * k * batch, False), draw(rng, "Z", k * n * batch, False),
               draw(rng, "Z", m * n * batch, False))
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC1, dC2 = torch.from_numpy(C).to(DEV), torch.from_numpy(C).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    al, be = 0.5 - 1j, 0.25 + 0.5j
    iaat.iaat_zgemm_strided_batched(ctx, 1, 0, m, n, k, al, dA.data_ptr(), k, m * k, dB.data_ptr(),
                                    k, k * n, be, dC1.data_ptr(), m, m * n, batch, s)
    for z in range(batch):
        iaat.iaat_zgemm(ctx, 1, 0, m, n, k, al, dA.data_ptr() + 16 * z * m * k, k,
                        dB.data_ptr() + 16 * z * k * n, k, be, dC2.data_ptr() + 16 * z * m * n, m, s)
    torch.cuda.synchronize(DEV)
    assert np.array_equal(dC1.cpu().numpy(), dC2.cpu().numpy())


def test_zgemm_argument_errors(ctx):
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_zgemm(ctx, 2, 0, 4, 4, 4, 1, 0, 4, 0, 4, 0, 0, 4)
    assert e.value.code == -2
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_zgemm(ctx, 0, 0, 4, 4, 4, 1, 0, 3, 0, 4, 0, 0, 4)
    assert e.value.code == -9


def uneven(ctx, dt, count, seed, integer):
    """An uneven batch of problems of type dt in one device buffer, plus the
    per-problem host copies.  Returns (descriptors, buffer, problems)."""
    dtc, np_t, esz, _ = DTYPES[dt]
    rng = np.random.Generator(np.random.PCG64(seed))
    probs, parts, off = [], [], 0
    for q in range(count):
        lay = LAYS[int(rng.integers(0, 4))]
        m, n, k = (int(x) for x in rng.integers(1, 97, 3))
        if q % 7 == 3:
            k = int(rng.integers(0, 3))  # K = 0 quick returns among them
        ta, tb = int(lay[0] == "T"), int(lay[1] == "T")
        ra, ca = (k, m) if ta else (m, k)
        rb, cb = (n, k) if tb else (k, n)
        lda, ldb, ldc = max(ra, 1) + (q % 2), max(rb, 1), m + (q % 3)
        A = draw(rng, dt, lda * max(ca, 1), integer)
        B = draw(rng, dt, ldb * max(cb, 1), integer)
        C = draw(rng, dt, ldc * n, integer)
        al, be = scalars(dt, integer)
        if q % 11 == 5:
            al = 0j
        if q % 13 == 6:
            be = 0j
        offs = []
        for x in (A, B, C):
            offs.append(off)
            parts.append(x)
            off += x.size
            pad = (-off) % 4
            if pad:
                parts.append(np.zeros(pad, np_t))
                off += pad
        probs.append(dict(ta=ta, tb=tb, m=m, n=n, k=k, lda=lda, ldb=ldb, ldc=ldc, al=al, be=be,
                          A=A, B=B, C=C, offs=offs))
    buf = torch.from_numpy(np.concatenate(parts)).to(DEV)
    base = buf.data_ptr()
    d = np.zeros(count, dtype=iaat.XPROBLEM_DTYPE)
    for q, p in enumerate(probs):
        d[q]["A"], d[q]["B"], d[q]["C"] = (base + esz * o for o in p["offs"])
        d[q]["trans"] = p["ta"] | (p["tb"] << 1)
        d[q]["m"], d[q]["n"], d[q]["k"] = p["m"], p["n"], p["k"]
        d[q]["lda"], d[q]["ldb"], d[q]["ldc"] = p["lda"], p["ldb"], p["ldc"]
        d[q]["alpha"] = (p["al"].real, p["al"].imag)
        d[q]["beta"] = (p["be"].real, p["be"].imag)
    return d, buf, probs


@pytest.mark.parametrize("dt", ["D", "C", "Z"])
def test_uneven_batch_integer_exact_and_equal_to_per_call(ctx, dt):
    dtc, np_t, esz, _ = DTYPES[dt]
    count = 120
    print("[xgemm vbatched] dt=%s count=%d" % (dt, count), flush=True)
    d, buf, probs = uneven(ctx, dt, count, 71 + dtc, True)
    ddev = torch.from_numpy(d.view(np.uint8)).to(DEV)
    status = torch.full((count,), -99, dtype=torch.int32, device=DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    iaat.iaat_xgemm_vbatched(ctx, dtc, ddev.data_ptr(), count, status.data_ptr(), s)
    torch.cuda.synchronize(DEV)
    assert (status.cpu().numpy() == 0).all()
    out = buf.cpu().numpy()
    # the same problems one call each, into a fresh copy of the inputs
    _, buf2, _ = uneven(ctx, dt, count, 71 + dtc, True)
    base2 = buf2.data_ptr()
    for p in probs:
        oA, oB, oC = p["offs"]
        gemm_call(ctx, dt, p["ta"], p["tb"], p["m"], p["n"], p["k"], p["al"], base2 + esz * oA,
                  p["lda"], base2 + esz * oB, p["ldb"], p["be"], base2 + esz * oC, p["ldc"], s)
    torch.cuda.synchronize(DEV)
    out2 = buf2.cpu().numpy()
    assert np.array_equal(out, out2)
    for q, p in enumerate(probs):
        oC = p["offs"][2]
        got = out[oC:oC + p["ldc"] * p["n"]].reshape(p["n"], p["ldc"]).T[:p["m"]]
        ref = oracle_call(dt, p["ta"], p["tb"], p["m"], p["n"], p["k"], p["al"], p["A"], p["lda"],
                          p["B"], p["ldb"], p["be"], p["C"], p["ldc"])
        assert np.array_equal(got, ref.astype(np_t)), (dt, q)


@pytest.mark.parametrize("dt", ["D", "Z"])
def test_uneven_batch_uniform_normwise(ctx, dt):
    dtc, np_t, esz, tol = DTYPES[dt]
    count = 60
    d, buf, probs = uneven(ctx, dt, count, 91 + dtc, False)
    ddev = torch.from_numpy(d.view(np.uint8)).to(DEV)
    s = torch.cuda.current_stream(DEV).cuda_stream
    iaat.iaat_xgemm_vbatched(ctx, dtc, ddev.data_ptr(), count, 0, s)
    torch.cuda.synchronize(DEV)
    out = buf.cpu().numpy()
    for q, p in enumerate(probs):
        oC = p["offs"][2]
        got = out[oC:oC + p["ldc"] * p["n"]].reshape(p["n"], p["ldc"]).T[:p["m"]]
        ref = oracle_call(dt, p["ta"], p["tb"], p["m"], p["n"], p["k"], p["al"], p["A"], p["lda"],
                          p["B"], p["ldb"], p["be"], p["C"], p["ldc"])
        assert normwise(got, ref) <= tol * max(p["k"], 1), (dt, q)


def test_uneven_batch_status_codes(ctx):
    d, buf, probs = uneven(ctx, "Z", 8, 7, True)
    d[1]["trans"] = 4          # -3
    d[2]["lda"] = 0            # -9 (lda < rows of A)
    d[3]["m"] = -1             # -4
    d[5]["ldc"] = d[5]["m"] - 1 if d[5]["m"] > 1 else 0  # -14
    ddev = torch.from_numpy(d.view(np.uint8)).to(DEV)
    status = torch.full((8,), -99, dtype=torch.int32, device=DEV)
    iaat.iaat_xgemm_vbatched(ctx, iaat.IAAT_DT_C128, ddev.data_ptr(), 8, status.data_ptr(),
                             torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize(DEV)
    st = status.cpu().numpy()
    assert st[1] == -3 and st[2] == -9 and st[3] == -4 and st[5] == -14
    assert st[0] == 0 and st[4] == 0 and st[6] == 0 and st[7] == 0
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_xgemm_vbatched(ctx, 9, ddev.data_ptr(), 8)
    assert e.value.code == -4
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_xgemm_vbatched(ctx, iaat.IAAT_DT_F64, 0, 8)
    assert e.value.code == -2


@pytest.mark.parametrize("dt", ["D", "C", "Z"])
def test_strided_batch_longer_than_one_grid_dimension(ctx, dt):
    """65,600 problems in one strided call, on a plan of small members (1 x 1)
    and on one that needs the full family (3 x 3, a 3 x 3 K-split block):
    problems on both sides of index 65,535 against the oracle, bit for bit
    (integer inputs)."""
    np_t = DTYPES[dt][1]
    batch, k = 65600, 5
    fns = {"D": iaat.iaat_dgemm_strided_batched, "C": iaat.iaat_cgemm_strided_batched,
           "Z": iaat.iaat_zgemm_strided_batched}
    s = torch.cuda.current_stream(DEV).cuda_stream
    for (m, n) in ((1, 1), (3, 3)):
        print("[strided-long] dt=%s m=%d n=%d batch=%d" % (dt, m, n, batch), flush=True)
        rng = np.random.Generator(np.random.PCG64(900 + m))
        A = draw(rng, dt, m * k * batch, True)
        B = draw(rng, dt, k * n * batch, True)
        C = draw(rng, dt, m * n * batch, True)
        al, be = scalars(dt, True)
        dA, dB, dC = (torch.from_numpy(x).to(DEV) for x in (A, B, C))
        if dt == "D":
            al, be = al.real, be.real
        fns[dt](ctx, 0, 0, m, n, k, al, dA.data_ptr(), m, m * k, dB.data_ptr(), k, k * n, be,
                dC.data_ptr(), m, m * n, batch, s)
        torch.cuda.synchronize(DEV)
        got = dC.cpu().numpy()
        for z in sorted({0, 1, 4999, 65533, 65534, 65535, 65536, 65537, batch - 1}):
            a0 = np.ascontiguousarray(A[z * m * k:(z + 1) * m * k])
            b0 = np.ascontiguousarray(B[z * k * n:(z + 1) * k * n])
            c0 = np.ascontiguousarray(C[z * m * n:(z + 1) * m * n])
            ref = oracle_call(dt, 0, 0, m, n, k, complex(al), a0, m, b0, k, complex(be), c0, m)
            want = np.asarray(ref).T.reshape(-1)  # column-major, ldc = m
            assert np.array_equal(got[z * m * n:(z + 1) * m * n], want.astype(np_t)), (dt, m, n, z)
