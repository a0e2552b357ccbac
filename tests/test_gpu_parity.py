"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Bar (stated for FP32 small GEMM): bit-exact on integer-valued inputs in
[-4, 4] with alpha, beta in {0, +-1/2, +-1, +-3/2, +-2} (every partial sum,
product and the epilogue are exact in FP32 for K <= 80, so every summation
order gives the same value); normwise relative error <= 1e-6 * K per problem
on uniform [-1, 1] inputs.
"""
import numpy as np
import pytest
import torch

from paper_2208_09822_amd import iaat, inputs
from _helpers import check_problem, oracle_all, oracle_one, result_of, fp32_equal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
LAYOUT_ID = {"NN": 0, "TN": 1, "NT": 2, "TT": 3}
EDGE = (1, 2, 3, 4, 5, 7, 8, 9, 12, 15, 16, 17, 20, 24, 31, 32, 33, 40, 47, 48, 49, 63, 64,
        65, 79, 80)


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def stream():
    return torch.cuda.current_stream(DEV).cuda_stream


def run_percall(ctx, ps):
    buf = torch.from_numpy(ps.buf).to(DEV)
    base = buf.data_ptr()
    s = stream()
    for q in range(ps.count):
        t = int(ps.trans[q])
        m, n, k = int(ps.m[q]), int(ps.n[q]), int(ps.k[q])
        iaat.iaat_gemm(ctx, t & 1, t >> 1, m, n, k, float(ps.alpha[q]),
                       base + 4 * int(ps.a_off[q]), int(ps.lda[q]),
                       base + 4 * int(ps.b_off[q]), int(ps.ldb[q]), float(ps.beta[q]),
                       base + 4 * int(ps.c_off[q]), int(ps.ldc[q]), s)
    torch.cuda.synchronize(DEV)
    return buf.cpu().numpy()


def run_vbatched(ctx, ps, host_form=False, status=False):
    buf = torch.from_numpy(ps.buf).to(DEV)
    desc = iaat.descriptors(ps, buf.data_ptr())
    st = torch.full((ps.count,), 12345, dtype=torch.int32, device=DEV) if status else None
    sp = st.data_ptr() if st is not None else 0
    if host_form:
        iaat.iaat_gemm_vbatched(ctx, desc, status=sp, stream=stream())
    else:
        dd = torch.from_numpy(desc.view(np.uint8)).to(DEV)
        iaat.iaat_gemm_vbatched_device(ctx, dd.data_ptr(), ps.count, status=sp, stream=stream())
    torch.cuda.synchronize(DEV)
    out = buf.cpu().numpy()
    return (out, st.cpu().numpy()) if status else out


def sample_shapes(layout, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        m, n, k = (int(x) for x in rng.choice(EDGE, 3))
        if inputs.in_small_domain(layout, m, n, k):
            out.append((layout, m, n, k))
    return out


@pytest.mark.parametrize("layout", ["NN", "NT", "TN", "TT"])
def test_percall_integer_bit_exact(ctx, layout):
    shapes = sample_shapes(layout, 160, seed=LAYOUT_ID[layout])
    rng = np.random.default_rng(100 + LAYOUT_ID[layout])
    al = rng.choice(inputs.EXACT_SCALARS, len(shapes))
    be = rng.choice(inputs.EXACT_SCALARS, len(shapes))
    ps = inputs.uniform_problems(shapes, seed=11 + LAYOUT_ID[layout], alpha=al, beta=be,
                                 integer=True)
    out = run_percall(ctx, ps)
    for q in range(ps.count):
        check_problem(ps, out, q, oracle_one(ps, q), exact=True)


@pytest.mark.parametrize("layout", ["NN", "NT", "TN", "TT"])
def test_percall_uniform_normwise(ctx, layout):
    shapes = sample_shapes(layout, 160, seed=20 + LAYOUT_ID[layout])
    rng = np.random.default_rng(200 + LAYOUT_ID[layout])
    ps = inputs.uniform_problems(shapes, seed=21 + LAYOUT_ID[layout],
                                 alpha=rng.uniform(-2, 2, len(shapes)),
                                 beta=rng.uniform(-2, 2, len(shapes)))
    out = run_percall(ctx, ps)
    for q in range(ps.count):
        check_problem(ps, out, q, oracle_one(ps, q), exact=False)


def test_percall_every_size_to_80_square(ctx):
    """M = N = K = 1..80 in all four layouts (TN up to 32), integer inputs."""
    shapes = [(l, s, s, s) for l in ("NN", "NT", "TN", "TT") for s in range(1, 81)
              if inputs.in_small_domain(l, s, s, s)]
    ps = inputs.uniform_problems(shapes, seed=31, alpha=1.5, beta=-0.5, integer=True)
    out = run_percall(ctx, ps)
    for q in range(ps.count):
        check_problem(ps, out, q, oracle_one(ps, q), exact=True)


def test_alpha_zero_k_zero_beta_zero(ctx):
    M, N = 19, 23
    C0 = np.arange(M * N, dtype=np.float32)
    C = torch.from_numpy(C0.copy()).to(DEV)
    # alpha == 0: A and B are not read (NULL)
    iaat.iaat_gemm(ctx, 0, 0, M, N, 7, 0.0, 0, M, 0, 7, 0.5, C.data_ptr(), M, stream())
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), 0.5 * C0)
    # K == 0
    iaat.iaat_gemm(ctx, 1, 1, M, N, 0, 2.0, 0, 1, 0, N, -1.0, C.data_ptr(), M, stream())
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), -0.5 * C0)
    # beta == 0: C holding NaN is overwritten, not read
    Cn = torch.full((M * N,), float("nan"), device=DEV)
    A = torch.ones(M * 5, device=DEV)
    B = torch.ones(5 * N, device=DEV)
    iaat.iaat_gemm(ctx, 0, 0, M, N, 5, 1.0, A.data_ptr(), M, B.data_ptr(), 5, 0.0,
                   Cn.data_ptr(), M, stream())
    torch.cuda.synchronize()
    assert np.all(Cn.cpu().numpy() == 5.0)
    # M == 0 / N == 0: no-op even with NULL pointers
    iaat.iaat_gemm(ctx, 0, 0, 0, N, 5, 1.0, 0, 1, 0, 5, 1.0, 0, 1, stream())
    iaat.iaat_gemm(ctx, 0, 0, M, 0, 5, 1.0, 0, M, 0, 5, 1.0, 0, M, stream())


def test_argument_errors(ctx):
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_gemm(ctx, 0, 0, 4, 4, 4, 1.0, 1, 3, 1, 4, 0.0, 1, 4, stream())
    assert e.value.code == -9
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_gemm(ctx, 2, 0, 4, 4, 4, 1.0, 1, 4, 1, 4, 0.0, 1, 4, stream())
    assert e.value.code == -2
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_gemm(ctx, 0, 0, 4, 4, 4, 1.0, 0, 4, 1, 4, 0.0, 1, 4, stream())
    assert e.value.code == -8
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_gemm(ctx, 0, 1, 4, 4, 4, 1.0, 1, 4, 1, 3, 0.0, 1, 4, stream())
    assert e.value.code == -11


def test_padded_ld_and_unaligned_offsets(ctx):
    shapes = sample_shapes("NN", 40, 41) + sample_shapes("TT", 40, 42) + \
        sample_shapes("NT", 40, 43) + sample_shapes("TN", 40, 44)
    for kw in ({"ld_pad": 3}, {"align": 1}, {"ld_pad": 1, "align": 3}):
        ps = inputs.uniform_problems(shapes, seed=45, alpha=-1.5, beta=2.0, integer=True, **kw)
        out = run_percall(ctx, ps)
        for q in range(ps.count):
            check_problem(ps, out, q, oracle_one(ps, q), exact=True)
        out2 = run_vbatched(ctx, ps)
        assert np.array_equal(out, out2)


def test_outside_small_domain(ctx):
    shapes = [("NN", 200, 170, 50), ("NT", 1000, 1, 7), ("TN", 3, 3, 1000), ("TT", 48, 48, 300),
              ("NN", 1, 1, 5000), ("TN", 81, 161, 33), ("NT", 7, 300, 19), ("TT", 250, 9, 64)]
    ps = inputs.uniform_problems(shapes, seed=51, alpha=1.0, beta=1.0)
    out = run_percall(ctx, ps)
    for q in range(ps.count):
        check_problem(ps, out, q, oracle_one(ps, q), exact=False)
    assert np.array_equal(out, run_vbatched(ctx, ps))


def test_leading_dimension_beyond_narrow_addressing(ctx):
    """lda > 2^22 takes the 64-bit path; results still match."""
    shapes = [("NN", 3, 5, 4), ("TT", 6, 2, 3)]
    for lay, m, n, k in shapes:
        ps = inputs.uniform_problems([(lay, m, n, k)], seed=61, integer=True,
                                     ld_pad=(1 << 22) + 5 - max(m, k))
        out = run_percall(ctx, ps)
        check_problem(ps, out, 0, oracle_one(ps, 0), exact=True)
        assert np.array_equal(out, run_vbatched(ctx, ps))


def test_vbatched_matches_oracle_and_percall(ctx):
    for integer in (True, False):
        ps = inputs.uneven_batch(3000, seed=71 + integer, integer=integer)
        outb = run_vbatched(ctx, ps)
        refs = oracle_all(ps)
        for q in range(ps.count):
            check_problem(ps, outb, q, refs[q], exact=integer)
        outp = run_percall(ctx, ps)
        assert np.array_equal(outb.view(np.uint32), outp.view(np.uint32)), \
            "batched and per-call results differ bitwise"
        outh = run_vbatched(ctx, ps, host_form=True)
        assert np.array_equal(outb.view(np.uint32), outh.view(np.uint32))


def test_vbatched_status_codes(ctx):
    ps = inputs.uneven_batch(50, seed=81, integer=True)
    buf = torch.from_numpy(ps.buf).to(DEV)
    desc = iaat.descriptors(ps, buf.data_ptr())
    desc["lda"][3] = 0          # -9
    desc["m"][7] = -1           # -4
    desc["B"][11] = 0           # -10 (alpha != 0 and k > 0 required)
    desc["trans"][13] = 5       # -3
    desc["ldc"][17] = desc["m"][17] - 1 if desc["m"][17] > 1 else 0  # -14
    st = torch.full((ps.count,), 77, dtype=torch.int32, device=DEV)
    dd = torch.from_numpy(desc.view(np.uint8)).to(DEV)
    iaat.iaat_gemm_vbatched_device(ctx, dd.data_ptr(), ps.count, status=st.data_ptr(),
                                   stream=stream())
    torch.cuda.synchronize()
    s = st.cpu().numpy()
    expect = np.zeros(ps.count, np.int32)
    if ps.alpha[11] != 0:
        expect[11] = -10
    expect[3], expect[7], expect[13], expect[17] = -9, -4, -3, -14
    assert np.array_equal(s, expect), s
    out = buf.cpu().numpy()
    for q in range(ps.count):
        if expect[q] == 0:
            check_problem(ps, out, q, oracle_one(ps, q), exact=True)
        else:  # skipped problems leave C untouched
            assert np.array_equal(result_of(ps, out, q), result_of(ps, ps.buf, q))


def test_full_size_uneven_batch(ctx):
    """The 65,536-problem uneven batch in the benchmark's launch form:
    every problem bit-exact on integer inputs; sampled problems within
    1e-6 K on uniform inputs."""
    ps = inputs.uneven_batch(65536, integer=True)
    out = run_vbatched(ctx, ps)
    refs = oracle_all(ps, nthreads=16)
    for q in range(ps.count):
        check_problem(ps, out, q, refs[q], exact=True)
    del refs
    ps = inputs.uneven_batch(65536)
    out = run_vbatched(ctx, ps)
    sel = np.random.default_rng(5).choice(ps.count, 3000, replace=False)
    refs = oracle_all(ps, select=sel)
    for q in sel:
        check_problem(ps, out, int(q), refs[int(q)], exact=False)


def test_graph_plan_replays_and_descriptor_updates(ctx):
    """A captured batch replays correctly several times, with eager library
    work between replays, and picks up descriptor edits made between them."""
    ps = inputs.uneven_batch(2000, seed=91, integer=True)
    ps.beta[:] = 0.0
    ps.alpha[:] = 1.0
    buf = torch.from_numpy(ps.buf).to(DEV)
    desc = iaat.descriptors(ps, buf.data_ptr())
    dd = torch.from_numpy(desc.view(np.uint8)).to(DEV)
    plan = iaat.iaat_vbplan_create(ctx, dd.data_ptr(), ps.count)
    try:
        refs = oracle_all(ps)
        other = inputs.uneven_batch(300, seed=92, integer=True)
        for rep in range(3):
            iaat.iaat_vbplan_launch(plan, stream())
            torch.cuda.synchronize()
            out = buf.cpu().numpy()
            for q in range(0, ps.count, 7):
                check_problem(ps, out, q, refs[q], exact=True)
            run_vbatched(ctx, other)  # eager work in between
        # change alpha to 2 in the device descriptors, replay
        desc["alpha"][:] = 2.0
        dd.copy_(torch.from_numpy(desc.view(np.uint8)))
        iaat.iaat_vbplan_launch(plan, stream())
        torch.cuda.synchronize()
        out = buf.cpu().numpy()
        for q in range(0, ps.count, 5):
            assert fp32_equal(result_of(ps, out, q), 2.0 * refs[q])
    finally:
        iaat.iaat_vbplan_destroy(plan)


def test_repeated_batched_calls_apply_once_each(ctx):
    """260 back-to-back batched calls each add A*B exactly once to C
    (alpha = beta = 1): no problem is skipped or computed twice."""
    ps = inputs.uneven_batch(100, seed=93, integer=True)
    ps.alpha[:] = 1.0
    ps.beta[:] = 1.0
    buf = torch.from_numpy(ps.buf).to(DEV)
    dd = torch.from_numpy(iaat.descriptors(ps, buf.data_ptr()).view(np.uint8)).to(DEV)
    reps = 260
    for _ in range(reps):
        iaat.iaat_gemm_vbatched_device(ctx, dd.data_ptr(), ps.count, stream=stream())
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    ab = ps.subset(np.arange(ps.count))
    ab.beta = np.zeros(ps.count, np.float32)
    for q in range(ps.count):
        expect = result_of(ps, ps.buf, q).astype(np.float64) + reps * oracle_one(ab, q)
        assert fp32_equal(result_of(ps, out, q), expect), q
