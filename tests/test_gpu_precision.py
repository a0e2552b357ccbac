"""Reduced-precision batched GEMM against the FP64 oracle, through the C ABI.

Inputs are quantised on the GPU (iaat_quantize_batch) and, independently, by
the oracle's quantisers from the same FP32 masters; codes must agree bit for
bit (decoded values equal, same scales).  Each product of two reduced inputs
is exact in FP32, so the GEMM gate is the FP32 one, against the oracle run
on the oracle's own dequantised inputs: normwise <= 1e-6 * K, and bit-exact
on integer inputs in [-4, 4] (exact in every format, with exact sums).
Split-bfloat16 is compared with the oracle's lo*hi + hi*lo + hi*hi.  The
error against the FP32 masters is measured and only loosely bounded (it is
the format's, not the kernel's).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import quant
from paper_2208_09822_amd import iaat, inputs
from oracle import lowp, metrics
from _helpers import fp32_equal, normwise, result_of

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
PRECS = [iaat.IAAT_PREC_BF16, iaat.IAAT_PREC_F16, iaat.IAAT_PREC_F8E4M3, iaat.IAAT_PREC_BF16X3]
CODE_DTYPE = {1: torch.int16, 2: torch.int16, 3: torch.uint8, 4: torch.int16}


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def stream():
    return torch.cuda.current_stream(DEV).cuda_stream


MODE = {iaat.IAAT_PREC_BF16: "bf16", iaat.IAAT_PREC_F16: "f16", iaat.IAAT_PREC_F8E4M3: "e4m3",
        iaat.IAAT_PREC_BF16X3: "bf16x3"}


def oracle_quant(prec, x):
    """(dequantised FP64 operand terms, scale) of an FP32 master array."""
    return lowp.dequant_terms(MODE[prec], x)


def decode(prec, codes):
    if prec == iaat.IAAT_PREC_BF16 or prec == iaat.IAAT_PREC_BF16X3:
        return quant.bf16_decode(codes.astype(np.int64) & 0xFFFF)
    if prec == iaat.IAAT_PREC_F16:
        return quant.f16_decode(codes.astype(np.int64) & 0xFFFF)
    return quant.e4m3_decode(codes)


def run_lowp(ctx, ps, prec):
    """Quantise and multiply on the GPU; returns (C buffer, codes, descriptors)."""
    buf = torch.from_numpy(ps.buf).to(DEV)
    n = iaat.PREC_SPAN[prec] * ps.buf.shape[0]
    codes = torch.zeros(n, dtype=CODE_DTYPE[prec], device=DEV)
    desc_dev = torch.zeros(ps.count * 64, dtype=torch.uint8, device=DEV)
    jobs, desc = iaat.lowp_layout(ps, prec, buf.data_ptr(), codes.data_ptr(), desc_dev.data_ptr())
    desc_dev.copy_(torch.from_numpy(desc.view(np.uint8)))
    jobs_dev = torch.from_numpy(jobs.view(np.uint8)).to(DEV)
    iaat.iaat_quantize_batch(ctx, prec, jobs_dev.data_ptr(), ps.count, stream())
    status = torch.full((ps.count,), 777, dtype=torch.int32, device=DEV)
    iaat.iaat_gemm_vbatched_device(ctx, desc_dev.data_ptr(), ps.count, prec=prec,
                                   status=status.data_ptr(), stream=stream())
    torch.cuda.synchronize(DEV)
    assert (status.cpu().numpy() == 0).all()
    return (buf.cpu().numpy(), codes.cpu().numpy(),
            desc_dev.cpu().numpy().view(iaat.PROBLEM_DTYPE))


def oracle_lowp(ps, q, prec):
    t = int(ps.trans[q])
    return lowp.gemm_lowp(MODE[prec], t & 1, t >> 1, int(ps.m[q]), int(ps.n[q]), int(ps.k[q]),
                          float(ps.alpha[q]), ps.A(q), int(ps.lda[q]), ps.B(q), int(ps.ldb[q]),
                          float(ps.beta[q]), ps.C(q), int(ps.ldc[q]))


def scaled_error(ps, q, prec, got, ref):
    """||C-hat - C*||_F / (|alpha| || |op(A)||op(B)| ||_F + |beta| ||C0||_F) on
    the dequantised operands (hi + lo magnitudes for split-bfloat16)."""
    t = int(ps.trans[q])
    return metrics.scaled_error(got, ref, t & 1, t >> 1, int(ps.m[q]), int(ps.n[q]), int(ps.k[q]),
                                float(ps.alpha[q]), lowp.abs_terms(MODE[prec], ps.A(q)),
                                int(ps.lda[q]), lowp.abs_terms(MODE[prec], ps.B(q)), int(ps.ldb[q]),
                                float(ps.beta[q]), ps.C(q), int(ps.ldc[q]))


def grid_shapes(step=3):
    shapes = inputs.sweep_shapes()
    return shapes[::step]


@pytest.mark.parametrize("prec", PRECS, ids=[iaat.PREC_NAMES[p] for p in PRECS])
def test_quantiser_codes_match_format_definitions(ctx, prec):
    """Codes of edge values (ties, subnormals, overflow, saturation, zeros,
    NaN) and of log-uniform values decode to the oracle's rounding."""
    rng = np.random.Generator(np.random.PCG64(inputs.SEED_BASE + 31))
    edge = np.array([0.0, -0.0, 1.0, -1.0, 1.00390625, 1.01171875, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8,
                     65504.0, 65519.99, 65520.0, 70000.0, -1e6, 6.0e-5, 6.1e-5, 2 ** -24, 2 ** -25,
                     3 * 2 ** -25, 1e-8, 448.0, 464.0, 480.0, 2 ** -9, 2 ** -10, 3 * 2 ** -11,
                     3.4e38, 1e-40, np.inf, -np.inf], np.float32)
    mags = (10.0 ** rng.uniform(-8, 8, 4000)).astype(np.float32)
    x = np.concatenate([edge, mags * np.where(rng.integers(0, 2, 4000) == 0, -1, 1)]).astype(np.float32)
    if prec == iaat.IAAT_PREC_F8E4M3:
        x = x[np.isfinite(x)]  # finite inputs (an infinite absmax gives scale 1 and saturation)
    nan = np.array([np.nan], np.float32)
    xs = [x, np.concatenate([x[:100], nan]) if prec != iaat.IAAT_PREC_F8E4M3 else x[:50] * 1e-3]
    src = [torch.from_numpy(v).to(DEV) for v in xs]
    span = iaat.PREC_SPAN[prec]
    dst = [torch.zeros(span * v.shape[0], dtype=CODE_DTYPE[prec], device=DEV) for v in xs]
    scales = torch.zeros(2, dtype=torch.float32, device=DEV)
    job = np.zeros(1, dtype=iaat.QJOB_DTYPE)
    job["a_src"], job["b_src"] = src[0].data_ptr(), src[1].data_ptr()
    job["a_dst"], job["b_dst"] = dst[0].data_ptr(), dst[1].data_ptr()
    job["a_n"], job["b_n"] = xs[0].shape[0], xs[1].shape[0]
    job["scales"] = scales.data_ptr()
    jd = torch.from_numpy(job.view(np.uint8)).to(DEV)
    iaat.iaat_quantize_batch(ctx, prec, jd.data_ptr(), 1, stream())
    torch.cuda.synchronize(DEV)
    sc = scales.cpu().numpy()
    for v, d, s_gpu in zip(xs, dst, sc):
        codes = d.cpu().numpy()
        terms, s = oracle_quant(prec, v)
        assert s_gpu == s
        if prec == iaat.IAAT_PREC_F8E4M3:
            assert not np.any(codes == 0x80), "negative zero code"
            got = [decode(prec, codes) / s]
        elif prec == iaat.IAAT_PREC_BF16X3:
            got = [decode(prec, codes[:v.shape[0]]), decode(prec, codes[v.shape[0]:])]
        else:
            got = [decode(prec, codes)]
        for g, e in zip(got, terms):
            same = (g == e) | (np.isnan(g) & np.isnan(e))
            bad = np.nonzero(~same)[0]
            assert bad.size == 0, (iaat.PREC_NAMES[prec], v[bad[:5]], g[bad[:5]], e[bad[:5]])


@pytest.mark.parametrize("prec", PRECS, ids=[iaat.PREC_NAMES[p] for p in PRECS])
def test_integer_inputs_bit_exact(ctx, prec):
    shapes = [(lay, m, n, k) for lay in ("NN", "TN", "NT", "TT")
              for (m, n, k) in [(1, 1, 1), (3, 5, 7), (16, 16, 16), (17, 9, 33), (32, 32, 32),
                                (80, 48, 40), (5, 80, 64), (33, 31, 17)]
              if inputs.in_small_domain(lay, m, n, k)]
    ps = inputs.uniform_problems(shapes, seed=inputs.SEED_BASE + 41, integer=True,
                                 alpha=1.5, beta=-0.5)
    out, _, desc = run_lowp(ctx, ps, prec)
    for q in range(ps.count):
        ref, sa, sb = oracle_lowp(ps, q, prec)
        assert desc["ab_scale"][q] == np.float32(1.0 / (sa * sb))
        got = result_of(ps, out, q)
        assert fp32_equal(got, ref), (iaat.PREC_NAMES[prec], ps.layout(q), ps.m[q], ps.n[q], ps.k[q])


@pytest.mark.parametrize("prec", PRECS, ids=[iaat.PREC_NAMES[p] for p in PRECS])
def test_loguniform_grid_parity_and_error(ctx, prec):
    """The sweep grid (every third shape, 2 problems each), |x| = 10^U(-3,3):
    parity with the oracle on dequantised inputs <= 1e-6 K in the scaled
    measure (with magnitudes over six decades a dot product can cancel far
    below its terms, and FP32 accumulation in any order is only bounded
    relative to |alpha| |op(A)||op(B)| + |beta| |C0|); error against the FP32
    masters recorded."""
    ps = inputs.precision_problems(per_shape=2, shapes=grid_shapes())
    out, _, _ = run_lowp(ctx, ps, prec)
    worst = 0.0
    errs = []
    for q in range(ps.count):
        ref, _, _ = oracle_lowp(ps, q, prec)
        got = result_of(ps, out, q)
        k = max(int(ps.k[q]), 1)
        err = scaled_error(ps, q, prec, got, ref)
        assert err <= 1e-6 * k, (iaat.PREC_NAMES[prec], q, ps.layout(q), ps.m[q], ps.n[q], ps.k[q], err)
        worst = max(worst, err / k)
        t = int(ps.trans[q])
        exact = oracle.gemm(t & 1, t >> 1, int(ps.m[q]), int(ps.n[q]), int(ps.k[q]),
                            float(ps.alpha[q]), ps.A(q), int(ps.lda[q]), ps.B(q), int(ps.ldb[q]),
                            float(ps.beta[q]), ps.C(q), int(ps.ldc[q]))
        errs.append(normwise(got, exact))
    errs = np.array(errs)
    # the formats' own accuracy (relative to the masters), far above the gate above
    loose = {1: 2e-2, 2: 5e-3, 3: 2.5e-1, 4: 2e-4}[prec]
    print("%s: parity (scaled) max err/K %.3g; vs FP32 masters: median %.3g p99 %.3g max %.3g" % (
        iaat.PREC_NAMES[prec], worst, np.median(errs), np.percentile(errs, 99), errs.max()))
    assert np.median(errs) <= loose


def test_quick_returns_and_status(ctx):
    shapes = [("NN", 7, 9, 0), ("NN", 0, 5, 5), ("TN", 6, 6, 6)]
    ps = inputs.uniform_problems(shapes, seed=inputs.SEED_BASE + 43, alpha=1.0, beta=2.0)
    ps.alpha[2] = 0.0
    prec = iaat.IAAT_PREC_BF16
    out, _, _ = run_lowp(ctx, ps, prec)
    for q in (0, 2):
        exp = 2.0 * ps.C(q).reshape(int(ps.n[q]), int(ps.ldc[q])).T[:int(ps.m[q]), :]
        assert fp32_equal(result_of(ps, out, q), exp.astype(np.float32))
