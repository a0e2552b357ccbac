"""Pins for the oracle's rounding helpers and its tile-algorithm reading.

Rounding: compared with library conversions (numpy float16, torch bfloat16
and float8_e4m3fn casts), with exhaustive code tables and with hand-picked
boundary values.  Tiler: the 15 x 15 SGEMM_NN example of Section V-A
(Fig. 2: 72K + 450 loads), the strip lower bound, Table 1's kernel counts,
and cover/membership invariants over every M, N <= 80.
"""
import os

import numpy as np
import pytest
import torch

from oracle import quant, tiler_ref, metrics


def _rand_f32(n, seed):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    return x[np.isfinite(x)]


def test_f16_matches_numpy():
    x = _rand_f32(400000, 1)
    x = np.concatenate([x, np.float32([65504, 65519.99, 65520, 65536, 2 ** -24, 2 ** -25,
                                       3 * 2 ** -26, 2 ** -14, 1 + 2 ** -11, 1 + 3 * 2 ** -11,
                                       -0.0, 0.0])])
    x = x[np.abs(x) < 1e6]
    lib = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(quant.f16_round(x), lib)
    # exhaustive decode vs numpy's binary16
    codes = np.arange(65536, dtype=np.uint16)
    ref = codes.view(np.float16).astype(np.float64)
    dec = quant.f16_decode(codes)
    same = (dec == ref) | (np.isnan(dec) & np.isnan(ref))
    assert same.all()


def test_bf16_matches_torch():
    x = _rand_f32(400000, 2)
    x = np.concatenate([x, np.float32([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20,
                                       3.3895314e38, 1e-40, -0.0])])
    lib = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    mine = quant.bf16_round(x)
    assert np.array_equal(mine, lib)
    codes = np.arange(65536, dtype=np.int32)
    ref = torch.from_numpy(codes.astype(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    dec = quant.bf16_decode(codes)
    assert ((dec == ref) | (np.isnan(dec) & np.isnan(ref))).all()


def test_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-448, 448, 200000),
                        np.sign(rng.standard_normal(50000)) * 2.0 ** rng.uniform(-12, 8.8, 50000)])
    x = x.astype(np.float32)
    x = x[np.abs(x) <= 448]
    lib = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(quant.e4m3_round(x), lib)
    # saturation instead of NaN above 448
    assert quant.e4m3_round(np.array([1e4, -500.0])).tolist() == [448.0, -448.0]


def test_e4m3_code_table():
    codes = np.arange(256)
    vals = quant.e4m3_decode(codes)
    assert np.isnan(vals[0x7F]) and np.isnan(vals[0xFF])
    fin = vals[np.isfinite(vals)]
    assert fin.max() == 448.0 and fin.min() == -448.0
    assert len(np.unique(fin)) == 253            # +0 and -0 coincide
    assert np.array_equal(quant.e4m3_round(fin), fin)   # every value is a fixed point
    assert vals[1] == 2.0 ** -9 and vals[8] == 2.0 ** -6
    # midpoint between 1.0 and 1.125 ties to even (1.0); 1.0625+eps goes up
    assert quant.e4m3_round(np.array([1.0625, 1.0625 + 1e-9, 1.1875]))[:3].tolist() == [1.0, 1.125, 1.25]
    # torch's own decode of every non-NaN code agrees
    t = torch.from_numpy(codes.astype(np.uint8)).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ok = np.isfinite(vals)
    assert np.array_equal(vals[ok], t[ok])


def test_fp8_scale_power_of_two_and_range():
    for absmax in (1e-3, 0.5, 1.0, 3.0, 447.0, 448.0, 449.0, 1e3, 12345.678):
        s = quant.fp8_scale(absmax)
        assert np.log2(s) == int(np.log2(s))
        assert 224.0 < absmax * s <= 448.0
    assert quant.fp8_scale(0.0) == 1.0


def test_split_bf16_properties():
    x = _rand_f32(100000, 4)
    x = x[(np.abs(x) > 1e-30) & (np.abs(x) < 1e30)]
    hi, lo = quant.split_bf16(x)
    x64 = x.astype(np.float64)
    # x - hi is exactly representable in FP32
    assert np.array_equal((x64 - hi).astype(np.float32).astype(np.float64), x64 - hi)
    rel = np.abs(hi + lo - x64) / np.abs(x64)
    assert rel.max() <= 2.0 ** -16


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_rows(name):
    rows = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].split()
        if line:
            rows[line[0]] = [int(x) for x in line[1:]]
    return rows


def test_fig2_fifteen_by_fifteen():
    a, b = golden_rows("fig2_15x15_loads.txt")["iaat"]
    blocks = tiler_ref.sgemm_nn_tile(15, 15)
    assert tiler_ref.memops_S(blocks) == a
    K = 37
    assert tiler_ref.memops(blocks, 15, 15, K) == a * K + b
    assert tiler_ref.strip_dp_optimum(15, 15) == a


def test_table1_kernel_sets():
    """The transcription in tiler_ref equals an independent row-by-row
    transcription of Table 1 (tests/golden/table1_kernels.txt) for every type
    and layout; the per-type totals are derived from the rows (the table
    prints none)."""
    rows = {}
    for line in open(os.path.join(GOLDEN, "table1_kernels.txt")):
        f = line.split("#")[0].split()
        if not f:
            continue
        typ, lay, fixed, cnt = f[0], f[1], int(f[2]), int(f[3])
        ks = rows.setdefault((typ, lay), set())
        for v in range(1, cnt + 1):
            ks.add((v, fixed) if lay == "TT" else (fixed, v))
    assert len(rows) == 16
    for (typ, lay), ks in rows.items():
        assert tiler_ref.kernel_set(typ, lay) == ks, (typ, lay)
    totals = {t: sum(len(rows[(t, l)]) for l in ("NN", "NT", "TN", "TT")) for t in "SDCZ"}
    assert [tiler_ref.kernel_count(t) for t in "SDCZ"] == [totals[t] for t in "SDCZ"]


@pytest.mark.parametrize("M", range(1, 81))
def test_tiler_cover_and_membership(M):
    ks = tiler_ref.kernel_set("S", "NN")
    for N in range(1, 81):
        blocks = tiler_ref.sgemm_nn_tile(M, N)
        cover = np.zeros((M, N), np.int32)
        for (i0, j0, m, n) in blocks:
            assert (m, n) in ks, (M, N, m, n)
            cover[i0:i0 + m, j0:j0 + n] += 1
        assert (cover == 1).all(), (M, N)
        assert tiler_ref.memops_S(blocks) >= tiler_ref.strip_dp_optimum(M, N)


def test_tile_single_dim():
    assert tiler_ref.tile_single_dim(15, range(1, 14)) == [(8, 1), (7, 1)]
    assert tiler_ref.tile_single_dim(26, range(1, 14)) == [(13, 2)]
    assert tiler_ref.tile_single_dim(15, range(1, 5)) == [(4, 3), (3, 1)]
    assert tiler_ref.tile_single_dim(5, [1, 2, 3, 4]) == [(3, 1), (2, 1)]


def test_metrics():
    c = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert metrics.normwise_rel(c, c) == 0.0
    assert metrics.normwise_rel(np.zeros(3), np.zeros(3)) == 0.0
    assert metrics.normwise_rel(np.ones(3), np.zeros(3)) == float("inf")
    d = c.copy(); d[0, 0] += 1e-3
    assert abs(metrics.normwise_rel(d, c) - 1e-3 / np.sqrt(30)) < 1e-15
