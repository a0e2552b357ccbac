"""The GPU tile table against the memory-operation cost of Section V-A.

For every (layout, M, N) of the small domain the test computes the plan's
S = sum(m_i + n_i) over its blocks (block extents clipped to the problem:
the K coefficient of the load count) and its block count, for the built-in
table and for the tuned table the benchmark applies, and sets them beside
the strip-DP optimum over the GPU family's strip heights (stored in
golden/gpu_strip_dp.txt by a script that calls only the oracle):

* S never falls below the optimum (the DP is a lower bound for the strip
  tilings the tiler produces -- a plan below it would be a wrong cover);
* a retuned or edited table cannot silently raise the cost: the mean and
  worst ratio S / S_opt stay within the bounds below, set just above the
  committed tables' values (built-in 1.346 mean, 2.000 worst; tuned 1.317
  mean, 2.185 worst -- matrix-core grids of 16 x 16 tiles on skinny shapes
  cost up to about twice the strip optimum, the price of the matrix cores);
* every plan has at most 15 blocks and covers M x N exactly (checked by the
  library when the table is built; recounted here).
"""
import itertools
import os

import numpy as np
import pytest

from oracle import tiler_ref
from paper_2208_09822_amd import autotune, iaat

HERE = os.path.dirname(os.path.abspath(__file__))
GPU_NMAX = {h: (64 if h <= 8 else 48 if h <= 48 else 8) for h in range(1, 65)}
BOUNDS = {"built-in": (1.36, 2.01), "tuned": (1.33, 2.20)}  # (mean, worst) of S / S_opt


def load_dp():
    dp = {}
    for line in open(os.path.join(HERE, "golden", "gpu_strip_dp.txt")):
        if line.startswith("#") or not line.strip():
            continue
        m, n, s = (int(x) for x in line.split())
        dp[(m, n)] = s
    return dp


def test_strip_dp_golden_pins():
    dp = load_dp()
    assert len(dp) == 80 * 80
    # one block covers: S_opt = M + N whenever N fits one piece of an M-high strip
    for (m, n), s in dp.items():
        if m <= 64 and n <= GPU_NMAX[m]:
            assert s == m + n, (m, n, s)
    # brute force over every composition of M into strip heights (M <= 6)
    for m in range(1, 7):
        for n in (1, 5, 49, 65, 80):
            best = None
            for parts in range(1, m + 1):
                for cut in itertools.combinations(range(1, m), parts - 1):
                    hs = np.diff((0,) + cut + (m,))
                    s = sum(-(-n // GPU_NMAX[int(h)]) * int(h) + n for h in hs)
                    best = s if best is None else min(best, s)
            assert dp[(m, n)] == best, (m, n)
    # the stored table is the oracle's DP
    for (m, n) in [(80, 80), (17, 33), (63, 9), (2, 79)]:
        assert dp[(m, n)] == tiler_ref.strip_dp_optimum(m, n, GPU_NMAX)


def _family():
    kids, ext = {}, {}
    for kid in range(iaat.iaat_family_size()):
        info = iaat.iaat_family_info(kid)
        kids[(info["family"], info["p1"], info["p2"])] = kid
        ext[kid] = (info["rows"], info["cols"])
    return kids, ext


def plan_stats(table):
    kids, ext = _family()
    choices = autotune.load(autotune.DEFAULT_TABLE) if table == "tuned" else {}
    out = []
    for lay in range(4):
        for m in range(1, 81):
            for n in range(1, 81):
                blocks = None
                if choices:
                    key, _ = autotune.class_of(lay, m, n)
                    blocks = autotune.plan_for(choices.get(key, "default"), m, n, kids)
                if blocks is None:
                    blocks = [(b[0], b[1], b[4]) for b in iaat.iaat_default_plan(lay, m, n)]
                cover = np.zeros((m, n), np.int32)
                s = 0
                for (i0, j0, kid) in blocks:
                    r, c = min(ext[kid][0], m - i0), min(ext[kid][1], n - j0)
                    cover[i0:i0 + r, j0:j0 + c] += 1
                    s += r + c
                out.append((lay, m, n, s, len(blocks), bool((cover == 1).all())))
    return out


@pytest.mark.parametrize("table", ["built-in", "tuned"])
def test_plan_cost_against_strip_optimum(table):
    dp = load_dp()
    ratios = []
    for (lay, m, n, s, nblk, exact) in plan_stats(table):
        assert exact, (table, lay, m, n)
        assert 1 <= nblk <= 15, (table, lay, m, n, nblk)
        opt = dp[(m, n)]
        assert s >= opt, (table, lay, m, n, s, opt)
        ratios.append(s / opt)
    ratios = np.array(ratios)
    mean_bound, worst_bound = BOUNDS[table]
    assert ratios.mean() <= mean_bound, (table, ratios.mean())
    assert ratios.max() <= worst_bound, (table, ratios.max())
