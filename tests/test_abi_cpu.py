"""Host-side checks of the C ABI (no GPU work is queued): the library loads,
exports every entry point the public header declares, rejects bad arguments
before touching a device, and its run-time tiler's built-in plans are valid
(exact cover, kernel membership) for every (layout, m, n) <= 80."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2208_09822_amd import iaat
from paper_2208_09822_amd.gen import gen_family

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iaat.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(iaat_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "iaat_gemm" in names and "iaat_gemm_vbatched_device" in names
    out = subprocess.run(["nm", "-D", "--defined-only", iaat.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = iaat.lib()
    for n in names:
        assert hasattr(lib, n)


def test_null_context_rejected_before_device_work():
    lib = iaat.lib()
    assert lib.iaat_gemm(None, 0, 0, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None) == -1
    assert lib.iaat_gemm_vbatched_device(None, None, 1, 0, None, None) == -1
    assert lib.iaat_gemm_vbatched(None, None, 1, 0, None, None) == -1
    assert "NULL" in iaat.iaat_last_error()


def test_small_domain_predicate_edges():
    d = iaat.iaat_in_small_domain
    assert d(0, 80, 80, 80) and not d(0, 80, 80, 81) and not d(3, 81, 80, 80)
    assert d(1, 32, 32, 32) and not d(1, 32, 32, 33)      # TN is layout 1
    assert d(2, 512000, 1, 1) and not d(2, 512001, 1, 1)
    assert not d(0, 2 ** 31 - 1, 2 ** 31 - 1, 2 ** 31 - 1)  # no overflow
    assert d(0, 0, 10 ** 9, 10 ** 9)
    with pytest.raises(iaat.IaatError):
        d(4, 1, 1, 1)


def test_family_matches_generator():
    kids = gen_family.family()
    assert iaat.iaat_family_size() == len(kids)
    for kid, (fam, p1, p2) in enumerate(kids):
        info = iaat.iaat_family_info(kid)
        assert (info["family"], info["p1"], info["p2"]) == (fam, p1, p2)
        assert (info["rows"], info["cols"]) == gen_family.extent(fam, p1, p2)


@pytest.mark.parametrize("layout", range(4))
def test_default_plans_cover_exactly(layout):
    infos = [iaat.iaat_family_info(k) for k in range(iaat.iaat_family_size())]
    for m in range(1, 81):
        for n in range(1, 81):
            blocks = iaat.iaat_default_plan(layout, m, n)
            cover = np.zeros((m, n), np.int32)
            for (i0, j0, rows, cols, kid) in blocks:
                info = infos[kid]
                assert rows == min(info["rows"], m - i0) and cols == min(info["cols"], n - j0)
                if info["family"] in ("ROWS", "KRED"):
                    assert i0 + info["rows"] <= m
                if info["family"] in ("COLS", "KRED"):
                    assert j0 + info["cols"] <= n
                cover[i0:i0 + rows, j0:j0 + cols] += 1
            assert (cover == 1).all(), (layout, m, n, blocks)


def test_default_plan_is_k_independent_and_minimal_for_mfma():
    """Matrix-core plans group ceil(m/16) x ceil(n/16) tiles into at most 3 x 3
    blocks; among such groupings the balanced one minimises sum(m_i + n_i)
    (the load-count principle of Section V-A) -- checked by brute force over
    all groupings into at most two groups per dimension."""
    for m in range(9, 81, 7):
        for n in range(9, 81, 5):
            blocks = iaat.iaat_default_plan(0, m, n)
            s = sum(r + c for (_, _, r, c, _) in blocks)
            tm, tn = -(-m // 16), -(-n // 16)

            def groupings(t):
                if t <= 3:
                    yield [t]
                for a in range(1, 4):
                    if 0 < t - a <= 3:
                        yield [a, t - a]

            best = None
            for gm in groupings(tm):
                for gn in groupings(tn):
                    rows = [min(16 * g, m - 16 * sum(gm[:i])) for i, g in enumerate(gm)]
                    cols = [min(16 * g, n - 16 * sum(gn[:i])) for i, g in enumerate(gn)]
                    cost = sum(r + c for r in rows for c in cols)
                    if len(gm) * len(gn) == len(blocks):
                        best = cost if best is None else min(best, cost)
            assert s == best, (m, n, s, best)
