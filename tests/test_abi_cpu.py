"""Host-side checks of the C ABI (no GPU work is queued): the library loads,
exports every entry point the public header declares, rejects bad arguments
before touching a device, and its run-time tiler's built-in plans are valid
(exact cover, kernel membership) for every (layout, m, n) <= 80."""
import ctypes
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


def test_generated_registry_matches_library():
    # the data types and staged units the library dispatches are exactly the
    # generator's lists
    assert iaat.iaat_family_dtypes() == [code for code, _ in gen_family.DTYPES]
    assert iaat.iaat_staged_units() == [(fam, p1, p2) for _, fam, p1, p2 in gen_family.staged_units()]
    assert iaat.lib().iaat_staged_unit_info(iaat.lib().iaat_staged_unit_count(), None, None,
                                            None) == -1


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


def test_default_matrix_core_plans_use_at_most_four_balanced_blocks():
    """Matrix-core plans split ceil(m/16) x ceil(n/16) tiles into at most two
    balanced groups per dimension (at most 3 tiles each), one block per
    wavefront of a four-wavefront work-group."""
    for layout in range(4):
        for m in range(9, 81):
            for n in range(9, 81):
                blocks = iaat.iaat_default_plan(layout, m, n)
                infos = [iaat.iaat_family_info(b[4]) for b in blocks]
                assert all(i["family"] == "MFMA" for i in infos)
                tm, tn = -(-m // 16), -(-n // 16)
                gm = sorted({i["p1"] for i in infos}, reverse=True)
                gn = sorted({i["p2"] for i in infos}, reverse=True)
                want = lambda t: [t] if t == 1 else sorted({t - t // 2, t // 2}, reverse=True)
                assert gm == want(tm) and gn == want(tn), (m, n, blocks)
                assert len(blocks) == (1 if tm == 1 else 2) * (1 if tn == 1 else 2)


def test_quantize_and_precision_arguments_rejected_before_device_work():
    lib = iaat.lib()
    assert lib.iaat_quantize_batch(None, iaat.IAAT_PREC_BF16, None, 1, None) == -1
    assert lib.iaat_gemm_vbatched_device(None, None, 1, iaat.IAAT_PREC_F8E4M3, None, None) == -1
    assert iaat.QJOB_DTYPE.itemsize == 64 and iaat.PROBLEM_DTYPE.itemsize == 64
    assert set(iaat.PREC_NAMES) == {0, 1, 2, 3, 4}


def test_serve_arguments_rejected_before_device_work():
    lib = iaat.lib()
    h = ctypes.c_void_p()
    cfg = iaat.ServeCfg(1 << 20, 1, 8, 0, 0)
    assert lib.iaat_serve_start(None, ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert lib.iaat_serve_submit(None, None, 1, -1.0, 0, None) == -1
    assert lib.iaat_serve_poll(None, 1, None) == -1
    assert lib.iaat_serve_stop(None) == 0
    assert ctypes.sizeof(iaat.ServeCfg) == 24 and ctypes.sizeof(iaat.ReqStatus) == 40


def test_tuned_table_file_is_valid():
    """Every class of the committed tuning has a choice the tuner offers, and
    the plans it implies cover every (layout, m, n) exactly with family kernels."""
    from paper_2208_09822_amd import autotune
    choices = autotune.load(autotune.DEFAULT_TABLE)
    kids = autotune._kids()
    infos = {k: iaat.iaat_family_info(k) for k in range(iaat.iaat_family_size())}
    seen = set()
    for layout in range(4):
        for m in range(1, 81):
            for n in range(1, 81):
                key, offered = autotune.class_of(layout, m, n)
                seen.add(key)
                ch = choices[key]
                assert ch in offered, (key, ch)
                blocks = autotune.plan_for(ch, m, n, kids)
                if blocks is None:
                    continue
                assert len(blocks) <= 15
                cover = np.zeros((m, n), np.int32)
                for (i0, j0, kid) in blocks:
                    r, c = infos[kid]["rows"], infos[kid]["cols"]
                    cover[i0:min(i0 + r, m), j0:min(j0 + c, n)] += 1
                assert (cover == 1).all(), (layout, m, n, ch)
    assert seen == set(choices)


def test_strided_batched_null_context():
    lib = iaat.lib()
    assert lib.iaat_gemm_strided_batched(None, 0, 0, 4, 4, 4, 1.0, None, 4, 16, None, 4, 16, 0.0,
                                         None, 4, 16, 2, None) == -1


def test_library_has_no_unresolved_internal_symbols():
    out = subprocess.run(["nm", "-D", "--undefined-only", iaat.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    bad = [l.split()[-1] for l in out.splitlines() if "iaat" in l]
    assert not bad, bad


def test_dgemm_null_context():
    lib = iaat.lib()
    assert lib.iaat_dgemm(None, 0, 0, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, None) == -1


def test_cgemm_null_context():
    lib = iaat.lib()
    assert lib.iaat_cgemm(None, 0, 0, 4, 4, 4, None, None, 4, None, 4, None, None, 4, None) == -1
