"""Tile-table editing and the autotuned table, through the C ABI."""
import os

import numpy as np
import pytest
import torch

from paper_2208_09822_amd import autotune, iaat, inputs
from _helpers import check_problem, oracle_all

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def run_batch(ctx, ps):
    buf = torch.from_numpy(ps.buf).to(DEV)
    d = torch.from_numpy(iaat.descriptors(ps, buf.data_ptr()).view(np.uint8)).to(DEV)
    iaat.iaat_gemm_vbatched_device(ctx, d.data_ptr(), ps.count,
                                   stream=torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize(DEV)
    return buf.cpu().numpy()


def test_tuned_table_parity():
    with iaat.Context(0) as c:
        changed = autotune.apply(c.handle)
        assert changed > 0
        ps = inputs.uneven_batch(8192, seed=inputs.SEED_BASE + 61, integer=True)
        out = run_batch(c.handle, ps)
        ref = oracle_all(ps)
        for q in range(ps.count):
            check_problem(ps, out, q, ref[q], exact=True)
        pu = inputs.uneven_batch(2048, seed=inputs.SEED_BASE + 62)
        out = run_batch(c.handle, pu)
        ref = oracle_all(pu)
        for q in range(pu.count):
            check_problem(pu, out, q, ref[q], exact=False)


def test_plan_set_validation_and_save_roundtrip(tmp_path):
    kids = autotune._kids()
    with iaat.Context(0) as c:
        h = c.handle
        with pytest.raises(iaat.IaatError) as e:  # does not cover the last column
            iaat.iaat_plan_set(h, 0, 40, 40, [(0, 0, kids[("MFMA", 2, 2)])])
        assert e.value.code == -5
        with pytest.raises(iaat.IaatError):
            iaat.iaat_plan_set(h, 0, 0, 40, [(0, 0, kids[("MFMA", 1, 1)])])
        blocks = autotune.mfma_blocks(40, 40, 3, 3, kids)
        iaat.iaat_plan_set(h, 0, 40, 40, blocks)
        # staged plans are not used before the commit
        assert len(iaat.iaat_plan_query(h, 0, 40, 40)) == len(iaat.iaat_default_plan(0, 40, 40))
        iaat.iaat_table_commit(h)
        got = [(b[0], b[1], b[4]) for b in iaat.iaat_plan_query(h, 0, 40, 40)]
        assert got == blocks
        path = str(tmp_path / "t.iaattbl")
        iaat.iaat_table_save(h, path)
    with iaat.Context(0, path) as c2:
        got = [(b[0], b[1], b[4]) for b in iaat.iaat_plan_query(c2.handle, 0, 40, 40)]
        assert got == blocks


def test_full_batch_in_the_benchmarked_configuration():
    """The uneven 65,536-problem batch exactly as bench.py times it (autotuned
    table, graph-replayed batched launch): integer inputs bit-exact on every
    problem, uniform inputs on a sample of 4,096 problems."""
    with iaat.Context(0) as c:
        autotune.apply(c.handle)
        s = torch.cuda.current_stream(DEV).cuda_stream
        for integer in (True, False):
            ps = inputs.uneven_batch(65536, integer=integer)
            buf = torch.from_numpy(ps.buf).to(DEV)
            d = torch.from_numpy(iaat.descriptors(ps, buf.data_ptr()).view(np.uint8)).to(DEV)
            plan = iaat.iaat_vbplan_create(c.handle, d.data_ptr(), ps.count)
            try:
                iaat.iaat_vbplan_launch(plan, s)
                torch.cuda.synchronize(DEV)
            finally:
                iaat.iaat_vbplan_destroy(plan)
            out = buf.cpu().numpy()
            sel = None if integer else np.random.Generator(np.random.PCG64(5)).choice(
                ps.count, 4096, replace=False)
            ref = oracle_all(ps, select=sel)
            for q, r in ref.items():
                check_problem(ps, out, q, r, exact=integer)
