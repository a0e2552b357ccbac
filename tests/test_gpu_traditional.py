"""The traditional pack + uniform-tile scheme (the ablation baseline) meets
the same oracle bar as the IAAT path, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2208_09822_amd import iaat, inputs
from _helpers import check_problem, oracle_all

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def run_trad(ctx, ps):
    buf = torch.from_numpy(ps.buf).to(DEV)
    desc = iaat.descriptors(ps, buf.data_ptr())
    plan = iaat.iaat_trad_create(ctx, desc)
    try:
        assert iaat.iaat_trad_workspace_bytes(plan) >= 0
        s = torch.cuda.current_stream(DEV).cuda_stream
        iaat.iaat_trad_pack(plan, s)
        iaat.iaat_trad_compute(plan, s)
        torch.cuda.synchronize(DEV)
    finally:
        iaat.iaat_trad_destroy(plan)
    return buf.cpu().numpy()


@pytest.mark.parametrize("integer", [True, False])
def test_traditional_matches_oracle(integer):
    with iaat.Context(0) as c:
        ps = inputs.uneven_batch(2048, seed=inputs.SEED_BASE + 81, integer=integer)
        out = run_trad(c.handle, ps)
        ref = oracle_all(ps)
        for q in range(ps.count):
            check_problem(ps, out, q, ref[q], exact=integer)


def test_traditional_alpha_zero_does_not_read_ab():
    with iaat.Context(0) as c:
        ps = inputs.uniform_problems([("NN", 9, 7, 5), ("TT", 3, 20, 33)], seed=5, alpha=0.0,
                                     beta=1.5)
        for q in range(ps.count):
            a = ps.A(q)
            a[:] = np.nan
        out = run_trad(c.handle, ps)
        for q in range(ps.count):
            m, n, ldc = int(ps.m[q]), int(ps.n[q]), int(ps.ldc[q])
            got = out[ps.c_off[q]:ps.c_off[q] + ldc * n].reshape(n, ldc).T[:m]
            exp = (1.5 * ps.C(q).reshape(n, ldc).T[:m]).astype(np.float32)
            assert np.array_equal(got, exp)
