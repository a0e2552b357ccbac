"""The allocation-free batched entry point (iaat_gemm_vbatched_noalloc)
through the C ABI: on two calls in a row, the second with a smaller batch,
its results equal those of the plan-replayed batched launch it varies
(iaat_vbplan_launch, whose window counter the plan allocates) bit for bit,
and each problem meets the FP32 bar against the FP64 oracle (bit-exact on
integer inputs, normwise <= 1e-6 * K otherwise)."""
import numpy as np
import pytest
import torch

from paper_2208_09822_amd import iaat, inputs
from _helpers import check_problem, oracle_all

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


def run_both(ctx, ps):
    """(plan-replay output, no-alloc output, their status arrays) for one set."""
    sp = torch.cuda.current_stream(DEV).cuda_stream
    buf_ref = torch.from_numpy(ps.buf).to(DEV)
    buf_new = torch.from_numpy(ps.buf).to(DEV)
    d_ref = torch.from_numpy(iaat.descriptors(ps, buf_ref.data_ptr()).view(np.uint8)).to(DEV)
    d_new = torch.from_numpy(iaat.descriptors(ps, buf_new.data_ptr()).view(np.uint8)).to(DEV)
    st_ref = torch.full((ps.count,), 777, dtype=torch.int32, device=DEV)
    st_new = torch.full((ps.count,), 777, dtype=torch.int32, device=DEV)
    plan = iaat.iaat_vbplan_create(ctx, d_ref.data_ptr(), ps.count, status=st_ref.data_ptr())
    try:
        iaat.iaat_vbplan_launch(plan, sp)
        iaat.iaat_gemm_vbatched_noalloc(ctx, d_new.data_ptr(), ps.count, status=st_new.data_ptr(),
                                        stream=sp)
        torch.cuda.synchronize(DEV)
    finally:
        iaat.iaat_vbplan_destroy(plan)
    return (buf_ref.cpu().numpy(), buf_new.cpu().numpy(), st_ref.cpu().numpy(),
            st_new.cpu().numpy())


@pytest.mark.parametrize("integer", [True, False])
def test_noalloc_equals_plan_replay_two_calls(ctx, integer):
    for count, seed in ((4000, 301), (700, 302)):  # second call: a smaller batch
        print("[no-alloc] integer=%s count=%d seed=%d" % (integer, count, seed), flush=True)
        ps = inputs.uneven_batch(count, seed=seed + 10 * integer, integer=integer)
        ref, new, st_ref, st_new = run_both(ctx, ps)
        assert (st_new == 0).all() and (st_ref == 0).all()
        for q in range(ps.count):
            lo, hi = int(ps.c_off[q]), int(ps.c_off[q] + ps.ldc[q] * ps.n[q])
            assert np.array_equal(ref[lo:hi].view(np.uint32), new[lo:hi].view(np.uint32)), q
        sample = np.arange(ps.count) if count <= 1000 else np.arange(0, ps.count, 7)
        refs = oracle_all(ps, select=sample)
        for q in sample:
            check_problem(ps, new, int(q), refs[int(q)], exact=integer)


def test_noalloc_statuses_and_limits(ctx):
    ps = inputs.uneven_batch(64, seed=303, integer=True)
    buf = torch.from_numpy(ps.buf).to(DEV)
    d = iaat.descriptors(ps, buf.data_ptr())
    d["lda"][5] = 0            # invalid: -9
    d["trans"][9] = 8          # invalid: -3
    dd = torch.from_numpy(d.view(np.uint8)).to(DEV)
    st = torch.full((ps.count,), 777, dtype=torch.int32, device=DEV)
    iaat.iaat_gemm_vbatched_noalloc(ctx, dd.data_ptr(), ps.count, status=st.data_ptr(),
                                    stream=torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize(DEV)
    s = st.cpu().numpy()
    assert s[5] == -9 and s[9] == -3
    assert (np.delete(s, [5, 9]) == 0).all()
    lib = iaat.lib()
    assert lib.iaat_gemm_vbatched_noalloc(ctx, dd.data_ptr(), 2 ** 31, None, None) == -3
    assert "2147483647" in iaat.iaat_last_error()
    assert lib.iaat_gemm_vbatched_noalloc(ctx, None, 5, None, None) == -2
    assert lib.iaat_gemm_vbatched_noalloc(None, dd.data_ptr(), 5, None, None) == -1
    assert lib.iaat_gemm_vbatched_noalloc(ctx, None, 0, None, None) == 0
