"""iaat_vbatched_plan / run / free: graph-replayed batches from host
descriptors (the upload is inside the captured graph), against the
device-descriptor plan replay bit for bit and against the FP64 oracle on
integer inputs; a run with another count re-captures, a run with edited
descriptors computes the edited problems."""
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


def device_replay(ctx, ps, desc_host):
    buf = torch.from_numpy(ps.buf).to(DEV)
    d = iaat.descriptors(ps, buf.data_ptr())
    d["alpha"], d["beta"] = desc_host["alpha"], desc_host["beta"]
    dd = torch.from_numpy(d.view(np.uint8)).to(DEV)
    plan = iaat.iaat_vbplan_create(ctx, dd.data_ptr(), ps.count)
    iaat.iaat_vbplan_launch(plan, torch.cuda.current_stream(DEV).cuda_stream)
    torch.cuda.synchronize(DEV)
    iaat.iaat_vbplan_destroy(plan)
    return buf.cpu().numpy()


def test_host_descriptor_plan_runs(ctx):
    s = torch.cuda.current_stream(DEV).cuda_stream
    plan = iaat.iaat_vbatched_plan(ctx, 4000)
    try:
        for count, seed, edit in ((3000, 401, False), (900, 402, False), (900, 403, True)):
            print("[hplan] count=%d seed=%d edit=%s" % (count, seed, edit), flush=True)
            ps = inputs.uneven_batch(count, seed=seed, integer=True)
            buf = torch.from_numpy(ps.buf).to(DEV)
            d = iaat.descriptors(ps, buf.data_ptr())
            if edit:  # same count as the previous run: the graph is replayed, not re-captured
                d["alpha"] = np.where(d["alpha"] == 0, 1.0, -d["alpha"]).astype(np.float32)
                ps.alpha[:] = d["alpha"]
            iaat.iaat_vbatched_run(plan, d, s)
            torch.cuda.synchronize(DEV)
            got = buf.cpu().numpy()
            assert np.array_equal(got.view(np.uint32), device_replay(ctx, ps, d).view(np.uint32))
            sel = list(range(0, count, 7))
            ref = oracle_all(ps, select=sel)
            for q in sel:
                check_problem(ps, got, q, ref[q], exact=True)
    finally:
        iaat.iaat_vbatched_free(plan)


def test_host_descriptor_plan_errors(ctx):
    plan = iaat.iaat_vbatched_plan(ctx, 8)
    try:
        ps = inputs.uneven_batch(9, seed=5)
        d = iaat.descriptors(ps, 0)
        with pytest.raises(iaat.IaatError) as e:
            iaat.iaat_vbatched_run(plan, d)
        assert e.value.code == -3
        iaat.iaat_vbatched_run(plan, d[:0])  # empty run
        torch.cuda.synchronize(DEV)
    finally:
        iaat.iaat_vbatched_free(plan)
    with pytest.raises(iaat.IaatError) as e:
        iaat.iaat_vbatched_plan(ctx, 0)
    assert e.value.code == -2
    assert iaat.lib().iaat_vbatched_run(None, None, 0, None) == -1
