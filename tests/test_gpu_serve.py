"""Serving loop (continuous batching) through the C ABI.

Every served GEMM must give bitwise the result the batched form gives for it
alone (the tile plan depends only on the problem and the block kernels not on
the batch), and that result must meet the oracle bar.  Admission must keep
the arena bytes in use under the cap, and the open-loop replay must complete
every request with consistent latency statistics.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

from paper_2208_09822_amd import iaat, inputs
from _helpers import normwise, oracle_one

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
_hip = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))


def d2h(ptr, nfloats):
    out = np.empty(nfloats, np.float32)
    assert _hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr),
                          ctypes.c_size_t(4 * nfloats), 2) == 0  # device to host
    return out


@pytest.fixture(scope="module")
def ctx():
    c = iaat.Context(0)
    yield c.handle
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def pool():
    ps = inputs.serve_pool(512, seed=inputs.SEED_BASE + 44)
    buf = torch.from_numpy(ps.buf).to(DEV)
    desc = iaat.descriptors(ps, buf.data_ptr())
    return ps, buf, desc


def alone_results(ctx, ps, desc):
    """Each pool GEMM alone through the batched form, on a private copy of C."""
    res = {}
    s = torch.cuda.current_stream(DEV).cuda_stream
    for q in range(ps.count):
        m, n, ldc = int(ps.m[q]), int(ps.n[q]), int(ps.ldc[q])
        c = torch.from_numpy(ps.C(q).copy()).to(DEV)
        d = desc[q:q + 1].copy()
        d["C"] = c.data_ptr()
        dd = torch.from_numpy(d.view(np.uint8)).to(DEV)
        iaat.iaat_gemm_vbatched_device(ctx, dd.data_ptr(), 1, stream=s)
        torch.cuda.synchronize(DEV)
        res[q] = c.cpu().numpy().reshape(n, ldc).T[:m, :].copy()
    return res


def test_served_results_equal_alone_results_bitwise(ctx, pool):
    ps, buf, desc = pool
    alone = alone_results(ctx, ps, desc)
    for q in range(0, ps.count, 37):  # the alone results meet the oracle bar
        k = max(int(ps.k[q]), 1)
        assert normwise(alone[q], oracle_one(ps, q)) <= 1e-6 * k
    srv = iaat.iaat_serve_start(ctx, 64 << 20, n_streams=4, max_batch_gemms=1024)
    try:
        rng = np.random.Generator(np.random.PCG64(7))
        reqs = []
        for _ in range(60):
            idx = rng.integers(0, ps.count, int(rng.integers(1, 65)))
            reqs.append((idx, iaat.iaat_serve_submit(srv, desc[idx], keep_output=True)))
        for idx, t in reqs:
            while True:
                done, st = iaat.iaat_serve_poll(srv, t)
                if done:
                    break
            assert st.err == 0 and st.state == iaat.IAAT_REQ_DONE and st.out
            assert st.t_arrival <= st.t_launch <= st.t_done
            g = desc[idx]
            off = iaat.out_offsets(g)
            span = lambda i: int(g["ldc"][i]) * (int(g["n"][i]) - 1) + int(g["m"][i])
            total = int(off[-1] + span(len(g) - 1))
            out = d2h(st.out, total)
            for i, q in enumerate(idx):
                m, n, ldc = int(ps.m[q]), int(ps.n[q]), int(ps.ldc[q])
                col = np.concatenate([out[off[i]:off[i] + span(i)], np.zeros(ldc - m, np.float32)])
                got = col.reshape(n, ldc).T[:m, :]
                assert np.array_equal(got.view(np.uint32), alone[int(q)].view(np.uint32)), (q, i)
            iaat.iaat_serve_release(srv, t)
        stats = iaat.iaat_serve_stats_get(srv)
        assert stats["done"] == 60 and stats["failed"] == 0
        assert stats["launches"] >= 1 and stats["gemms_done"] == sum(len(i) for i, _ in reqs)
    finally:
        iaat.iaat_serve_stop(srv)
    # pool operands are untouched (outputs went to the arena)
    assert np.array_equal(buf.cpu().numpy(), ps.buf)


def test_admission_respects_memory_cap(ctx, pool):
    ps, _, desc = pool
    cap = 1 << 20
    srv = iaat.iaat_serve_start(ctx, cap, n_streams=2, max_batch_gemms=256)
    try:
        rng = np.random.Generator(np.random.PCG64(8))
        tickets = [iaat.iaat_serve_submit(srv, desc[rng.integers(0, ps.count, 16)])
                   for _ in range(80)]
        for t in tickets:
            while not iaat.iaat_serve_poll(srv, t)[0]:
                pass
        stats = iaat.iaat_serve_stats_get(srv)
        assert stats["done"] == 80 and stats["failed"] == 0
        assert 0 < stats["peak_admitted_bytes"] <= cap
        assert stats["peak_queue_depth"] >= 1
    finally:
        iaat.iaat_serve_stop(srv)


def test_open_loop_replay(ctx, pool):
    ps, _, desc = pool
    t_arr, counts = inputs.poisson_trace(20000.0, 0.05, seed=inputs.SEED_BASE + 45, max_gemms=32)
    idx = inputs.pool_indices(int(counts.sum()), ps.count, seed=inputs.SEED_BASE + 46)
    srv = iaat.iaat_serve_start(ctx, 256 << 20, n_streams=4, max_batch_gemms=4096)
    try:
        lat = iaat.iaat_serve_replay(srv, t_arr, counts, idx, desc)
        stats = iaat.iaat_serve_stats_get(srv)
    finally:
        iaat.iaat_serve_stop(srv)
    assert lat.shape[0] == t_arr.shape[0] and (lat > 0).all()
    assert stats["done"] == t_arr.shape[0] and stats["failed"] == 0
    assert stats["gemms_done"] == int(counts.sum())
    assert 0 < stats["p50"] <= stats["p99"] <= stats["max_latency"]
    assert stats["gflops"] > 0


def test_submit_errors(ctx, pool):
    ps, _, desc = pool
    srv = iaat.iaat_serve_start(ctx, 1 << 20, n_streams=1, max_batch_gemms=8)
    try:
        with pytest.raises(iaat.IaatError) as e:
            iaat.iaat_serve_submit(srv, desc[:9])
        assert e.value.code == -3
        bad = desc[:2].copy()
        bad["lda"][1] = 0
        with pytest.raises(iaat.IaatError) as e:
            iaat.iaat_serve_submit(srv, bad)
        assert e.value.code == -4
        t = iaat.iaat_serve_submit(srv, desc[:2])
        while not iaat.iaat_serve_poll(srv, t)[0]:
            pass
        with pytest.raises(iaat.IaatError):
            iaat.iaat_serve_release(srv, t)  # not kept
        with pytest.raises(iaat.IaatError):
            iaat.iaat_serve_poll(srv, 999)
    finally:
        iaat.iaat_serve_stop(srv)
