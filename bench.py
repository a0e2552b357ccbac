#!/usr/bin/env python3
"""Benchmark of the batched small-GEMM path on one MI355X.

Workload: 65,536 uneven FP32 problems C = alpha*op(A)*op(B) + beta*C;
M, N, K uniform over 1..80, redrawn until cbrt(MNK) <= 80 (<= 32 for TN);
layout uniform over NN/NT/TN/TT; entries U[-1,1]; alpha, beta U[-2,2];
ld = stored row count; seeded synthetic data.  Operands and the descriptor
array are resident in device memory before timing starts.

One step = one replay of the graph-captured persistent launch
(iaat_vbplan_launch) over the whole batch: on-device validation, tile-plan
lookup, work queue, block kernels and epilogue.  GFLOP/s = sum 2MNK / t
(the paper's Eq. 1).

Also reported (not the headline value): the same batch through
iaat_gemm_vbatched_device without a graph, through the host-descriptor form
(PCIe copy of the descriptors included), through one iaat_gemm call per
problem, and the FP64 oracle on the host's cores.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]
    python bench.py --profile           # short run for rocprofv3
    python bench.py --calibrate-copy    # a plain 1 GiB device copy (counter scale)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "vbatched small-GEMM GFLOP/s + %roofline vs per-call; p50/p99 serve latency"
KERNEL = "vbatched_f32_kernel"


def source_hash() -> str:
    """Hash of the sources the batched FP32 kernel is compiled from (its
    file and every local header it includes, transitively): a stored counter
    profile applies only to the kernel it was taken on."""
    import re
    csrc = os.path.join(ROOT, "paper_2208_09822_amd", "csrc")
    todo, seen = [os.path.join(csrc, "batched.hip")], set()
    while todo:
        path = os.path.normpath(todo.pop())
        if path in seen or not os.path.exists(path):
            continue
        seen.add(path)
        text = open(path, "rb").read()
        for inc in re.findall(rb'#include "([^"]+)"', text):
            todo.append(os.path.join(os.path.dirname(path), inc.decode()))
    h = hashlib.sha256()
    for path in sorted(seen):
        h.update(os.path.relpath(path, ROOT).encode())
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str):
    """HBM bytes per launch from the committed counter profile, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "vbatched_f32_kernel_uneven65536_counters.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash() or d.get("workload") != workload:
        return None
    return d.get("hbm_bytes_per_launch")


def _events_ms(torch, stream, fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def plain_nn16(iaat, inputs, h, dev, stream):
    """1,000 NN problems of 16 x 16 x 16 (alpha 1.5, beta 0.5): one iaat_gemm
    launch per problem, and the same problems as one batched launch."""
    import numpy as np
    import torch
    ps = inputs.plain_nn16()
    buf = torch.from_numpy(ps.buf).to(dev)
    base, sp, L = buf.data_ptr(), stream.cuda_stream, iaat.lib()
    ao = (base + 4 * ps.a_off).tolist(); bo = (base + 4 * ps.b_off).tolist()
    co = (base + 4 * ps.c_off).tolist()

    def calls():
        for q in range(ps.count):
            L.iaat_gemm(h, 0, 0, 16, 16, 16, 1.5, ao[q], 16, bo[q], 16, 0.5, co[q], 16, sp)

    ms = _events_ms(torch, stream, calls, 5)
    d = torch.from_numpy(iaat.descriptors(ps, base).view(np.uint8)).to(dev)
    ms_b = _events_ms(torch, stream, lambda: iaat.iaat_gemm_vbatched_device(
        h, d.data_ptr(), ps.count, stream=sp), 50)
    fl = ps.flops()
    return {"per_call_us": round(ms * 1e3 / ps.count, 3), "per_call_gflops": round(fl / ms / 1e6, 2),
            "batched_us": round(ms_b * 1e3, 2), "batched_gflops": round(fl / ms_b / 1e6, 1)}


def strided_leg(iaat, h, dev, stream):
    """Same-size batches (iaat_gemm_strided_batched, one shared plan) against
    the same problems through the uneven batched kernel."""
    import numpy as np
    import torch
    res = {}
    sp = stream.cuda_stream
    for (m, n, k, batch) in ((16, 16, 16, 65536), (32, 32, 32, 32768), (80, 80, 80, 8192)):
        g = torch.Generator(device="cpu").manual_seed(m)
        A = (torch.rand(batch * m * k, generator=g) * 2 - 1).to(dev)
        B = (torch.rand(batch * k * n, generator=g) * 2 - 1).to(dev)
        C = (torch.rand(batch * m * n, generator=g) * 2 - 1).to(dev)
        ms = _events_ms(torch, stream, lambda: iaat.iaat_gemm_strided_batched(
            h, 0, 0, m, n, k, 1.0, A.data_ptr(), m, m * k, B.data_ptr(), k, k * n, 1.0,
            C.data_ptr(), m, m * n, batch, sp), 10)
        d = np.zeros(batch, dtype=iaat.PROBLEM_DTYPE)
        z = np.arange(batch, dtype=np.uint64)
        d["A"] = A.data_ptr() + 4 * z * (m * k)
        d["B"] = B.data_ptr() + 4 * z * (k * n)
        d["C"] = C.data_ptr() + 4 * z * (m * n)
        d["m"], d["n"], d["k"], d["lda"], d["ldb"], d["ldc"] = m, n, k, m, k, m
        d["alpha"], d["beta"], d["ab_scale"] = 1.0, 1.0, 1.0
        dd = torch.from_numpy(d.view(np.uint8)).to(dev)
        mb = _events_ms(torch, stream, lambda: iaat.iaat_gemm_vbatched_device(
            h, dd.data_ptr(), batch, stream=sp), 10)
        byt = 4.0 * batch * (m * k + k * n + 2 * m * n)
        fl = 2.0 * batch * m * n * k
        res["nn%d_x%d" % (m, batch)] = {
            "strided_us": round(ms * 1e3, 1), "strided_gbs": round(byt / ms / 1e6, 1),
            "strided_gflops": round(fl / ms / 1e6, 1),
            "vbatched_us": round(mb * 1e3, 1), "vbatched_gbs": round(byt / mb / 1e6, 1)}
    return res


def traditional_leg(iaat, h, ps, desc, iaat_ms, dev, stream):
    """The same uneven batch through the traditional scheme: pack op(A) and
    op(B) into zero-padded tile-contiguous buffers, then one uniform 16 x 16
    tile with a masked C store (the scheme IAAT removes)."""
    import numpy as np
    import torch
    plan = iaat.iaat_trad_create(h, desc)
    sp = stream.cuda_stream
    try:
        ms_pack = _events_ms(torch, stream, lambda: iaat.iaat_trad_pack(plan, sp), 10)
        ms_comp = _events_ms(torch, stream, lambda: iaat.iaat_trad_compute(plan, sp), 10)
        ws = iaat.iaat_trad_workspace_bytes(plan)
    finally:
        iaat.iaat_trad_destroy(plan)
    m, n, k = (x.astype(np.float64) for x in (ps.m, ps.n, ps.k))
    ab = 4.0 * float(np.sum(m * k + k * n))
    c = 4.0 * float(np.sum(m * n * np.where(ps.beta != 0, 2, 1)))
    total = ms_pack + ms_comp
    return {"pack_us": round(ms_pack * 1e3, 1), "compute_us": round(ms_comp * 1e3, 1),
            "total_us": round(total * 1e3, 1), "pack_share": round(ms_pack / total, 3),
            "iaat_us": round(iaat_ms * 1e3, 1), "iaat_speedup": round(total / iaat_ms, 2),
            "packed_workspace_mb": round(ws / 2 ** 20, 1),
            "algorithmic_bytes": {"iaat": int(ab + c), "traditional": int(2 * ab + 2 * ws + c)}}


XGEMM_TYPES = {  # name: (IAAT_DT_*, bytes per element, real flops per multiply-add)
    "dgemm": (1, 8, 2.0), "cgemm": (2, 8, 8.0), "zgemm": (3, 16, 8.0)}


def xgemm_leg(iaat, inputs, h, dev, stream, name):
    """DGEMM / CGEMM / ZGEMM (Table 1 rows D, C, Z) on the plan-driven path:
    same-size strided batches, and an uneven batch of 16,384 problems (M, N,
    K uniform in 1..80, layouts uniform) through iaat_xgemm_vbatched.  Flops
    count 2MNK real or 8MNK complex (Eq. 2); bytes count A, B and C read
    plus C written once each."""
    import numpy as np
    import torch
    dt, eb, fpm = XGEMM_TYPES[name]
    real = torch.float64 if eb == 16 or name == "dgemm" else torch.float32
    per = 2 if name != "dgemm" else 1  # reals per element
    res = {}
    sp = stream.cuda_stream
    fns = {"dgemm": iaat.iaat_dgemm_strided_batched, "cgemm": iaat.iaat_cgemm_strided_batched,
           "zgemm": iaat.iaat_zgemm_strided_batched}
    for (m, n, k, batch) in ((16, 16, 16, 65536), (80, 80, 80, 4096)):
        g = torch.Generator(device="cpu").manual_seed(m + dt)
        mk = lambda c: (torch.rand(per * c, generator=g, dtype=real) * 2 - 1).to(dev)
        A, B, C = mk(batch * m * k), mk(batch * k * n), mk(batch * m * n)
        ms = _events_ms(torch, stream, lambda: fns[name](
            h, 0, 0, m, n, k, 1.0, A.data_ptr(), m, m * k, B.data_ptr(), k, k * n, 1.0,
            C.data_ptr(), m, m * n, batch, sp), 10)
        byt = float(eb) * batch * (m * k + k * n + 2 * m * n)
        res["nn%d_x%d" % (m, batch)] = {"us": round(ms * 1e3, 1), "gbs": round(byt / ms / 1e6, 1),
                                        "hbm_frac": round(byt / ms / 1e6 / HBM_PEAK_GBS, 4),
                                        "gflops": round(fpm * batch * m * n * k / ms / 1e6, 1)}
    # uneven batch
    count = 16384
    rng = np.random.Generator(np.random.PCG64(inputs.SEED_BASE + 40 + dt))
    shp = inputs.uneven_shapes(count, rng)
    lay = np.array([inputs.LAYOUT_BITS[x[0]] for x in shp], np.int32)
    M, N, K = (np.array([x[i] for x in shp], np.int64) for i in (1, 2, 3))
    ta, tb = (lay & 1).astype(bool), (lay & 2).astype(bool)
    lda = np.where(ta, K, M)
    ldb = np.where(tb, N, K)
    sa, sb, sc = M * K, K * N, M * N
    tot = np.cumsum(np.stack([sa, sb, sc], 1).ravel())
    start = np.concatenate([[0], tot[:-1]]).reshape(count, 3)
    g = torch.Generator(device="cpu").manual_seed(77 + dt)
    buf = (torch.rand(per * int(tot[-1]), generator=g, dtype=real) * 2 - 1).to(dev)
    d = np.zeros(count, dtype=iaat.XPROBLEM_DTYPE)
    base = buf.data_ptr()
    d["A"], d["B"], d["C"] = (base + eb * start[:, i].astype(np.uint64) for i in range(3))
    d["trans"], d["m"], d["n"], d["k"] = lay, M, N, K
    d["lda"], d["ldb"], d["ldc"] = lda, ldb, M
    d["alpha"][:, 0] = 1.0
    d["beta"][:, 0] = 1.0
    dd = torch.from_numpy(d.view(np.uint8)).to(dev)
    ms = _events_ms(torch, stream, lambda: iaat.iaat_xgemm_vbatched(h, dt, dd.data_ptr(), count, 0, sp), 5)
    byt = float(eb) * float(np.sum(sa + sb + 2 * sc))
    fl = fpm * float(np.sum(M * N * K))
    res["uneven%d" % count] = {"us": round(ms * 1e3, 1), "gbs": round(byt / ms / 1e6, 1),
                               "hbm_frac": round(byt / ms / 1e6 / HBM_PEAK_GBS, 4),
                               "gflops": round(fl / ms / 1e6, 1)}
    print("[bench] %s uneven %d: %.1f us" % (name, count, ms * 1e3), file=sys.stderr, flush=True)
    return res


def precision_leg(iaat, inputs, h, dev, stream):
    """Reduced-precision inputs on the sweep grid (16 problems per shape,
    |x| = 10^U(-3,3)): on-device quantisation and the batched GEMM, per type.
    Bytes count A and B at the stored width (4 bytes for a bf16 hi/lo pair)."""
    import numpy as np
    import torch
    ps = inputs.precision_problems(per_shape=16)
    buf = torch.from_numpy(ps.buf).to(dev)
    sp = stream.cuda_stream
    fl = ps.flops()
    m, n, k = (x.astype(np.float64) for x in (ps.m, ps.n, ps.k))
    ab_elems = float(np.sum(m * k + k * n))
    c_bytes = float(np.sum(4.0 * m * n * 2))  # beta = 1: C read and written
    res = {"workload": "sweep grid x16 (%d problems), log-uniform entries" % ps.count}
    for prec in (iaat.IAAT_PREC_BF16, iaat.IAAT_PREC_F16, iaat.IAAT_PREC_F8E4M3, iaat.IAAT_PREC_BF16X3):
        eb = iaat.PREC_ELEM_BYTES[prec] * iaat.PREC_SPAN[prec]
        codes = torch.zeros(iaat.PREC_SPAN[prec] * ps.buf.shape[0] * iaat.PREC_ELEM_BYTES[prec],
                            dtype=torch.uint8, device=dev)
        desc_dev = torch.zeros(ps.count * 64, dtype=torch.uint8, device=dev)
        jobs, desc = iaat.lowp_layout(ps, prec, buf.data_ptr(), codes.data_ptr(), desc_dev.data_ptr())
        desc_dev.copy_(torch.from_numpy(desc.view(np.uint8)))
        jd = torch.from_numpy(jobs.view(np.uint8)).to(dev)
        ms_q = _events_ms(torch, stream, lambda: iaat.iaat_quantize_batch(h, prec, jd.data_ptr(),
                                                                            ps.count, sp), 3)
        ms = _events_ms(torch, stream, lambda: iaat.iaat_gemm_vbatched_device(
            h, desc_dev.data_ptr(), ps.count, prec=prec, stream=sp), 5)
        gbs = (ab_elems * eb + c_bytes) / ms / 1e6
        res[iaat.PREC_NAMES[prec]] = {"gemm_us": round(ms * 1e3, 1), "gflops": round(fl / ms / 1e6, 1),
                                      "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                      "quantize_us": round(ms_q * 1e3, 1)}
        print("[bench] precision %s: %.1f us" % (iaat.PREC_NAMES[prec], ms * 1e3), file=sys.stderr,
              flush=True)
    return res


def serve_leg(iaat, inputs, h, dev, seconds):
    """Open-loop Poisson traces at 20k, 50k and 100k requests/s, 1..256 GEMMs
    per request from a resident pool (sweep-grid shapes, alpha = beta = 1),
    8 GB admission cap; latency = completion - scheduled arrival."""
    import numpy as np
    import torch
    ps = inputs.serve_pool(16384)
    buf = torch.from_numpy(ps.buf).to(dev)
    desc = iaat.descriptors(ps, buf.data_ptr())
    pf = 2.0 * ps.m.astype(np.float64) * ps.n * ps.k
    res = {"pool_gemms": ps.count, "seconds": seconds, "mem_cap_gb": 8, "streams": 4}
    for i, rate in enumerate((20000.0, 50000.0, 100000.0)):
        t, cnt = inputs.poisson_trace(rate, seconds, seed=inputs.SEED_BASE + 4 + 10 * (i + 1))
        idx = inputs.pool_indices(int(cnt.sum()), ps.count, seed=inputs.SEED_BASE + 5 + 10 * (i + 1))
        srv = iaat.iaat_serve_start(h, 8 << 30, n_streams=4, max_batch_gemms=16384)
        try:
            lat = iaat.iaat_serve_replay(srv, t, cnt, idx, desc)
            st = iaat.iaat_serve_stats_get(srv)
        finally:
            iaat.iaat_serve_stop(srv)
        offered = float(pf[idx].sum()) / seconds / 1e9
        res["%dk_req_s" % int(rate / 1000)] = {
            "requests": int(t.shape[0]), "gemms": int(cnt.sum()),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "max_ms": round(float(lat.max()) * 1e3, 3),
            "achieved_gflops": round(st["gflops"], 1), "offered_gflops": round(offered, 1),
            "launches": st["launches"], "gemms_per_launch": round(st["gemms_done"] / max(st["launches"], 1), 1),
            "peak_admitted_mb": round(st["peak_admitted_bytes"] / 2 ** 20, 1),
            "peak_queue_depth": st["peak_queue_depth"], "failed": st["failed"],
            "p99_submit_lag_ms": round(st["p99_submit_lag"] * 1e3, 3)}
        print("[bench] serve %dk req/s: p50 %.3f ms p99 %.3f ms (p99 submit lag %.3f ms)" % (
            rate / 1000, np.percentile(lat, 50) * 1e3, np.percentile(lat, 99) * 1e3,
            st["p99_submit_lag"] * 1e3), file=sys.stderr, flush=True)
    # the per-call baseline: the 20k req/s trace's first requests, closed loop
    # (no arrival waits), one iaat_gemm launch per GEMM on one stream -- the
    # most requests per second that path sustains, to set beside the offered
    # rates above
    t, cnt = inputs.poisson_trace(20000.0, seconds, seed=inputs.SEED_BASE + 14)
    idx = inputs.pool_indices(int(cnt.sum()), ps.count, seed=inputs.SEED_BASE + 15)
    nreq = min(int(t.shape[0]), 4000)
    ng = int(cnt[:nreq].sum())
    base = buf.data_ptr()
    L = iaat.lib()
    sp = torch.cuda.current_stream(dev).cuda_stream
    qs = idx[:ng].tolist()
    tr = ps.trans.tolist(); mm = ps.m.tolist(); nn = ps.n.tolist(); kk = ps.k.tolist()
    la = ps.lda.tolist(); lb = ps.ldb.tolist(); lc = ps.ldc.tolist()
    ao = (base + 4 * ps.a_off).tolist(); bo = (base + 4 * ps.b_off).tolist()
    co = (base + 4 * ps.c_off).tolist()
    torch.cuda.synchronize(dev)
    w0 = time.perf_counter()
    for q in qs:
        tq = tr[q]
        L.iaat_gemm(h, tq & 1, tq >> 1, mm[q], nn[q], kk[q], 1.0, ao[q], la[q], bo[q], lb[q], 1.0,
                    co[q], lc[q], sp)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - w0
    res["per_call_baseline"] = {
        "requests": nreq, "gemms": ng, "seconds": round(wall, 3),
        "req_per_s": round(nreq / wall, 1), "gemms_per_s": round(ng / wall, 1),
        "gflops": round(float(pf[idx[:ng]].sum()) / wall / 1e9, 1),
        "note": "closed loop, one launch per GEMM; compare req_per_s with the offered rates"}
    print("[bench] serve per-call baseline: %.0f req/s" % (nreq / wall), file=sys.stderr, flush=True)
    return res


def sweep(iaat, inputs, dev, per_shape, out_path=None, percall_sample=16, chunk_shapes=1024):
    """The plain-method sweep (every (layout, M, N, K) of the grid, ld =
    stored rows, U[-1,1], alpha = beta = 1): each shape's `per_shape`
    problems as one batched launch, and the first `percall_sample` of them
    one iaat_gemm call each (timing sampled; parity over every problem is a
    GPU test).  Problems are generated a chunk of shapes at a time, so memory
    stays bounded at 256 per shape.  Writes the per-shape CSV when
    `out_path` is given; returns the per-layout summary."""
    import numpy as np
    import torch
    from paper_2208_09822_amd import autotune
    shapes = inputs.sweep_shapes()
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    ctx = iaat.Context(0)
    autotune.apply(ctx.handle)
    L = iaat.lib()
    rows = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    ns = min(percall_sample, per_shape)
    for c0 in range(0, len(shapes), chunk_shapes):
        chunk = shapes[c0:c0 + chunk_shapes]
        ps = inputs.sweep_problems(per_shape=per_shape, shapes=chunk, seed=inputs.SEED_BASE + 1 + c0)
        buf = torch.from_numpy(ps.buf).to(dev)
        base = buf.data_ptr()
        desc = torch.from_numpy(iaat.descriptors(ps, base).view(np.uint8)).to(dev)
        ao = (base + 4 * ps.a_off).tolist(); bo = (base + 4 * ps.b_off).tolist()
        co = (base + 4 * ps.c_off).tolist()
        for si, (lay, m, n, k) in enumerate(chunk):
            q0 = si * per_shape
            t = inputs.LAYOUT_BITS[lay]
            lda, ldb = int(ps.lda[q0]), int(ps.ldb[q0])

            def calls():
                for q in range(q0, q0 + ns):
                    L.iaat_gemm(ctx.handle, t & 1, t >> 1, m, n, k, 1.0, ao[q], lda, bo[q], ldb, 1.0,
                                co[q], m, sp)
            calls()
            a.record(stream)
            calls()
            b.record(stream)
            b.synchronize()
            ms_pc = a.elapsed_time(b) / ns
            dptr = desc.data_ptr() + 64 * q0
            iaat.iaat_gemm_vbatched_device(ctx.handle, dptr, per_shape, stream=sp)
            a.record(stream)
            iaat.iaat_gemm_vbatched_device(ctx.handle, dptr, per_shape, stream=sp)
            b.record(stream)
            b.synchronize()
            ms_b = a.elapsed_time(b)
            fl = 2.0 * m * n * k
            rows.append((lay, m, n, k, ms_pc * 1e3, fl / ms_pc / 1e6, ms_b * 1e3,
                         fl * per_shape / ms_b / 1e6))
        del buf, desc
        print("[sweep] %d/%d shapes, %.0fs" % (c0 + len(chunk), len(shapes), time.time() - t0),
              file=sys.stderr, flush=True)
    ctx.close()
    if out_path:
        os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
        with open(out_path, "w") as f:
            f.write("layout,m,n,k,percall_us,percall_gflops,batched_us,batched_gflops\n")
            for r in rows:
                f.write("%s,%d,%d,%d,%.3f,%.3f,%.3f,%.3f\n" % r)
    summ = {"per_shape": per_shape, "percall_timed_per_shape": ns, "shapes": len(rows)}
    for lay in ("NN", "NT", "TN", "TT"):
        rr = np.array([r[4:] for r in rows if r[0] == lay])
        summ[lay] = {"shapes": int(rr.shape[0]), "percall_us_median": round(float(np.median(rr[:, 0])), 2),
                     "percall_gflops_median": round(float(np.median(rr[:, 1])), 2),
                     "percall_gflops_max": round(float(np.max(rr[:, 1])), 1),
                     "batched_gflops_median": round(float(np.median(rr[:, 3])), 1),
                     "batched_gflops_max": round(float(np.max(rr[:, 3])), 1)}
    return summ


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--count", type=int, default=65536)
    ap.add_argument("--profile", action="store_true",
                    help="short run (5 steps) with no side measurements, for rocprofv3")
    ap.add_argument("--only", choices=["traditional", "strided", "dgemm", "cgemm", "zgemm",
                                       "precision", "serve"],
                    help="run one side leg alone (after a single headline step), for profiling; "
                         "prints that leg's JSON")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-percall", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of each open-loop serving trace (seconds)")
    ap.add_argument("--sweep", action="store_true",
                    help="only the shape sweep: every grid shape, one call per problem vs one "
                         "batched launch; per-shape CSV to --sweep-out, summary JSON to stdout")
    ap.add_argument("--sweep-per-shape", type=int, default=256)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the shape sweep leg of the default run")
    ap.add_argument("--sweep-out", default="sweep.csv")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the benchmark measures one GPU only (no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2208_09822_amd import iaat, inputs

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # two reference kernels of known traffic: a 1 GiB device copy (reads
        # 1 GiB, writes 1 GiB) and an elementwise add (reads 2 GiB, writes 1 GiB)
        n = (1 << 30) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        src2 = torch.full((n,), 2.0, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        for _ in range(3):
            torch.add(src, src2, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 1 << 30, "launches": 3,
                          "calibrate_add_read_bytes": 2 << 30, "add_launches": 3}))
        return 0

    if args.sweep:
        summ = sweep(iaat, inputs, dev, args.sweep_per_shape, args.sweep_out)
        print(json.dumps({"sweep": summ, "csv": args.sweep_out}), flush=True)
        return 0

    if args.profile or args.only:
        args.steps, args.warmup = (5, 1) if args.profile else (1, 1)
        args.no_cpu_baseline = args.no_percall = args.no_precision = args.no_serve = True
        args.no_sweep = True

    t0 = time.time()
    ps = inputs.uneven_batch(args.count)
    workload = "uneven_vbatched_%d" % ps.count
    flops = ps.flops()
    alg_bytes = ps.algorithmic_bytes()
    print("[bench] generated %d problems (%.3f GFLOP, %.3f GB algorithmic) in %.1fs"
          % (ps.count, flops / 1e9, alg_bytes / 1e9, time.time() - t0), file=sys.stderr, flush=True)

    buf = torch.from_numpy(ps.buf).to(dev)
    desc = iaat.descriptors(ps, buf.data_ptr())
    desc_dev = torch.from_numpy(desc.view(np.uint8)).to(dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    ctx = iaat.Context(0)
    from paper_2208_09822_amd import autotune
    tuned = autotune.apply(ctx.handle)  # the install-time autotuned tile table
    plan = iaat.iaat_vbplan_create(ctx.handle, desc_dev.data_ptr(), ps.count)

    # --- timed region: graph replays of the persistent batched launch
    for _ in range(args.warmup):
        iaat.iaat_vbplan_launch(plan, sp)
    torch.cuda.synchronize(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for s in range(args.steps):
        iaat.iaat_vbplan_launch(plan, sp)
        ev[s + 1].record(stream)
    torch.cuda.synchronize(dev)
    per = [ev[s].elapsed_time(ev[s + 1]) for s in range(args.steps)]
    ms_total = ev[0].elapsed_time(ev[-1])
    ms = ms_total / args.steps
    value = flops / (ms * 1e-3) / 1e9
    print("[bench] graph replay: %.1f us/step (median %.1f, min %.1f)"
          % (ms * 1e3, float(np.median(per)) * 1e3, min(per) * 1e3), file=sys.stderr, flush=True)

    achieved = alg_bytes / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": stored_traffic(workload),
            "kernel": KERNEL, "algorithmic_bytes_per_launch": int(alg_bytes),
            "avg_launch_us": round(ms * 1e3, 2)}

    if args.only:
        h = ctx.handle
        if args.only == "traditional":
            r = traditional_leg(iaat, h, ps, desc, ms, dev, stream)
        elif args.only == "strided":
            r = strided_leg(iaat, h, dev, stream)
        elif args.only == "precision":
            r = precision_leg(iaat, inputs, h, dev, stream)
        elif args.only == "serve":
            r = serve_leg(iaat, inputs, h, dev, args.serve_seconds)
        else:
            r = xgemm_leg(iaat, inputs, h, dev, stream, args.only)
        iaat.iaat_vbplan_destroy(plan)
        ctx.close()
        print(json.dumps({"only": args.only, "result": r}), flush=True)
        return 0

    extra = {}
    if not args.profile:
        # the same batch without the graph, and with host-resident descriptors
        def timed(fn, reps):
            fn()
            torch.cuda.synchronize(dev)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize(dev)
            return a.elapsed_time(b) / reps

        ms_dev = timed(lambda: iaat.iaat_gemm_vbatched_device(ctx.handle, desc_dev.data_ptr(),
                                                              ps.count, stream=sp), 20)
        ms_host = timed(lambda: iaat.iaat_gemm_vbatched(ctx.handle, desc, stream=sp), 10)
        extra["device_descriptor_form"] = {"gflops": round(flops / ms_dev / 1e6, 1),
                                           "us_per_call": round(ms_dev * 1e3, 1)}
        extra["host_descriptor_form_pcie_inclusive"] = {
            "gflops": round(flops / ms_host / 1e6, 1), "us_per_call": round(ms_host * 1e3, 1)}

    if not args.no_percall:
        # one iaat_gemm launch per problem, same problems, same stream
        base = buf.data_ptr()
        L = iaat.lib()
        tr = ps.trans.tolist(); mm = ps.m.tolist(); nn = ps.n.tolist(); kk = ps.k.tolist()
        al = ps.alpha.tolist(); be = ps.beta.tolist()
        la = ps.lda.tolist(); lb = ps.ldb.tolist(); lc = ps.ldc.tolist()
        ao = (base + 4 * ps.a_off).tolist(); bo = (base + 4 * ps.b_off).tolist()
        co = (base + 4 * ps.c_off).tolist()
        h = ctx.handle

        def percall():
            g = L.iaat_gemm
            for q in range(ps.count):
                t = tr[q]
                g(h, t & 1, t >> 1, mm[q], nn[q], kk[q], al[q], ao[q], la[q], bo[q], lb[q],
                  be[q], co[q], lc[q], sp)

        percall()
        torch.cuda.synchronize(dev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        a.record(stream)
        percall()
        b.record(stream)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - w0
        ms_pc = a.elapsed_time(b)
        extra["per_call"] = {"gflops": round(flops / ms_pc / 1e6, 2),
                             "us_per_problem": round(ms_pc * 1e3 / ps.count, 3),
                             "launches": ps.count, "host_wall_s": round(wall, 3),
                             "speedup_of_value": round(value / (flops / ms_pc / 1e6), 1)}
        print("[bench] per-call: %.2f us/problem" % (ms_pc * 1e3 / ps.count), file=sys.stderr,
              flush=True)

    if not args.no_percall:
        extra["plain_nn16_1000"] = plain_nn16(iaat, inputs, ctx.handle, dev, stream)
    if not args.no_percall:
        extra["strided_same_size"] = strided_leg(iaat, ctx.handle, dev, stream)
        extra["ablation_traditional"] = traditional_leg(iaat, ctx.handle, ps, desc, ms, dev, stream)
        for name in ("dgemm", "cgemm", "zgemm"):
            extra[name] = xgemm_leg(iaat, inputs, ctx.handle, dev, stream, name)
    if not args.no_precision:
        extra["precision"] = precision_leg(iaat, inputs, ctx.handle, dev, stream)
    if not args.no_serve:
        extra["serve"] = serve_leg(iaat, inputs, ctx.handle, dev, args.serve_seconds)
    if not args.no_sweep:
        extra["sweep"] = sweep(iaat, inputs, dev, args.sweep_per_shape)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # at most 16 threads: the host CPU share that comes with one GPU
        cores = min(len(os.sched_getaffinity(0)), 16)
        # repeat the full batch until about 1.5 s of wall time (tens of
        # CPU-seconds on the host's cores) so the rate is stable
        secs, reps = 0.0, 0
        while secs < 1.5 and reps < 50:
            _, t1, _ = oracle.gemm_batch(ps, nthreads=cores)
            secs += t1
            reps += 1
        cpu = {"value": round(reps * flops / secs / 1e9, 3), "unit": "GFLOP/s", "cores": cores,
               "kind": "oracle",
               "sample": "the full %d-problem batch x %d, FP64 triple loop, %d threads (the "
                         "host CPU share of one GPU), %.2f s" % (ps.count, reps, cores, secs)}

    iaat.iaat_vbplan_destroy(plan)
    ctx.close()
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "problems": ps.count,
                   "shapes": "M,N,K ~ U{1..80}, cbrt(MNK)<=80 (<=32 for TN)",
                   "layouts": "NN/NT/TN/TT uniform", "values": "U[-1,1]",
                   "scalars": "alpha,beta ~ U[-2,2]", "form": "iaat_vbplan_launch (hipGraph)",
                   "tile_table": "autotuned (%d plans from tables/gfx950.txt)" % tuned,
                   "gflop_per_step": round(flops / 1e9, 4),
                   "algorithmic_gb_per_step": round(alg_bytes / 1e9, 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
