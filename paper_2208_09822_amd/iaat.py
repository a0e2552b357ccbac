"""ctypes binding of libiaat (include/iaat.h).

Argument marshalling only: every function has the name of the C entry point
it calls, takes plain integers for device pointers and streams (for example
``tensor.data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``), and
raises ``IaatError`` on a non-zero status.  All GEMM work runs in the HIP
library; if ``libiaat.so`` has not been built, loading fails loudly.

torch (when importable) is imported before the library is loaded so that the
process has a single HIP runtime: torch's bundled ``libamdhip64.so.7`` then
satisfies the library's dependency of the same soname.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

import numpy as np

try:  # share torch's HIP runtime when torch is used for memory and streams
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libiaat.so")

IAAT_OP_N, IAAT_OP_T = 0, 1
IAAT_PREC_F32, IAAT_PREC_BF16, IAAT_PREC_F16, IAAT_PREC_F8E4M3, IAAT_PREC_BF16X3 = 0, 1, 2, 3, 4
PREC_NAMES = {0: "f32", 1: "bf16", 2: "f16", 3: "f8e4m3", 4: "bf16x3"}
IAAT_OK = 0
IAAT_ERR_HIP = -100
IAAT_ERR_NOMEM = -101
IAAT_ERR_TABLE = -102
IAAT_ERR_UNSUPPORTED = -103

FAMILY_NAMES = {0: "MFMA", 1: "ROWS", 2: "COLS", 3: "KRED"}

# iaat_problem, 64 bytes
PROBLEM_DTYPE = np.dtype([
    ("A", "<u8"), ("B", "<u8"), ("C", "<u8"),
    ("trans", "<i4"), ("m", "<i4"), ("n", "<i4"), ("k", "<i4"),
    ("lda", "<i4"), ("ldb", "<i4"), ("ldc", "<i4"),
    ("alpha", "<f4"), ("beta", "<f4"), ("ab_scale", "<f4"),
])
assert PROBLEM_DTYPE.itemsize == 64


# iaat_qjob, 64 bytes
QJOB_DTYPE = np.dtype([
    ("a_src", "<u8"), ("b_src", "<u8"), ("a_dst", "<u8"), ("b_dst", "<u8"),
    ("a_n", "<i8"), ("b_n", "<i8"), ("prob", "<u8"), ("scales", "<u8"),
])
assert QJOB_DTYPE.itemsize == 64


class ServeCfg(ctypes.Structure):
    _fields_ = [("mem_cap_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_int32),
                ("max_batch_gemms", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ReqStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("err", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double), ("out", ctypes.c_void_p)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("done", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("gemms_done", ctypes.c_uint64),
                ("p50", ctypes.c_double), ("p99", ctypes.c_double), ("max_latency", ctypes.c_double),
                ("gflops", ctypes.c_double), ("peak_admitted_bytes", ctypes.c_uint64),
                ("peak_queue_depth", ctypes.c_int64), ("p99_submit_lag", ctypes.c_double)]


IAAT_REQ_QUEUED, IAAT_REQ_ADMITTED, IAAT_REQ_DONE = 0, 1, 3


class IaatBlock(ctypes.Structure):
    _fields_ = [("i0", ctypes.c_int32), ("j0", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("kid", ctypes.c_int32)]


class IaatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("iaat error %d: %s" % (code, msg))
        self.code = code


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libiaat.so is not built (%s); run "
                                   "`python -m paper_2208_09822_amd.build`" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            i32, i64, f32, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p
            sig = {
                "iaat_create": (i32, [ctypes.POINTER(vp), i32, ctypes.c_char_p]),
                "iaat_destroy": (i32, [vp]),
                "iaat_last_error": (ctypes.c_char_p, []),
                "iaat_gemm": (i32, [vp, i32, i32, i64, i64, i64, f32, vp, i64, vp, i64, f32,
                                    vp, i64, vp]),
                "iaat_gemm_vbatched_device": (i32, [vp, vp, i64, i32, vp, vp]),
                "iaat_gemm_vbatched": (i32, [vp, vp, i64, i32, vp, vp]),
                "iaat_gemm_vbatched_noalloc": (i32, [vp, vp, i64, vp, vp]),
                "iaat_vbplan_create": (i32, [vp, vp, i64, i32, vp, ctypes.POINTER(vp)]),
                "iaat_quantize_batch": (i32, [vp, i32, vp, i64, vp]),
                "iaat_trad_create": (i32, [vp, vp, i64, ctypes.POINTER(vp)]),
                "iaat_cgemm": (i32, [vp, i32, i32, i64, i64, i64, vp, vp, i64, vp, i64, vp, vp, i64,
                                     vp]),
                "iaat_cgemm_strided_batched": (i32, [vp, i32, i32, i64, i64, i64, vp, vp, i64, i64,
                                                     vp, i64, i64, vp, vp, i64, i64, i64, vp]),
                "iaat_dgemm": (i32, [vp, i32, i32, i64, i64, i64, ctypes.c_double, vp, i64, vp, i64,
                                     ctypes.c_double, vp, i64, vp]),
                "iaat_dgemm_strided_batched": (i32, [vp, i32, i32, i64, i64, i64, ctypes.c_double,
                                                     vp, i64, i64, vp, i64, i64, ctypes.c_double,
                                                     vp, i64, i64, i64, vp]),
                "iaat_zgemm": (i32, [vp, i32, i32, i64, i64, i64, vp, vp, i64, vp, i64, vp, vp, i64,
                                     vp]),
                "iaat_zgemm_strided_batched": (i32, [vp, i32, i32, i64, i64, i64, vp, vp, i64, i64,
                                                     vp, i64, i64, vp, vp, i64, i64, i64, vp]),
                "iaat_xgemm_vbatched": (i32, [vp, i32, vp, i64, vp, vp]),
                "iaat_vbatched_plan": (i32, [vp, i64, i32, ctypes.POINTER(vp)]),
                "iaat_vbatched_run": (i32, [vp, vp, i64, vp]),
                "iaat_vbatched_free": (i32, [vp]),
                "iaat_trad_pack": (i32, [vp, vp]),
                "iaat_trad_compute": (i32, [vp, vp]),
                "iaat_trad_workspace_bytes": (i64, [vp]),
                "iaat_trad_destroy": (i32, [vp]),
                "iaat_gemm_strided_batched": (i32, [vp, i32, i32, i64, i64, i64, f32, vp, i64, i64,
                                                    vp, i64, i64, f32, vp, i64, i64, i64, vp]),
                "iaat_plan_set": (i32, [vp, i32, i32, i32, ctypes.POINTER(IaatBlock), i32]),
                "iaat_table_commit": (i32, [vp]),
                "iaat_table_save": (i32, [vp, ctypes.c_char_p]),
                "iaat_serve_start": (i32, [vp, ctypes.POINTER(ServeCfg), ctypes.POINTER(vp)]),
                "iaat_serve_submit": (i32, [vp, vp, i64, ctypes.c_double, i32,
                                            ctypes.POINTER(ctypes.c_uint64)]),
                "iaat_serve_poll": (i32, [vp, ctypes.c_uint64, ctypes.POINTER(ReqStatus)]),
                "iaat_serve_release": (i32, [vp, ctypes.c_uint64]),
                "iaat_serve_clock": (ctypes.c_double, [vp]),
                "iaat_serve_stats_get": (i32, [vp, ctypes.POINTER(ServeStats)]),
                "iaat_serve_replay": (i32, [vp, i64, vp, vp, vp, vp, i64, vp]),
                "iaat_serve_stop": (i32, [vp]),
                "iaat_vbplan_launch": (i32, [vp, vp]),
                "iaat_vbplan_destroy": (i32, [vp]),
                "iaat_plan_query": (i32, [vp, i32, i32, i32, ctypes.POINTER(IaatBlock), i32]),
                "iaat_default_plan": (i32, [i32, i32, i32, ctypes.POINTER(IaatBlock), i32]),
                "iaat_family_size": (i32, []),
                "iaat_family_info": (i32, [i32] + [ctypes.POINTER(ctypes.c_int32)] * 5),
                "iaat_family_dtypes": (i32, [vp, i32]),
                "iaat_staged_unit_count": (i32, []),
                "iaat_staged_unit_info": (i32, [i32] + [ctypes.POINTER(ctypes.c_int32)] * 3),
                "iaat_in_small_domain": (i32, [i32, i64, i64, i64]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != IAAT_OK:
        raise IaatError(rc, iaat_last_error())
    return rc


def iaat_last_error() -> str:
    return (lib().iaat_last_error() or b"").decode()


def iaat_create(device: int = 0, tile_table_path: Optional[str] = None) -> int:
    h = ctypes.c_void_p()
    p = tile_table_path.encode() if tile_table_path else None
    _check(lib().iaat_create(ctypes.byref(h), int(device), p))
    return h.value


def iaat_destroy(ctx: int) -> None:
    _check(lib().iaat_destroy(ctx))


def iaat_gemm(ctx, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=0) -> None:
    _check(lib().iaat_gemm(ctx, int(ta), int(tb), int(m), int(n), int(k), float(alpha),
                           A or None, int(lda), B or None, int(ldb), float(beta), C or None,
                           int(ldc), stream or None))


def iaat_gemm_vbatched_device(ctx, probs_dev, count, prec=IAAT_PREC_F32, status=0,
                              stream=0) -> None:
    _check(lib().iaat_gemm_vbatched_device(ctx, probs_dev or None, int(count), int(prec),
                                           status or None, stream or None))


def iaat_gemm_vbatched_noalloc(ctx, probs_dev, count, status=0, stream=0) -> None:
    _check(lib().iaat_gemm_vbatched_noalloc(ctx, probs_dev or None, int(count), status or None,
                                            stream or None))


def iaat_gemm_vbatched(ctx, probs_host: np.ndarray, count=None, prec=IAAT_PREC_F32, status=0,
                       stream=0) -> None:
    arr = np.ascontiguousarray(probs_host, dtype=PROBLEM_DTYPE)
    count = len(arr) if count is None else int(count)
    _check(lib().iaat_gemm_vbatched(ctx, arr.ctypes.data if count else None, count, int(prec),
                                    status or None, stream or None))


def iaat_gemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, stride_a, B, ldb, stride_b,
                              beta, C, ldc, stride_c, batch, stream=0) -> None:
    _check(lib().iaat_gemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A or None, lda, stride_a,
                                           B or None, ldb, stride_b, beta, C or None, ldc,
                                           stride_c, batch, stream or None))


def iaat_dgemm(ctx, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=0) -> None:
    _check(lib().iaat_dgemm(ctx, ta, tb, m, n, k, alpha, A or None, lda, B or None, ldb, beta,
                            C or None, ldc, stream or None))


def iaat_dgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, stride_a, B, ldb, stride_b,
                               beta, C, ldc, stride_c, batch, stream=0) -> None:
    _check(lib().iaat_dgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A or None, lda, stride_a,
                                            B or None, ldb, stride_b, beta, C or None, ldc,
                                            stride_c, batch, stream or None))


def _cscalar(x):
    x = complex(x)
    return (ctypes.c_float * 2)(x.real, x.imag)


def iaat_cgemm(ctx, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=0) -> None:
    _check(lib().iaat_cgemm(ctx, ta, tb, m, n, k, _cscalar(alpha), A or None, lda, B or None, ldb,
                            _cscalar(beta), C or None, ldc, stream or None))


def iaat_cgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, stride_a, B, ldb, stride_b,
                               beta, C, ldc, stride_c, batch, stream=0) -> None:
    _check(lib().iaat_cgemm_strided_batched(ctx, ta, tb, m, n, k, _cscalar(alpha), A or None, lda,
                                            stride_a, B or None, ldb, stride_b, _cscalar(beta),
                                            C or None, ldc, stride_c, batch, stream or None))


def _zscalar(x):
    x = complex(x)
    return (ctypes.c_double * 2)(x.real, x.imag)


def iaat_zgemm(ctx, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=0) -> None:
    _check(lib().iaat_zgemm(ctx, ta, tb, m, n, k, _zscalar(alpha), A or None, lda, B or None, ldb,
                            _zscalar(beta), C or None, ldc, stream or None))


def iaat_zgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, stride_a, B, ldb, stride_b,
                               beta, C, ldc, stride_c, batch, stream=0) -> None:
    _check(lib().iaat_zgemm_strided_batched(ctx, ta, tb, m, n, k, _zscalar(alpha), A or None, lda,
                                            stride_a, B or None, ldb, stride_b, _zscalar(beta),
                                            C or None, ldc, stride_c, batch, stream or None))


IAAT_DT_F64, IAAT_DT_C64, IAAT_DT_C128 = 1, 2, 3

# iaat_xproblem (96 bytes)
XPROBLEM_DTYPE = np.dtype([("A", np.uint64), ("B", np.uint64), ("C", np.uint64),
                           ("trans", np.int32), ("m", np.int32), ("n", np.int32), ("k", np.int32),
                           ("lda", np.int32), ("ldb", np.int32), ("ldc", np.int32),
                           ("reserved0", np.int32), ("alpha", np.float64, (2,)),
                           ("beta", np.float64, (2,)), ("reserved1", np.int64)])
assert XPROBLEM_DTYPE.itemsize == 96


def iaat_xgemm_vbatched(ctx, dtype, probs_dev, count, status_dev=0, stream=0) -> None:
    _check(lib().iaat_xgemm_vbatched(ctx, dtype, probs_dev or None, count, status_dev or None,
                                     stream or None))


def iaat_vbatched_plan(ctx, capacity, prec=IAAT_PREC_F32) -> int:
    h = ctypes.c_void_p()
    _check(lib().iaat_vbatched_plan(ctx, int(capacity), int(prec), ctypes.byref(h)))
    return h.value


def iaat_vbatched_run(plan, probs_host: np.ndarray, stream=0) -> None:
    d = np.ascontiguousarray(probs_host, dtype=PROBLEM_DTYPE)
    _check(lib().iaat_vbatched_run(plan, d.ctypes.data if d.shape[0] else None, d.shape[0],
                                   stream or None))


def iaat_vbatched_free(plan) -> None:
    _check(lib().iaat_vbatched_free(plan))


def iaat_trad_create(ctx, probs_host: np.ndarray) -> int:
    d = np.ascontiguousarray(probs_host, dtype=PROBLEM_DTYPE)
    h = ctypes.c_void_p()
    _check(lib().iaat_trad_create(ctx, d.ctypes.data, d.shape[0], ctypes.byref(h)))
    return h.value


def iaat_trad_pack(plan, stream=0) -> None:
    _check(lib().iaat_trad_pack(plan, stream or None))


def iaat_trad_compute(plan, stream=0) -> None:
    _check(lib().iaat_trad_compute(plan, stream or None))


def iaat_trad_workspace_bytes(plan) -> int:
    return lib().iaat_trad_workspace_bytes(plan)


def iaat_trad_destroy(plan) -> None:
    _check(lib().iaat_trad_destroy(plan))


def iaat_quantize_batch(ctx, prec, jobs_dev, count, stream=0) -> None:
    _check(lib().iaat_quantize_batch(ctx, prec, jobs_dev or None, count, stream or None))


def iaat_serve_start(ctx, mem_cap_bytes, n_streams=4, max_batch_gemms=8192,
                     prec=IAAT_PREC_F32) -> int:
    cfg = ServeCfg(mem_cap_bytes, n_streams, max_batch_gemms, prec, 0)
    h = ctypes.c_void_p()
    _check(lib().iaat_serve_start(ctx, ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def iaat_serve_submit(srv, gemms: np.ndarray, t_arrival=-1.0, keep_output=False) -> int:
    g = np.ascontiguousarray(gemms, dtype=PROBLEM_DTYPE)
    t = ctypes.c_uint64()
    _check(lib().iaat_serve_submit(srv, g.ctypes.data, g.shape[0], float(t_arrival),
                                   int(bool(keep_output)), ctypes.byref(t)))
    return t.value


def iaat_serve_poll(srv, ticket):
    """(done: bool, ReqStatus)."""
    st = ReqStatus()
    rc = lib().iaat_serve_poll(srv, ticket, ctypes.byref(st))
    if rc < 0:
        raise IaatError(rc, iaat_last_error())
    return rc == 0, st


def iaat_serve_release(srv, ticket) -> None:
    _check(lib().iaat_serve_release(srv, ticket))


def iaat_serve_clock(srv) -> float:
    return lib().iaat_serve_clock(srv)


def iaat_serve_stats_get(srv) -> dict:
    st = ServeStats()
    _check(lib().iaat_serve_stats_get(srv, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in ServeStats._fields_}


def iaat_serve_replay(srv, t_arrival, n_gemms, pool_idx, pool: np.ndarray):
    """Replays an open-loop trace; returns per-request latencies (seconds)."""
    t = np.ascontiguousarray(t_arrival, dtype=np.float64)
    n = np.ascontiguousarray(n_gemms, dtype=np.int32)
    idx = np.ascontiguousarray(pool_idx, dtype=np.int64)
    p = np.ascontiguousarray(pool, dtype=PROBLEM_DTYPE)
    lat = np.zeros(t.shape[0], dtype=np.float64)
    _check(lib().iaat_serve_replay(srv, t.shape[0], t.ctypes.data, n.ctypes.data, idx.ctypes.data,
                                   p.ctypes.data, p.shape[0], lat.ctypes.data))
    return lat


def iaat_serve_stop(srv) -> None:
    _check(lib().iaat_serve_stop(srv))


def out_offsets(gemms: np.ndarray) -> np.ndarray:
    """Float offset of each GEMM's output inside a served request's output
    region (C spans ldc*(n-1)+m, each rounded up to 64 floats, in order)."""
    g = np.asarray(gemms, dtype=PROBLEM_DTYPE)
    f = np.where((g["m"] > 0) & (g["n"] > 0),
                 g["ldc"].astype(np.int64) * (g["n"].astype(np.int64) - 1) + g["m"], 0)
    f = (f + 63) // 64 * 64
    return np.concatenate([[0], np.cumsum(f)[:-1]]).astype(np.int64)


def iaat_vbplan_create(ctx, probs_dev, count, prec=IAAT_PREC_F32, status=0) -> int:
    h = ctypes.c_void_p()
    _check(lib().iaat_vbplan_create(ctx, probs_dev or None, int(count), int(prec), status or None,
                                    ctypes.byref(h)))
    return h.value


def iaat_vbplan_launch(plan, stream=0) -> None:
    _check(lib().iaat_vbplan_launch(plan, stream or None))


def iaat_vbplan_destroy(plan) -> None:
    _check(lib().iaat_vbplan_destroy(plan))


def _blocks(fn, *args, cap=16):
    out = (IaatBlock * cap)()
    n = fn(*args, out, cap)
    if n < 0:
        raise IaatError(n, iaat_last_error())
    return [(b.i0, b.j0, b.rows, b.cols, b.kid) for b in out[:min(n, cap)]]


def iaat_plan_query(ctx, layout, m, n):
    """Blocks (i0, j0, rows, cols, kid) of the context's plan."""
    return _blocks(lib().iaat_plan_query, ctx, int(layout), int(m), int(n))


def iaat_default_plan(layout, m, n):
    return _blocks(lib().iaat_default_plan, int(layout), int(m), int(n))


def iaat_plan_set(ctx, layout, m, n, blocks) -> None:
    """blocks: sequence of (i0, j0, kid)."""
    arr = (IaatBlock * len(blocks))(*[IaatBlock(i0, j0, 0, 0, kid) for (i0, j0, kid) in blocks])
    _check(lib().iaat_plan_set(ctx, layout, m, n, arr, len(blocks)))


def iaat_table_commit(ctx) -> None:
    _check(lib().iaat_table_commit(ctx))


def iaat_table_save(ctx, path: str) -> None:
    _check(lib().iaat_table_save(ctx, path.encode()))


def iaat_family_size() -> int:
    return lib().iaat_family_size()


def iaat_family_info(kid: int):
    vals = [ctypes.c_int32() for _ in range(5)]
    _check(lib().iaat_family_info(int(kid), *[ctypes.byref(v) for v in vals]))
    fam, p1, p2, br, bc = (v.value for v in vals)
    return {"family": FAMILY_NAMES[fam], "p1": p1, "p2": p2, "rows": br, "cols": bc}


def iaat_family_dtypes():
    n = lib().iaat_family_dtypes(None, 0)
    arr = (ctypes.c_int32 * n)()
    lib().iaat_family_dtypes(arr, n)
    return list(arr)


def iaat_staged_units():
    out = []
    for u in range(lib().iaat_staged_unit_count()):
        vals = [ctypes.c_int32() for _ in range(3)]
        _check(lib().iaat_staged_unit_info(u, *[ctypes.byref(v) for v in vals]))
        out.append((FAMILY_NAMES[vals[0].value], vals[1].value, vals[2].value))
    return out


def iaat_in_small_domain(layout, m, n, k) -> bool:
    rc = lib().iaat_in_small_domain(int(layout), int(m), int(n), int(k))
    if rc < 0:
        raise IaatError(rc, iaat_last_error())
    return bool(rc)


# ------------------------------------------------------------ marshalling

def descriptors(ps, base_ptr: int, elem_bytes: int = 4, ab_scale=None) -> np.ndarray:
    """iaat_problem array for a ProblemSet whose buffer sits in device memory
    at ``base_ptr`` (element offsets scaled by ``elem_bytes``)."""
    d = np.zeros(ps.count, dtype=PROBLEM_DTYPE)
    d["A"] = base_ptr + ps.a_off.astype(np.uint64) * elem_bytes
    d["B"] = base_ptr + ps.b_off.astype(np.uint64) * elem_bytes
    d["C"] = base_ptr + ps.c_off.astype(np.uint64) * 4
    d["trans"] = ps.trans
    d["m"], d["n"], d["k"] = ps.m, ps.n, ps.k
    d["lda"], d["ldb"], d["ldc"] = ps.lda, ps.ldb, ps.ldc
    d["alpha"], d["beta"] = ps.alpha, ps.beta
    d["ab_scale"] = 1.0 if ab_scale is None else ab_scale
    return d


PREC_ELEM_BYTES = {IAAT_PREC_BF16: 2, IAAT_PREC_F16: 2, IAAT_PREC_F8E4M3: 1, IAAT_PREC_BF16X3: 2}
# elements of destination per source element (a hi/lo pair for BF16X3)
PREC_SPAN = {IAAT_PREC_BF16: 1, IAAT_PREC_F16: 1, IAAT_PREC_F8E4M3: 1, IAAT_PREC_BF16X3: 2}


def lowp_layout(ps, prec, src_base: int, dst_base: int, desc_dev: int):
    """Quantisation jobs and reduced-precision descriptors for a ProblemSet
    whose FP32 buffer is at ``src_base``; codes go to a device buffer at
    ``dst_base`` holding ``PREC_SPAN[prec] * len(ps.buf)`` elements of
    ``PREC_ELEM_BYTES[prec]`` bytes, each operand at its FP32 element offset
    times the span.  ``desc_dev`` is where the descriptor array will live (the
    jobs point at its ab_scale fields).  Returns (jobs, descriptors)."""
    eb, sp = PREC_ELEM_BYTES[prec], PREC_SPAN[prec]
    jobs = np.zeros(ps.count, dtype=QJOB_DTYPE)
    lda, ldb = ps.lda.astype(np.int64), ps.ldb.astype(np.int64)
    ta, tb = (ps.trans & 1).astype(bool), (ps.trans & 2).astype(bool)
    cols_a = np.where(ta, ps.m, ps.k).astype(np.int64)
    cols_b = np.where(tb, ps.k, ps.n).astype(np.int64)
    jobs["a_src"] = src_base + ps.a_off.astype(np.uint64) * 4
    jobs["b_src"] = src_base + ps.b_off.astype(np.uint64) * 4
    jobs["a_dst"] = dst_base + ps.a_off.astype(np.uint64) * (eb * sp)
    jobs["b_dst"] = dst_base + ps.b_off.astype(np.uint64) * (eb * sp)
    jobs["a_n"], jobs["b_n"] = lda * cols_a, ldb * cols_b
    jobs["prob"] = desc_dev + np.arange(ps.count, dtype=np.uint64) * PROBLEM_DTYPE.itemsize
    d = descriptors(ps, src_base)
    d["A"], d["B"] = jobs["a_dst"], jobs["b_dst"]
    return jobs, d


class Context:
    """Owns an iaat context (``with Context() as ctx: ...``)."""

    def __init__(self, device: int = 0, tile_table_path: Optional[str] = None):
        self.handle = iaat_create(device, tile_table_path)

    def close(self):
        if self.handle:
            iaat_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
