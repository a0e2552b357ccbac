"""The oracle: plain, slow, obviously correct CPU implementations of what the
small-GEMM path computes.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import, call, link or execute
anything under ``oracle/``.  The product library never does, and shares no
code with it: no kernels, headers, helpers, tables or generators.

Contents
  gemm_f64.c   FP64 triple-loop GEMM (Section I statement, Table 1 note for the
               layouts) for FP32 inputs, and the same loop with FP64 operands
               (DGEMM, Table 1 row D), and the complex loops (CGEMM, row C,
               FP32 storage; ZGEMM, row Z, FP64 storage), built with gcc
               into ``_build/liboracle.so``.
  quant.py     BF16 / FP16 / FP8-E4M3 rounding from the format definitions,
               the split-BF16 pair, the power-of-two FP8 scale.
  tiler_ref.py A reading of the SGEMM_NN tile algorithm (Section V-A,
               Algorithm 2) and its load-count cost model.
  metrics.py   Normwise error measures.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gemm_f64.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, strict IEEE)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    stale = (not os.path.exists(_LIB_PATH)
             or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-pthread", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
            vp = ctypes.c_void_p
            lib.oracle_gemm_f64.argtypes = [i32, i32, i64, i64, i64, dbl, vp, i64,
                                            vp, i64, dbl, vp, i64, vp, i64]
            lib.oracle_gemm_f64.restype = None
            lib.oracle_gemm_f64_d.argtypes = lib.oracle_gemm_f64.argtypes
            lib.oracle_gemm_f64_d.restype = None
            lib.oracle_dgemm.argtypes = lib.oracle_gemm_f64.argtypes
            lib.oracle_dgemm.restype = None
            lib.oracle_cgemm.argtypes = [i32, i32, i64, i64, i64, dbl, dbl, vp, i64, vp, i64,
                                         dbl, dbl, vp, i64, vp, i64]
            lib.oracle_cgemm.restype = None
            lib.oracle_zgemm.argtypes = lib.oracle_cgemm.argtypes
            lib.oracle_zgemm.restype = None
            lib.oracle_gemm_batch.argtypes = [i64] + [vp] * 15 + [i32]
            lib.oracle_gemm_batch.restype = dbl
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def gemm(ta: int, tb: int, m: int, n: int, k: int, alpha: float, A, lda: int,
         B, ldb: int, beta: float, C0, ldc: int) -> np.ndarray:
    """C* = alpha*op(A)*op(B) + beta*C0 in FP64 (Section I).

    A, B, C0 are flat FP32 arrays in column-major storage (A may be None when
    alpha == 0 or k == 0; C0 may be None when beta == 0).  Returns C* as an
    (m, n) float64 array (numpy C-order indexing ``out[i, j]``).
    """
    lib = _load()
    out = np.zeros((max(n, 1), max(m, 1)), dtype=np.float64)  # column-major m x n
    a = None if A is None else np.ascontiguousarray(A, dtype=np.float32)
    b = None if B is None else np.ascontiguousarray(B, dtype=np.float32)
    c = None if C0 is None else np.ascontiguousarray(C0, dtype=np.float32)
    if m > 0 and n > 0:
        lib.oracle_gemm_f64(int(ta), int(tb), m, n, k, float(alpha), _ptr(a), lda,
                            _ptr(b), ldb, float(beta), _ptr(c), ldc, _ptr(out), max(m, 1))
    return out[:n, :m].T.copy()


def gemm_dequant(ta, tb, m, n, k, alpha, A64, lda, B64, ldb, beta, C0, ldc):
    """Same definition with FP64 operand arrays (already dequantized values)."""
    lib = _load()
    out = np.zeros((max(n, 1), max(m, 1)), dtype=np.float64)
    a = np.ascontiguousarray(A64, dtype=np.float64)
    b = np.ascontiguousarray(B64, dtype=np.float64)
    c = None if C0 is None else np.ascontiguousarray(C0, dtype=np.float32)
    if m > 0 and n > 0:
        lib.oracle_gemm_f64_d(int(ta), int(tb), m, n, k, float(alpha), _ptr(a), lda,
                              _ptr(b), ldb, float(beta), _ptr(c), ldc, _ptr(out), max(m, 1))
    return out[:n, :m].T.copy()


def dgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc):
    """DGEMM (Table 1, row D): FP64 operands and C0, FP64 result (m x n)."""
    lib = _load()
    out = np.zeros((max(n, 1), max(m, 1)), dtype=np.float64)
    a = None if A is None else np.ascontiguousarray(A, dtype=np.float64)
    b = None if B is None else np.ascontiguousarray(B, dtype=np.float64)
    c = None if C0 is None else np.ascontiguousarray(C0, dtype=np.float64)
    if m > 0 and n > 0:
        lib.oracle_dgemm(int(ta), int(tb), m, n, k, float(alpha), _ptr(a), lda, _ptr(b), ldb,
                         float(beta), _ptr(c), ldc, _ptr(out), max(m, 1))
    return out[:n, :m].T.copy()


def cgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc):
    """CGEMM (Table 1, row C): complex64 operands (numpy arrays of the stored
    matrices, column-major, flat), complex alpha/beta; complex128 m x n result."""
    lib = _load()
    out = np.zeros((max(n, 1), max(m, 1)), dtype=np.complex128)
    a = None if A is None else np.ascontiguousarray(A, dtype=np.complex64)
    b = None if B is None else np.ascontiguousarray(B, dtype=np.complex64)
    c = None if C0 is None else np.ascontiguousarray(C0, dtype=np.complex64)
    al, be = complex(alpha), complex(beta)
    if m > 0 and n > 0:
        lib.oracle_cgemm(int(ta), int(tb), m, n, k, al.real, al.imag, _ptr(a), lda, _ptr(b), ldb,
                         be.real, be.imag, _ptr(c), ldc, _ptr(out), max(m, 1))
    return out[:n, :m].T.copy()


def zgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc):
    """ZGEMM (Table 1, row Z; Eq. 2's complex product): complex128 operands
    (numpy arrays of the stored matrices, column-major, flat), complex
    alpha/beta; complex128 m x n result."""
    lib = _load()
    out = np.zeros((max(n, 1), max(m, 1)), dtype=np.complex128)
    a = None if A is None else np.ascontiguousarray(A, dtype=np.complex128)
    b = None if B is None else np.ascontiguousarray(B, dtype=np.complex128)
    c = None if C0 is None else np.ascontiguousarray(C0, dtype=np.complex128)
    al, be = complex(alpha), complex(beta)
    if m > 0 and n > 0:
        lib.oracle_zgemm(int(ta), int(tb), m, n, k, al.real, al.imag, _ptr(a), lda, _ptr(b), ldb,
                         be.real, be.imag, _ptr(c), ldc, _ptr(out), max(m, 1))
    return out[:n, :m].T.copy()


def gemm_batch(batch, nthreads: int = 1, select=None):
    """Run the FP64 oracle over a problem set.

    ``batch`` is a problem set from the input generators (struct-of-arrays
    with element offsets into one FP32 buffer).  ``select`` optionally limits
    the run to a subset of problem indices.  Returns ``(outputs, seconds)``:
    ``outputs`` is a flat float64 array, problem q's M x N column-major result
    at ``out_off[q]`` (returned as the third element), and ``seconds`` the
    wall time of the threaded run.
    """
    lib = _load()
    idx = np.arange(batch.count) if select is None else np.asarray(select, dtype=np.int64)
    sub = {f: np.ascontiguousarray(getattr(batch, f)[idx]) for f in
           ("trans", "m", "n", "k", "lda", "ldb", "ldc", "alpha", "beta",
            "a_off", "b_off", "c_off")}
    sizes = sub["m"].astype(np.int64) * sub["n"].astype(np.int64)
    out_off = np.zeros(len(idx), dtype=np.int64)
    if len(idx) > 1:
        out_off[1:] = np.cumsum(sizes)[:-1]
    out = np.zeros(int(sizes.sum()) + 1, dtype=np.float64)
    i32 = lambda f: np.ascontiguousarray(sub[f], dtype=np.int32)
    f32 = lambda f: np.ascontiguousarray(sub[f], dtype=np.float32)
    i64 = lambda f: np.ascontiguousarray(sub[f], dtype=np.int64)
    arrs = [i32("trans"), i32("m"), i32("n"), i32("k"), i32("lda"), i32("ldb"),
            i32("ldc"), f32("alpha"), f32("beta"), i64("a_off"), i64("b_off"),
            i64("c_off"), out_off, np.ascontiguousarray(batch.buf, dtype=np.float32), out]
    secs = lib.oracle_gemm_batch(len(idx), *[_ptr(a) for a in arrs], int(nthreads))
    return out, secs, out_off
