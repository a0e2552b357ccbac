"""Shared test helpers: run problem sets through the HIP library (through the
C ABI binding) and compare with the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle


def fp32_equal(got, exp):
    got = np.asarray(got, np.float32)
    exp = np.asarray(exp, np.float32)
    return bool(np.all((got == exp) | (np.isnan(got) & np.isnan(exp))))


def result_of(ps, out_buf, q):
    m, n = int(ps.m[q]), int(ps.n[q])
    ldc = int(ps.ldc[q])
    c = out_buf[ps.c_off[q]:ps.c_off[q] + ldc * n].reshape(n, ldc).T
    return c[:m, :]


def oracle_one(ps, q):
    t = int(ps.trans[q])
    return oracle.gemm(t & 1, t >> 1, int(ps.m[q]), int(ps.n[q]), int(ps.k[q]),
                       float(ps.alpha[q]), ps.A(q), int(ps.lda[q]), ps.B(q), int(ps.ldb[q]),
                       float(ps.beta[q]), ps.C(q), int(ps.ldc[q]))


def oracle_all(ps, nthreads=16, select=None):
    """{q: FP64 result} for all (or selected) problems, threaded C oracle."""
    idx = np.arange(ps.count) if select is None else np.asarray(select)
    out, _, off = oracle.gemm_batch(ps, nthreads=nthreads, select=idx)
    res = {}
    for t, q in enumerate(idx):
        m, n = int(ps.m[q]), int(ps.n[q])
        res[int(q)] = out[off[t]:off[t] + m * n].reshape(n, m).T
    return res


def normwise(got, ref):
    got = np.asarray(got, np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def check_problem(ps, out_buf, q, ref, exact):
    got = result_of(ps, out_buf, q)
    if exact:
        assert fp32_equal(got, ref), "problem %d (%s %dx%dx%d) not bit-exact" % (
            q, ps.layout(q), ps.m[q], ps.n[q], ps.k[q])
    else:
        k = max(int(ps.k[q]), 1)
        err = normwise(got, ref)
        assert err <= 1e-6 * k, "problem %d (%s %dx%dx%d): normwise %.3g > %.3g" % (
            q, ps.layout(q), ps.m[q], ps.n[q], ps.k[q], err, 1e-6 * k)
