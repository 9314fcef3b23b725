"""CPU oracle for the CB-SpMV hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product path (the HIP library and its Python
binding) never imports it, and it imports nothing from the product.

* ``spmv_oracle.c`` (built to ``liboracle.so`` with plain gcc, no fast-math):
  the plain FP64 sparse product over COO triplets (Section 2.1-2.2), the same
  product over CSR rows on several threads (the all-core CPU reference), its
  Neumaier-compensated checking variant, the |A||x| scale of the accuracy
  metric, the k-right-hand-side product, and FP64 -> FP32 / BF16
  round-to-nearest-even of stored values.
* ``cb_model.py``: the conversion steps of Section 3 (partition, th0 decision,
  column aggregation, format selection, packing, Algorithm 2).
* ``scaled_error`` below: the accuracy metric |y - y_ref| / (|alpha||A||x| +
  |beta||y0|) with exact-match rules for zero scale and non-finite results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spmv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64, _i32, _dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
_p = ctypes.c_void_p


def build() -> str:
    """Compile the C oracle with gcc (no -ffast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-fopenmp", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_spmv_coo.argtypes = [_i64, _i64, _p, _p, _p, _p, _dbl, _dbl, _p, _p, _p]
        L.oracle_spmv_coo_comp.argtypes = [_i64, _i64, _p, _p, _p, _p, _dbl, _dbl, _p, _p, _p, _p]
        L.oracle_scale_coo.argtypes = [_i64, _i64, _p, _p, _p, _p, _dbl, _dbl, _p, _p]
        L.oracle_spmm_coo.argtypes = [_i64, _i64, _i32, _p, _p, _p, _p, _i64, _dbl, _dbl, _p, _p, _i64,
                                      ctypes.c_int, _p]
        L.oracle_spmv_csr_par.argtypes = [_i64, _p, _p, _p, _p, _dbl, _p, ctypes.c_int]
        L.oracle_round_f32_bits.argtypes = [_dbl]
        L.oracle_round_f32_bits.restype = ctypes.c_uint32
        L.oracle_round_bf16_bits.argtypes = [_dbl]
        L.oracle_round_bf16_bits.restype = ctypes.c_uint16
        L.oracle_round_f32_array.argtypes = [_i64, _p, _p]
        L.oracle_round_bf16_array.argtypes = [_i64, _p, _p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_p) if a is not None and a.size else None


def _coo(csr):
    rows = np.ascontiguousarray(np.repeat(np.arange(csr.m, dtype=np.int32), np.diff(csr.row_ptr)))
    return rows, np.ascontiguousarray(csr.col_idx, dtype=np.int32), np.ascontiguousarray(csr.values, dtype=np.float64)


def spmv(csr, x, alpha=1.0, beta=0.0, y0=None, comp=False, values=None, coo=None):
    """y = alpha * A x + beta * y0 over the COO triplets of ``csr``.
    ``values`` overrides the stored values (e.g. the rounded storage values)."""
    m = csr.m
    rows, cols, vals = coo if coo is not None else _coo(csr)
    if values is not None:
        vals = np.ascontiguousarray(values, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y0a = np.ascontiguousarray(y0 if y0 is not None else np.zeros(m), dtype=np.float64)
    y = np.empty(m, dtype=np.float64)
    if m == 0:
        return y
    L = lib()
    if comp:
        s, c = np.empty(m), np.empty(m)
        L.oracle_spmv_coo_comp(m, vals.shape[0], _ptr(rows), _ptr(cols), _ptr(vals), _ptr(x), alpha, beta,
                               _ptr(y0a), _ptr(y), _ptr(s), _ptr(c))
    else:
        w = np.empty(m)
        L.oracle_spmv_coo(m, vals.shape[0], _ptr(rows), _ptr(cols), _ptr(vals), _ptr(x), alpha, beta,
                          _ptr(y0a), _ptr(y), _ptr(w))
    return y


def scale(csr, x, alpha=1.0, beta=0.0, y0=None, values=None, coo=None):
    m = csr.m
    rows, cols, vals = coo if coo is not None else _coo(csr)
    if values is not None:
        vals = np.ascontiguousarray(values, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y0a = np.ascontiguousarray(y0 if y0 is not None else np.zeros(m), dtype=np.float64)
    s = np.empty(m)
    if m:
        lib().oracle_scale_coo(m, vals.shape[0], _ptr(rows), _ptr(cols), _ptr(vals), _ptr(x), alpha, beta,
                               _ptr(y0a), _ptr(s))
    return s


def spmm(csr, X, alpha=1.0, beta=0.0, Y0=None, comp=False, values=None, coo=None):
    """Y = alpha * A X + beta * Y0; X is n x k row-major, result m x k."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    k = X.shape[1]
    m = csr.m
    rows, cols, vals = coo if coo is not None else _coo(csr)
    if values is not None:
        vals = np.ascontiguousarray(values, dtype=np.float64)
    Y0a = np.ascontiguousarray(Y0 if Y0 is not None else np.zeros((m, k)), dtype=np.float64)
    Y = np.empty((m, k))
    if m == 0 or k == 0:
        return Y
    work = np.empty(2 * m * k)
    lib().oracle_spmm_coo(m, vals.shape[0], k, _ptr(rows), _ptr(cols), _ptr(vals), _ptr(X), k, alpha, beta,
                          _ptr(Y0a), _ptr(Y), k, 1 if comp else 0, _ptr(work))
    return Y


def spmm_scale(csr, X, alpha=1.0, beta=0.0, Y0=None, values=None):
    """|alpha| |A| |X| + |beta| |Y0| column by column."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    k = X.shape[1]
    out = np.empty((csr.m, k))
    coo = _coo(csr)
    for j in range(k):
        out[:, j] = scale(csr, X[:, j], alpha, beta, None if Y0 is None else Y0[:, j], values=values, coo=coo)
    return out


def round_f32_bits(v) -> np.ndarray:
    v = np.ascontiguousarray(np.atleast_1d(v), dtype=np.float64)
    out = np.empty(v.shape, dtype=np.uint32)
    lib().oracle_round_f32_array(v.size, _ptr(v), _ptr(out))
    return out


def round_bf16_bits(v) -> np.ndarray:
    v = np.ascontiguousarray(np.atleast_1d(v), dtype=np.float64)
    out = np.empty(v.shape, dtype=np.uint16)
    lib().oracle_round_bf16_array(v.size, _ptr(v), _ptr(out))
    return out


def f32_values(v) -> np.ndarray:
    """The FP32 storage values as float64."""
    return round_f32_bits(v).view(np.float32).astype(np.float64)


def bf16_values(v) -> np.ndarray:
    """The BF16 storage values as float64 (bf16 bits are the top half of an f32)."""
    b = round_bf16_bits(v).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def scaled_error(y, yref, scl, tol):
    """Return (max_e, violations, worst_index) for e_i = |y_i - yref_i| / scl_i.

    Rules: where scl_i == 0 the result must equal yref_i exactly; where yref_i is
    NaN the result must be NaN; where yref_i is +-Inf the result must be the same
    infinity.  Any breach of these rules counts as e_i = inf."""
    y = np.asarray(y, dtype=np.float64).ravel()
    yref = np.asarray(yref, dtype=np.float64).ravel()
    scl = np.asarray(scl, dtype=np.float64).ravel()
    e = np.zeros(y.shape[0])
    nan_ref = np.isnan(yref)
    inf_ref = np.isinf(yref)
    fin = ~(nan_ref | inf_ref)
    zero = fin & (scl == 0)
    reg = fin & (scl != 0) & np.isfinite(scl)
    e[nan_ref & ~np.isnan(y)] = np.inf
    e[inf_ref & (y != yref)] = np.inf
    e[zero & (y != yref)] = np.inf
    with np.errstate(invalid="ignore", over="ignore"):
        d = np.abs(y[reg] - yref[reg]) / scl[reg]
    d[np.isnan(d)] = np.inf
    e[reg] = d
    # a finite reference with an overflowing scale only has to be a number
    big = fin & ~np.isfinite(scl)
    e[big & np.isnan(y)] = np.inf
    viol = int((e > tol).sum())
    worst = int(np.argmax(e)) if e.size else -1
    return (float(e.max()) if e.size else 0.0), viol, worst
