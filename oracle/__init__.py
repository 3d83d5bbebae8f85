"""Oracle for the Radic determinant -- TEST INFRASTRUCTURE ONLY.

Plain CPU evaluation of Definition 3, eq. (1): enumerate every ascending column
sequence in dictionary order (Sections 3-5), evaluate each m x m minor (FP64
Gaussian elimination with partial pivoting, or exact Bareiss for integers), apply
(-1)^(r+s) and sum.  The C part is ``radic_oracle.c``; this module only loads it
and converts arguments.  ``exact.py`` holds independent exact evaluators used to
pin it.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does, and nothing here imports the GPU library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if _build.stale():
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u64, i64, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_binomial.argtypes = [i32, i32, ip]
        L.oracle_binomial.restype = u64
        L.oracle_unrank.argtypes = [u64, i32, i32, ip]
        L.oracle_unrank.restype = None
        L.oracle_unrank_trace.argtypes = [u64, i32, i32, ip, ip, ip, u64p, ip]
        L.oracle_unrank_trace.restype = i32
        L.oracle_successor.argtypes = [ip, i32, i32]
        L.oracle_successor.restype = i32
        L.oracle_subset_term_f64.argtypes = [dp, i32, i32, i64, u64, ip]
        L.oracle_subset_term_f64.restype = ctypes.c_double
        L.oracle_subset_terms_f64.argtypes = [dp, i32, i32, i64, u64, u64, dp]
        L.oracle_subset_terms_f64.restype = i32
        L.oracle_radic_f64_range.argtypes = [dp, i32, i32, i64, u64, u64, i32, dp]
        L.oracle_radic_f64_range.restype = i32
        L.oracle_radic_int_range.argtypes = [i32p, i32, i32, i64, u64, u64, i32, u32p, i32, ip, ip]
        L.oracle_radic_int_range.restype = i32
        L.oracle_subset_term_int.argtypes = [i32p, i32, i32, i64, u64, u32p, i32, ip, ip]
        L.oracle_subset_term_int.restype = i32
        _lib = L
    return _lib


def _threads(nthreads):
    if nthreads is None:
        nthreads = min(os.cpu_count() or 1, 16)
    return int(nthreads)


def binomial(a, b):
    ovf = ctypes.c_int(0)
    v = lib().oracle_binomial(a, b, ctypes.byref(ovf))
    if ovf.value:
        raise OverflowError(f"C({a},{b}) does not fit in 64 bits")
    return int(v)


def unrank(q, m, n):
    """q-th (0-based) ascending sequence of {1..n} of length m, 1-based values."""
    B = (ctypes.c_int * m)()
    lib().oracle_unrank(q, m, n, B)
    return list(B)


def unrank_trace(q, m, n):
    """Moves of the combinatorial addition: list of (k, p, q_after, B_after)."""
    B = (ctypes.c_int * m)()
    tk = (ctypes.c_int * m)()
    tp = (ctypes.c_int * m)()
    tq = (ctypes.c_uint64 * m)()
    tB = (ctypes.c_int * (m * m))()
    moves = lib().oracle_unrank_trace(q, m, n, B, tk, tp, tq, tB)
    out = [(tk[i], tp[i], int(tq[i]), list(tB[i * m:(i + 1) * m])) for i in range(moves)]
    return list(B), out


def successor(B, n):
    """Dictionary-order successor of a 1-based ascending sequence, or None at the end."""
    m = len(B)
    arr = (ctypes.c_int * m)(*B)
    ok = lib().oracle_successor(arr, m, n)
    return list(arr) if ok else None


def _as_f64(A):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    return A


def _as_i32(A):
    A = np.asarray(A)
    if A.dtype.kind not in "iu":
        raise ValueError("integer matrix expected")
    if A.size and (A.min() < -(2 ** 31) or A.max() >= 2 ** 31):
        raise ValueError("entries must fit in int32")
    A = np.ascontiguousarray(A.astype(np.int32))
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    return A


def radic_f64(A, q0=0, count=0, nthreads=None):
    """FP64 oracle.  Returns dict(value, hi, lo, abs_sum) over ranks [q0, q0+count)
    (count = 0: all remaining ranks)."""
    A = _as_f64(A)
    m, n = A.shape
    out = (ctypes.c_double * 4)()
    rc = lib().oracle_radic_f64_range(A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m, n, n,
                                      q0, count, _threads(nthreads), out)
    if rc != 0:
        raise ValueError(f"oracle_radic_f64_range failed with {rc}")
    return {"value": out[0], "hi": out[1], "lo": out[2], "abs_sum": out[3]}


def subset_term_f64(A, q):
    """(-1)^(r+s) det(A_J) in FP64 for the q-th sequence J, and J (1-based)."""
    A = _as_f64(A)
    m, n = A.shape
    B = (ctypes.c_int * m)()
    v = lib().oracle_subset_term_f64(A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m, n, n, q, B)
    return v, list(B)


def subset_terms_f64(A, q0=0, count=None):
    """The signed FP64 terms (-1)^(r+s) det(A_J) of ranks [q0, q0 + count) in rank
    order (count None: to the end), as a numpy array; the same values the
    summing enumerator adds."""
    A = _as_f64(A)
    m, n = A.shape
    total = binomial(n, m)
    if count is None:
        count = total - q0
    out = np.empty(int(count), dtype=np.float64)
    rc = lib().oracle_subset_terms_f64(A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m, n, n, q0, count,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError(f"oracle_subset_terms_f64 failed with {rc}")
    return out


def _limbs_to_int(mag, length, sign):
    v = 0
    for i in reversed(range(length)):
        v = (v << 32) | int(mag[i])
    return -v if sign < 0 else v


def radic_int(A, q0=0, count=0, nthreads=None, cap=256):
    """Exact integer oracle (Bareiss in multi-precision integers); returns a Python int."""
    A = _as_i32(A)
    m, n = A.shape
    mag = (ctypes.c_uint32 * cap)()
    length, sign = ctypes.c_int(0), ctypes.c_int(0)
    rc = lib().oracle_radic_int_range(A.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), m, n, n, q0, count,
                                      _threads(nthreads), mag, cap, ctypes.byref(length), ctypes.byref(sign))
    if rc != 0:
        raise ValueError(f"oracle_radic_int_range failed with {rc}")
    return _limbs_to_int(mag, length.value, sign.value)


def subset_term_int(A, q, cap=256):
    A = _as_i32(A)
    m, n = A.shape
    mag = (ctypes.c_uint32 * cap)()
    length, sign = ctypes.c_int(0), ctypes.c_int(0)
    rc = lib().oracle_subset_term_int(A.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), m, n, n, q, mag, cap,
                                      ctypes.byref(length), ctypes.byref(sign))
    if rc != 0:
        raise ValueError(f"oracle_subset_term_int failed with {rc}")
    return _limbs_to_int(mag, length.value, sign.value)
