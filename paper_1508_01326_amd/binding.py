"""ctypes binding of ``libradic.so`` (argument marshalling only).

Every function named like a C entry point takes PyTorch tensors for device
buffers, passes raw pointers and the current HIP stream, and returns what the C
call returns.  All arithmetic runs in the library's HIP kernels.  Loading fails
loudly when the library has not been built.
"""
import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libradic.so")

RADIC_OK = 0
RADIC_EINVAL = -1
RADIC_ENOTSUP = -2
RADIC_EOVERFLOW = -3
RADIC_ENOMEM = -4
RADIC_EDEVICE = -5
RADIC_EWORKSPACE = -6
RADIC_ENONFINITE = -7

RADIC_FP64 = 0
RADIC_FP32_BULK = 1
PRECISIONS = {"fp64": RADIC_FP64, "fp32_bulk": RADIC_FP32_BULK}

RADIC_WS_DET = 0
RADIC_WS_INT = 1
RADIC_WS_BATCHED = 2

RADIC_ENUM_AUTO = 0
RADIC_ENUM_PER_MINOR = 1
RADIC_ENUM_PREFIX_SHARED = 2
RADIC_ENUM_GROUP_SHARED = 3

RADIC_MAX_M = 12
RADIC_MAX_M_WIDE = 32
RADIC_MAX_N = 1024
RADIC_MAX_PRIMES = 24

F64_RESULT_DTYPE = np.dtype([("value", "<f8"), ("hi", "<f8"), ("lo", "<f8"), ("abs_sum", "<f8"),
                             ("n_subsets", "<u8"), ("n_fallback", "<u8"), ("status", "<i4"),
                             ("reserved", "<i4")])
DESC_DTYPE = np.dtype([("m", "<i4"), ("n", "<i4"), ("dtype", "<i4"), ("reserved", "<i4"),
                       ("offset", "<i8"), ("lda", "<i8")])
BATCH_RESULT_DTYPE = np.dtype([("value", "<f8"), ("hi", "<f8"), ("lo", "<f8"), ("abs_sum", "<f8"),
                               ("n_subsets", "<u8"), ("n_fallback", "<u8"), ("status", "<i4"),
                               ("sign", "<i4"), ("mag_len", "<i4"), ("n_primes", "<i4"),
                               ("mag", "<u4", (RADIC_MAX_PRIMES,))])
assert F64_RESULT_DTYPE.itemsize == 56
assert DESC_DTYPE.itemsize == 32
assert BATCH_RESULT_DTYPE.itemsize == 160

# (name, restype, argtypes) of every exported function
_vp, _i, _i64, _u64, _sz, _d = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                ctypes.c_size_t, ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "radic_status_string": (ctypes.c_char_p, [_i]),
    "radic_version": (_i, []),
    "radic_last_error": (ctypes.c_char_p, []),
    "radic_workspace_bytes": (_sz, [_i, _i, _i, _i]),
    "radic_det": (_i, [_vp, _i, _i, _i64, _i, _vp, _vp, _sz, _vp]),
    "radic_det_range": (_i, [_vp, _i, _i, _i64, _i, _u64, _u64, _vp, _vp, _sz, _vp]),
    "radic_det_subsets": (_i, [_vp, _i, _i, _i64, _i, _u64, _u64, _vp, _vp, _vp]),
    "radic_det_int_exact": (_i, [_vp, _i, _i, _i64, _u32p, _i, _ip, _ip, _vp, _sz, _vp]),
    "radic_det_batched": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _sz, _vp]),
    "radic_det_batched_noalloc": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp]),
    "radic_batched_graph_create": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _sz, ctypes.POINTER(_vp)]),
    "radic_graph_launch": (_i, [_vp, _vp]),
    "radic_graph_destroy": (_i, [_vp]),
    "radic_autotune": (_i, [_i, _i, _i, _i, _ip, _vp]),
    "radic_autotune_batched": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _sz, _ip, _vp]),
    "radic_tune_save": (_i, [ctypes.c_char_p]),
    "radic_tune_load": (_i, [ctypes.c_char_p]),
    "radic_set_launch": (_i, [_i, _i]),
    "radic_set_fallback_tau": (_i, [_d]),
    "radic_fallback_tau_for": (_d, [_u64]),
    "radic_set_enumeration": (_i, [_i]),
    "radic_det_2xn": (_i, [_vp, _i64, _i64, _vp, _vp, _sz, _vp]),
    "radic_profile_enable": (_i, [_i]),
    "radic_profile_read": (_i, [_dp, _ip]),
    "radic_profile_read_launches": (_i, [_dp, _i, _ip]),
    "radic_host_binomial": (_i, [_i, _i, _u64p]),
    "radic_host_unrank": (_i, [_i, _i, _u64, _ip]),
    "radic_host_prime": (_i, [_i, _u32p]),
    "radic_host_batch_chunking": (_i, [_i, _i, _i, _i, _u64p, _u64p]),
    "radic_host_split_count": (_i, [_i, _i, _i, _i, _u64p]),
    "radic_host_split_prefix": (_i, [_i, _i, _i, _i, _u64, _ip]),
    "radic_host_split_blocks": (_i, [_i, _i, _i, _u64p]),
    "radic_set_prime_set": (_i, [_u32p, _i]),
}

_lib = None


class RadicError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        if _lib is not None and status == RADIC_EDEVICE:
            msg += " [" + _lib.radic_last_error().decode() + "]"
        super().__init__(f"{where}: {msg}" if where else msg)


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with paper_1508_01326_amd/build.py "
                              "(there is no CPU fallback)")
        # Load PyTorch first: its wheel carries its own HIP runtime under the same
        # soname as the system one, and the library must bind to the runtime that
        # owns PyTorch's streams and allocations (one runtime per process).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(status):
    return lib().radic_status_string(int(status)).decode()


def _check(rc, where):
    if rc != RADIC_OK:
        raise RadicError(rc, where)


# ------------------------------------------------------------------ torch plumbing
def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require_cuda(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")


def _matrix_args(A, dtype):
    _require_cuda(A, dtype, "A")
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    if A.stride(1) != 1:
        raise ValueError("A must be row-major with unit column stride")
    m, n = A.shape
    lda = A.stride(0) if m > 1 else n
    return m, n, lda


def workspace(kind, m=0, n=0, batch=0, device=None):
    torch = _torch()
    nbytes = int(lib().radic_workspace_bytes(kind, m, n, batch))
    if nbytes == 0:
        raise RadicError(RADIC_EINVAL, "radic_workspace_bytes")
    # torch's caching allocator returns 256-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


def new_f64_result(device=None, pinned=False):
    """A radic_f64_result buffer in device memory, or (pinned=True) in pinned
    host memory, which the library's kernel writes directly."""
    torch = _torch()
    if pinned:
        return torch.zeros(F64_RESULT_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
    return torch.zeros(F64_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=device or "cuda")


_per_thread = threading.local()


def _result_buffer(out, sync, device):
    """The caller's buffer; else, for a synchronous call, this thread's pinned
    host buffer (the result needs no copy back), or a new device buffer."""
    if out is not None:
        return out
    if not sync:
        return new_f64_result(device)
    buf = getattr(_per_thread, "f64_result", None)
    if buf is None:
        buf = _per_thread.f64_result = new_f64_result(pinned=True)
    return buf


def read_f64_result(out):
    raw = (out.cpu() if out.is_cuda else out).numpy().tobytes()
    r = np.frombuffer(raw, dtype=F64_RESULT_DTYPE)[0]
    return {k: (r[k].item()) for k in F64_RESULT_DTYPE.names if k != "reserved"}


# ------------------------------------------------------------------ entry points
def radic_det(A, precision="fp64", out=None, work=None, stream=None, sync=True):
    """Radic determinant of a float64 CUDA matrix.  Returns the result dict
    (sync=True) or the device result buffer (sync=False)."""
    torch = _torch()
    m, n, lda = _matrix_args(A, torch.float64)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    out = _result_buffer(out, sync, A.device)
    work = work if work is not None else workspace(RADIC_WS_DET, max(m, 1), max(n, 1), device=A.device)
    rc = lib().radic_det(ctypes.c_void_p(A.data_ptr()), m, n, lda, prec, ctypes.c_void_p(out.data_ptr()),
                         ctypes.c_void_p(work.data_ptr()), work.numel(), _stream_handle(stream))
    _check(rc, "radic_det")
    if not sync:
        return out
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return read_f64_result(out)


def radic_det_2xn(A, out=None, work=None, stream=None, sync=True):
    """O(n) Radic determinant of a 2 x n float64 CUDA matrix; abs_sum in the
    result is an upper bound on sum |det(A_J)| (see include/radic.h)."""
    torch = _torch()
    _require_cuda(A, torch.float64, "A")
    if A.dim() != 2 or A.shape[0] != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2 x n matrix with unit column stride")
    n, lda = A.shape[1], A.stride(0)
    out = _result_buffer(out, sync, A.device)
    work = work if work is not None else workspace(RADIC_WS_DET, 2, 2, device=A.device)
    rc = lib().radic_det_2xn(ctypes.c_void_p(A.data_ptr()), n, lda, ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(work.data_ptr()), work.numel(), _stream_handle(stream))
    _check(rc, "radic_det_2xn")
    if not sync:
        return out
    torch.cuda.synchronize(A.device)
    return read_f64_result(out)


def radic_det_range(A, q_begin, count, precision="fp64", out=None, work=None, stream=None, sync=True):
    torch = _torch()
    m, n, lda = _matrix_args(A, torch.float64)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    out = _result_buffer(out, sync, A.device)
    work = work if work is not None else workspace(RADIC_WS_DET, max(m, 1), max(n, 1), device=A.device)
    rc = lib().radic_det_range(ctypes.c_void_p(A.data_ptr()), m, n, lda, prec, int(q_begin), int(count),
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                               work.numel(), _stream_handle(stream))
    _check(rc, "radic_det_range")
    if not sync:
        return out
    torch.cuda.synchronize(A.device)
    return read_f64_result(out)


def radic_det_subsets(A, q_begin, count, precision="fp64", with_cols=False, stream=None):
    """Signed terms (-1)^(r+s) det(A_J) for ranks [q_begin, q_begin+count) (and
    the 1-based columns when with_cols).  Returns CPU numpy arrays."""
    torch = _torch()
    m, n, lda = _matrix_args(A, torch.float64)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    terms = torch.empty(int(count), dtype=torch.float64, device=A.device)
    cols = torch.empty(int(count) * m if with_cols else 1, dtype=torch.uint8, device=A.device)
    rc = lib().radic_det_subsets(ctypes.c_void_p(A.data_ptr()), m, n, lda, prec, int(q_begin), int(count),
                                 ctypes.c_void_p(terms.data_ptr()),
                                 ctypes.c_void_p(cols.data_ptr()) if with_cols else None,
                                 _stream_handle(stream))
    _check(rc, "radic_det_subsets")
    torch.cuda.synchronize(A.device)
    t = terms.cpu().numpy()
    if with_cols:
        return t, cols.cpu().numpy().reshape(int(count), m)
    return t


def radic_det_int_exact(A, work=None, stream=None, cap=RADIC_MAX_PRIMES + 2):
    """Exact Radic determinant of an int32 CUDA matrix; returns a Python int."""
    torch = _torch()
    m, n, lda = _matrix_args(A, torch.int32)
    work = work if work is not None else workspace(RADIC_WS_INT, max(m, 1), max(n, 1), device=A.device)
    mag = (ctypes.c_uint32 * cap)()
    length, sign = ctypes.c_int(0), ctypes.c_int(0)
    rc = lib().radic_det_int_exact(ctypes.c_void_p(A.data_ptr()), m, n, lda, mag, cap, ctypes.byref(length),
                                   ctypes.byref(sign), ctypes.c_void_p(work.data_ptr()), work.numel(),
                                   _stream_handle(stream))
    _check(rc, "radic_det_int_exact")
    v = 0
    for i in reversed(range(length.value)):
        v = (v << 32) | int(mag[i])
    return -v if sign.value < 0 else v


def autotune(kind, m=0, n=0, precision="fp64", stream=None):
    """Time launch shapes for (kind, m, n, precision) and keep the fastest;
    returns (subsets_per_lane, block).  For RADIC_WS_BATCHED, precision "exact"
    tunes the exact persistent kernels."""
    prec = {"fp64": 0, "fp32_bulk": 1, "exact": 2}[precision] if isinstance(precision, str) else int(precision)
    best = (ctypes.c_int * 2)()
    _check(lib().radic_autotune(int(kind), int(m), int(n), prec, best, _stream_handle(stream)), "radic_autotune")
    return best[0], best[1]


def autotune_batched(batch, precision="fp64", stream=None):
    """Time the batched chunk sizes on this Batch itself and keep the fastest for
    later batched calls; returns (subsets_per_lane, block)."""
    best = (ctypes.c_int * 2)()
    desc, nb, f64, i32, prec, out, work, nwork = batch.args(precision)
    _check(lib().radic_autotune_batched(desc, nb, f64, i32, prec, out, work, nwork, best, _stream_handle(stream)),
           "radic_autotune_batched")
    return best[0], best[1]


def tune_save(path):
    _check(lib().radic_tune_save(str(path).encode()), "radic_tune_save")


def tune_load(path):
    _check(lib().radic_tune_load(str(path).encode()), "radic_tune_load")


def set_launch(subsets_per_lane=0, block_size=0):
    _check(lib().radic_set_launch(int(subsets_per_lane), int(block_size)), "radic_set_launch")


def set_fallback_tau(tau):
    _check(lib().radic_set_fallback_tau(float(tau)), "radic_set_fallback_tau")


def fallback_tau_for(minors):
    """The FP32-bulk threshold a sum over `minors` minors uses under the current setting."""
    return lib().radic_fallback_tau_for(int(minors))


ENUMERATIONS = {"auto": RADIC_ENUM_AUTO, "per_minor": RADIC_ENUM_PER_MINOR,
                "prefix_shared": RADIC_ENUM_PREFIX_SHARED, "group_shared": RADIC_ENUM_GROUP_SHARED}


def set_enumeration(mode="auto"):
    """Enumeration used by radic_det / radic_det_range: "auto", "per_minor",
    "prefix_shared" or "group_shared" (or the RADIC_ENUM_* value)."""
    code = ENUMERATIONS[mode] if isinstance(mode, str) else int(mode)
    _check(lib().radic_set_enumeration(code), "radic_set_enumeration")


def profile_enable(on=True):
    _check(lib().radic_profile_enable(1 if on else 0), "radic_profile_enable")


def profile_read():
    ms, launches = ctypes.c_double(0.0), ctypes.c_int(0)
    _check(lib().radic_profile_read(ctypes.byref(ms), ctypes.byref(launches)), "radic_profile_read")
    return ms.value, launches.value


def profile_read_launches(capacity=4096):
    buf = (ctypes.c_double * capacity)()
    count = ctypes.c_int(0)
    _check(lib().radic_profile_read_launches(buf, capacity, ctypes.byref(count)), "radic_profile_read_launches")
    return [buf[i] for i in range(min(count.value, capacity))]


def host_binomial(a, b):
    out = ctypes.c_uint64(0)
    rc = lib().radic_host_binomial(int(a), int(b), ctypes.byref(out))
    _check(rc, "radic_host_binomial")
    return int(out.value)


def host_unrank(m, n, q):
    cols = (ctypes.c_int * m)()
    _check(lib().radic_host_unrank(int(m), int(n), int(q), cols), "radic_host_unrank")
    return list(cols)


def set_prime_set(primes=()):
    primes = list(primes)
    arr = (ctypes.c_uint32 * max(len(primes), 1))(*primes)
    _check(lib().radic_set_prime_set(arr, len(primes)), "radic_set_prime_set")


def host_prime(i):
    p = ctypes.c_uint32(0)
    _check(lib().radic_host_prime(int(i), ctypes.byref(p)), "radic_host_prime")
    return int(p.value)


def host_batch_chunking(dtype, m, n, subsets_per_lane):
    """(ranks per chunk, chunks) of one matrix in radic_det_batched."""
    c, k = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().radic_host_batch_chunking(int(dtype), int(m), int(n), int(subsets_per_lane), ctypes.byref(c),
                                           ctypes.byref(k)), "radic_host_batch_chunking")
    return int(c.value), int(k.value)


def host_split_count(m, n, side, v):
    """Prefixes of one side of the two-sided blocks with last column v."""
    c = ctypes.c_uint64(0)
    _check(lib().radic_host_split_count(int(m), int(n), int(side), int(v), ctypes.byref(c)), "radic_host_split_count")
    return int(c.value)


def host_split_prefix(m, n, side, v, j):
    """The j-th such prefix: m-2 columns, 0-based, in that side's coordinates."""
    cols = (ctypes.c_int * (m - 2))()
    _check(lib().radic_host_split_prefix(int(m), int(n), int(side), int(v), int(j), cols), "radic_host_split_prefix")
    return list(cols)


def host_split_blocks(m, n, minors_per_block):
    """Blocks a whole rank space is taken in, about minors_per_block minors each."""
    c = ctypes.c_uint64(0)
    _check(lib().radic_host_split_blocks(int(m), int(n), int(minors_per_block), ctypes.byref(c)),
           "radic_host_split_blocks")
    return int(c.value)


# ------------------------------------------------------------------ batched
class Batch:
    """Device buffers for radic_det_batched: entry pools, descriptors, results and
    workspace, built from a list of 2-D numpy arrays (float64 or int32).  With
    work=False no workspace is made (for radic_det_batched_noalloc)."""

    def __init__(self, matrices, device="cuda", work=True):
        torch = _torch()
        f64, i32, desc = [], [], np.zeros(len(matrices), dtype=DESC_DTYPE)
        foff = ioff = 0
        for b, A in enumerate(matrices):
            A = np.asarray(A)
            m, n = A.shape
            if A.dtype == np.float64:
                desc[b] = (m, n, 0, 0, foff, n)
                f64.append(np.ascontiguousarray(A).ravel())
                foff += A.size
            elif A.dtype == np.int32:
                desc[b] = (m, n, 1, 0, ioff, n)
                i32.append(np.ascontiguousarray(A).ravel())
                ioff += A.size
            else:
                raise ValueError("matrices must be float64 or int32")
        self.batch = len(matrices)
        self.desc_host = desc
        self.desc = torch.from_numpy(desc.view(np.uint8).copy()).to(device)
        self.f64 = torch.from_numpy(np.concatenate(f64) if f64 else np.zeros(1)).to(device)
        self.i32 = torch.from_numpy(np.concatenate(i32) if i32 else np.zeros(1, np.int32)).to(device)
        self.out = torch.zeros(self.batch * BATCH_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.work = workspace(RADIC_WS_BATCHED, batch=self.batch, device=device) if work else None

    def args(self, precision):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        return (ctypes.c_void_p(self.desc.data_ptr()), self.batch, ctypes.c_void_p(self.f64.data_ptr()),
                ctypes.c_void_p(self.i32.data_ptr()), prec, ctypes.c_void_p(self.out.data_ptr()),
                ctypes.c_void_p(self.work.data_ptr()), self.work.numel())

    def results(self):
        raw = self.out.cpu().numpy().tobytes()
        rows = np.frombuffer(raw, dtype=BATCH_RESULT_DTYPE)
        res = []
        for r in rows:
            d = {k: r[k].item() for k in ("value", "hi", "lo", "abs_sum", "n_subsets", "n_fallback", "status",
                                          "sign", "mag_len", "n_primes")}
            v = 0
            for l in reversed(range(int(r["mag_len"]))):
                v = (v << 32) | int(r["mag"][l])
            d["exact"] = -v if r["sign"] < 0 else v
            res.append(d)
        return res


def radic_det_batched(batch, precision="fp64", stream=None, sync=True):
    """Run radic_det_batched on a Batch; returns the per-matrix result dicts."""
    torch = _torch()
    rc = lib().radic_det_batched(*batch.args(precision), _stream_handle(stream))
    _check(rc, "radic_det_batched")
    if not sync:
        return None
    torch.cuda.synchronize()
    return batch.results()


def radic_det_batched_noalloc(batch, precision="fp64", stream=None, sync=True):
    """Run radic_det_batched_noalloc on a Batch (its workspace, if any, is not
    used: the library's static scratch is); returns the per-matrix results."""
    torch = _torch()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    rc = lib().radic_det_batched_noalloc(ctypes.c_void_p(batch.desc.data_ptr()), batch.batch,
                                         ctypes.c_void_p(batch.f64.data_ptr()), ctypes.c_void_p(batch.i32.data_ptr()),
                                         prec, ctypes.c_void_p(batch.out.data_ptr()), _stream_handle(stream))
    _check(rc, "radic_det_batched_noalloc")
    if not sync:
        return None
    torch.cuda.synchronize()
    return batch.results()


class BatchGraph:
    """A HIP graph holding one radic_det_batched call (radic_batched_graph_create)."""

    def __init__(self, batch, precision="fp64"):
        self.handle = ctypes.c_void_p(0)
        rc = lib().radic_batched_graph_create(*batch.args(precision), ctypes.byref(self.handle))
        _check(rc, "radic_batched_graph_create")

    def launch(self, stream=None):
        _check(lib().radic_graph_launch(self.handle, _stream_handle(stream)), "radic_graph_launch")

    def destroy(self):
        if self.handle:
            _check(lib().radic_graph_destroy(self.handle), "radic_graph_destroy")
            self.handle = ctypes.c_void_p(0)
