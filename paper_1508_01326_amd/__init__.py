"""MI355X-native (gfx950) Radic determinant of non-square matrices.

The determinant of an m x n matrix (m <= n) in Radic's sense is the signed sum,
over all C(n, m) column sequences in dictionary order, of (-1)^(r+s) times the
m x m minor.  The work runs in hand-written HIP kernels behind the C ABI of
``include/radic.h``; this package is a thin ctypes binding with the same names.
"""
from .binding import (  # noqa: F401
    Batch, BatchGraph, autotune, autotune_batched, radic_det_batched, tune_load, tune_save,
    PRECISIONS, RADIC_EDEVICE, RADIC_EINVAL, RADIC_ENONFINITE, RADIC_ENOTSUP, RADIC_EOVERFLOW, RADIC_EWORKSPACE,
    RADIC_FP32_BULK, RADIC_FP64, RADIC_MAX_M, RADIC_MAX_N, RADIC_OK, RADIC_WS_BATCHED, RADIC_WS_DET, RADIC_WS_INT,
    RadicError, host_binomial, host_prime, host_unrank, lib, profile_enable, profile_read, profile_read_launches, radic_det,
    radic_det_int_exact, radic_det_range, radic_det_subsets, set_fallback_tau, set_launch, set_prime_set, status_string, workspace,
    RADIC_ENUM_AUTO, RADIC_ENUM_PER_MINOR, RADIC_ENUM_PREFIX_SHARED, RADIC_ENUM_GROUP_SHARED, set_enumeration, radic_det_2xn,
    host_batch_chunking, host_split_blocks, host_split_count, host_split_prefix, radic_det_batched_noalloc,
    fallback_tau_for,
)
