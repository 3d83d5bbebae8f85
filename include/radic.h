/*
 * radic.h -- C ABI of the MI355X (gfx950) Radic-determinant library.
 *
 * The Radic determinant of a real m x n matrix A with m <= n (Definition 3,
 * eq. (1) of Abdollahi, Jafari, Bayat, Amiri and Fathy, "An efficient parallel
 * algorithm for computing determinant of non-square matrices based on Radic's
 * definition"):
 *
 *     det(A) = sum over 1 <= j1 < ... < jm <= n of (-1)^(r+s) det(A[:, j1..jm])
 *     r = 1 + 2 + ... + m,   s = j1 + ... + jm   (1-based column indices),
 *     det(A) = 0 when m > n.
 *
 * The library evaluates the sum the way the paper's parallel algorithm does
 * (Sections 4-5): every GPU lane unranks its first column sequence in dictionary
 * order, walks a contiguous range of ranks with the dictionary successor, gathers
 * each m x m minor, factors it by LU with partial pivoting (FP64, or FP32 with an
 * FP64 rerun of badly conditioned minors) or by fraction-free elimination modulo
 * 31-bit primes (integers), and feeds a compensated wave -> block -> grid tree
 * reduction (the CREW tree sum of Section 6).
 *
 * Conventions shared by every entry point
 *  - Every function is extern "C", never throws and never aborts.
 *  - Pointers named d* are device memory, h* are host memory.  The caller owns
 *    every buffer; the library allocates no device memory per call.  Scratch
 *    space is the caller's workspace (size from radic_workspace_bytes), which
 *    must be 256-byte aligned and must not be shared by calls that may overlap.
 *    The first call on a device (any entry point) uploads the library's
 *    constant tables (binomial coefficients, primes) synchronously; make it
 *    outside stream capture.  After that, radic_det, radic_det_range and
 *    radic_det_batched allocate nothing, never synchronise with the host and
 *    can be captured into a HIP graph.
 *  - Matrices are row-major with leading dimension lda >= n (elements).
 *  - Work is enqueued on `stream` (0 = the null stream).  Functions documented
 *    as asynchronous return after enqueueing; their device-side result,
 *    including the device-detected status, is valid once the stream reaches
 *    that point.  Nothing here uses stream priorities.
 *  - Return values are radic_status codes for host-detected conditions.
 *  - Limits: 1 <= m <= RADIC_MAX_M (RADIC_MAX_M_WIDE for radic_det and
 *    radic_det_range), n <= RADIC_MAX_N, C(n, m) < 2^63.
 */
#ifndef RADIC_H
#define RADIC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RADIC_MAX_M 12
/* radic_det / radic_det_range also take 12 < m <= RADIC_MAX_M_WIDE: such minors
 * are factored by a group of 32 lanes each (one row per lane, partial pivoting
 * by a group max-reduction, true division), in double for both precisions
 * (FP32_BULK reports n_fallback = 0). */
#define RADIC_MAX_M_WIDE 32
#define RADIC_MAX_N 1024
#define RADIC_MAX_PRIMES 24

typedef enum {
    RADIC_OK = 0,
    RADIC_EINVAL = -1,      /* null pointer, m < 1, n < 1, lda < n, bad enum */
    RADIC_ENOTSUP = -2,     /* m > RADIC_MAX_M, n > RADIC_MAX_N, shape too big for on-chip staging */
    RADIC_EOVERFLOW = -3,   /* C(n, m) >= 2^63, or an output buffer too small for the exact result */
    RADIC_ENOMEM = -4,      /* host allocation failed (bookkeeping, or a pinned result buffer) */
    RADIC_EDEVICE = -5,     /* a HIP call failed */
    RADIC_EWORKSPACE = -6,  /* workspace null, misaligned or smaller than radic_workspace_bytes */
    RADIC_ENONFINITE = -7   /* a NaN or infinity in a floating-point input (device-detected) */
} radic_status;

typedef enum {
    RADIC_FP64 = 0,      /* every minor factored in IEEE double */
    RADIC_FP32_BULK = 1  /* minors factored in float on rows pre-scaled by exact powers of two;
                            minors whose product of capped pivot ratios falls below the
                            threshold (radic_set_fallback_tau) are refactored in double;
                            all accumulation in double.  A call (or a
                            batch matrix) over fewer than 4096 minors refactors every minor
                            in double (n_fallback = its minor count): only a sum over many
                            minors absorbs the float error within the tolerance */
} radic_precision;

/* Workspace kinds for radic_workspace_bytes. */
typedef enum {
    RADIC_WS_DET = 0,      /* radic_det, radic_det_subsets */
    RADIC_WS_INT = 1,      /* radic_det_int_exact */
    RADIC_WS_BATCHED = 2   /* radic_det_batched */
} radic_ws_kind;

/* Result of a floating-point Radic determinant (written to device memory).
 * value   = hi + lo rounded to double: the signed sum of eq. (1).
 * hi, lo  = unevaluated double-double sum (|lo| <= ulp(hi)/2 after normalisation).
 * abs_sum = sum of |det(A_J)| over the same subsets (the tolerance normaliser).
 * n_subsets  = number of minors evaluated (C(n, m), or the requested rank count).
 * n_fallback = FP32_BULK only: minors refactored in double.
 * status  = RADIC_OK, or RADIC_ENONFINITE (then value is NaN). */
typedef struct {
    double value;
    double hi;
    double lo;
    double abs_sum;
    uint64_t n_subsets;
    uint64_t n_fallback;
    int32_t status;
    int32_t reserved;
} radic_f64_result;

/* One matrix of a batch.  dtype 0: float64 entries at dF64 + offset; dtype 1: int32
 * entries at dI32 + offset (offset and lda in elements of that type). */
typedef struct {
    int32_t m;
    int32_t n;
    int32_t dtype;
    int32_t reserved;
    int64_t offset;
    int64_t lda;
} radic_matrix_desc;

/* Per-matrix result of a batch (device memory).
 * Float matrices: value/hi/lo/abs_sum/n_fallback as in radic_f64_result.
 * Integer matrices: the exact result is sign * sum_i mag[i] 2^(32 i) with
 * mag_len significant little-endian limbs; value is that integer rounded to double.
 * status: per-matrix radic_status (EINVAL/ENOTSUP for a bad descriptor,
 * EOVERFLOW when the exact result needs more than 24 limbs, ENONFINITE). */
typedef struct {
    double value;
    double hi;
    double lo;
    double abs_sum;
    uint64_t n_subsets;
    uint64_t n_fallback;
    int32_t status;
    int32_t sign;
    int32_t mag_len;
    int32_t n_primes;
    uint32_t mag[RADIC_MAX_PRIMES];
} radic_batch_result;

/* Human-readable name of a status code (static string). */
const char *radic_status_string(int status);

/* Description of the last HIP failure seen by the library on the calling
 * thread (which call failed and HIP's message), or "" if none. */
const char *radic_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int radic_version(void);

/* Bytes of device workspace needed by one call of the given kind.
 * RADIC_WS_DET / RADIC_WS_INT: for an m x n matrix (batch ignored).  The
 * RADIC_WS_DET size grows with C(n, m): it holds the FP32-bulk queue of minors
 * awaiting a double refactorisation, 16 bytes per 64 minors, between 64 MiB
 * and 512 MiB (about 68 MiB for 8 x 32, 313 MiB for 12 x 36).  A larger
 * workspace than asked for gives the queue more room.
 * RADIC_WS_BATCHED: for `batch` matrices (m, n ignored).
 * Returns 0 for invalid arguments. */
size_t radic_workspace_bytes(int kind, int m, int n, int batch);

/*
 * radic_det -- Radic determinant of one float64 matrix (Definition 3, eq. (1)),
 * evaluated over all C(n, m) column sequences in dictionary order.
 *   dA     device, m x n float64, row-major, leading dimension lda (elements).
 *   prec   RADIC_FP64 or RADIC_FP32_BULK.
 *   dOut   one radic_f64_result in device memory, or in pinned host memory
 *          (hipHostMalloc): a kernel writes it, so read it once the stream has
 *          synchronised.
 *   dWork  device workspace of at least radic_workspace_bytes(RADIC_WS_DET, m, n, 0) bytes.
 * Asynchronous.  m > n writes value 0 (Definition 3) and returns RADIC_OK.
 * The minors are summed in an order fixed by the shape and the launch shape
 * (in prefix-shared mode, blocks of minors sharing their first or their last
 * columns, taken over the shared columns' last index upwards, heaviest first),
 * so repeated calls, eager or replayed from a captured graph, give the same bits.
 * Errors: EINVAL, ENOTSUP, EOVERFLOW, EWORKSPACE, EDEVICE (nothing enqueued
 * except for EDEVICE).  Non-finite entries give dOut->status = ENONFINITE.
 */
int radic_det(const double *dA, int m, int n, int64_t lda, int prec, radic_f64_result *dOut,
              void *dWork, size_t work_bytes, hipStream_t stream);

/*
 * radic_det_range -- as radic_det, restricted to the dictionary ranks
 * [q_begin, q_begin + count) (count clipped to C(n, m) - q_begin).  This is one
 * processor's share in the granularity scheme of Section 5 (and one GPU's share
 * when the rank space is split across devices).  dOut->n_subsets = ranks done.
 */
int radic_det_range(const double *dA, int m, int n, int64_t lda, int prec, uint64_t q_begin,
                    uint64_t count, radic_f64_result *dOut, void *dWork, size_t work_bytes,
                    hipStream_t stream);

/*
 * radic_det_subsets -- export the individual signed terms of eq. (1):
 * dTerms[t] = (-1)^(r+s) det(A_J) of the dictionary rank q_begin + t, for
 * t < count, computed like radic_det in the given precision (FP32_BULK terms are
 * rounded float results widened to double, or the double refactorisation when
 * the fallback fires).  Optional dCols (may be null) receives the m 1-based column
 * indices of each sequence as uint8 (requires n <= 255), row t at dCols + t*m.
 * Asynchronous; no workspace.  count must be <= 2^31.
 */
int radic_det_subsets(const double *dA, int m, int n, int64_t lda, int prec, uint64_t q_begin,
                      uint64_t count, double *dTerms, uint8_t *dCols, hipStream_t stream);

/*
 * radic_det_2xn -- Radic determinant of a 2 x n float64 matrix in O(n), the
 * two-row case the paper's introduction cites: with u_j = (-1)^j a_1j and
 * v_j = (-1)^j a_2j, eq. (1) with r = 3 is -sum_k (U_{k-1} v_k - V_{k-1} u_k),
 * U, V the prefix sums.  Runs of columns are combined in column order in
 * double-double arithmetic.  n may exceed RADIC_MAX_N (any n >= 1 whose 2 x n
 * input fits in memory).
 *   dA     device, 2 x n float64, row-major, leading dimension lda >= n.
 *   dOut   device, one radic_f64_result: value/hi/lo as in radic_det; abs_sum
 *          holds the O(n) upper bound sum_{j<k} (|u_j||v_k| + |u_k||v_j|) on
 *          sum |det(A_J)| (the exact sum of absolute minors needs every pair);
 *          n_subsets = n(n-1)/2, n_fallback = 0.
 *   dWork  device workspace of at least radic_workspace_bytes(RADIC_WS_DET, 2, n, 0).
 * Asynchronous.  n = 1 writes 0 (m > n).  Errors: EINVAL (null pointers, n < 1,
 * lda < n), EWORKSPACE, EDEVICE; non-finite entries give status ENONFINITE.
 */
int radic_det_2xn(const double *dA, int64_t n, int64_t lda, radic_f64_result *dOut, void *dWork,
                  size_t work_bytes, hipStream_t stream);

/*
 * radic_det_int_exact -- exact Radic determinant of one int32 matrix: the sum of
 * Definition 3, eq. (1) over all C(n, m) column sequences of Sections 3-5, as an
 * exact integer.  (The multi-modular evaluation is this library's, not the
 * paper's.)  Each minor is eliminated fraction-free modulo k 31-bit primes (k
 * chosen on the device from a Hadamard-type bound so that the product of the
 * primes exceeds twice the largest possible |result|), residues are summed per
 * prime and combined by Garner's mixed-radix CRT into a signed integer.
 *   dA         device, m x n int32, row-major, leading dimension lda (elements).
 *   dWork      device workspace of at least radic_workspace_bytes(RADIC_WS_INT, m, n, 0).
 *   hMag       host, capacity mag_capacity little-endian 32-bit limbs of |result|.
 *   hMagLen    host, number of significant limbs written (0 for a zero result);
 *              on RADIC_EOVERFLOW the number of limbs needed.
 *   hSign      host, -1, 0 or +1.
 * Synchronous: returns after the result is in host memory.  The last kernel
 * writes the result into a pinned host buffer of the library's (one per call in
 * flight, allocated on first need and kept until the process ends), so the
 * read-back is the wait for the stream and no copy command.
 * Errors: EINVAL, ENOTSUP, EOVERFLOW (C(n,m) too large, or mag_capacity too small),
 * EWORKSPACE, ENOMEM (the pinned buffer could not be allocated), EDEVICE.
 */
int radic_det_int_exact(const int32_t *dA, int m, int n, int64_t lda, uint32_t *hMag,
                        int mag_capacity, int *hMagLen, int *hSign, void *dWork, size_t work_bytes,
                        hipStream_t stream);

/*
 * radic_det_batched -- Radic determinants of `batch` matrices of mixed shapes and
 * types in one persistent kernel.  The rank spaces of all matrices are cut into
 * chunks; resident workgroups take chunks from one global atomic queue (the
 * granularity scheme of Section 5 applied to the whole batch); float matrices use
 * `prec`, int32 matrices use the exact multi-modular path.  Per-matrix partial
 * sums are reduced in a fixed order, so results do not depend on scheduling.
 *   dDesc  device, batch descriptors.   dF64 / dI32  device entry pools (either may
 *          be null if no descriptor uses it).   dOut  device, batch results.
 * Asynchronous and capturable into a HIP graph (no allocation, no host
 * synchronisation, no memset nodes).  Bad descriptors are reported per matrix.
 */
int radic_det_batched(const radic_matrix_desc *dDesc, int batch, const double *dF64,
                      const int32_t *dI32, int prec, radic_batch_result *dOut, void *dWork,
                      size_t work_bytes, hipStream_t stream);

/*
 * radic_det_batched_noalloc -- radic_det_batched for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results as
 * radic_det_batched, without dWork/work_bytes: the workspace is a static
 * device array of the library (36 MiB, held on every device the library runs
 * on until the process ends), sized for at most 4096 matrices.
 *   batch > 4096 -> RADIC_ENOTSUP (radic_last_error says why); nothing enqueued.
 * Allocates nothing (no hipMalloc, no allocating library call; the timing hook
 * of radic_profile_enable does not time it).  The first call on a device takes
 * the array's address with hipGetSymbolAddress and uploads the library's
 * tables, like any first call: make it outside stream capture.
 * All calls on one device share that device's array, and every kernel of a
 * call rewrites what it reads (no state is carried between calls), but calls
 * that may overlap on one device (other streams, other threads) race on it.
 * Asynchronous.
 */
int radic_det_batched_noalloc(const radic_matrix_desc *dDesc, int batch, const double *dF64,
                              const int32_t *dI32, int prec, radic_batch_result *dOut,
                              hipStream_t stream);

/*
 * Captured launch of radic_det_batched: records the same work into a HIP graph
 * once and replays it with a single launch.  *hGraph receives an opaque handle.
 * Arguments are bound at creation; replaying reuses them (contents of the
 * buffers may change between replays, shapes in dDesc may too as long as
 * `batch` is unchanged).  radic_graph_launch enqueues one replay on `stream`.
 */
int radic_batched_graph_create(const radic_matrix_desc *dDesc, int batch, const double *dF64,
                               const int32_t *dI32, int prec, radic_batch_result *dOut, void *dWork,
                               size_t work_bytes, void **hGraph);
int radic_graph_launch(void *hGraph, hipStream_t stream);
int radic_graph_destroy(void *hGraph);

/*
 * Launch-shape tuning (the granularity knob of Section 5).  radic_autotune times
 * candidate (subsets per lane, workgroup size) pairs for the given shape and
 * precision on the current device with HIP events, on a synthetic matrix of
 * that shape, and records the fastest for later calls.  Synchronous.  For the
 * prefix-shared kernels the subsets per lane set the block of minors that
 * shares its prefixes (64 x subsets per lane; candidates 16 ... 128 for the
 * float kernels, 8 ... 64 for the exact one) and the workgroup size is fixed.
 * kind: RADIC_WS_DET (prec applies), RADIC_WS_INT or RADIC_WS_BATCHED (m and n
 * ignored; prec 0 or 1 tunes the float classes on a synthetic float batch, prec 2
 * the exact classes on a synthetic int32 batch).  A shape tuned for n serves
 * every n of its bucket (each n up to 16, runs of 8 up to 64, then of 32), under
 * the enumeration (radic_set_enumeration) it was tuned with.
 * hBest (may be null) receives {subsets_per_lane, block_size}.
 * radic_tune_save/load persist the table as text; the table names the device
 * architecture and the library version (radic_version), and radic_tune_load
 * refuses (RADIC_EINVAL) a table of another version or, when a device is
 * current, of another architecture.
 */
int radic_autotune(int kind, int m, int n, int prec, int *hBest, hipStream_t stream);
/*
 * radic_autotune_batched -- launch-shape tuning of radic_det_batched on the
 * caller's own batch (Section 5's granularity for that workload): times each
 * candidate subsets-per-lane value (the chunks of both the float and the exact
 * classes hold at least 64 x that many ranks) with radic_det_batched on the given
 * arguments, and records the fastest for later batched calls of any batch in
 * this process (both the `prec` float classes and the exact classes).  Same
 * arguments as radic_det_batched (dOut and dWork are overwritten), plus hBest
 * (may be null) receiving {subsets_per_lane, block_size}.  Synchronous.
 * Errors: as radic_det_batched; EDEVICE if no candidate ran.
 */
int radic_autotune_batched(const radic_matrix_desc *dDesc, int batch, const double *dF64,
                           const int32_t *dI32, int prec, radic_batch_result *dOut, void *dWork,
                           size_t work_bytes, int *hBest, hipStream_t stream);
int radic_tune_save(const char *path);
int radic_tune_load(const char *path);
/* Force a launch shape (0 = tuned/default) for subsequent calls; for tests and sweeps. */
int radic_set_launch(int subsets_per_lane, int block_size);
/* FP32_BULK fallback threshold tau (default 2^-10): a minor is refactored in double
 * when prod_k min(1, |u_kk| / s_k) < tau', with u_kk the float pivots and s_k the
 * largest |entry| of the minor's k-th column in the row-scaled matrix (so it also
 * fires whenever a single pivot ratio is below tau').  A sum over N minors (a
 * radic_det or radic_det_range call, or one batch matrix) uses
 * tau' = tau * min(1, (8192 / N)^(1/4)): the errors of the minors kept in float
 * add up with independent signs, so their share of sum |det| falls as N grows.
 * radic_det_subsets, whose terms are not summed, uses tau' = tau.  tau = 0
 * disables the fallback, tau = +inf refactors every minor. */
int radic_set_fallback_tau(double tau);
/* The threshold tau' a sum over `minors` minors uses under the current setting. */
double radic_fallback_tau_for(uint64_t minors);

/*
 * Which enumeration radic_det / radic_det_range use for float matrices.
 *  RADIC_ENUM_AUTO            prefix-shared where supported (default).
 *  RADIC_ENUM_PER_MINOR       every minor unranked/advanced and factored on its
 *                             own by one lane (the scheme of Sections 4-6).
 *  RADIC_ENUM_PREFIX_SHARED   the minors sharing their first m-2 columns (which
 *                             the dictionary order of Section 3 makes
 *                             consecutive) share the first m-2 steps of their
 *                             LU with partial pivoting, whose pivots and
 *                             multipliers depend on those columns only; each
 *                             minor then costs its last two elimination steps.
 *                             Used for 3 <= m <= 12; other shapes fall back
 *                             to per-minor.
 *  RADIC_ENUM_GROUP_SHARED    the minors sharing their first m-3 columns share
 *                             those m-3 steps; each minor then costs the
 *                             determinant of its last 3 x 3 block, a dot
 *                             product with a cross product formed once per
 *                             pair of its last three columns.  Used for
 *                             4 <= m <= 12; m = 3 falls back to prefix-shared.
 * RADIC_ENUM_AUTO takes prefix-shared where supported.  All give every minor's
 * determinant (the terms of eq. (1)) individually; they differ in rounding only.
 * radic_det_subsets always uses per-minor.  The same switch applies to
 * radic_det_int_exact (any shared mode: prefix-shared for 3 <= m <= 10: the
 * minors of a prefix share its fraction-free elimination steps modulo p; the
 * result is the same exact integer either way).
 * Returns RADIC_EINVAL for an unknown mode.
 */
#define RADIC_ENUM_AUTO 0
#define RADIC_ENUM_PER_MINOR 1
#define RADIC_ENUM_PREFIX_SHARED 2
#define RADIC_ENUM_GROUP_SHARED 3
int radic_set_enumeration(int mode);

/*
 * Timing hook for benchmarks: while enabled, the library times every launch of
 * its main enumeration kernels with HIP events on the launch stream.  For the
 * single-matrix float and exact calls the events are bound to the kernel's own
 * dispatch (hipExtLaunchKernel; created without the system-scope fence); for
 * the two-row, batched and graph calls they are recorded around the launches.
 * A timed launch still delays the stream by a few microseconds.
 * radic_profile_read waits for them and returns the summed duration in ms and
 * the number of launches since the last read, then clears.
 */
int radic_profile_enable(int on);
int radic_profile_read(double *hTotalMs, int *hLaunches);
/* Same, but returns each launch's duration (ms) in launch order: up to capacity
 * values in hMs, *hCount = launches recorded (may exceed capacity; extra are
 * dropped).  Clears like radic_profile_read. */
int radic_profile_read_launches(double *hMs, int capacity, int *hCount);

/* Prime set of the exact path: by default the 24 largest primes below 2^31,
 * in decreasing order.  Tests may substitute other odd primes (e.g. tiny ones,
 * so that zero pivots modulo p occur): hPrimes[0..count-1], each prime,
 * 3 <= p < 2^31, distinct, count <= RADIC_MAX_PRIMES; count = 0 restores the
 * default.  Applies to later calls on every device.  EINVAL on a bad list. */
int radic_set_prime_set(const uint32_t *hPrimes, int count);

/* Host-side combinatorics used by the launchers, exported for testing:
 * binomial with overflow detection (returns EOVERFLOW), dictionary-order
 * unranking (1-based columns into hCols), and the i-th prime used by the exact path. */
int radic_host_binomial(int a, int b, uint64_t *hOut);
int radic_host_unrank(int m, int n, uint64_t q, int *hCols);
int radic_host_prime(int i, uint32_t *hPrime);
/* How radic_det_batched cuts the rank space of one matrix (dtype 0 float64,
 * 1 int32) into chunks, the unit a wave takes from its class queue (the
 * granularity scheme of Section 5).  Float matrices with m >= 7 and int32
 * matrices with 5 <= m <= 6 are taken in the two-sided blocks of radic_det
 * (radic_host_split_blocks with 64 * subsets_per_lane minors per block):
 * *hChunk blocks per chunk.  The others are cut into rank windows: *hChunk
 * ranks per chunk (a multiple of 64, at least 64 * subsets_per_lane).
 * *hChunks chunks; float matrices have at most 256 (one partial-sum slot
 * each), int32 matrices at most 2^16.  EINVAL for bad arguments, EOVERFLOW
 * when C(n, m) >= 2^63. */
int radic_host_batch_chunking(int dtype, int m, int n, int subsets_per_lane, uint64_t *hChunk,
                              uint64_t *hChunks);
/* The blocks radic_det and radic_det_int_exact take a whole rank space in
 * (3 <= m <= RADIC_MAX_M), computed on the host by the kernels' own code.  Each
 * minor j_0 < ... < j_{m-1} (0-based) is grouped either with the minors that
 * share its first m-2 columns (side 0, n-1-j_{m-3} columns after them) or with
 * those that share its last m-2 (side 1, j_2 columns before them), whichever
 * leaves more (side 0 on a tie); side 1 is side 0 of the column-reversed matrix
 * (column c read as n-1-c).  A side's prefixes c_0 < ... < c_{m-3} (0-based, in
 * that side's coordinates) are grouped by their last column v = c_{m-3},
 * m-3 <= v <= n-3.
 *   radic_host_split_count: *hCount prefixes of side `side` with last column v.
 *   radic_host_split_prefix: the j-th of them (j < that count) into
 *     hCols[0..m-3] (m-2 entries).
 *   radic_host_split_blocks: *hBlocks blocks of about minors_per_block minors
 *     (the launchers use 64 * subsets_per_lane).
 * EINVAL for bad arguments, EOVERFLOW when C(n, m) >= 2^63. */
int radic_host_split_count(int m, int n, int side, int v, uint64_t *hCount);
int radic_host_split_prefix(int m, int n, int side, int v, uint64_t j, int *hCols);
int radic_host_split_blocks(int m, int n, int minors_per_block, uint64_t *hBlocks);

#ifdef __cplusplus
}
#endif

#endif /* RADIC_H */
