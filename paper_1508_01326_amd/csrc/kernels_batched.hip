// Batched Radic determinants: many matrices of mixed shape and type in
// persistent kernels fed by global work queues.
//
// The rank space [0, C(n_b, m_b)) of every matrix b is cut into chunks (the
// granularity scheme of Section 5 applied to the whole batch).  A setup kernel
// validates the descriptors, sizes the chunks and sorts the matrices into
// classes by (type, m); a scan per class turns the per-matrix chunk counts into
// queue prefixes, and one persistent kernel per class (compiled for that m, so
// its register and LDS footprint is that of its own minors) takes chunk indices
// from the class's global atomic counter until the queue is empty.  A wave that takes a
// chunk of a matrix other than the one it holds stages that matrix in its own
// LDS region, then runs the same per-lane enumeration and LU (or modular
// elimination) as the single-matrix kernels.  Float chunks write their partial
// sums to per-(matrix, chunk) slots, which a final kernel reduces in chunk
// order, so float results do not depend on the order in which waves took chunks;
// exact chunks add residues into per-(matrix, prime) 64-bit sums, which is exact
// and order independent.  No kernel allocates or clears memory through the
// runtime, so the whole sequence can be captured in a HIP graph.
#include <type_traits>

#include "lu_float.h"
#include "modp.h"
#include "shared_int.h"
#include "shared_int3.h"
#include "shared_round.h"

namespace radic {

constexpr int kBatchMaxN = 64;           // widest matrix a wave stages in LDS
static_assert(kBatchMaxN <= kWave, "the setup kernel reads one column per lane");
constexpr int kBatchWaves = 4;           // waves per workgroup of the persistent kernels

struct BatchMeta {
    unsigned long long total;    // C(n, m)
    unsigned long long chunk;    // ranks per chunk (a multiple of 64), or blocks per chunk (blocks > 0)
    unsigned long long nchunks;
    unsigned long long blocks;   // two-sided blocks of the matrix (batch_uses_blocks), else 0
    int status;                  // per-matrix radic status
    int kind;                    // 0 float, 1 exact, -1 no work (error or m > n)
    int n_primes;
    int scale_exp;               // FP32_BULK: sum of the row exponents
    int all_double;              // FP32_BULK with fewer than kF32MinMinors minors: every minor in double
};

// Work classes: (kind, m), kind 0 float / 1 exact, m = 1..RADIC_MAX_M.  Each
// class has its own queue and its own persistent kernel, compiled for that m
// only, so a kernel's register allocation is that of its own minor size.
constexpr int kClasses = 2 * RADIC_MAX_M;
__host__ __device__ inline int class_of(int kind, int m) { return kind * RADIC_MAX_M + (m - 1); }

// Queue counters are 64-bit: a class's chunk total is a sum over its matrices
// of up to 2^16 chunks each (see k_batch_setup), so it can pass 2^32, and a
// 32-bit counter would wrap and never reach it.
struct BatchHeader {
    unsigned long long chunks[kClasses];   // queue length per class
    unsigned long long queue[kClasses];    // next chunk index per class
};

static_assert(sizeof(BatchHeader) == 16 * kClasses, "batch header layout");

// Exact chunks hold at least 64 * spl_int ranks and are made larger for big
// rank spaces, so that no matrix has more than kExactChunksMax of them.
constexpr unsigned long long kExactChunksMax = 1ull << 16;

// Chunk size (a multiple of 64 ranks, at least 64 * spl) and chunk count of one
// matrix with `total` ranks: float chunks are at most kBatchChunksPerMatrix per
// matrix (each has a partial-sum slot), exact chunks at most kExactChunksMax.
__host__ __device__ inline void batch_chunking(int kind, unsigned long long total, int spl,
                                               unsigned long long& chunk, unsigned long long& nchunks) {
    const unsigned long long most = kind == 0 ? (unsigned long long)kBatchChunksPerMatrix : kExactChunksMax;
    const unsigned long long minc = 64ull * (unsigned long long)(spl > 0 ? spl : 1);
    unsigned long long c = (total + most - 1) / most;
    c = (c + 63) & ~63ull;
    chunk = c > minc ? c : minc;
    nchunks = (total + chunk - 1) / chunk;
}

struct BatchJob {
    const radic_matrix_desc* desc;
    int batch;
    const double* f64;
    const int* i32;
    int prec;
    double tau;
    int spl_float;
    int spl_int;
    int prime_count;
    radic_batch_result* out;
    BatchHeader* header;
    BatchMeta* meta;
    unsigned long long* prefix;         // [kClasses][batch + 1]
    Partial* partials;                  // [batch][kBatchChunksPerMatrix]
    unsigned long long* residues;       // [batch][RADIC_MAX_PRIMES]
};

// Workspace layout (offsets in bytes, all 256-byte aligned)
__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
__host__ __device__ inline size_t off_meta() { return align256(sizeof(BatchHeader)); }
__host__ __device__ inline size_t off_prefix(int batch) { return off_meta() + align256(sizeof(BatchMeta) * batch); }
__host__ __device__ inline size_t off_partials(int batch) {
    return off_prefix(batch) + align256(8 * (size_t)kClasses * (batch + 1));
}
__host__ __device__ inline size_t off_residues(int batch) {
    return off_partials(batch) + align256(sizeof(Partial) * (size_t)kBatchChunksPerMatrix * batch);
}
__host__ __device__ inline size_t batch_ws_bytes(int batch) {
    return off_residues(batch) + align256(8 * (size_t)RADIC_MAX_PRIMES * batch);
}

// Two-sided blocks of about K minors of an m x n matrix (the single-matrix
// kernels' split_block order), counted by the wave: lanes take (v, side) pairs.
template <int P>
__device__ unsigned long long split_blocks_wave_p(int n, unsigned K, int lane) {
    unsigned long long nb = 0;
    for (int v0 = P - 1; v0 <= n - 3; v0 += kWave / 2) {
        const int v = v0 + lane / 2;
        if (v <= n - 3) nb += split_blocks_at<P>(n, lane & 1, v, K, g_binom, kBinomCols);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) nb += __shfl_xor(nb, o, kWave);
    return nb;
}

__device__ unsigned long long split_blocks_wave(int m, int n, unsigned K, int lane) {
    switch (m - 2) {
#define RADIC_CASE(PP) \
    case PP: return split_blocks_wave_p<PP>(n, K, lane);
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10)
#undef RADIC_CASE
        default: return 0ull;
    }
}

// Chunking of one matrix: runs of two-sided blocks (batch_uses_blocks), else
// rank windows (batch_chunking).
__device__ void chunk_matrix(int kind, int m, int n, unsigned long long total, int spl, int lane, BatchMeta& mt) {
    if (batch_uses_blocks(kind, m)) {
        const unsigned K = 64u * (unsigned)(spl > 0 ? spl : 1);
        mt.blocks = split_blocks_wave(m, n, K, lane);
        batch_block_chunking(mt.blocks, kind == 0 ? (unsigned long long)kBatchChunksPerMatrix : kExactChunksMax,
                             mt.chunk, mt.nchunks);
    } else {
        mt.blocks = 0;
        batch_chunking(kind, total, spl, mt.chunk, mt.nchunks);
    }
}

// ---------------------------------------------------------------- setup
// One wave per matrix: its lanes read the matrix together (lane j column j, for
// j < n), and the wave reduces what the matrix's meta needs.
__global__ __launch_bounds__(256) void k_batch_setup(BatchJob J) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int b = blockIdx.x * (blockDim.x / kWave) + wave;
    if (b >= J.batch) return;
    const radic_matrix_desc d = J.desc[b];
    BatchMeta mt{};
    mt.kind = -1;
    mt.status = RADIC_OK;
    if (lane < RADIC_MAX_PRIMES) J.residues[(size_t)b * RADIC_MAX_PRIMES + lane] = 0ull;
    const bool bad_dtype = d.dtype != 0 && d.dtype != 1;
    const bool no_pool = (d.dtype == 0 && !J.f64) || (d.dtype == 1 && !J.i32);
    if (d.m < 1 || d.n < 1 || d.lda < d.n || d.offset < 0 || bad_dtype || no_pool) {
        mt.status = RADIC_EINVAL;
    } else if (d.m > d.n) {
        mt.status = RADIC_OK;   // Definition 3: zero
    } else if (d.m > RADIC_MAX_M || d.n > kBatchMaxN) {
        mt.status = RADIC_ENOTSUP;
    } else {
        const unsigned long long total = g_binom[d.n * kBinomCols + d.m];
        const bool col = lane < d.n;   // kBatchMaxN <= 64: one column per lane
        if (total >= (1ull << 63)) {
            mt.status = RADIC_EOVERFLOW;
        } else if (d.dtype == 0) {
            mt.kind = 0;
            mt.total = total;
            chunk_matrix(0, d.m, d.n, total, J.spl_float, lane, mt);
            const double* A = J.f64 + d.offset;
            int se = 0;
            bool bad = false;
            for (int i = 0; i < d.m; ++i) {
                const double v = col ? A[(long long)i * d.lda + lane] : 0.0;
                bad |= !isfinite(v);
                double mx = fabs(v);
#pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
                int e = 0;
                if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
                se += e;
            }
            mt.scale_exp = J.prec == RADIC_FP32_BULK ? se : 0;
            mt.all_double = J.prec == RADIC_FP32_BULK && total < kF32MinMinors;
            if (__ballot(bad)) {
                mt.status = RADIC_ENONFINITE;
                mt.kind = -1;
            }
        } else {
            // exact: primes for the bound e_m(column norms) (Hadamard per minor)
            const int* A = J.i32 + d.offset;
            double s = 0.0;
            for (int i = 0; i < d.m; ++i) {
                const double a = col ? (double)A[(long long)i * d.lda + lane] : 0.0;
                s = __builtin_fma(a, a, s);
            }
            const double xl = sqrt(s) * (1.0 + 1e-12);
            double e[RADIC_MAX_M + 1];
            e[0] = 1.0;
#pragma unroll
            for (int k = 1; k <= RADIC_MAX_M; ++k) e[k] = 0.0;
            for (int j = 0; j < d.n; ++j) {   // every lane the same recurrence, column j's norm from lane j
                const double x = __shfl(xl, j, kWave);
#pragma unroll
                for (int k = RADIC_MAX_M; k >= 1; --k)
                    if (k <= d.m) e[k] = __builtin_fma(x, e[k - 1], e[k]);
            }
            double em = 0.0;
#pragma unroll
            for (int k = 0; k <= RADIC_MAX_M; ++k) em = k == d.m ? e[k] : em;
            const double need = log2(em * (1.0 + 1e-9) + 1.0) + 1.0 + 1e-6;
            double have = 0.0;
            int k = 0;
            while (k < J.prime_count && have <= need) have += log2(g_prime[k++]);
            if (have <= need || k > RADIC_MAX_PRIMES) {
                mt.status = RADIC_EOVERFLOW;
            } else {
                mt.kind = 1;
                mt.total = total;
                mt.n_primes = k;
                chunk_matrix(1, d.m, d.n, total, J.spl_int, lane, mt);
            }
        }
    }
    if (lane == 0) J.meta[b] = mt;
}

// One workgroup per class: prefix sums of the class's chunk counts in matrix
// order, and the class queue reset.
__global__ __launch_bounds__(1024) void k_batch_scan(BatchJob J) {
    __shared__ unsigned long long sf[1024];
    const int cls = blockIdx.x;
    unsigned long long* prefix = J.prefix + (size_t)cls * (J.batch + 1);
    const int per = (J.batch + blockDim.x - 1) / blockDim.x;
    const int b0 = threadIdx.x * per;
    auto count = [&](int b) -> unsigned long long {
        const BatchMeta& mt = J.meta[b];
        return (mt.kind >= 0 && class_of(mt.kind, J.desc[b].m) == cls) ? mt.nchunks : 0ull;
    };
    unsigned long long f = 0;
    for (int b = b0; b < b0 + per && b < J.batch; ++b) f += count(b);
    sf[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {   // inclusive Hillis-Steele scan
        const unsigned long long a = threadIdx.x >= (unsigned)off ? sf[threadIdx.x - off] : 0ull;
        __syncthreads();
        sf[threadIdx.x] += a;
        __syncthreads();
    }
    f = threadIdx.x ? sf[threadIdx.x - 1] : 0ull;
    for (int b = b0; b < b0 + per && b < J.batch; ++b) {
        prefix[b] = f;
        f += count(b);
    }
    if (threadIdx.x == blockDim.x - 1) {
        prefix[J.batch] = sf[blockDim.x - 1];
        J.header->chunks[cls] = sf[blockDim.x - 1];
        J.header->queue[cls] = 0ull;
    }
}

// ---------------------------------------------------------------- queue helpers
__device__ __forceinline__ unsigned long long take_chunk(unsigned long long* queue, int lane) {
    unsigned long long g = 0;
    if (lane == 0) g = atomicAdd(queue, 1ull);
    return __shfl(g, 0, kWave);
}

// matrix b with prefix[b] <= g < prefix[b + 1] (prefix nondecreasing, prefix[0] = 0)
__device__ __forceinline__ int find_matrix(const unsigned long long* prefix, int batch, unsigned long long g) {
    int lo = 0, hi = batch;   // invariant: prefix[lo] <= g < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- float chunks
// Per-wave LDS of a float class: the double copy of the staged matrix, and for
// FP32_BULK the float copy (with the column-scale slot), the queue of minors to
// refactor in double and the row exponents.
template <int M, bool F32> struct FloatWaveLds {
    double cd[kBatchMaxN * Layout<M>::st64];
    float cf[F32 ? kBatchMaxN * Layout<M>::st32 : 1];
    unsigned queue[F32 ? 4 * kFallbackCap : 1];
    int rowexp[M];
};

template <int M, bool F32>
__device__ void stage_float(const BatchJob& J, const radic_matrix_desc& d, FloatWaveLds<M, F32>& L, int lane) {
    constexpr int ST64 = Layout<M>::st64, ST32 = Layout<M>::st32;
    const double* A = J.f64 + d.offset;
    const int n = d.n;
    if (F32 && lane < M) {   // exponent of row `lane`'s maximum, max |a_ij| = f 2^e with f in [0.5, 1)
        double mx = 0.0;
        for (int j = 0; j < n; ++j) mx = fmax(mx, fabs(A[(long long)lane * d.lda + j]));
        int e_row = 0;
        if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e_row);
        L.rowexp[lane] = e_row;
    }
    wave_lds_sync();
    for (int e = lane; e < M * n; e += kWave) {
        const int i = e / n, j = e - i * n;
        double v = A[(long long)i * d.lda + j];
        if (F32) v = ldexp(v, -L.rowexp[i]);
        L.cd[j * ST64 + i] = v;
        if (F32) L.cf[j * ST32 + i] = (float)v;
    }
    wave_lds_sync();
    if (F32) {
        for (int j = lane; j < n; j += kWave) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) s = fmaxf(s, fabsf(L.cf[j * ST32 + i]));
            L.cf[j * ST32 + M] = s > 0.f ? 1.0f / s : 0.f;
        }
        wave_lds_sync();
    }
}

template <int M, bool F32>
__device__ void float_chunk(const BatchJob& J, const radic_matrix_desc& d, const BatchMeta& mt,
                            unsigned long long c, FloatWaveLds<M, F32>& L, int lane, bool restage, Partial& out) {
    using T = typename std::conditional<F32, float, double>::type;
    constexpr int ST64 = Layout<M>::st64, ST32 = Layout<M>::st32;
    if (restage) stage_float<M, F32>(J, d, L, lane);
    const int n = d.n;
    const T* colbase = F32 ? reinterpret_cast<const T*>(L.cf) : reinterpret_cast<const T*>(L.cd);
    const int colstride = F32 ? ST32 : ST64;
    const T tau = mt.all_double ? (T)__builtin_inf() : (T)effective_tau(J.tau, mt.total);
    const unsigned long long sub = mt.chunk / kWave;          // ranks per lane
    const unsigned long long q0 = c * mt.chunk + (unsigned long long)lane * sub;
    const int cnt = q0 < mt.total ? (int)((mt.total - q0) < sub ? (mt.total - q0) : sub) : 0;
    int col[M];
    unrank_strided<M>(q0 < mt.total ? q0 : mt.total - 1, n, g_binom, kBinomCols, col);
    unsigned long long perm = 0;   // natural row order (no wave copy in the batched kernel)
    int perm_odd = 0;
#pragma unroll
    for (int r = 0; r < M; ++r) perm |= (unsigned long long)r << (4 * r);
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    int qcount = 0;
    for (unsigned long long s = 0; s < sub; ++s) {
        const bool valid = s < (unsigned long long)cnt;
        T a[M][M];
        gather<M, T>(a, colbase, colstride, col);
        T sc[M];
        if (F32) {
#pragma unroll
            for (int j = 0; j < M; ++j) sc[j] = colbase[col[j] * colstride + M];
        }
        bool neg = radic_sign_odd<M>(col);
        bool flag = false;
        const T det = lu_det<M, T, F32>(a, neg, flag, sc, tau, perm, perm_odd);
        perm_odd = 0;   // rows are always gathered in their natural order here
#pragma unroll
        for (int r = 0; r < M; ++r) perm = (perm & ~(15ull << (4 * r))) | ((unsigned long long)r << (4 * r));
        flag = flag && valid;
        if (valid && !flag) {
            const double dd = (double)det;
            const double term = neg ? -dd : dd;
            double sum, err;
            two_sum(hi, term, sum, err);
            hi = sum;
            lo += err;
            ab += fabs(dd);
        }
        if (F32) {
            const unsigned long long fm = __ballot(flag);
            if (fm) {
                if (flag) {
                    const int pos = qcount + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                    unsigned w[4];
                    pack_cols<M>(col, w);
                    L.queue[4 * pos + 0] = w[0];
                    L.queue[4 * pos + 1] = w[1];
                    L.queue[4 * pos + 2] = w[2];
                    L.queue[4 * pos + 3] = w[3];
                    nfb += 1;
                }
                qcount += __popcll(fm);
                if (qcount > kFallbackCap - kWave) {
                    wave_lds_sync();
                    refactor_queue_f64<M>(L.cd, L.queue, qcount, lane, hi, lo, ab);
                    qcount = 0;
                }
            }
        }
        successor<M>(col, n);
    }
    if (F32 && qcount > 0) {
        wave_lds_sync();
        refactor_queue_f64<M>(L.cd, L.queue, qcount, lane, hi, lo, ab);
    }
    wave_reduce_partial(hi, lo, ab, nfb);
    out = Partial{hi, lo, ab, nfb};
}

// ---------------------------------------------------------------- float chunks, prefix-shared (m >= 3)
// From m = 3 a float chunk runs the prefix-shared round of the single-matrix
// kernels: the minors of a prefix (first m-2 columns of its side) share its
// elimination steps and end with a 2 x 2 determinant.  From m = 7 the chunk is
// a run of the matrix's two-sided blocks (as the single-matrix kernels take a
// whole rank space, see split_shape), below a rank window in dictionary order.  FP32-bulk
// queues its flagged minors in the wave's LDS and refactors them in double by
// lane groups (between rounds once the queue is half full, and at the end of
// the chunk); a round whose flagged minors would not fit is done again in
// double.  Matrices with fewer than kF32MinMinors minors run the double round.
constexpr int kBatchSharedCap = 256;   // projected-column slots per wave
constexpr int kBatchDefer = 128;       // FP32-bulk queue entries per wave
constexpr int kBatchBS = RADIC_MAX_M + 1;   // stride of the float kernels' binomial table (C(x, y), y <= m)

template <int M, bool F32> struct FloatSharedLds {
    double cd[kBatchMaxN * SharedLayout<M>::s64];   // (row-scaled for FP32-bulk) double copy
    float cf[F32 ? kBatchMaxN * SharedLayout<M>::s32 : 1];   // float copy, reciprocal column scale in slot m
    alignas(16) unsigned char rec[kHdrBytes + kScanBytes + (F32 ? kF32Extra : 0)];
    uint4 tv[kBatchSharedCap];
    uint4 queue[F32 ? kBatchDefer : 1];
    int rowexp[M];
};

// Stage matrix d into the wave's copies, with the layout and scaling of the
// single-matrix prefix-shared kernels: FP32-bulk rows scaled by 2^-e_i (e_i the
// exponent of the row maximum), the float copy, and its reciprocal column
// scales.
template <int M, bool F32>
__device__ void stage_float_shared(const BatchJob& J, const radic_matrix_desc& d, FloatSharedLds<M, F32>& L,
                                   int lane) {
    constexpr int S64 = SharedLayout<M>::s64, S32 = SharedLayout<M>::s32;
    const double* A = J.f64 + d.offset;
    const int n = d.n;
    wave_lds_sync();
    if (F32 && lane < M) {
        double mx = 0.0;
        for (int j = 0; j < n; ++j) mx = fmax(mx, fabs(A[(long long)lane * d.lda + j]));
        int e_row = 0;
        if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e_row);
        L.rowexp[lane] = e_row;
    }
    wave_lds_sync();
    for (int e = lane; e < M * n; e += kWave) {
        const int i = e / n, j = e - i * n;
        double v = A[(long long)i * d.lda + j];
        if (F32) v = ldexp(v, -L.rowexp[i]);
        L.cd[j * S64 + i] = v;
        if (F32) L.cf[j * S32 + i] = (float)v;
    }
    wave_lds_sync();
    if (F32) {
        for (int j = lane; j < n; j += kWave) {
            float sc = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) sc = fmaxf(sc, fabsf(L.cf[j * S32 + i]));
            L.cf[j * S32 + M] = sc > 0.f ? 1.0f / sc : 0.f;
        }
        wave_lds_sync();
    }
}

template <int M, bool F32>
__device__ void float_chunk_shared(const BatchJob& J, const radic_matrix_desc& d, const BatchMeta& mt,
                                   unsigned long long c, FloatSharedLds<M, F32>& L, const unsigned long long* bt,
                                   int lane, bool restage, Partial& out) {
    constexpr int S64 = SharedLayout<M>::s64;
    if (restage) stage_float_shared<M, F32>(J, d, L, lane);
    const int n = d.n;
    // the chunk is the run [b0, b1) of the matrix's two-sided blocks, each
    // taken as by the single-matrix kernel (its whole rank space, no clipping),
    // or (mt.blocks == 0) the rank window [R0, R1) in dictionary order, the
    // round clipping its minors to it
    // (a function of the class, so each class kernel holds one of the two)
    constexpr bool blocks = batch_uses_blocks(0, M);
    const unsigned K = 64u * (unsigned)(J.spl_float > 0 ? J.spl_float : 1);
    const unsigned long long b0 = c * mt.chunk;
    const unsigned long long b1 = blocks ? (b0 + mt.chunk < mt.blocks ? b0 + mt.chunk : mt.blocks) : b0 + 1;
    const unsigned long long R1 = b0 + mt.chunk < mt.total ? b0 + mt.chunk : mt.total;
    FloatJob FJ{};
    FJ.n = n;
    FJ.q_begin = blocks ? 0ull : b0;
    FJ.count = blocks ? mt.total : R1 - b0;
    FJ.total = mt.total;
    FJ.tau = effective_tau(J.tau, mt.total);
    FJ.colex = blocks ? 1 : 0;
    FJ.colex_pairs = K;
    FJ.n_prefix = g_binom[(n - 2) * kBinomCols + (M - 2)];
    FJ.cap = kBatchSharedCap;
    FJ.defer_cap = kBatchDefer;
    FJ.fb_entries = reinterpret_cast<unsigned*>(L.queue);   // the wave's queue (segment 0)
    RoundLds W;
    W.hdr = reinterpret_cast<PairHdr*>(L.rec);
    W.incl = reinterpret_cast<unsigned*>(L.rec + kHdrBytes);
    W.cincl = W.incl + kPrefixBlock;
    W.ratios = reinterpret_cast<float*>(L.rec + kHdrBytes + kScanBytes);
    W.wcols = reinterpret_cast<uint4*>(L.rec + kHdrBytes + kScanBytes + kPrefixBlock * 4);
    W.tv = reinterpret_cast<unsigned char*>(L.tv);
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    int gcount = 0;
    unsigned minors;
    const bool f32 = F32 && !mt.all_double;
    for (unsigned long long blk = b0; blk < b1; ++blk) {
        unsigned long long next, pi1;
        int side = 0, vlast = 0;
        if constexpr (blocks) {
            int cnt;
            split_block<M - 2>(blk, n, bt, kBatchBS, K, lane, side, vlast, next, cnt);
            pi1 = next + (unsigned long long)cnt;
        } else {
            // the prefixes holding the window's first and last ranks
            next = prefix_of_rank<M>(b0, n, bt, kBatchBS);
            pi1 = prefix_of_rank<M>(R1 - 1, n, bt, kBatchBS) + 1;
        }
        if constexpr (F32) {
            if (f32) {
                while (next < pi1) {
                    const double shi = hi, slo = lo, sab = ab;
                    const unsigned long long snfb = nfb;
                    const int sg = gcount;
                    const int ntake = shared_round<M, true, kBatchBS>(FJ, bt, L.cf, next, pi1, side, vlast, W, lane,
                                                                      0ull, hi, lo, ab, nfb, gcount, minors);
                    if (gcount > FJ.defer_cap) {
                        // the round's flagged minors do not fit the queue: the
                        // round again, in double (every one of its minors counted
                        // as refactored)
                        hi = shi;
                        lo = slo;
                        ab = sab;
                        nfb = snfb;
                        gcount = sg;
                        wave_lds_sync();
                        (void)shared_round<M, false, kBatchBS>(FJ, bt, L.cd, next, pi1, side, vlast, W, lane, 0ull, hi,
                                                               lo, ab, nfb, gcount, minors);
                        if (lane == 0) nfb += minors;
                    }
                    next += (unsigned long long)ntake;
                    wave_lds_sync();
                    relieve_segment<M, S64>(FJ, L.cd, 0ull, gcount, lane, hi, lo, ab);
                }
                continue;
            }
        }
        // double rounds (FP64, or FP32-bulk under kF32MinMinors minors: every
        // minor counted as done in double)
        while (next < pi1) {
            const int ntake = shared_round<M, false, kBatchBS>(FJ, bt, L.cd, next, pi1, side, vlast, W, lane, 0ull, hi,
                                                               lo, ab, nfb, gcount, minors);
            if (F32 && lane == 0) nfb += minors;
            next += (unsigned long long)ntake;
            wave_lds_sync();
        }
    }
    if constexpr (F32) {
        if (gcount > 0) {
            __threadfence_block();   // the entries other lanes of the wave stored
            refactor_queue_groups<M, S64>(L.cd, L.queue, gcount, lane, hi, lo, ab);
        }
    }
    wave_reduce_partial(hi, lo, ab, nfb);
    out = Partial{hi, lo, ab, nfb};
}

template <bool F32, int M>
__global__ __launch_bounds__(kBatchWaves * kWave) void k_batch_float(BatchJob J) {
    constexpr bool SHARED = M >= 3;
    using Lds = typename std::conditional<SHARED, FloatSharedLds<M, F32>, FloatWaveLds<M, F32>>::type;
    __shared__ Lds lds[kBatchWaves];
    // binomial table C(x, y), x < kBatchMaxN, y <= RADIC_MAX_M, for the prefix rounds
    __shared__ unsigned long long bt[SHARED ? kBatchMaxN * kBatchBS : 1];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    constexpr int cls = M - 1;   // class_of(0, M)
    const unsigned long long total = J.header->chunks[cls];
    // waves numbered past the class's chunk count would find the queue drained:
    // a workgroup of only such waves leaves at once, the others after the barrier
    if ((unsigned long long)blockIdx.x * kBatchWaves >= total) return;
    if constexpr (SHARED) {
        for (int e = threadIdx.x; e < kBatchMaxN * kBatchBS; e += blockDim.x) {
            const int x = e / kBatchBS, y = e - x * kBatchBS;
            bt[e] = g_binom[x * kBinomCols + y];
        }
        __syncthreads();
    }
    if ((unsigned long long)blockIdx.x * kBatchWaves + wave >= total) return;
    Lds& L = lds[wave];
    const unsigned long long* prefix = J.prefix + (size_t)cls * (J.batch + 1);
    int staged = -1;
    for (;;) {
        const unsigned long long g = take_chunk(&J.header->queue[cls], lane);
        if (g >= total) break;
        const int b = find_matrix(prefix, J.batch, g);
        const unsigned long long c = g - prefix[b];
        const radic_matrix_desc d = J.desc[b];
        const BatchMeta mt = J.meta[b];
        const bool restage = b != staged;
        staged = b;
        Partial p{};
        if constexpr (SHARED) float_chunk_shared<M, F32>(J, d, mt, c, L, bt, lane, restage, p);
        else float_chunk<M, F32>(J, d, mt, c, L, lane, restage, p);
        if (lane == 0) J.partials[(size_t)b * kBatchChunksPerMatrix + c] = p;
    }
}

// ---------------------------------------------------------------- exact chunks
// Exact chunks share elimination steps: the minors of a prefix (first m-2
// columns; rank windows for m = 3, 4, two-sided blocks for 5 <= m <
// kGroupExactMin), of a group (first m-3 columns, rank windows) from there to
// m = 10 (groups hold C(r, 3) minors against C(r, 2) per prefix).
// projected-column slots (16 bytes) per wave: enough for 64 prefixes or groups
// of the narrow matrices a batch holds
template <int M> constexpr int batch_cap() { return M >= kGroupExactMin ? 512 : 256; }

template <int M> struct IntWaveLds {
    double cr[kBatchMaxN * IntLayout<M>::st];
    IntSlot slot[M >= 3 && M <= 10 ? kPrefixBlock : 1];
    unsigned incl[M >= 3 && M <= 10 ? 2 * kPrefixBlock : 1];   // minor and column scans
    double2 tv[M >= 3 && M <= 10 ? batch_cap<M>() : 1];
};

template <int M>
__device__ void int_chunk(const BatchJob& J, const radic_matrix_desc& d, const BatchMeta& mt, unsigned long long c,
                          int b, IntWaveLds<M>& L, const unsigned long long* bt, int lane, bool restage) {
    constexpr int ST = IntLayout<M>::st;
    const int n = d.n;
    (void)restage;   // residues are restaged per prime
    const int* A = J.i32 + d.offset;
    if constexpr (M >= kGroupExactMin && M <= 10) {
        // group-shared: the chunk's ranks [R0, R1), groups from the one holding R0
        const unsigned long long R0 = c * mt.chunk;
        const unsigned long long R1 = R0 + mt.chunk < mt.total ? R0 + mt.chunk : mt.total;
        PrefixSpace sp;
        sp.n = n;
        sp.total = mt.total;
        sp.n_prefix = g_binom[(n - 3) * kBinomCols + (M - 3)];
        const unsigned long long first = group_of_rank<M>(R0, n, bt, RADIC_MAX_M);
        const unsigned long long rbase = first_completion_rank<M, PrefixSpace, 3>(first, sp, bt, RADIC_MAX_M);
        for (int pi = 0; pi < mt.n_primes; ++pi) {
            const double p = g_prime[pi], pinv = g_prime_inv[pi];
            wave_lds_sync();
            for (int e = lane; e < M * n; e += kWave) {
                const int i = e / n, j = e - i * n;
                const double v = (double)A[(long long)i * d.lda + j];
                const double q = __builtin_floor(v * pinv);
                L.cr[j * ST + i] = mod_fix(__builtin_fma(-q, p, v), p);
            }
            wave_lds_sync();
            double acc = 0.0;
            int_group_range<M>(L.cr, n, bt, RADIC_MAX_M, first, sp.n_prefix, sp.n_prefix, rbase, R0, R1, p, pinv,
                               batch_cap<M>(), L.slot, L.incl, reinterpret_cast<uint4*>(L.tv), lane, acc);
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) acc = addmod(acc, __shfl_xor(acc, o, kWave), p);
            if (lane == 0) atomicAdd(&J.residues[(size_t)b * RADIC_MAX_PRIMES + pi], (unsigned long long)acc);
        }
        return;
    } else if constexpr (M >= 3 && M <= 10) {
        // prefix-shared: the chunk is the run [b0, b1) of the matrix's
        // two-sided blocks, each its whole rank space's as in the single-matrix
        // kernel, or (mt.blocks == 0) the rank window [R0, R1), prefixes from
        // the one holding R0 in dictionary order
        constexpr bool blocks = batch_uses_blocks(1, M);   // a function of the class
        const unsigned K = 64u * (unsigned)(J.spl_int > 0 ? J.spl_int : 1);
        const unsigned long long b0 = c * mt.chunk;
        const unsigned long long b1 = blocks ? (b0 + mt.chunk < mt.blocks ? b0 + mt.chunk : mt.blocks) : b0 + 1;
        const unsigned long long R1 = b0 + mt.chunk < mt.total ? b0 + mt.chunk : mt.total;
        PrefixSpace sp;
        sp.n = n;
        sp.total = mt.total;
        sp.n_prefix = g_binom[(n - 2) * kBinomCols + (M - 2)];
        unsigned long long first = 0, rbase = 0;
        if constexpr (!blocks) {
            first = prefix_of_rank<M>(b0, n, bt, RADIC_MAX_M);
            rbase = first_completion_rank<M>(first, sp, bt, RADIC_MAX_M);
        }
        for (int pi = 0; pi < mt.n_primes; ++pi) {
            const double p = g_prime[pi], pinv = g_prime_inv[pi];
            wave_lds_sync();
            for (int e = lane; e < M * n; e += kWave) {
                const int i = e / n, j = e - i * n;
                const double v = (double)A[(long long)i * d.lda + j];
                const double q = __builtin_floor(v * pinv);
                L.cr[j * ST + i] = mod_fix(__builtin_fma(-q, p, v), p);
            }
            wave_lds_sync();
            double acc = 0.0;
            if constexpr (blocks) {
                for (unsigned long long blk = b0; blk < b1; ++blk) {
                    unsigned long long next;
                    int cnt, side, vlast;
                    split_block<M - 2>(blk, n, bt, RADIC_MAX_M, K, lane, side, vlast, next, cnt);
                    int_prefix_range<M, true>(L.cr, n, bt, RADIC_MAX_M, next, next + (unsigned long long)cnt,
                                              sp.n_prefix, 0ull, 0ull, mt.total, p, pinv, batch_cap<M>(), L.slot,
                                              L.incl, L.tv, lane, acc, side, vlast);
                }
            } else {
                int_prefix_range<M>(L.cr, n, bt, RADIC_MAX_M, first, sp.n_prefix, sp.n_prefix, rbase, b0, R1, p, pinv,
                                    batch_cap<M>(), L.slot, L.incl, L.tv, lane, acc);
            }
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) acc = addmod(acc, __shfl_xor(acc, o, kWave), p);
            if (lane == 0) atomicAdd(&J.residues[(size_t)b * RADIC_MAX_PRIMES + pi], (unsigned long long)acc);
        }
        return;
    }
    const unsigned long long sub = mt.chunk / kWave;
    const unsigned long long q0 = c * mt.chunk + (unsigned long long)lane * sub;
    const int cnt = q0 < mt.total ? (int)((mt.total - q0) < sub ? (mt.total - q0) : sub) : 0;
    for (int pi = 0; pi < mt.n_primes; ++pi) {
        const double p = g_prime[pi], pinv = g_prime_inv[pi];
        wave_lds_sync();
        for (int e = lane; e < M * n; e += kWave) {
            const int i = e / n, j = e - i * n;
            const double v = (double)A[(long long)i * d.lda + j];
            const double q = __builtin_floor(v * pinv);
            L.cr[j * ST + i] = mod_fix(__builtin_fma(-q, p, v), p);
        }
        wave_lds_sync();
        int col[M];
        unrank_strided<M>(q0 < mt.total ? q0 : mt.total - 1, n, g_binom, kBinomCols, col);
        double num = 0.0, den = 1.0;
        for (unsigned long long s = 0; s < sub; ++s) {
            double a[M][M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double* src = L.cr + col[j] * ST;
#pragma unroll
                for (int i = 0; i + 1 < M; i += 2) {
                    const double2 v = *reinterpret_cast<const double2*>(src + i);
                    a[i][j] = v.x;
                    a[i + 1][j] = v.y;
                }
                if (M & 1) a[M - 1][j] = src[M - 1];
            }
            double N = 1.0, P = 1.0, D = 1.0;
            bool zero = false;
            bool neg = radic_sign_odd<M>(col);
            elim_steps_mod<M, 0>(a, p, pinv, N, P, D, zero, neg);
            if (s < (unsigned long long)cnt && !zero) {
                const double t = neg ? (N == 0.0 ? 0.0 : p - N) : N;
                frac_add(num, den, t, D, p, pinv);
            }
            successor<M>(col, n);
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double n2 = shfl_xor_d(num, off), d2 = shfl_xor_d(den, off);
            frac_add(num, den, n2, d2, p, pinv);
        }
        if (lane == 0) {
            const double r = mulmod(num, invmod(den, p, pinv), p, pinv);
            atomicAdd(&J.residues[(size_t)b * RADIC_MAX_PRIMES + pi], (unsigned long long)r);
        }
    }
}

template <int M>
__device__ __forceinline__ void batch_int_body(const BatchJob& J) {
    __shared__ IntWaveLds<M> lds[kBatchWaves];
    // binomial table C(x, y), x < kBatchMaxN, y < RADIC_MAX_M, for the prefix walk
    __shared__ unsigned long long bt[M >= 3 && M <= 10 ? kBatchMaxN * RADIC_MAX_M : 1];
    constexpr int cls = RADIC_MAX_M + M - 1;   // class_of(1, M)
    const unsigned long long total = J.header->chunks[cls];
    // waves numbered past the class's chunk count would find the queue drained:
    // a workgroup of only such waves leaves at once, the others after the barrier
    if ((unsigned long long)blockIdx.x * kBatchWaves >= total) return;
    if constexpr (M >= 3 && M <= 10) {
        for (int e = threadIdx.x; e < kBatchMaxN * RADIC_MAX_M; e += blockDim.x) {
            const int x = e / RADIC_MAX_M, y = e - x * RADIC_MAX_M;
            bt[e] = g_binom[x * kBinomCols + y];
        }
        __syncthreads();
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if ((unsigned long long)blockIdx.x * kBatchWaves + wave >= total) return;
    IntWaveLds<M>& L = lds[wave];
    const unsigned long long* prefix = J.prefix + (size_t)cls * (J.batch + 1);
    int staged = -1;
    for (;;) {
        const unsigned long long g = take_chunk(&J.header->queue[cls], lane);
        if (g >= total) break;
        const int b = find_matrix(prefix, J.batch, g);
        const unsigned long long c = g - prefix[b];
        const radic_matrix_desc d = J.desc[b];
        const BatchMeta mt = J.meta[b];
        const bool restage = b != staged;
        staged = b;
        int_chunk<M>(J, d, mt, c, b, L, bt, lane, restage);
    }
}

// Up to m = 10 the class is compiled for two waves per SIMD (256 VGPRs; a few
// bytes spill at m = 10); above, the register need is left to the compiler.
template <int M>
__global__ __launch_bounds__(kBatchWaves * kWave) void k_batch_int(BatchJob J) {
    batch_int_body<M>(J);
}
template <int M>
__global__ __launch_bounds__(kBatchWaves * kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_int_w2(BatchJob J) {
    batch_int_body<M>(J);
}

// ---------------------------------------------------------------- finalize (one wave per matrix)
__global__ __launch_bounds__(256) void k_batch_finalize(BatchJob J) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (wave >= J.batch) return;
    const int b = wave;
    const BatchMeta mt = J.meta[b];
    radic_batch_result r{};
    r.status = mt.status;
    r.n_subsets = mt.kind >= 0 ? mt.total : 0;
    if (mt.kind == 0) {
        double hi = 0.0, lo = 0.0, ab = 0.0;
        unsigned long long nfb = 0;
        for (unsigned long long c = lane; c < mt.nchunks; c += kWave) {
            const Partial p = J.partials[(size_t)b * kBatchChunksPerMatrix + c];
            dd_add(hi, lo, p.hi, p.lo);
            ab += p.abs;
            nfb += p.nfb;
        }
        wave_reduce_partial(hi, lo, ab, nfb);
        r.hi = ldexp(hi, mt.scale_exp);
        r.lo = ldexp(lo, mt.scale_exp);
        r.abs_sum = ldexp(ab, mt.scale_exp);
        r.value = r.hi + r.lo;
        r.n_fallback = nfb;
    } else if (mt.kind == 1) {
        // the whole wave: Chinese remaindering with lane i on prime i
        const int k = mt.n_primes;
        const int li = lane < k ? lane : 0;
        const unsigned long long pr = (unsigned long long)g_prime[li];
        const double res = lane < k ? (double)(J.residues[(size_t)b * RADIC_MAX_PRIMES + lane] % pr) : 0.0;
        int sign = 0, len = 0;
        unsigned limb = 0;
        wave_crt(res, k, lane, sign, len, limb);
        r.n_primes = k;
        r.sign = sign;
        if (len > RADIC_MAX_PRIMES) {
            r.status = RADIC_EOVERFLOW;
        } else {
            r.mag_len = len;
            double v = 0.0;
#pragma unroll
            for (int l = RADIC_MAX_PRIMES - 1; l >= 0; --l) {
                r.mag[l] = l < len ? (unsigned)__shfl((int)limb, l, kWave) : 0u;
                if (l < len) v = v * 4294967296.0 + (double)r.mag[l];
            }
            r.value = sign < 0 ? -v : v;
            r.hi = r.value;
        }
    } else if (mt.status == RADIC_ENONFINITE) {
        r.value = __builtin_nan("");
    }
    if (lane == 0) J.out[b] = r;
}

// ---------------------------------------------------------------- host side
hipError_t upload_binomials_batched(const unsigned long long* t) { return upload_binomial_table(t); }
hipError_t upload_primes_batched(const unsigned* primes, int count) { return upload_prime_table(primes, count); }
size_t batched_workspace_bytes(int batch) { return batch_ws_bytes(batch); }
void host_batch_chunking(int kind, unsigned long long total, int spl, unsigned long long* chunk,
                         unsigned long long* nchunks) {
    batch_chunking(kind, total, spl, *chunk, *nchunks);
}

// Persistent grid: as many workgroups as fit on the current device at once,
// cached per (kernel, device).
constexpr int kMaxDevices = 64;
static int persistent_grid(const void* kernel, int block, int (&cache)[kMaxDevices]) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    if (cache[dev] > 0) return cache[dev];
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || per <= 0) per = 1;
    cache[dev] = cus * per;
    return cache[dev];
}

template <bool F32, int M>
static hipError_t launch_float_class(const BatchJob& J, hipStream_t s) {
    static int grid[kMaxDevices] = {};
    const int block = kBatchWaves * kWave;
    const int g = persistent_grid(reinterpret_cast<const void*>(k_batch_float<F32, M>), block, grid);
    hipLaunchKernelGGL((k_batch_float<F32, M>), dim3(g), dim3(block), 0, s, J);
    return hipGetLastError();
}

template <int M>
static hipError_t launch_int_class(const BatchJob& J, hipStream_t s) {
    static int grid[kMaxDevices] = {};
    const int block = kBatchWaves * kWave;
    if constexpr (M <= 10) {
        const int g = persistent_grid(reinterpret_cast<const void*>(k_batch_int_w2<M>), block, grid);
        hipLaunchKernelGGL(k_batch_int_w2<M>, dim3(g), dim3(block), 0, s, J);
    } else {
        const int g = persistent_grid(reinterpret_cast<const void*>(k_batch_int<M>), block, grid);
        hipLaunchKernelGGL(k_batch_int<M>, dim3(g), dim3(block), 0, s, J);
    }
    return hipGetLastError();
}

template <int M>
static hipError_t launch_classes(const BatchJob& J, int prec, hipStream_t s) {
    hipError_t e = prec == RADIC_FP32_BULK ? launch_float_class<true, M>(J, s) : launch_float_class<false, M>(J, s);
    if (e == hipSuccess) e = launch_int_class<M>(J, s);
    if (e != hipSuccess) return e;
    if constexpr (M < RADIC_MAX_M) return launch_classes<M + 1>(J, prec, s);
    return hipSuccess;
}

hipError_t launch_batched(const radic_matrix_desc* desc, int batch, const double* f64, const int* i32, int prec,
                          double tau, int spl_float, int spl_int, int prime_count, radic_batch_result* out,
                          void* ws, hipStream_t s) {
    unsigned char* w = static_cast<unsigned char*>(ws);
    BatchJob J{};
    J.desc = desc;
    J.batch = batch;
    J.f64 = f64;
    J.i32 = i32;
    J.prec = prec;
    J.tau = tau;
    J.spl_float = spl_float;
    J.spl_int = spl_int;
    J.prime_count = prime_count;
    J.out = out;
    J.header = reinterpret_cast<BatchHeader*>(w);
    J.meta = reinterpret_cast<BatchMeta*>(w + off_meta());
    J.prefix = reinterpret_cast<unsigned long long*>(w + off_prefix(batch));
    J.partials = reinterpret_cast<Partial*>(w + off_partials(batch));
    J.residues = reinterpret_cast<unsigned long long*>(w + off_residues(batch));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_batch_setup, dim3((batch + 3) / 4), dim3(256), 0, s, J);
    hipLaunchKernelGGL(k_batch_scan, dim3(kClasses), dim3(1024), 0, s, J);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_classes<1>(J, prec, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_finalize, dim3((batch * kWave + 255) / 256), dim3(256), 0, s, J);
    return hipGetLastError();
}

}  // namespace radic
