// Internal definitions shared by the HIP translation units of the Radic library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <tuple>

#include "radic.h"

namespace radic {

constexpr int kWave = 64;            // CDNA4 wavefront width
constexpr int kMaxBlock = 256;       // __launch_bounds__ of every enumeration kernel
constexpr int kMaxGrid = 8192;       // partial-sum slots (one per workgroup) for single-matrix launches
constexpr int kPrefixBlock = 64;     // prefixes of m-2 columns per wave block (prefix-shared kernels)
constexpr int kGroupBlock = 16;      // prefixes of m-3 columns per wave block (group-shared kernel)
// Blocks of a whole rank space (prefix-shared kernels, see split_shape): about
// this many minors per block, so that the heaviest prefixes do not make one
// block the whole launch's critical path.
constexpr unsigned kColexPairs = 2048;

// Prefixes per block for prefixes with r later columns (C(r, 2) minors each):
// about K minors, between 1 and kPrefixBlock prefixes.
__host__ __device__ inline int colex_run(int r, unsigned K) {
    const unsigned pairs = (unsigned)(r * (r - 1) / 2);
    const unsigned k = pairs ? K / pairs : (unsigned)kPrefixBlock;
    return k < 1u ? 1 : (k > (unsigned)kPrefixBlock ? kPrefixBlock : (int)k);
}
// Two-sided prefix sharing over a whole rank space.  A minor with columns
// j_0 < ... < j_{m-1} can share its first m-2 columns with the minors that
// differ only in the last two (side 0: r = n-1-j_{m-3} free columns after
// them), or its last m-2 columns with those that differ only in the first two
// (side 1: j_2 free columns before them).  Each minor goes to the side with
// more free columns (side 0 on a tie).  Side 1 is side 0 of the column-reversed
// matrix (column c read as n-1-c): there a minor's shared columns come first
// again, and with m >= 5 both choices depend only on the shared columns, so a
// side-s prefix c_0 < ... < c_{m-3} (last column v, r = n-1-v) is taken
// exactly when c_2 <= r - s.  Below m = 5 every prefix is on side 0.
// The side-s prefixes with last column v: their other m-3 columns hold at
// least `imin` below a and the rest in [a, v); `on` false when there are none.
__host__ __device__ inline void split_shape(int P, int n, int side, int v, int& a, int& b, int& imin, bool& on) {
    const int L = n - 1 - v - side;   // largest admissible c_2
    if (P >= 4) {
        a = L + 1 < v ? L + 1 : v;
        b = v - a;
        imin = 3;
        on = true;
    } else {
        a = v;
        b = 0;
        imin = P - 1;
        on = P == 3 ? v <= L : side == 0;
    }
}
// FP32-bulk in the shared kernels: up to m = 8 a workgroup refactors its
// flagged minors in double when its waves are done (eight lanes per minor, one
// row each); above, the refactorisation kernel does it.
__host__ __device__ constexpr bool shared_tail_refactor(int m) { return m <= 8; }
constexpr int kFallbackCap = 128;    // per-wave queue of minors awaiting an FP64 refactorisation
constexpr int kBatchChunksPerMatrix = 256;
// Batched exact chunks share the first m-3 elimination steps per group (3 x 3
// determinant per minor) from this m on, up to m = 10.
constexpr int kGroupExactMin = 7;
// Batched matrices whose chunks are runs of the two-sided blocks of the
// single-matrix kernels (float m >= 7, exact 5 <= m < kGroupExactMin); the
// others are cut into rank windows.  For smaller m a batch matrix (n <= 64)
// has few prefixes per last column, and blocks, which never span two last
// columns, would leave most lanes of a round idle.
__host__ __device__ constexpr bool batch_uses_blocks(int kind, int m) {
    return kind == 0 ? m >= 7 : (m >= 5 && m < kGroupExactMin);
}
// Chunks of a matrix taken in two-sided blocks: runs of chunk blocks, at most
// most_chunks of them.
__host__ __device__ inline void batch_block_chunking(unsigned long long nblocks, unsigned long long most_chunks,
                                                     unsigned long long& chunk, unsigned long long& nchunks) {
    chunk = (nblocks + most_chunks - 1) / most_chunks;
    if (chunk < 1) chunk = 1;
    nchunks = (nblocks + chunk - 1) / chunk;
}
constexpr int kDeferEntries = 1 << 22;   // 16-byte deferral entries in a single-matrix workspace
// FP32-bulk keeps a float result only over at least this many minors: a float
// minor carries a relative error up to about u_f times its condition, which
// the tolerance on the sum (relative to sum |det|) absorbs only when many
// minors with independent rounding are added.  A call (or a batch matrix) with
// fewer minors refactors every minor in double (threshold tau = +inf).
constexpr unsigned long long kF32MinMinors = 4096;

// The threshold an FP32-bulk sum over `minors` minors uses, from the set tau:
// the errors of the minors kept in float add up with independent signs, so
// their share of sum |det| falls as the count grows, and the threshold falls
// with the fourth root of the count beyond kTauMinors (on uniformly
// ill-conditioned matrices this kept the worst error near its level at 8192
// minors).  0 (never) and +inf (always) are kept as they are.
constexpr double kTauMinors = 8192.0;
__host__ __device__ inline double effective_tau(double tau, unsigned long long minors) {
    if (!(tau > 0.0) || tau > 1.7976931348623157e308 || (double)minors <= kTauMinors) return tau;
    return tau * sqrt(sqrt(kTauMinors / (double)minors));
}

// Per-workgroup partial of a floating-point enumeration (32 bytes).
struct Partial {
    double hi;
    double lo;
    double abs;
    unsigned long long nfb;
};

// Header at the start of a single-matrix workspace.
struct DetHeader {
    int nonfinite;     // set by workgroup 0 while staging A
    int scale_exp;     // FP32_BULK: sum of the row exponents e_i
    int n_primes;      // exact path: primes used
    int pad;
    double bound_log2; // exact path: log2 of the bound on |result|
};

// Launch description of one single-matrix float enumeration.
struct FloatJob {
    const double* A;
    long long lda;
    int m, n;
    unsigned long long q_begin;   // first dictionary rank
    unsigned long long count;     // ranks to evaluate
    unsigned long long chunks;    // ceil(count / spl)
    int spl;                      // ranks per lane chunk ("subsets per lane")
    double tau;                   // FP32_BULK fallback threshold
    Partial* partials;            // [gridDim.x], unless exporting
    DetHeader* header;
    double* terms;                // export mode: [count]
    unsigned char* cols;          // export mode: [count * m] or null
    // FP32_BULK with deferral: per global wave, the number of queued minors and
    // defer_cap 16-byte entries; per workgroup, the double partials of the
    // refactorisation kernel
    int defer_cap;
    unsigned* fb_count;
    unsigned* fb_entries;
    Partial* fb_partials;
    // Prefix-shared enumeration: the ranks are grouped by their first m-2
    // (mapping 1, m >= 3) or m-3 (mapping 2, m >= 4) columns ("prefixes",
    // numbered in dictionary order among the (m-k)-subsets of the first n-k
    // columns); waves take blocks of prefixes.
    int mapping;                  // 0: lane chunks of ranks; 1: blocks of m-2 column prefixes; 2: of m-3
    int cap;                      // projected-column slots per wave (mappings 1, 2)
    unsigned long long total;     // C(n, m)
    unsigned long long n_prefix;  // C(n-2, m-2) (mapping 1) or C(n-3, m-3) (mapping 2)
    unsigned long long p_begin;   // prefixes [p_begin, p_end) cover [q_begin, q_begin + count)
    unsigned long long p_end;
    // Mapping 1 over the whole rank space: 1 when the blocks are two-sided
    // blocks (split_block: each minor shared through its first or its last m-2
    // columns, blocks of prefixes with one last column and side, about
    // colex_pairs minors each, heaviest first; colex_blocks of them), 0 when
    // block blk holds the prefixes p_begin + blk*64 ... in dictionary order.
    int colex;
    unsigned colex_pairs;
    unsigned long long colex_blocks;
};

// ---------------------------------------------------------------- timed launches
// Start and stop events for the next launch_timed call on this thread: they
// are bound to that kernel's own dispatch (hipExtLaunchKernel), so timing puts
// no extra packets on the stream.  Null when launches are not being timed.
struct TimedLaunch {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    bool used = false;
};
TimedLaunch& timed_launch();

// Launch of a main enumeration kernel: timed by the pending events when there
// are some, a plain launch otherwise.
template <typename... Params, typename... Args>
hipError_t launch_timed(void (*kernel)(Params...), dim3 grid, dim3 block, unsigned lds, hipStream_t s,
                        Args... args) {
    static_assert(sizeof...(Params) == sizeof...(Args), "argument count");
    TimedLaunch& t = timed_launch();
    (void)hipGetLastError();   // clear an error left by an earlier, unrelated call
    if (t.start && !t.used) {
        // the arguments converted to the kernel's own parameter types
        std::tuple<Params...> held(args...);
        void* argv[sizeof...(Params)];
        std::apply([&argv](auto&... a) {
            int i = 0;
            ((argv[i++] = static_cast<void*>(&a)), ...);
        }, held);
        const hipError_t e = hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, lds, s,
                                                t.start, t.stop, 0);
        t.used = e == hipSuccess;
        return e;
    }
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    return hipGetLastError();
}

// ---------------------------------------------------------------- arithmetic helpers
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += (h2, l2), renormalised so that |lo| <= ulp(hi)/2.
__device__ __forceinline__ void dd_add(double& hi, double& lo, double h2, double l2) {
    double s, e;
    two_sum(hi, h2, s, e);
    e += lo + l2;
    hi = s + e;
    lo = e - (hi - s);
}

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    return __shfl_xor(v, mask, kWave);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int mask) {
    return __shfl_xor(v, mask, kWave);
}

// Compiler-level ordering of LDS traffic issued by a single wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wave-wide combination of lane partials in a fixed butterfly order.
__device__ __forceinline__ void wave_reduce_partial(double& hi, double& lo, double& ab, unsigned long long& nfb) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        double h2 = shfl_xor_d(hi, off);
        double l2 = shfl_xor_d(lo, off);
        double a2 = shfl_xor_d(ab, off);
        unsigned long long n2 = shfl_xor_u64(nfb, off);
        dd_add(hi, lo, h2, l2);
        ab += a2;
        nfb += n2;
    }
}

// Pivot key: the magnitude's leading bits with the row index in the low 4 bits,
// arranged so that an unsigned max picks the largest magnitude and, among
// magnitudes equal in the kept bits, the lowest row.  For double the kept bits
// are the exponent and 16 mantissa bits (the high word with sign and the four
// lowest bits cleared); for float the exponent and 19 mantissa bits.
__device__ __forceinline__ unsigned pivot_key(double x, int row) {
    unsigned hi = (unsigned)__double2hiint(x);
    return (hi & 0x7FFFFFF0u) | (unsigned)(15 - row);
}
__device__ __forceinline__ unsigned pivot_key(float x, int row) {
    unsigned b = (unsigned)__float_as_int(x);
    return (b & 0x7FFFFFF0u) | (unsigned)(15 - row);
}
__device__ __forceinline__ int pivot_row(unsigned key) { return 15 - (int)(key & 15u); }

// Reciprocal for the elimination multipliers: hardware estimate refined by two
// Newton-Raphson steps (double) or used as is (float, where its error is below
// the float rounding of the products it feeds).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Fused multiply-add in the operand type (the generic builtin is double-only).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------- host helpers
int host_binomial(int a, int b, unsigned long long* out);   // 0 or RADIC_EOVERFLOW

}  // namespace radic
