// Pieces shared by the prefix-shared floating-point kernels: the per-wave
// prefix records, the workgroup's LDS copies of the matrix, and the pivoted LU
// of a prefix's m x P block.
#pragma once

#include <type_traits>

#include "prefix.h"
#include "stage.h"

namespace radic {

// Per-prefix record in the wave's LDS, read by the minor loop (16 bytes).  A
// prefix here is the first m-k columns (k = 2 or 3 trailing columns).
struct PairHdr {
    double prodS;     // product of the prefix's pivots with its sign parity applied
    unsigned lo;      // first minor (in the prefix's own order) inside the call's rank range
    unsigned rt;      // r | toff << kRBits: r columns after the prefix, toff its first slot
};
static_assert(sizeof(PairHdr) == 16, "pair header size");
constexpr int kRBits = 11;
constexpr unsigned kRMask = (1u << kRBits) - 1u;

constexpr int kHdrBytes = kPrefixBlock * (int)sizeof(PairHdr);
constexpr int kScanBytes = 2 * kPrefixBlock * 4;
constexpr int kF32Extra = kPrefixBlock * 4 + kPrefixBlock * 16;   // FP32-bulk: capped ratios, packed prefix columns

// Column strides of the workgroup's matrix copies: odd (in 4- or 8-byte words),
// so that lanes reading consecutive columns, or runs of an odd number of
// columns apart, hit different LDS banks.  The float copy keeps the column's
// reciprocal scale in slot m.
template <int M> struct SharedLayout {
    static constexpr int s64 = M | 1;
    static constexpr int s32 = (M + 1) | 1;
};

// The LDS binomial slice holds C(x, y) for y <= m (stride m + 1): the prefix
// unranking reads y <= m-2, the rank of a prefix's first sequence y <= m.  Then
// the double copy and, for FP32-bulk, the row-scaled float copy.
template <int M, bool F32> __host__ __device__ int shared_common_bytes(int n) {
    int b = binom_bytes<M + 1>(n) + align16(n * SharedLayout<M>::s64 * 8);
    if (F32) b += align16(n * SharedLayout<M>::s32 * 4);
    return b;
}

// Step K of LU with partial pivoting of the m x P prefix block, column by
// column (left-looking): column c_K is read in the lane's current row order
// `rel` (4 bits per position), the earlier steps are applied to it with the
// stored multipliers L, its pivot is chosen, and an exchange swaps the two rows
// of L and of the column and is recorded in `rel`, so that later columns are read
// already exchanged.  Every entry sees the same operations in the same order as
// in the row-by-row (right-looking) form, P A = L U, with only L kept: U enters
// through the pivot product.
template <int M, int P, int K, typename T, bool CHECK>
__device__ __forceinline__ void left_steps(T (&L)[M][P], const T* src, int stride, const int (&c)[P], double& prod,
                                           bool& neg, float& ratio, unsigned long long& rel) {
    if constexpr (K < P) {
        const T* colp = src + c[K] * stride;
        T x[M];
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] = colp[(int)((rel >> (4 * i)) & 15ull)];
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = k + 1; i < M; ++i) x[i] = fma_t(-L[i][k], x[k], x[i]);
        }
        unsigned best = pivot_key(x[K], K);
#pragma unroll
        for (int i = K + 1; i < M; ++i) best = max(best, pivot_key(x[i], i));
        const int p = pivot_row(best);
        neg ^= (p != K);
        if (__ballot(p != K)) {
            const unsigned long long d = ((rel >> (4 * K)) ^ (rel >> (4 * p))) & 15ull;
            rel ^= (d << (4 * K)) | (d << (4 * p));
        }
#pragma unroll
        for (int i = K + 1; i < M; ++i) {
            const bool e = (p == i);
            if (__ballot(e)) {
                {
                    const T u = x[K], v = x[i];
                    x[K] = e ? v : u;
                    x[i] = e ? u : v;
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const T u = L[K][k], v = L[i][k];
                    L[K][k] = e ? v : u;
                    L[i][k] = e ? u : v;
                }
            }
        }
        const T piv = x[K];
        if (CHECK) ratio *= __saturatef(__builtin_fabsf((float)piv) * (float)colp[M]);
        prod *= (double)piv;
        const T rp = piv == T(0) ? T(0) : recip(piv);   // a zero pivot column: every minor is 0
#pragma unroll
        for (int i = K + 1; i < M; ++i) L[i][K] = x[i] * rp;
        left_steps<M, P, K + 1, T, CHECK>(L, src, stride, c, prod, neg, ratio, rel);
    }
}


// Every rank of [lo, hi) factored in double by the wave's groups of G =
// refactor_group<M>() lanes (group_refactor_cols_f64: one row per lane, no
// per-lane matrix): group g takes the g-th of 64/G contiguous sub-ranges,
// unranks its first sequence (Section 4) and walks the rest with the successor
// (Section 5); its first lane adds the terms.  bt[x*BS + y] = C(x, y).  Counts
// the ranks in nvalid.  With side 1 the ranks are those of the column-reversed
// matrix (see split_shape), each minor evaluated through the matrix's columns.
template <int M, int BS, int S64>
__device__ void redo_ranks_group_f64(const FloatJob& J, const unsigned long long* bt, const double* cd,
                                     unsigned long long lo, unsigned long long hi, int lane, double& h, double& l,
                                     double& ab, unsigned long long& nvalid, int side = 0) {
    constexpr int G = refactor_group<M>(), NG = kWave / G;
    if (hi <= lo) return;
    const int g = lane / G;
    const unsigned long long per = (hi - lo + NG - 1) / NG;
    const unsigned long long s0 = lo + (unsigned long long)g * per;
    const unsigned long long s1 = s0 + per < hi ? s0 + per : hi;
    int col[M];
    unrank_strided<M>(s0 < hi ? s0 : lo, J.n, bt, BS, col);
    for (unsigned long long s = 0; s < per; ++s) {
        int cm[M];
        side_to_matrix<M>(col, J.n, side, cm);
        double ad;
        const double term = group_refactor_cols_f64<M, S64>(cd, cm, lane, ad);
        if (s0 + s < s1 && (lane & (G - 1)) == 0) {
            double sum, err;
            two_sum(h, term, sum, err);
            h = sum;
            l += err;
            ab += ad;
            nvalid += 1;
        }
        successor<M>(col, J.n);
    }
}

// Entries [0, count) of a wave's queue q of packed minors (count wave-uniform),
// refactored in double by the wave's groups of G = refactor_group<M>() lanes:
// group g takes entries g, g + 64/G, ...; a group past the last entry works on
// entry 0 and adds nothing; the group's first lane adds the term.  Every lane
// calls this.
template <int M, int S64>
__device__ void refactor_queue_groups(const double* cd, const uint4* q, int count, int lane, double& hi, double& lo,
                                      double& ab) {
    constexpr int G = refactor_group<M>(), NG = kWave / G;
    for (int e0 = 0; e0 < count; e0 += NG) {
        const int e = e0 + lane / G;
        const bool ok = e < count;
        double ad;
        const double term = group_refactor_f64<M, S64>(cd, reinterpret_cast<const unsigned*>(q + (ok ? e : 0)), lane, ad);
        if (ok && (lane & (G - 1)) == 0) {
            double sum, err;
            two_sum(hi, term, sum, err);
            hi = sum;
            lo += err;
            ab += ad;
        }
    }
}

// FP32-bulk, prefix-shared: every minor of one round (the prefixes next ...
// next + ntake - 1, of a two-sided block or dictionary numbers, clipped to the
// call's rank window) refactored in double by the wave's lane groups, each
// counted in nvalid.  Used when a round flags more minors than the wave's
// segment holds.  Every lane calls this.
template <int M, int BS, int S64>
__device__ void redo_round_groups(const FloatJob& J, const unsigned long long* bt, const double* cd,
                                  unsigned long long next, int ntake, int side, int vlast, int lane, double& hi,
                                  double& lo, double& ab, unsigned long long& nvalid) {
    if (J.colex) {
        for (int t = 0; t < ntake; ++t) {
            unsigned long long r0, r1;
            split_prefix_ranks<M, BS>(J, bt, side, vlast, next + (unsigned long long)t, r0, r1);
            redo_ranks_group_f64<M, BS, S64>(J, bt, cd, r0, r1, lane, hi, lo, ab, nvalid, side);
        }
    } else {
        unsigned long long r0 = first_completion_rank<M, FloatJob, 2>(next, J, bt, BS);
        unsigned long long r1 = first_completion_rank<M, FloatJob, 2>(next + (unsigned long long)ntake, J, bt, BS);
        const unsigned long long qe = J.q_begin + J.count;
        if (r0 < J.q_begin) r0 = J.q_begin;
        if (r1 > qe) r1 = qe;
        redo_ranks_group_f64<M, BS, S64>(J, bt, cd, r0, r1, lane, hi, lo, ab, nvalid, 0);
    }
}

// FP32-bulk, between two rounds of a prefix-shared wave: when the wave's segment
// of J.fb_entries is more than half full (gcount entries, wave-uniform), the
// wave refactors them in double here, in whole passes of its lane groups
// (refactor_queue_groups), and moves the fewer than 64/G left to the front of
// the segment; gcount becomes their number.  This keeps a wave that meets many
// flagged minors from overflowing its segment.  Every lane calls this.
template <int M, int S64>
__device__ void relieve_segment(const FloatJob& J, const double* cd, unsigned long long gwave, int& gcount, int lane,
                                double& hi, double& lo, double& ab) {
    constexpr int NG = kWave / refactor_group<M>();   // groups per wave
    if (2 * gcount <= J.defer_cap) return;
    const int F = gcount - gcount % NG;
    uint4* seg = reinterpret_cast<uint4*>(J.fb_entries) + (size_t)gwave * J.defer_cap;
    __threadfence_block();   // the entries other lanes of the wave stored
    refactor_queue_groups<M, S64>(cd, seg, F, lane, hi, lo, ab);
    // entries [F, gcount) to [0, gcount - F): disjoint, since gcount - F < NG <= F
    const int rest = gcount - F;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (lane < rest) v = seg[F + lane];
    if (lane < rest) seg[lane] = v;
    gcount = rest;
}

// FP32-bulk tail of a prefix-shared workgroup.  Each wave queued its flagged
// minors in its segment of J.fb_entries (gcount, wave-uniform).  With m-3
// column prefixes (KT = 3) a wave whose segment overflowed drops its float sums
// and redoes its own blocks (BLOCK prefixes: gwave, gwave + nwaves, ...) in
// double, a group of refactor_group<M>() lanes per minor; with m-2 column
// prefixes a round that would overflow is redone at once (redo_round_groups),
// so no segment overflows.  The
// entries of the other waves are pooled and refactored in double by such groups
// of the workgroup's threads, in a fixed order (group g takes entries g, g + NG,
// ...; its first lane adds the term).  segn: a workgroup LDS array of 16.  Every thread of the workgroup calls this.  Reads the binomial
// slice bt (stride BS) and the row-scaled double copy cd (column stride S64).
template <int M, int KT, int BLOCK, int BS, int S64>
__device__ void shared_fp32_tail(const FloatJob& J, const unsigned long long* bt, const double* cd, int gcount,
                                 unsigned long long gwave, unsigned long long nwaves, unsigned long long nblk,
                                 unsigned* segn, double& hi, double& lo, double& ab, unsigned long long& nfb) {
    const int waves = blockDim.x / kWave, wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) segn[wave] = (unsigned)gcount;
    __syncthreads();
    if constexpr (KT == 3) {
        if (gcount > J.defer_cap) {
            hi = lo = ab = 0.0;
            nfb = 0;
            // one contiguous rank range per block
            for (unsigned long long blk = gwave; blk < nblk; blk += nwaves) {
                unsigned long long r0, r1;
                prefix_block_ranks<M, FloatJob, KT, BLOCK>(J, bt, blk, r0, r1, BS);
                redo_ranks_group_f64<M, BS, S64>(J, bt, cd, r0, r1, lane, hi, lo, ab, nfb);
            }
        }
    }
    unsigned E = 0;
    for (int w = 0; w < waves; ++w)
        if (segn[w] <= (unsigned)J.defer_cap) E += segn[w];
    const unsigned long long w0 = (unsigned long long)blockIdx.x * waves;
    // a group of GL lanes per entry: group g of the workgroup takes entries g,
    // g + NG, ...
    constexpr unsigned GL = refactor_group<M>();
    const unsigned g = threadIdx.x / GL, NG = blockDim.x / GL;
    for (unsigned e = g; e < E; e += NG) {
        // the segment holding entry e (overflowed segments skipped)
        int w = 0;
        unsigned pos = e;
        for (;; ++w) {
            const unsigned c = segn[w] <= (unsigned)J.defer_cap ? segn[w] : 0u;
            if (pos < c) break;
            pos -= c;
        }
        const unsigned* ent = J.fb_entries + ((size_t)(w0 + w) * J.defer_cap + pos) * 4;
        double ad;
        const double term = group_refactor_f64<M, S64>(cd, ent, lane, ad);
        if ((lane & (GL - 1)) == 0) {
            double sum, err;
            two_sum(hi, term, sum, err);
            hi = sum;
            lo += err;
            ab += ad;
        }
    }
}

}  // namespace radic
