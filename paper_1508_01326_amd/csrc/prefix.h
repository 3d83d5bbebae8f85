// Prefix structure of the dictionary order used by the prefix-shared kernels.
//
// In the dictionary order of Section 3 all sequences that share their first
// m-2 columns c_0 < ... < c_{m-3} (a "prefix") are consecutive: the pairs
// (a, b), c_{m-3} < a < b < n, in dictionary order.  Prefixes are numbered in
// the dictionary order of the (m-2)-subsets of the first n-2 columns (0-based),
// so consecutive prefixes own consecutive rank ranges.  Waves take blocks of
// kPrefixBlock consecutive prefixes.
#pragma once

#include "lu_float.h"
#include "split.h"

namespace radic {


// Prefix number pi to its columns c_0 < ... < c_{m-3}, through the
// combinatorial number system: with x_k = n - 3 - c_k (strictly decreasing),
// the prefixes after pi in dictionary order number
// N = n_prefix - 1 - pi = sum_k C(x_k, m-2-k), so each x_k is the largest x below
// x_{k-1} with C(x, m-2-k) <= what is left of N.  A binary search over the LDS
// binomial slice (bt[x*stride + y] = C(x, y)) finds the leading digits; the last
// two have closed forms.
template <int P>
__device__ __forceinline__ void unrank_prefix(unsigned long long pi, int n, unsigned long long n_prefix,
                                              const unsigned long long* bt, int stride, int (&c)[P]) {
    unsigned long long N = n_prefix - 1 - pi;
    int hi = n - 3;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int j = P - k;
        int x;
        if (j == 1) {
            x = (int)N;
        } else if (j == 2) {
            x = (int)((1.0 + sqrt(1.0 + 8.0 * (double)N)) * 0.5);
            if ((unsigned long long)x * (unsigned long long)(x - 1) / 2 > N) --x;
            if ((unsigned long long)(x + 1) * (unsigned long long)x / 2 <= N) ++x;
            N -= (unsigned long long)x * (unsigned long long)(x - 1) / 2;
        } else {
            int lo = j - 1, h = hi;
            while (lo < h) {
                const int mid = (lo + h + 1) >> 1;
                if (bt[mid * stride + j] <= N) lo = mid;
                else h = mid - 1;
            }
            x = lo;
            N -= bt[x * stride + j];
        }
        c[k] = n - 3 - x;
        hi = x - 1;
    }
}

// Inclusive scan over the wave of 64-bit counts.
__device__ __forceinline__ unsigned long long wave_scan_u64(unsigned long long v, int lane) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned long long u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

// Block blk of the two-sided blocks: its side, last column v, first index j0
// among the side's prefixes with that v, and prefix count (0 past the last
// block).  The wave's lanes take 32 values of v (two sides each) at a time and
// scan their block counts; every lane of the wave calls this and gets the same
// answer.
template <int P>
__device__ void split_block(unsigned long long blk, int n, const unsigned long long* bt, int stride, unsigned K,
                            int lane, int& side, int& v, unsigned long long& j0, int& count) {
    unsigned long long acc = 0;
    side = 0;
    v = P - 1;
    j0 = 0;
    count = 0;
    for (int v0 = P - 1; v0 <= n - 3; v0 += kWave / 2) {
        const int vv = v0 + lane / 2, sd = lane & 1;
        unsigned long long nb = 0, cnt = 0;
        int k = 1;
        if (vv <= n - 3) {
            cnt = split_count<P>(n, sd, vv, bt, stride);
            k = colex_run(n - 1 - vv, K);
            nb = (cnt + (unsigned long long)k - 1) / (unsigned long long)k;
        }
        const unsigned long long incl = wave_scan_u64(nb, lane);
        const unsigned long long tot = __shfl(incl, kWave - 1, kWave);
        if (blk < acc + tot) {
            const bool mine = nb > 0 && blk >= acc + incl - nb && blk < acc + incl;
            const int owner = __ffsll((long long)__ballot(mine)) - 1;
            unsigned long long st = 0;
            int c = 0;
            if (mine) {
                st = (blk - (acc + incl - nb)) * (unsigned long long)k;
                const unsigned long long rem = cnt - st;
                c = (int)(rem < (unsigned long long)k ? rem : (unsigned long long)k);
            }
            // wave-uniform results, kept in scalar registers
            const unsigned long long sj = __shfl(st, owner, kWave);
            j0 = ((unsigned long long)__builtin_amdgcn_readfirstlane((int)(sj >> 32)) << 32) |
                 (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)sj);
            count = __builtin_amdgcn_readfirstlane(__shfl(c, owner, kWave));
            side = __builtin_amdgcn_readfirstlane(owner & 1);
            v = __builtin_amdgcn_readfirstlane(v0 + owner / 2);
            return;
        }
        acc += tot;
    }
}

// Column list of a side-s minor, from its side's coordinates (ascending) to the
// matrix's (ascending): side 1 reads column c as n-1-c.
template <int M>
__device__ __forceinline__ void side_to_matrix(const int (&cs)[M], int n, int side, int (&c)[M]) {
#pragma unroll
    for (int k = 0; k < M; ++k) c[k] = side ? n - 1 - cs[M - 1 - k] : cs[k];
}

// Dictionary rank of the first sequence (c, c_{m-3}+1, c_{m-3}+2) of a prefix c
// of m-2 columns: the sequences after it number sum_k C(n-1-c_k, m-k) (read from
// the full binomial table).
template <int M>
__device__ __forceinline__ unsigned long long prefix_first_rank(const int (&c)[M - 2], int n,
                                                                unsigned long long total) {
    constexpr int P = M - 2;
    const int r = n - 1 - c[P - 1];
    unsigned long long after = g_binom[(r - 1) * kBinomCols + 2] + g_binom[(r - 2) * kBinomCols + 1];
#pragma unroll
    for (int k = 0; k < P; ++k) after += g_binom[(n - 1 - c[k]) * kBinomCols + (M - k)];
    return total - 1 - after;
}

// Dictionary rank of the first sequence with prefix number pi: the prefix c of
// m-KT columns (numbered among the (m-KT)-subsets of the first n-KT columns)
// followed by c_last+1, ..., c_last+KT; J.total when pi is past the last
// prefix.  Reads the LDS binomial slice bt[x*stride + y] = C(x, y), y < m-KT.
template <int M, class Job, int KT = 2>
__device__ unsigned long long first_completion_rank(unsigned long long pi, const Job& J,
                                                    const unsigned long long* bt, int stride = M) {
    constexpr int P = M - KT;
    if (pi >= J.n_prefix) return J.total;
    const int n = J.n;
    int c[P];
    unrank_prefix<P>(pi, n - KT + 2, J.n_prefix, bt, stride, c);
    int full[M];
#pragma unroll
    for (int k = 0; k < P; ++k) full[k] = c[k];
#pragma unroll
    for (int j = 0; j < KT; ++j) full[P + j] = c[P - 1] + 1 + j;
    // dictionary rank from the complement count: the sequences after `full`
    // number sum_k C(n-1-c_k, M-k), read from the full binomial table
    unsigned long long after = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) after += g_binom[(n - 1 - full[k]) * kBinomCols + (M - k)];
    const unsigned long long q = J.total - 1 - after;
    return q;
}

// Inclusive scan over the wave (lanes in order).
__device__ __forceinline__ unsigned wave_scan_u32(unsigned v, int lane) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

// Pair number x (dictionary order of the pairs ia < ib < r) to (ia, ib).
__device__ __forceinline__ void unrank_pair(unsigned x, int r, int& ia, int& ib) {
    const double b = 2.0 * r - 1.0;
    int i = (int)((b - sqrt(b * b - 8.0 * (double)x)) * 0.5);
    i = i < 0 ? 0 : (i > r - 2 ? r - 2 : i);
    // row i starts at i (2r - i - 1) / 2; correct a rounding step either way
    if ((unsigned)(i * (2 * r - i - 1) / 2) > x) --i;
    if (i + 1 <= r - 2 && (unsigned)((i + 1) * (2 * r - i - 2) / 2) <= x) ++i;
    ia = i;
    ib = i + 1 + (int)(x - (unsigned)(i * (2 * r - i - 1) / 2));
}

// The rank space of one m x n matrix, for the prefix helpers.
struct PrefixSpace {
    int n;
    unsigned long long total;      // C(n, m)
    unsigned long long n_prefix;   // C(n-2, m-2)
};

// Number of the prefix of the sequence of rank q (bt[x*stride + y] = C(x, y)).
template <int M>
__device__ unsigned long long prefix_of_rank(unsigned long long q, int n, const unsigned long long* bt, int stride) {
    constexpr int P = M - 2;
    int c[M];
    unrank_strided<M>(q, n, bt, stride, c);
    unsigned long long pi = 0;
    int prev = -1;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        for (int v = prev + 1; v < c[k]; ++v) pi += bt[(n - 3 - v) * stride + (P - 1 - k)];
        prev = c[k];
    }
    return pi;
}

// Ranks [lo, hi) owned by prefix block blk (BLOCK prefixes of m-KT columns),
// clipped to the call's rank range.
template <int M, class Job, int KT = 2, int BLOCK = kPrefixBlock>
__device__ void prefix_block_ranks(const Job& J, const unsigned long long* bt, unsigned long long blk,
                                   unsigned long long& lo, unsigned long long& hi, int stride = M) {
    const unsigned long long pi0 = J.p_begin + blk * BLOCK;
    const unsigned long long pe = pi0 + BLOCK;
    const unsigned long long pi1 = pe < J.p_end ? pe : J.p_end;
    lo = first_completion_rank<M, Job, KT>(pi0, J, bt, stride);
    hi = first_completion_rank<M, Job, KT>(pi1, J, bt, stride);
    const unsigned long long qe = J.q_begin + J.count;
    if (lo < J.q_begin) lo = J.q_begin;
    if (hi > qe) hi = qe;
    if (hi < lo) hi = lo;
}

// Every rank of [lo, hi) factored in double by the wave, minor by minor (rows in
// natural order, from the row-scaled double copy cd, column stride ST64): lane l
// takes the l-th of 64 contiguous sub-ranges.  bt[x*BSTRIDE + y] = C(x, y).
// Counts the ranks in nvalid.
// With side 1 the ranks are those of the column-reversed matrix (see
// split_shape) and each minor is evaluated through the matrix's own columns.
template <int M, int BSTRIDE = M, int ST64 = Layout<M>::st64>
__device__ void redo_ranks_f64(const FloatJob& J, const unsigned long long* bt, const double* cd,
                               unsigned long long lo, unsigned long long hi, int lane, double& h, double& l,
                               double& ab, unsigned long long& nvalid, int side = 0) {
    if (hi <= lo) return;
    const unsigned long long per = (hi - lo + kWave - 1) / kWave;
    const unsigned long long s0 = lo + (unsigned long long)lane * per;
    const unsigned long long s1 = s0 + per < hi ? s0 + per : hi;
    const double none[M] = {};
    int col[M];
    unrank_strided<M>(s0 < hi ? s0 : lo, J.n, bt, BSTRIDE, col);
    for (unsigned long long s = 0; s < per; ++s) {
        int cm[M];
        side_to_matrix<M>(col, J.n, side, cm);
        double a[M][M];
        gather_f64<M, ST64>(a, cd, cm);
        bool neg = radic_sign_odd<M>(cm);
        bool flag = false;
        unsigned long long perm = 0;
        int perm_odd = 0;
        const double d = lu_det<M, double, false>(a, neg, flag, none, 0.0, perm, perm_odd);
        if (s0 + s < s1) {
            const double term = neg ? -d : d;
            double sum, err;
            two_sum(h, term, sum, err);
            h = sum;
            l += err;
            ab += fabs(d);
            nvalid += 1;
        }
        successor<M>(col, J.n);
    }
}

// Ranks [r0, r1), in the coordinates of its side, of the minors of the j-th
// side-s prefix with last column v (see split_block).  bt[x*BSTRIDE + y] =
// C(x, y) for y <= m-3.
template <int M, int BSTRIDE = M>
__device__ void split_prefix_ranks(const FloatJob& J, const unsigned long long* bt, int side, int v,
                                   unsigned long long j, unsigned long long& r0, unsigned long long& r1) {
    constexpr int P = M - 2;
    int c[P];
    split_unrank<P>(j, J.n, side, v, bt, BSTRIDE, c);
    const int r = J.n - 1 - v;
    r0 = prefix_first_rank<M>(c, J.n, J.total);
    r1 = r0 + (unsigned long long)(r * (r - 1) / 2);
}

}  // namespace radic
