// Dictionary-order enumeration helpers shared by the Radic kernels.
//
// Sequences are 0-based column indices c_0 < ... < c_{M-1} held in registers.
// Ranks are 0-based positions in the dictionary order of Section 3
// (Definitions 1-2): rank 0 is the First Member [0, 1, ..., M-1].
#pragma once

#include "radic_internal.h"

namespace radic {

// Binomial coefficients C(x, y), x < kBinomRows, y < kBinomCols, saturated at
// 2^64-1.  Device code is compiled per translation unit, so every kernel source
// holds its own copy, filled by the host at first use on each device through
// that unit's upload function.
constexpr int kBinomRows = RADIC_MAX_N + 1;
constexpr int kBinomCols = 33;
static __device__ unsigned long long g_binom[kBinomRows * kBinomCols];

static inline hipError_t upload_binomial_table(const unsigned long long* host_table) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_binom), host_table,
                             sizeof(unsigned long long) * kBinomRows * kBinomCols);
}

__host__ __device__ constexpr int align16(int b) { return (b + 15) & ~15; }

template <int M> __host__ __device__ constexpr int binom_bytes(int n) { return align16(n * M * 8); }

// The slice C(x, y), x < n, y < W of the table, staged in LDS as bt[x*W + y].
template <int W>
__device__ void stage_binomials(unsigned long long* bt, int n) {
    for (int e = threadIdx.x; e < n * W; e += blockDim.x) {
        int x = e / W, y = e - x * W;
        bt[e] = g_binom[x * kBinomCols + y];
    }
}

// Dictionary-order unranking (Section 4): at place k the sequences that put the
// value c there number C(n-1-c, M-1-k) (0-based c); step c to the right while q
// can pay for them.
template <int M>
__device__ __forceinline__ void unrank_strided(unsigned long long q, int n, const unsigned long long* bt, int stride,
                                               int (&col)[M]) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        for (;;) {
            unsigned long long w = bt[(n - 1 - c) * stride + (M - 1 - k)];
            if (q < w) break;
            q -= w;
            ++c;
        }
        col[k] = c;
        ++c;
    }
}

// Same, reading the LDS slice bt[x*M + y] = C(x, y).
template <int M>
__device__ __forceinline__ void unrank(unsigned long long q, int n, const unsigned long long* bt, int (&col)[M]) {
    unrank_strided<M>(q, n, bt, M, col);
}

// Dictionary successor (Section 5): the rightmost place still below its maximum
// n-M+j moves up by one and the places after it follow consecutively.  Written
// without branches; from the last member it wraps to the first (callers never
// use that value).
template <int M>
__device__ __forceinline__ void successor(int (&col)[M], int n) {
    int ip = -1, t = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        bool nf = col[j] < n - M + j;
        ip = nf ? j : ip;
        t = nf ? col[j] - j + 1 : t;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) col[j] = (j >= ip) ? t + j : col[j];
}

// Parity of r + s in (-1)^(r+s) of eq. (1): r = M(M+1)/2, s = sum of 1-based columns.
template <int M>
__device__ __forceinline__ bool radic_sign_odd(const int (&col)[M]) {
    int s = M * (M + 1) / 2 + M;
#pragma unroll
    for (int j = 0; j < M; ++j) s += col[j];
    return s & 1;
}

}  // namespace radic
