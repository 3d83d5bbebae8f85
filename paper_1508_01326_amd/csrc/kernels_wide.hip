// Radic determinant for minors wider than the per-lane register kernels
// (12 < m <= 32): a group of 32 lanes (half a wave) factors one minor at a time,
// lane r holding row r of the minor in the group's LDS block.  Each
// elimination step takes the pivot by a max-reduction over the group (first
// largest |entry| of the column, as in the oracle), exchanges the two rows in
// LDS, and updates the rows below with true division; the group walks its
// chunk of ranks with the dictionary successor (Section 5) from the unranked
// first member (Section 4), and lane 0 of the group adds the signed terms of
// eq. (1) by TwoSum.  Computed in double for both precisions.
#include "lu_float.h"

namespace radic {

constexpr int kWideGroup = 32;   // lanes per minor
constexpr int kWideMax = 32;     // largest m

struct WideGroupLds {
    double W[kWideMax * kWideMax];
    int col[kWideMax];
};

__global__ __launch_bounds__(128) void k_radic_wide(FloatJob J, int spl) {
    __shared__ WideGroupLds lds[128 / kWideGroup];
    __shared__ double red[3 * (128 / kWideGroup)];
    const int m = J.m, n = J.n;
    const int groups = blockDim.x / kWideGroup;
    const int grp = threadIdx.x / kWideGroup;
    const int r = threadIdx.x % kWideGroup;   // the row this lane holds
    WideGroupLds& L = lds[grp];
    double hi = 0.0, lo = 0.0, ab = 0.0;
    // non-finite entries anywhere in A (every workgroup sees the same answer)
    int bad = 0;
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        bad |= !isfinite(J.A[(long long)i * J.lda + j]);
    }
    bad = __syncthreads_or(bad);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.header->nonfinite = bad;
        J.header->scale_exp = 0;
    }

    const unsigned long long chunks = (J.count + spl - 1) / spl;
    const unsigned long long ggrp = (unsigned long long)blockIdx.x * groups + grp;
    const unsigned long long ngrp = (unsigned long long)gridDim.x * groups;
    for (unsigned long long ch = ggrp; ch < chunks; ch += ngrp) {
        const unsigned long long q0 = J.q_begin + ch * spl;
        const unsigned long long left = J.q_begin + J.count - q0;
        const int cnt = left < (unsigned long long)spl ? (int)left : spl;
        // first member of the chunk: combinatorial addition (Section 4), lane 0
        if (r == 0) {
            unsigned long long q = q0;
            int c = 0;
            for (int k = 0; k < m; ++k) {
                for (;;) {
                    const unsigned long long w = g_binom[(n - 1 - c) * kBinomCols + (m - 1 - k)];
                    if (q < w) break;
                    q -= w;
                    ++c;
                }
                L.col[k] = c++;
            }
        }
        wave_lds_sync();
        for (int s = 0; s < cnt; ++s) {
            // gather: lane r loads row r of the minor
            if (r < m)
                for (int j = 0; j < m; ++j) L.W[r * m + j] = J.A[(long long)r * J.lda + L.col[j]];
            wave_lds_sync();
            double det = 1.0;
            bool neg = false, zero = false;
            for (int k = 0; k < m; ++k) {
                // pivot: first row attaining the largest |entry| of column k
                double v = (r >= k && r < m) ? fabs(L.W[r * m + k]) : -1.0;
                if (v != v) v = __builtin_inf();
                int idx = r;
#pragma unroll
                for (int off = kWideGroup / 2; off > 0; off >>= 1) {
                    const double v2 = __shfl_xor(v, off, kWideGroup);
                    const int i2 = __shfl_xor(idx, off, kWideGroup);
                    if (v2 > v || (v2 == v && i2 < idx)) {
                        v = v2;
                        idx = i2;
                    }
                }
                if (v == 0.0) {
                    zero = true;
                    break;
                }
                const int p = (idx >= k && idx < m) ? idx : k;
                if (p != k) {
                    neg = !neg;
                    if (r < m) {   // lane r exchanges entry r of rows k and p
                        const double x = L.W[k * m + r];
                        L.W[k * m + r] = L.W[p * m + r];
                        L.W[p * m + r] = x;
                    }
                    wave_lds_sync();
                }
                const double piv = L.W[k * m + k];
                det *= piv;
                if (r > k && r < m) {
                    const double l = L.W[r * m + k] / piv;
                    for (int j = k + 1; j < m; ++j) L.W[r * m + j] -= l * L.W[k * m + j];
                }
                wave_lds_sync();
            }
            if (r == 0) {
                int sgn = m * (m + 1) / 2 + m;
                for (int j = 0; j < m; ++j) sgn += L.col[j];
                const double d = zero ? 0.0 : det;
                const double term = ((sgn & 1) != neg) ? -d : d;
                double sum, err;
                two_sum(hi, term, sum, err);
                hi = sum;
                lo += err;
                ab += fabs(d);
                // dictionary successor (Section 5)
                int ip = -1;
                for (int j = 0; j < m; ++j)
                    if (L.col[j] < n - m + j) ip = j;
                if (ip >= 0) {
                    const int t = L.col[ip] + 1;
                    for (int j = ip; j < m; ++j) L.col[j] = t + (j - ip);
                }
            }
            wave_lds_sync();
        }
    }
    if (r == 0) {
        red[3 * grp + 0] = hi;
        red[3 * grp + 1] = lo;
        red[3 * grp + 2] = ab;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double h = red[0], l = red[1], a2 = red[2];
        for (int g = 1; g < groups; ++g) {
            dd_add(h, l, red[3 * g + 0], red[3 * g + 1]);
            a2 += red[3 * g + 2];
        }
        J.partials[blockIdx.x] = Partial{h, l, a2, 0ull};
    }
}

hipError_t upload_binomials_wide(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

hipError_t launch_wide(const FloatJob& J, int spl, int grid, hipStream_t s) {
    return launch_timed(k_radic_wide, dim3(grid), dim3(128), 0, s, J, spl);
}

}  // namespace radic
