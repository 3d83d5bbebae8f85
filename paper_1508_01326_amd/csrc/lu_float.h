// LU with partial pivoting of register-resident minors, shared by the
// single-matrix and batched floating-point kernels.
#pragma once

#include "enumerate.h"

namespace radic {

// ---------------------------------------------------------------- LDS layout
// Columns are stored contiguously with a stride (in 16-byte groups) chosen odd so
// that lanes reading different columns start on different bank groups.
template <int M> struct Layout {
    static constexpr int g64 = (((M + 1) / 2) % 2 == 0) ? (M + 1) / 2 + 1 : (M + 1) / 2;
    static constexpr int st64 = 2 * g64;                  // doubles per column
    static constexpr int g32 = (((M + 4) / 4) % 2 == 0) ? (M + 4) / 4 + 1 : (M + 4) / 4;
    static constexpr int st32 = 4 * g32;                  // floats per column (+1 slot: column scale)
};

// Per-wave fallback region of the export kernel: queue of rank offsets followed
// by the M x M double scratch of the wave-cooperative LU.
template <int M> __host__ __device__ constexpr int fallback_wave_bytes() {
    return kFallbackCap * 4 + align16(M * M * 8);
}

// ---------------------------------------------------------------- LU building blocks
template <int M, typename T>
__device__ __forceinline__ void gather(T (&a)[M][M], const T* base, int stride, const int (&col)[M]) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const T* src = base + col[j] * stride;
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int i = 0; i + 1 < M; i += 2) {
                double2 v = *reinterpret_cast<const double2*>(src + i);
                a[i][j] = v.x;
                a[i + 1][j] = v.y;
            }
            if (M & 1) a[M - 1][j] = src[M - 1];
        } else {
#pragma unroll
            for (int i = 0; i + 3 < M; i += 4) {
                float4 v = *reinterpret_cast<const float4*>(src + i);
                a[i][j] = v.x;
                a[i + 1][j] = v.y;
                a[i + 2][j] = v.z;
                a[i + 3][j] = v.w;
            }
#pragma unroll
            for (int i = (M / 4) * 4; i < M; ++i) a[i][j] = src[i];
        }
    }
}

// Double minor gather from a column-major copy with column stride ST64: pairs of
// rows by 16-byte loads where the stride keeps them aligned, else one by one.
template <int M, int ST64>
__device__ __forceinline__ void gather_f64(double (&a)[M][M], const double* base, const int (&col)[M]) {
    if constexpr (ST64 % 2 == 0) {
        gather<M, double>(a, base, ST64, col);
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int i = 0; i < M; ++i) a[i][j] = base[col[j] * ST64 + i];
        }
    }
}

// Bring each lane's pivot row p into row K with selects.  Only candidate rows
// that some lane of the wave chose are visited (a wave-uniform test), so a step
// on which the whole wave keeps row K costs one ballot per candidate.  When every
// lane of the wave chose the same row i, the exchange (K, i) is recorded in the
// wave's row order `perm` (4 bits per position) and its parity flipped, so that
// the next minors are gathered with that exchange already applied.
template <int M, int K, typename T>
__device__ __forceinline__ void exchange_rows(T (&a)[M][M], int p, unsigned long long& perm, int& perm_odd) {
#pragma unroll
    for (int i = K + 1; i < M; ++i) {
        const bool c = (p == i);
        const unsigned long long mask = __ballot(c);
        if (mask) {
            if (mask == ~0ull) {
                const unsigned long long x = ((perm >> (4 * K)) ^ (perm >> (4 * i))) & 15ull;
                perm ^= (x << (4 * K)) | (x << (4 * i));
                perm_odd ^= 1;
            }
#pragma unroll
            for (int j = K; j < M; ++j) {
                const T x = a[K][j], y = a[i][j];
                a[K][j] = c ? y : x;
                a[i][j] = c ? x : y;
            }
        }
    }
}

// LU with partial pivoting of the register-resident minor, one step per
// template level K so that every register index is a compile-time constant.
// Accumulates the pivots into det, raises `zero` for an exactly zero pivot
// column, flips `neg` once per row exchange and, for FP32 (CHECK), raises `flag`
// when a pivot falls below tau * s_k.
template <int M, int K, typename T, bool CHECK>
__device__ __forceinline__ void lu_steps(T (&a)[M][M], T& det, bool& zero, bool& neg, float& ratio,
                                         const T (&s)[M], unsigned long long& perm, int& perm_odd) {
    if constexpr (K < M - 1) {
        unsigned best = pivot_key(a[K][K], K);
#pragma unroll
        for (int i = K + 1; i < M; ++i) best = max(best, pivot_key(a[i][K], i));
        const int p = pivot_row(best);
        neg ^= (p != K);
        exchange_rows<M, K, T>(a, p, perm, perm_odd);
        const T piv = a[K][K];
        zero |= (piv == T(0));
        if (CHECK) ratio *= __saturatef(__builtin_fabsf((float)piv) * (float)s[K]);
        det *= piv;
        const T r = recip(piv);
#pragma unroll
        for (int i = K + 1; i < M; ++i) {
            const T l = a[i][K] * r;
#pragma unroll
            for (int j = K + 1; j < M; ++j) a[i][j] = fma_t(-l, a[K][j], a[i][j]);
        }
        lu_steps<M, K + 1, T, CHECK>(a, det, zero, neg, ratio, s, perm, perm_odd);
    }
}

// Determinant of the minor (0 for an exactly zero pivot column).  For FP32
// (CHECK) `flag` is raised when prod_k min(1, |u_kk| / s_k) < tau, s_k the largest
// magnitude in the minor's k-th column of the row-scaled matrix (s holds 1/s_k):
// the minor is then relatively ill-conditioned, float elimination may have lost
// too many digits, and the minor is refactored in double.
template <int M, typename T, bool CHECK>
__device__ __forceinline__ T lu_det(T (&a)[M][M], bool& neg, bool& flag, const T (&s)[M], T tau,
                                    unsigned long long& perm, int& perm_odd) {
    T det = T(1);
    bool zero = false;
    float ratio = 1.0f;
    lu_steps<M, 0, T, CHECK>(a, det, zero, neg, ratio, s, perm, perm_odd);
    const T last = a[M - 1][M - 1];
    if (CHECK) {
        ratio *= __saturatef(__builtin_fabsf((float)last) * (float)s[M - 1]);
        flag |= !(ratio >= (float)tau);
    }
    det *= last;
    return zero ? T(0) : det;
}

// ---------------------------------------------------------------- FP64 refactorisation (wave-cooperative)
// One minor at a time, factored by the whole wave in LDS: exact first-maximum
// partial pivoting and true division, as in the textbook algorithm.
template <int M>
__device__ double coop_det_f64(const double* cd, const int (&c)[M], double* W, int lane) {
    constexpr int ST64 = Layout<M>::st64;
    for (int t = lane; t < M * M; t += kWave) {
        int i = t / M, j = t - i * M;
        W[t] = cd[c[j] * ST64 + i];
    }
    wave_lds_sync();
    double det = 1.0;
    bool neg = false, zero = false;
    for (int k = 0; k < M; ++k) {
        double v = (lane >= k && lane < M) ? fabs(W[lane * M + k]) : -1.0;
        if (v != v) v = __builtin_inf();   // a NaN entry is taken as the largest
        int idx = lane;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            double v2 = shfl_xor_d(v, off);
            int i2 = __shfl_xor(idx, off, kWave);
            if (v2 > v || (v2 == v && i2 < idx)) { v = v2; idx = i2; }
        }
        if (v == 0.0) { zero = true; break; }
        const int p = (idx >= k && idx < M) ? idx : k;
        if (p != k) {
            neg = !neg;
            if (lane >= k && lane < M) {
                double x = W[k * M + lane];
                W[k * M + lane] = W[p * M + lane];
                W[p * M + lane] = x;
            }
        }
        wave_lds_sync();
        const double piv = W[k * M + k];
        det *= piv;
        const int w = M - 1 - k;
        for (int t = lane; t < w * w; t += kWave) {
            int i = k + 1 + t / w, j = k + 1 + t % w;
            double l = W[i * M + k] / piv;
            W[i * M + j] -= l * W[k * M + j];
        }
        wave_lds_sync();
    }
    return zero ? 0.0 : (neg ? -det : det);
}

// A queued minor is 16 bytes: its M 0-based column indices in 10-bit fields,
// three per 32-bit word (M <= 12, n <= 1024).
constexpr int kColBits = 10;
// Bit 31 of an entry's first word: its columns are stored in descending order
// (the minor's determinant in that order is (-1)^(m(m-1)/2) times its own).
constexpr unsigned kColsDescending = 1u << 31;

template <int M>
__device__ __forceinline__ void pack_cols(const int (&col)[M], unsigned (&w)[4]) {
    w[0] = w[1] = w[2] = w[3] = 0u;
#pragma unroll
    for (int j = 0; j < M; ++j) w[j / 3] |= (unsigned)col[j] << (kColBits * (j % 3));
}

template <int M>
__device__ __forceinline__ void unpack_cols(const unsigned* w, int (&col)[M]) {
#pragma unroll
    for (int j = 0; j < M; ++j) col[j] = (w[j / 3] >> (kColBits * (j % 3))) & ((1u << kColBits) - 1u);
}

// Signed term of one queued minor refactored in double (rows in natural order,
// from the row-scaled double copy cd).
template <int M, int ST64 = Layout<M>::st64>
__device__ __forceinline__ double refactor_entry_f64(const double* cd, const unsigned* entry, double& absdet) {
    int c[M];
    unpack_cols<M>(entry, c);
    double a[M][M];
    gather_f64<M, ST64>(a, cd, c);
    bool neg = radic_sign_odd<M>(c) ^ ((entry[0] & kColsDescending) && ((M * (M - 1) / 2) & 1));
    bool flag = false;
    unsigned long long perm = 0;
    int perm_odd = 0;
    const double unused[M] = {};
    const double d = lu_det<M, double, false>(a, neg, flag, unused, 0.0, perm, perm_odd);
    absdet = fabs(d);
    return neg ? -d : d;
}

// Lanes per minor of the group refactorisation: one row per lane, in groups of
// eight up to m = 8 and of sixteen beyond.
template <int M> constexpr int refactor_group() { return M <= 8 ? 8 : 16; }

// Signed term of one queued minor refactored in double by a group of G =
// refactor_group<M>() lanes (G-aligned in the wave; all G call together): lane r
// holds row r of the minor (rows in natural order, from the row-scaled double
// copy cd), so no register is indexed by a run-time row.  Partial pivoting
// without exchanges: step k takes the unused row with the largest key |a_rk|
// (the key of lu_steps, ties to the lower row; the group maximum by DPP lane
// moves: pairs, quads, half rows of 8, rows of 16), broadcasts that row to the
// group and eliminates the other unused rows with the multipliers and fused
// multiply-adds of lu_steps.  The permutation's parity is the number of unused
// rows above each pivot row, summed.  Every lane returns the term.
template <int M, int ST64 = Layout<M>::st64>
__device__ __forceinline__ double group_refactor_cols_f64(const double* cd, const int (&c)[M], int lane,
                                                          double& absdet) {
    constexpr int G = refactor_group<M>();
    static_assert(M <= G && G <= 16, "one row per lane of a group");
    const int r = lane & (G - 1), base = lane & ~(G - 1);
    double a[M];
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] = r < M ? cd[c[j] * ST64 + r] : 0.0;
    bool used = r >= M;
    bool zero = false, odd = false;
    double det = 1.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        unsigned key = used ? 0u : pivot_key(a[k], r);   // an unused row's key is >= 16 - M > 0
        key = max(key, (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0xB1, 0xF, 0xF, false));
        key = max(key, (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x4E, 0xF, 0xF, false));
        key = max(key, (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x141, 0xF, 0xF, false));
        if constexpr (G == 16)
            key = max(key, (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x140, 0xF, 0xF, false));
        const int p = pivot_row(key);
        const unsigned gm = (unsigned)(__ballot(!used) >> base) & ((1u << G) - 1u);
        odd ^= (__popc(gm & ((1u << p) - 1u)) & 1) != 0;
        const double piv = __shfl(a[k], base + p, kWave);
        if (k < M - 1) zero |= (piv == 0.0);
        det *= piv;
        const bool elim = !used && r != p;
        used |= (r == p);
        if (k < M - 1) {
            const double l = a[k] * recip(piv);
#pragma unroll
            for (int j = k + 1; j < M; ++j) {
                const double pj = __shfl(a[j], base + p, kWave);
                const double v = __builtin_fma(-l, pj, a[j]);
                a[j] = elim ? v : a[j];
            }
        }
    }
    const double d = zero ? 0.0 : det;
    absdet = fabs(d);
    return (radic_sign_odd<M>(c) ^ odd) ? -d : d;
}

// The same for a queued (packed) minor.
template <int M, int ST64 = Layout<M>::st64>
__device__ __forceinline__ double group_refactor_f64(const double* cd, const unsigned* entry, int lane,
                                                     double& absdet) {
    int c[M];
    unpack_cols<M>(entry, c);
    const double t = group_refactor_cols_f64<M, ST64>(cd, c, lane, absdet);
    return ((entry[0] & kColsDescending) && ((M * (M - 1) / 2) & 1)) ? -t : t;
}

// Refactor queued minors in double, one minor per lane; lane l takes entries
// l, l + 64, ...  Each lane adds its terms to its own double-double sum.
template <int M>
__device__ void refactor_queue_f64(const double* cd, const unsigned* queue, int count, int lane, double& hi,
                                   double& lo, double& ab) {
    for (int base = 0; base < count; base += kWave) {
        const int e = base + lane;
        const bool valid = e < count;
        double ad;
        const double term = refactor_entry_f64<M>(cd, queue + 4 * (valid ? e : base), ad);
        if (valid) {
            double s, err;
            two_sum(hi, term, s, err);
            hi = s;
            lo += err;
            ab += ad;
        }
    }
}

}  // namespace radic
