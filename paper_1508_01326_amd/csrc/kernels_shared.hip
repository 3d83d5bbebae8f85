// Prefix-shared floating-point Radic kernels (m >= 3) for gfx950.
//
// Gaussian elimination with partial pivoting chooses the pivot and the
// multipliers of step k from the first k+1 columns only.  In the dictionary
// order (Section 3) every minor with the same first m-2 columns (a prefix) is
// consecutive, and GEPP of all those minors performs the same first m-2 steps.
// Those steps are done once per prefix here; what is left of each minor is the
// last two steps on a 2 x 2 block.
//
// A wave takes a block of 64 consecutive prefixes and works in rounds:
//  A. Each lane takes one prefix and factors the m x (m-2) block of its columns
//     by LU with partial pivoting in registers (the first m-2 steps of every
//     minor with that prefix).  From the multipliers it forms the two rows of
//     the projection onto the two rows left after those steps, W = rows m-2 and
//     m-1 of L^{-1} P.  It writes W x_c for every later column c (2 values per
//     column, the column read in the lane's row order) to its slot in the
//     wave's LDS, with the signed product of the m-2 pivots.
//  B. The wave's minors (the column pairs (a, b) after each prefix, in
//     dictionary order) are split evenly over the 64 lanes.  Each minor is
//     det(A_J) = (signed pivot product) * det([W x_a, W x_b]).  Its last two
//     elimination steps reduce to that 2 x 2 determinant: the pivot choice
//     between the two rows changes only the sign bookkeeping, which cancels.
//     The signed term (-1)^(r+s) det(A_J) of eq. (1) is added by TwoSum.
// Every minor's determinant is still formed individually, so sum |det(A_J)| and
// the FP32-bulk conditioning test per minor are available.
//
// FP32-bulk runs both phases in float on the power-of-two row-scaled matrix.
// The capped pivot-ratio product of a minor is the prefix's product times the
// factors of the last two pivots.  Flagged minors are queued for the double
// refactorisation kernel exactly as in the per-minor kernel.
#include <type_traits>

#include "prefix.h"
#include "stage.h"

namespace radic {

// Per-prefix record in the wave's LDS (48 bytes).
struct SlotHdr {
    double prodS;     // product of the m-2 pivots with the prefix's sign parity applied
    int r;            // columns after the prefix: n - 1 - c_{m-3}
    int toff;         // first projected-column slot of this prefix
    unsigned lo;      // first pair (in the prefix's pair order) inside the call's rank range
    float ratio;      // FP32-bulk: capped pivot-ratio product of the m-2 prefix steps
    unsigned w[4];    // packed prefix columns (FP32-bulk deferral entries)
    int pad[2];
};
static_assert(sizeof(SlotHdr) == 48, "slot header size");

template <int M, bool F32> __host__ __device__ int shared_common_bytes(int n) {
    int b = binom_bytes<M>(n) + align16(n * Layout<M>::st64 * 8);
    if (F32) b += align16(n * Layout<M>::st32 * 4);
    return b;
}

template <int M, bool F32> __host__ __device__ int shared_wave_bytes(int n, int cap) {
    return wave_copy_bytes<M, F32>(n) + kPrefixBlock * (int)sizeof(SlotHdr) + kPrefixBlock * 4 +
           align16(cap * 2 * (F32 ? 4 : 8));
}

template <int M, bool F32> __host__ __device__ int shared_lds_bytes(int n, int waves, int cap) {
    return shared_common_bytes<M, F32>(n) + waves * shared_wave_bytes<M, F32>(n, cap);
}

// m x P block of the prefix columns, rows in the order of the LDS copy.
template <int M, int P, typename T>
__device__ __forceinline__ void gather_prefix(T (&a)[M][P], const T* base, int stride, const int (&col)[P]) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const T* src = base + col[j] * stride;
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int i = 0; i + 1 < M; i += 2) {
                const double2 v = *reinterpret_cast<const double2*>(src + i);
                a[i][j] = v.x;
                a[i + 1][j] = v.y;
            }
            if (M & 1) a[M - 1][j] = src[M - 1];
        } else {
#pragma unroll
            for (int i = 0; i + 3 < M; i += 4) {
                const float4 v = *reinterpret_cast<const float4*>(src + i);
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

// The two values left in rows m-2, m-1 after the prefix's elimination steps,
// for one column of the copy: with the lane's rows read in the lane's order
// (copy row off[i] at position i), t_q = x_{m-2+q} + sum_{i<m-2} z_q[i] x_i,
// z_q the rows m-2+q of -L21 L11^{-1}.
template <int M, int P, typename T>
__device__ __forceinline__ void project(const T (&z0)[P], const T (&z1)[P], const int (&off)[M], const T* src,
                                        T& t0, T& t1) {
    T x[M];
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] = src[off[i]];
    T s0 = x[P], s1 = x[P + 1];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        s0 = fma_t(z0[i], x[i], s0);
        s1 = fma_t(z1[i], x[i], s1);
    }
    t0 = s0;
    t1 = s1;
}

// Step K of LU with partial pivoting on the m x P prefix block, multipliers
// stored below the diagonal (whole rows exchanged, so that P A = L U).  `rel`
// tracks the lane's row order relative to the copy (4 bits per position);
// exchanges made by every lane alike are also recorded in the wave's order
// `perm` for later rounds, as in the per-minor kernel.
template <int M, int P, int K, typename T, bool CHECK>
__device__ __forceinline__ void prefix_steps(T (&a)[M][P], double& prod, bool& neg, float& ratio, const T (&s)[P],
                                             unsigned long long& perm, int& perm_odd, unsigned long long& rel) {
    if constexpr (K < P) {
        unsigned best = pivot_key(a[K][K], K);
#pragma unroll
        for (int i = K + 1; i < M; ++i) best = max(best, pivot_key(a[i][K], i));
        const int p = pivot_row(best);
        neg ^= (p != K);
        if (__ballot(p != K)) {
            const unsigned long long x = ((rel >> (4 * K)) ^ (rel >> (4 * p))) & 15ull;
            rel ^= (x << (4 * K)) | (x << (4 * p));
        }
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
                for (int j = 0; j < P; ++j) {
                    const T x = a[K][j], y = a[i][j];
                    a[K][j] = c ? y : x;
                    a[i][j] = c ? x : y;
                }
            }
        }
        const T piv = a[K][K];
        if (CHECK) ratio *= __saturatef(__builtin_fabsf((float)piv) * (float)s[K]);
        prod *= (double)piv;
        const T rp = piv == T(0) ? T(0) : recip(piv);   // a zero pivot column: every minor is 0
#pragma unroll
        for (int i = K + 1; i < M; ++i) {
            const T l = a[i][K] * rp;
            a[i][K] = l;
#pragma unroll
            for (int j = K + 1; j < P; ++j) a[i][j] = fma_t(-l, a[K][j], a[i][j]);
        }
        prefix_steps<M, P, K + 1, T, CHECK>(a, prod, neg, ratio, s, perm, perm_odd, rel);
    }
}

template <int M, bool F32>
__global__ __launch_bounds__(kMaxBlock) void k_radic_shared(FloatJob J) {
    using T = typename std::conditional<F32, float, double>::type;
    using T2 = typename std::conditional<F32, float2, double2>::type;
    constexpr int P = M - 2;
    constexpr int ST64 = Layout<M>::st64, ST32 = Layout<M>::st32;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rowexp[RADIC_MAX_M];
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];

    const int n = J.n;
    const int waves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int colstride = F32 ? ST32 : ST64;

    unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
    double* cd = reinterpret_cast<double*>(smem + binom_bytes<M>(n));
    float* cf = reinterpret_cast<float*>(smem + binom_bytes<M>(n) + align16(n * ST64 * 8));
    unsigned char* wr = smem + shared_common_bytes<M, F32>(n) + wave * shared_wave_bytes<M, F32>(n, J.cap);
    T* wcopy = reinterpret_cast<T*>(wr);
    SlotHdr* hdr = reinterpret_cast<SlotHdr*>(wr + wave_copy_bytes<M, F32>(n));
    unsigned* incl = reinterpret_cast<unsigned*>(wr + wave_copy_bytes<M, F32>(n) + kPrefixBlock * sizeof(SlotHdr));
    T2* tv = reinterpret_cast<T2*>(wr + wave_copy_bytes<M, F32>(n) + kPrefixBlock * sizeof(SlotHdr) +
                                   kPrefixBlock * 4);

    stage_binomials<M>(bt, n);
    const int bad = stage_matrix<M, F32>(J, cd, cf, rowexp);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.header->nonfinite = bad;
        int se = 0;
        if (F32)
            for (int i = 0; i < M; ++i) se += rowexp[i];
        J.header->scale_exp = se;
    }

    const T* master = F32 ? reinterpret_cast<const T*>(cf) : reinterpret_cast<const T*>(cd);
    const T tau = (T)J.tau;
    unsigned long long perm = 0;
#pragma unroll
    for (int r = 0; r < M; ++r) perm |= (unsigned long long)r << (4 * r);
    int perm_odd = 0;
    write_wave_copy<M, T>(wcopy, master, colstride, n, perm, lane, F32);

    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    int gcount = 0;          // wave-uniform number of flagged minors (FP32-bulk)
    bool overflow = false;   // wave-uniform: more flagged minors than the segment holds
    const unsigned long long qend = J.q_begin + J.count;
    const unsigned long long nblk = (J.p_end - J.p_begin + kPrefixBlock - 1) / kPrefixBlock;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const unsigned long long nwaves = (unsigned long long)gridDim.x * waves;

    for (unsigned long long blk = gwave; blk < nblk && !overflow; blk += nwaves) {
        unsigned long long next = J.p_begin + blk * kPrefixBlock;
        const unsigned long long pe = next + kPrefixBlock;
        const unsigned long long pi1 = pe < J.p_end ? pe : J.p_end;
        unsigned long long rbase = first_completion_rank<M>(next, J, bt);
        while (next < pi1 && !overflow) {
            // ---------------- the round's prefixes: lane l takes prefix next + l
            const unsigned long long pi = next + lane;
            const bool have = pi < pi1;
            int c[P];
            unrank_strided<P>(have ? pi : next, n - 2, bt, M, c);
            const int r = n - 1 - c[P - 1];
            // projected-column slots: lanes take prefixes while the slots last
            // (lane 0 always fits: cap >= n - m + 2 >= r)
            const unsigned rs = wave_scan_u32(have ? (unsigned)r : 0u, lane);
            const bool take = have && rs <= (unsigned)J.cap;
            const int ntake = __popcll(__ballot(take));
            const unsigned cnt = take ? (unsigned)(r * (r - 1) / 2) : 0u;
            const unsigned cincl = wave_scan_u32(cnt, lane);
            const unsigned round_total = __shfl(cincl, kWave - 1, kWave);
            const unsigned long long base = rbase + (cincl - cnt);
            // the prefix's pairs inside [q_begin, q_begin + count)
            unsigned lo_c = 0, hi_c = cnt;
            if (base < J.q_begin) {
                const unsigned long long d = J.q_begin - base;
                lo_c = d < cnt ? (unsigned)d : cnt;
            }
            if (base + cnt > qend) {
                const unsigned long long d = qend > base ? qend - base : 0ull;
                hi_c = d < cnt ? (unsigned)d : cnt;
            }
            if (hi_c < lo_c) hi_c = lo_c;
            const unsigned cc = hi_c - lo_c;
            const unsigned ccincl = wave_scan_u32(cc, lane);
            const unsigned Tr = __shfl(ccincl, kWave - 1, kWave);

            // ---------------- phase A: the prefix's m-2 elimination steps
            const int perm_odd_round = perm_odd;
            const unsigned long long perm_round = perm;
            {
                T a[M][P];
                gather_prefix<M, P, T>(a, wcopy, colstride, c);
                T sc[P];
#pragma unroll
                for (int k = 0; k < P; ++k) sc[k] = F32 ? wcopy[c[k] * colstride + M] : T(0);
                unsigned long long rel = 0;
#pragma unroll
                for (int q = 0; q < M; ++q) rel |= (unsigned long long)q << (4 * q);
                double prod = 1.0;
                bool neg = false;
                float ratio = 1.0f;
                prefix_steps<M, P, 0, T, F32>(a, prod, neg, ratio, sc, perm, perm_odd, rel);
                // z_t = -l_{m-2+t} L11^{-1}: rows m-2, m-1 of L^{-1} in the lane's row order
                T z0[P], z1[P];
#pragma unroll
                for (int k = P - 1; k >= 0; --k) {
                    T s0 = -a[P][k], s1 = -a[P + 1][k];
#pragma unroll
                    for (int i = k + 1; i < P; ++i) {
                        s0 = fma_t(-z0[i], a[i][k], s0);
                        s1 = fma_t(-z1[i], a[i][k], s1);
                    }
                    z0[k] = s0;
                    z1[k] = s1;
                }
                // the lane's row order: position i holds copy row rel_i
                int off[M];
#pragma unroll
                for (int i = 0; i < M; ++i) off[i] = (int)((rel >> (4 * i)) & 15ull);
                // sign: row order (lane exchanges, copy order) and the prefix's share of (-1)^(r+s)
                int ps = M * (M + 1) / 2 + P;
#pragma unroll
                for (int k = 0; k < P; ++k) ps += c[k];
                const bool sg = neg ^ (perm_odd_round != 0) ^ ((ps & 1) != 0);
                const int toff = (int)rs - r;
                if (take) {
                    SlotHdr h;
                    h.prodS = sg ? -prod : prod;
                    h.r = r;
                    h.toff = toff;
                    h.lo = lo_c;
                    h.ratio = ratio;
                    h.w[0] = h.w[1] = h.w[2] = h.w[3] = 0u;
#pragma unroll
                    for (int k = 0; k < P; ++k) h.w[k / 3] |= (unsigned)c[k] << (kColBits * (k % 3));
                    h.pad[0] = h.pad[1] = 0;
                    hdr[lane] = h;
                    incl[lane] = ccincl;
                }
                int rmax = take ? r : 0;
#pragma unroll
                for (int off = kWave / 2; off > 0; off >>= 1) rmax = max(rmax, __shfl_xor(rmax, off, kWave));
                for (int j = 0; j < rmax; ++j) {
                    const int col = min(c[P - 1] + 1 + j, n - 1);
                    T t0, t1;
                    project<M, P, T>(z0, z1, off, wcopy + col * colstride, t0, t1);
                    if (take && j < r) {
                        T2 v;
                        v.x = t0;
                        v.y = t1;
                        tv[toff + j] = v;
                    }
                }
            }
            wave_lds_sync();
            if (perm != perm_round) write_wave_copy<M, T>(wcopy, master, colstride, n, perm, lane, false);

            // ---------------- phase B: the round's minors, split evenly over the lanes
            const unsigned chunk = (Tr + kWave - 1) / kWave;
            if (chunk > 0) {
                const unsigned g0 = (unsigned)lane * chunk;
                const unsigned gend = min(g0 + chunk, Tr);
                const bool active = g0 < Tr;
                int s = 0;
                {
                    int l2 = 0, h2 = ntake - 1;
                    while (l2 < h2) {
                        const int mid = (l2 + h2) >> 1;
                        if (incl[mid] > g0) h2 = mid;
                        else l2 = mid + 1;
                    }
                    s = active ? l2 : 0;
                }
                SlotHdr h = hdr[s];
                int ia = 0, ib = 1;
                if (active) {
                    const unsigned excl = s > 0 ? incl[s - 1] : 0u;
                    unrank_pair(g0 - excl + h.lo, h.r, ia, ib);
                }
                T2 ta = tv[h.toff + ia];
                for (unsigned k = 0; k < chunk; ++k) {
                    const bool valid = g0 + k < gend;
                    const T2 tb = tv[h.toff + ib];
                    const T d = fma_t(ta.x, tb.y, -(ta.y * tb.x));
                    double term = (double)d * h.prodS;
                    if ((ia + ib) & 1) term = -term;
                    bool flag = false;
                    if (F32) {
                        // last two pivots of the minor: max(|t_a|) and det / that pivot
                        const int ca = n - h.r + ia, cb = n - h.r + ib;
                        const float pa = fmaxf(fabsf((float)ta.x), fabsf((float)ta.y));
                        const float sa = cf[ca * ST32 + M], sb = cf[cb * ST32 + M];
                        const float q = pa > 0.f ? fabsf((float)d) * __builtin_amdgcn_rcpf(pa) : 0.f;
                        const float rt = h.ratio * __saturatef(pa * sa) * __saturatef(q * sb);
                        flag = valid && !(rt >= (float)tau);
                        const unsigned long long fm = __ballot(flag);
                        if (fm) {
                            const int pos = gcount + (int)__builtin_amdgcn_mbcnt_hi(
                                                         (unsigned)(fm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                            if (flag && pos < J.defer_cap) {
                                unsigned w[4] = {h.w[0], h.w[1], h.w[2], h.w[3]};
                                w[P / 3] |= (unsigned)ca << (kColBits * (P % 3));
                                w[(P + 1) / 3] |= (unsigned)cb << (kColBits * ((P + 1) % 3));
                                unsigned* ent = J.fb_entries + ((size_t)gwave * J.defer_cap + pos) * 4;
                                ent[0] = w[0];
                                ent[1] = w[1];
                                ent[2] = w[2];
                                ent[3] = w[3];
                                nfb += 1;
                            }
                            gcount += __popcll(fm);
                            if (gcount > J.defer_cap) {
                                overflow = true;
                                break;
                            }
                        }
                    }
                    if (valid && !flag) {
                        double sum, err;
                        two_sum(hi, term, sum, err);
                        hi = sum;
                        lo += err;
                        ab += fabs(term);
                    }
                    // next pair; past the prefix's last pair, the next prefix
                    if (++ib >= h.r) {
                        ++ia;
                        ib = ia + 1;
                        if (ib >= h.r) {
                            s = min(s + 1, ntake - 1);
                            h = hdr[s];
                            ia = 0;
                            ib = 1;
                        }
                        ta = tv[h.toff + ia];
                    }
                }
            }
            rbase += round_total;
            next += (unsigned long long)ntake;
            wave_lds_sync();
        }
    }
    if (F32 && lane == 0) J.fb_count[gwave] = (unsigned)gcount;   // above J.defer_cap: overflowed

    wave_reduce_partial(hi, lo, ab, nfb);
    if (lane == 0) {
        red[4 * wave + 0] = hi;
        red[4 * wave + 1] = lo;
        red[4 * wave + 2] = ab;
        redn[wave] = nfb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double h = red[0], l = red[1], a2 = red[2];
        unsigned long long nf = redn[0];
        for (int w = 1; w < waves; ++w) {
            dd_add(h, l, red[4 * w + 0], red[4 * w + 1]);
            a2 += red[4 * w + 2];
            nf += redn[w];
        }
        J.partials[blockIdx.x] = Partial{h, l, a2, nf};
    }
}

// ---------------------------------------------------------------- host side
hipError_t upload_binomials_shared(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

int shared_lds(int m, int n, int prec, int waves, int cap) {
    switch (m) {
#define RADIC_CASE(MM)                                                                            \
    case MM:                                                                                      \
        return prec == RADIC_FP32_BULK ? shared_lds_bytes<MM, true>(n, waves, cap)                \
                                       : shared_lds_bytes<MM, false>(n, waves, cap);
        RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return 1 << 30;
    }
}

hipError_t launch_shared(int m, int prec, const FloatJob& J, int grid, int block, hipStream_t s) {
    const int lds = shared_lds(m, J.n, prec, block / kWave, J.cap);
    (void)hipGetLastError();
    switch (m) {
#define RADIC_CASE(MM)                                                                                  \
    case MM:                                                                                            \
        if (prec == RADIC_FP32_BULK)                                                                    \
            hipLaunchKernelGGL((k_radic_shared<MM, true>), dim3(grid), dim3(block), lds, s, J);         \
        else                                                                                            \
            hipLaunchKernelGGL((k_radic_shared<MM, false>), dim3(grid), dim3(block), lds, s, J);        \
        break;
        RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace radic
