// Group-shared floating-point Radic kernels (4 <= m <= 12) for gfx950.
//
// The prefix-shared kernel lets the minors with equal first m-2 columns share
// the first m-2 steps of their LU with partial pivoting.  This kernel shares one
// step fewer among many more minors: every minor with the same first m-3
// columns (a group) is consecutive in the dictionary order (Section 3), and GEPP
// of all of them performs the same first m-3 steps.  What is left of a minor is
// a 3 x 3 block.  With W the rows m-3, m-2, m-1 of L^{-1} P and u_c = W x_c,
//   det(A_J) = (signed pivot product) * det([u_a, u_b, u_c])
//            = (signed pivot product) * u_c . (u_a x u_b).
// The cross product is formed once per pair (a, b); each minor then costs one
// dot product.  The 3 x 3 determinant is taken without further pivoting: the
// pivot choice on the block changes only the bookkeeping of its value.
//
// A wave takes a block of kGroupBlock consecutive groups and works in rounds:
//  A. Lanes 0 .. kGroupBlock-1 each factor one group's m x (m-3) block (the
//     left-looking LU with the multipliers only) and form W.
//  P. The round's later columns (r per group) are split evenly over the 64
//     lanes; a lane fetches W of the group owning its column from the owner lane
//     and writes (-1)^j u_c to the wave's LDS.
//  B. The round's minors (the triples a < b < c after each group's columns, in
//     dictionary order) are split evenly over the 64 lanes; the signed term
//     (-1)^(r+s) det(A_J) of eq. (1) is added by TwoSum.
//
// FP32-bulk: the capped pivot-ratio product of a minor is the group's product
// times the factors of the three pivots partial pivoting takes on the 3 x 3
// block: p1 = max|u_a| (row i), p1 p2 = the largest 2 x 2 minor of [u_a u_b]
// through row i, p1 p2 p3 = |det|.  The test rho < tau becomes a threshold on
// |det| s_c fixed per pair (a, b).  Flagged minors are queued for the double
// refactorisation kernel as in the other float kernels.
#include <type_traits>

#include "shared_lu.h"

namespace radic {

// A projected-column slot: u_c, and for FP32-bulk the column's reciprocal scale.
template <bool F32> struct Slot3;
template <> struct alignas(16) Slot3<false> {
    double u0, u1, u2, pad;
};
template <> struct alignas(16) Slot3<true> {
    float u0, u1, u2, s;
};

template <int M, bool F32> __host__ __device__ int shared3_wave_bytes(int cap) {
    return kHdrBytes + kScanBytes + (F32 ? kF32Extra : 0) + cap * (int)sizeof(Slot3<F32>);
}

template <int M, bool F32> __host__ __device__ int shared3_lds_bytes(int n, int waves, int cap) {
    return shared_common_bytes<M, F32>(n) + waves * shared3_wave_bytes<M, F32>(cap);
}

// The three values left in rows m-3 .. m-1 after the group's elimination steps,
// for one column read in the lane's row order (row off[i] at position i):
// u_q = x_{m-3+q} + sum_{i<m-3} z_q[i] x_i, z_q the rows m-3+q of -L21 L11^{-1}.
template <int M, int P, typename T>
__device__ __forceinline__ void project3(const T (&z0)[P], const T (&z1)[P], const T (&z2)[P], const int (&off)[M],
                                         const T* src, T& t0, T& t1, T& t2) {
    T x[M];
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] = src[off[i]];
    T s0 = x[P], s1 = x[P + 1], s2 = x[P + 2];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        s0 = fma_t(z0[i], x[i], s0);
        s1 = fma_t(z1[i], x[i], s1);
        s2 = fma_t(z2[i], x[i], s2);
    }
    t0 = s0;
    t1 = s1;
    t2 = s2;
}

template <int M, bool F32>
__global__ __launch_bounds__(kMaxBlock) void k_radic_shared3(FloatJob J) {
    using T = typename std::conditional<F32, float, double>::type;
    using SV = Slot3<F32>;
    constexpr int P = M - 3;
    constexpr int S64 = SharedLayout<M>::s64, S32 = SharedLayout<M>::s32;
    constexpr int ST = F32 ? S32 : S64;
    constexpr int BS = M + 1;   // stride of the LDS binomial slice
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rowexp[RADIC_MAX_M];
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];
    __shared__ unsigned segn[16];   // FP32-bulk: flagged minors per wave

    const int n = J.n;
    const int waves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;

    unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
    double* cd = reinterpret_cast<double*>(smem + binom_bytes<BS>(n));
    float* cf = reinterpret_cast<float*>(smem + binom_bytes<BS>(n) + align16(n * S64 * 8));
    unsigned char* wr = smem + shared_common_bytes<M, F32>(n) + wave * shared3_wave_bytes<M, F32>(J.cap);
    PairHdr* hdr = reinterpret_cast<PairHdr*>(wr);
    unsigned* incl = reinterpret_cast<unsigned*>(wr + kHdrBytes);   // minors, inclusive scan over the lanes
    unsigned* cincl = incl + kPrefixBlock;                           // columns, inclusive scan
    float* ratios = reinterpret_cast<float*>(wr + kHdrBytes + kScanBytes);
    uint4* wcols = reinterpret_cast<uint4*>(wr + kHdrBytes + kScanBytes + kPrefixBlock * 4);
    SV* tv = reinterpret_cast<SV*>(wr + kHdrBytes + kScanBytes + (F32 ? kF32Extra : 0));

    stage_binomials<BS>(bt, n);
    const int bad = stage_matrix<M, F32, F32, S64, S32>(J, cd, cf, rowexp);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.header->nonfinite = bad;
        int se = 0;
        if (F32)
            for (int i = 0; i < M; ++i) se += rowexp[i];
        J.header->scale_exp = se;
    }

    const T* src = F32 ? reinterpret_cast<const T*>(cf) : reinterpret_cast<const T*>(cd);
    const float tau = (float)J.tau;
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    int gcount = 0;          // wave-uniform number of flagged minors (FP32-bulk)
    bool overflow = false;   // wave-uniform: more flagged minors than the segment holds
    const unsigned long long qend = J.q_begin + J.count;
    const unsigned long long nblk = (J.p_end - J.p_begin + kGroupBlock - 1) / kGroupBlock;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const unsigned long long nwaves = (unsigned long long)gridDim.x * waves;

    for (unsigned long long blk = gwave; blk < nblk && !overflow; blk += nwaves) {
        unsigned long long next = J.p_begin + blk * kGroupBlock;
        const unsigned long long pe = next + kGroupBlock;
        const unsigned long long pi1 = pe < J.p_end ? pe : J.p_end;
        while (next < pi1 && !overflow) {
            // ---------------- the round's groups: lane l < kGroupBlock takes group next + l
            const unsigned long long pi = next + lane;
            const bool have = lane < kGroupBlock && pi < pi1;
            int c[P];
            unrank_prefix<P>(have ? pi : next, n - 1, J.n_prefix, bt, BS, c);
            const int r = n - 1 - c[P - 1];   // columns after the group's, >= 3
            // dictionary rank of the group's first sequence (c, c+1, c+2, c+3)
            // (c = c_{m-4}): the sequences after it number sum_k C(n-1-c_k, m-k)
            unsigned long long after = bt[(r - 1) * BS + 3] + bt[(r - 2) * BS + 2] + bt[(r - 3) * BS + 1];
#pragma unroll
            for (int k = 0; k < P; ++k) after += bt[(n - 1 - c[k]) * BS + (M - k)];
            const unsigned long long base = J.total - 1 - after;
            // projected-column slots: lanes take groups while the slots last
            // (lane 0 always fits: cap >= n - m + 3 >= r)
            const unsigned rs = wave_scan_u32(have ? (unsigned)r : 0u, lane);
            const bool take = have && rs <= (unsigned)J.cap;
            const int ntake = __popcll(__ballot(take));
            const unsigned ncols = __shfl(rs, ntake - 1, kWave);
            const unsigned cnt = take ? (unsigned)r * (unsigned)(r - 1) * (unsigned)(r - 2) / 6u : 0u;
            // the group's minors inside [q_begin, q_begin + count)
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

            // ---------------- phase A: the group's m-3 elimination steps
            T pz0[P], pz1[P], pz2[P];   // the group's projection rows, kept for the exchange below
            unsigned long long prel;     // and its row order
            {
                T L[M][P];
                unsigned long long rel = 0;
#pragma unroll
                for (int q = 0; q < M; ++q) rel |= (unsigned long long)q << (4 * q);
                double prod = 1.0;
                bool neg = false;
                float ratio = 1.0f;
                left_steps<M, P, 0, T, F32>(L, src, ST, c, prod, neg, ratio, rel);
                // z_t = -l_{m-3+t} L11^{-1}: rows m-3 .. m-1 of L^{-1} in the lane's row order
#pragma unroll
                for (int k = P - 1; k >= 0; --k) {
                    T s0 = -L[P][k], s1 = -L[P + 1][k], s2 = -L[P + 2][k];
#pragma unroll
                    for (int i = k + 1; i < P; ++i) {
                        s0 = fma_t(-pz0[i], L[i][k], s0);
                        s1 = fma_t(-pz1[i], L[i][k], s1);
                        s2 = fma_t(-pz2[i], L[i][k], s2);
                    }
                    pz0[k] = s0;
                    pz1[k] = s1;
                    pz2[k] = s2;
                }
                prel = rel;
                // sign: the lane's exchanges and the group's share of (-1)^(r+s); the
                // three later columns add 3 (n - r) + 3 + (their offsets), the
                // offsets carried by the stored columns
                int ps = M * (M + 1) / 2 + P + 1 + (n - r);
#pragma unroll
                for (int k = 0; k < P; ++k) ps += c[k];
                const bool sg = neg ^ ((ps & 1) != 0);
                if (take) {
                    PairHdr h;
                    h.prodS = sg ? -prod : prod;
                    h.lo = lo_c;
                    h.rt = (unsigned)r | ((rs - (unsigned)r) << kRBits);
                    hdr[lane] = h;
                    incl[lane] = ccincl;
                    cincl[lane] = rs;
                    if (F32) {
                        ratios[lane] = ratio;
                        uint4 w = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            const unsigned v = (unsigned)c[k] << (kColBits * (k % 3));
                            if (k / 3 == 0) w.x |= v;
                            else if (k / 3 == 1) w.y |= v;
                            else w.z |= v;
                        }
                        wcols[lane] = w;
                    }
                }
            }
            wave_lds_sync();

            // ---------------- projection: the round's columns split evenly over the lanes
            {
                // runs of an odd number of columns start the lanes on different LDS banks
                const unsigned per = ((ncols + kWave - 1) / kWave) | 1u;
                const unsigned g0 = (unsigned)lane * per;
                const unsigned g1 = min(g0 + per, ncols);
                // group owning column g0: the first s with cincl[s] > g0 (the last
                // taken group for a lane without columns)
                int s = ntake - 1;
                if (g0 < ncols) {
                    int l2 = 0, h2 = ntake - 1;
                    while (l2 < h2) {
                        const int mid = (l2 + h2) >> 1;
                        if (cincl[mid] > g0) h2 = mid;
                        else l2 = mid + 1;
                    }
                    s = l2;
                }
                unsigned send = cincl[s];
                unsigned sbeg = s > 0 ? cincl[s - 1] : 0u;
                T z0[P], z1[P], z2[P];
                int off[M];
                // the projection rows of group s, from its owner lane (every lane
                // takes part in the exchange)
                auto fetch = [&]() {
#pragma unroll
                    for (int i = 0; i < P; ++i) {
                        z0[i] = __shfl(pz0[i], s, kWave);
                        z1[i] = __shfl(pz1[i], s, kWave);
                        z2[i] = __shfl(pz2[i], s, kWave);
                    }
                    const unsigned long long rl = __shfl(prel, s, kWave);
#pragma unroll
                    for (int i = 0; i < M; ++i) off[i] = (int)((rl >> (4 * i)) & 15ull);
                };
                fetch();
                for (unsigned it = 0; it < per; ++it) {
                    const unsigned g = g0 + it;
                    const bool act = g < g1;
                    const bool cross = act && g >= send;
                    if (__ballot(cross)) {
                        if (cross) {
                            ++s;
                            sbeg = send;
                            send = cincl[s];
                        }
                        fetch();
                    }
                    if (act) {
                        // slot g holds column c_{m-4} + 1 + (g - sbeg) = n - send + g
                        const T* colp = src + (n - (int)send + (int)g) * ST;
                        T t0, t1, t2;
                        project3<M, P, T>(z0, z1, z2, off, colp, t0, t1, t2);
                        // (-1)^j folded in for the j-th column after the group's
                        if ((g - sbeg) & 1u) {
                            t0 = -t0;
                            t1 = -t1;
                            t2 = -t2;
                        }
                        SV v;
                        v.u0 = t0;
                        v.u1 = t1;
                        v.u2 = t2;
                        if constexpr (F32) v.s = colp[M];   // reciprocal column scale
                        else v.pad = 0.0;
                        tv[g] = v;
                    }
                }
            }
            wave_lds_sync();

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
                PairHdr h = hdr[s];
                int hr = (int)(h.rt & kRMask), toff = (int)(h.rt >> kRBits);
                float hratio = F32 ? ratios[s] : 1.0f;
                // the lane's first triple: its number inside the group's C(r, 3)
                // triples, unranked like a prefix of three columns out of r + 2
                int ia = 0, ib = 1, ic = 2;
                if (active) {
                    const unsigned excl = s > 0 ? incl[s - 1] : 0u;
                    int t3[3];
                    unrank_prefix<3>(g0 - excl + h.lo, hr + 2, bt[hr * BS + 3], bt, BS, t3);
                    ia = t3[0];
                    ib = t3[1];
                    ic = t3[2];
                }
                const unsigned kend = active ? gend - g0 : 0u;
                SV ua = tv[toff + ia], ub = tv[toff + ib];
                T w0, w1, w2;
                float thr = 0.f;
                // the pair (a, b): u_a x u_b, and for FP32-bulk the threshold on
                // |det| s_c: rho = h * min(|det| s_c / (p1 p2), 1) with
                // h = (group ratios) * min(p1 s_a, 1) * min(p2 s_b, 1)
                auto pair = [&]() {
                    w0 = fma_t(ua.u1, ub.u2, -(ua.u2 * ub.u1));
                    w1 = fma_t(ua.u2, ub.u0, -(ua.u0 * ub.u2));
                    w2 = fma_t(ua.u0, ub.u1, -(ua.u1 * ub.u0));
                    if constexpr (F32) {
                        const float a0 = fabsf(ua.u0), a1 = fabsf(ua.u1), a2 = fabsf(ua.u2);
                        const float p1 = fmaxf(a0, fmaxf(a1, a2));
                        // partial pivoting takes the first row holding p1; the 2 x 2
                        // minors through it are the other two components of u_a x u_b
                        const float p12 = a0 == p1 ? fmaxf(fabsf(w1), fabsf(w2))
                                                   : (a1 == p1 ? fmaxf(fabsf(w0), fabsf(w2))
                                                               : fmaxf(fabsf(w0), fabsf(w1)));
                        const float q2 = p1 > 0.f ? p12 * __builtin_amdgcn_rcpf(p1) * ub.s : 0.f;
                        const float h2 = hratio * fminf(p1 * ua.s, 1.f) * fminf(q2, 1.f);
                        thr = !(h2 >= tau) ? __builtin_inff() : (tau > 0.f ? tau * p12 * __builtin_amdgcn_rcpf(h2) : 0.f);
                    }
                };
                pair();
                for (unsigned k = 0; k < chunk; ++k) {
                    const bool valid = k < kend;
                    const SV uc = tv[toff + ic];
                    // det([u_a u_b u_c]) = u_c . (u_a x u_b); (-1)^(a+b+c) is carried by the columns
                    const T d = fma_t(w2, uc.u2, fma_t(w1, uc.u1, w0 * uc.u0));
                    bool keep = valid;
                    if constexpr (F32) {
                        const bool flag = valid && (fabsf(d) * uc.s < thr);
                        keep = valid && !flag;
                        const unsigned long long fm = __ballot(flag);
                        if (fm) {
                            const int pos = gcount + (int)__builtin_amdgcn_mbcnt_hi(
                                                         (unsigned)(fm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                            if (flag && pos < J.defer_cap) {
                                const int base_c = n - hr;
                                const uint4 pw = wcols[s];
                                unsigned w[4] = {pw.x, pw.y, pw.z, pw.w};
                                w[P / 3] |= (unsigned)(base_c + ia) << (kColBits * (P % 3));
                                w[(P + 1) / 3] |= (unsigned)(base_c + ib) << (kColBits * ((P + 1) % 3));
                                w[(P + 2) / 3] |= (unsigned)(base_c + ic) << (kColBits * ((P + 2) % 3));
                                unsigned* ent = J.fb_entries + ((size_t)gwave * J.defer_cap + pos) * 4;
                                ent[0] = w[0];
                                ent[1] = w[1];
                                ent[2] = w[2];
                                ent[3] = w[3];
                                nfb += 1;
                            }
                            gcount += __popcll(fm);
                        }
                    }
                    // a minor outside the lane's share, or queued, adds an exact 0
                    const double term = keep ? (double)d * h.prodS : 0.0;
                    double sum, err;
                    two_sum(hi, term, sum, err);
                    hi = sum;
                    lo += err;
                    ab += fabs(term);
                    // next triple: c, then b, then a, then the next group
                    if (++ic >= hr) {
                        if (++ib >= hr - 1) {
                            if (++ia >= hr - 2) {
                                s = min(s + 1, ntake - 1);
                                h = hdr[s];
                                hr = (int)(h.rt & kRMask);
                                toff = (int)(h.rt >> kRBits);
                                if (F32) hratio = ratios[s];
                                ia = 0;
                            }
                            ib = ia + 1;
                            ua = tv[toff + ia];
                        }
                        ic = ib + 1;
                        ub = tv[toff + ib];
                        pair();
                    }
                }
            }
            // a full segment: the workgroup is redone in double by the
            // refactorisation kernel, so the rest is not needed
            if (F32 && gcount > J.defer_cap) overflow = true;
            next += (unsigned long long)ntake;
            wave_lds_sync();
            if constexpr (F32 && shared_tail_refactor(M)) {
                if (!overflow) relieve_segment<M, S64>(J, cd, gwave, gcount, lane, hi, lo, ab);
            }
        }
    }
    if constexpr (F32 && shared_tail_refactor(M)) {
        shared_fp32_tail<M, 3, kGroupBlock, BS, S64>(J, bt, cd, gcount, gwave, nwaves, nblk, segn, hi, lo, ab, nfb);
    } else if (F32 && lane == 0) {
        J.fb_count[gwave] = (unsigned)gcount;   // above J.defer_cap: overflowed
    }

    wave_reduce_partial(hi, lo, ab, nfb);
    if (lane == 0) {
        red[4 * wave + 0] = hi;
        red[4 * wave + 1] = lo;
        red[4 * wave + 2] = ab;
        redn[wave] = nfb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double h2 = red[0], l2 = red[1], a2 = red[2];
        unsigned long long nf = redn[0];
        for (int w = 1; w < waves; ++w) {
            dd_add(h2, l2, red[4 * w + 0], red[4 * w + 1]);
            a2 += red[4 * w + 2];
            nf += redn[w];
        }
        J.partials[blockIdx.x] = Partial{h2, l2, a2, nf};
    }
}

// ---------------------------------------------------------------- host side
hipError_t upload_binomials_shared3(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

int shared3_lds(int m, int n, int prec, int waves, int cap) {
    switch (m) {
#define RADIC_CASE(MM)                                                                            \
    case MM:                                                                                      \
        return prec == RADIC_FP32_BULK ? shared3_lds_bytes<MM, true>(n, waves, cap)               \
                                       : shared3_lds_bytes<MM, false>(n, waves, cap);
        RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return 1 << 30;
    }
}

int shared3_slot_bytes(int prec) { return prec == RADIC_FP32_BULK ? (int)sizeof(Slot3<true>) : (int)sizeof(Slot3<false>); }

template <int M, bool F32>
static hipError_t launch_shared3_m(const FloatJob& J, int grid, int block, int lds, hipStream_t s) {
    // beyond 64 KiB of dynamic LDS the kernel has to be allowed it first
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_radic_shared3<M, F32>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return launch_timed(k_radic_shared3<M, F32>, dim3(grid), dim3(block), lds, s, J);
}

hipError_t launch_shared3(int m, int prec, const FloatJob& J, int grid, int block, hipStream_t s) {
    const int lds = shared3_lds(m, J.n, prec, block / kWave, J.cap);
    switch (m) {
#define RADIC_CASE(MM)                                                                              \
    case MM:                                                                                        \
        return prec == RADIC_FP32_BULK ? launch_shared3_m<MM, true>(J, grid, block, lds, s)         \
                                       : launch_shared3_m<MM, false>(J, grid, block, lds, s);
        RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace radic
