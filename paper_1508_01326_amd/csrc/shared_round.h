// The round of a prefix-shared floating-point wave (phases A, P and B of the
// prefix-shared kernels: the prefixes' elimination steps, the projection of their
// later columns, the minors' 2 x 2 determinants), shared by the single-matrix
// kernel and the batched float chunks.
#pragma once

#include <type_traits>

#include "shared_lu.h"

namespace radic {

// A projected-column slot is 16 bytes: (t0, t1) in double, or in float with the
// FP32-bulk conditioning threshold of the minors whose first later column it is
// and the column's reciprocal scale.
constexpr int kSlotBytes = 16;

template <int M, bool F32> __host__ __device__ int shared_wave_bytes(int cap) {
    return kHdrBytes + kScanBytes + (F32 ? kF32Extra : 0) + cap * kSlotBytes;
}

template <int M, bool F32> __host__ __device__ int shared_lds_bytes(int n, int waves, int cap) {
    return shared_common_bytes<M, F32>(n) + waves * shared_wave_bytes<M, F32>(cap);
}

// The two values left in rows m-2, m-1 after the prefix's elimination steps,
// for one column: with the lane's rows read in the lane's order (row off[i] at
// position i), t_q = x_{m-2+q} + sum_{i<m-2} z_q[i] x_i, z_q the rows m-2+q of
// -L21 L11^{-1}.
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

// The wave's LDS records of a round: per prefix its header (PairHdr) and the
// two inclusive scans over the lanes (minors, projected columns), for FP32-bulk
// its capped ratio product and packed columns, then the projected-column slots.
struct RoundLds {
    PairHdr* hdr;
    unsigned* incl;
    unsigned* cincl;
    float* ratios;
    uint4* wcols;
    unsigned char* tv;
};

// One round of a wave over the prefixes next, next + 1, ... below pi1 (as many
// as the wave's projected-column slots hold), on the matrix copy src (float or
// double, column stride of SharedLayout<M>): A. lane l factors prefix next + l
// (m x (m-2) block, LU with partial pivoting) and forms its two projection rows
// and signed pivot product; P. the later columns of the taken prefixes, split
// evenly over the lanes, are projected into the slots; B. the minors (pairs of
// later columns after each prefix, dictionary order) are split evenly over the
// lanes, each a 2 x 2 determinant times its prefix's signed pivot product.
// J supplies n, the rank window [q_begin, q_begin + count) of C(n, m) = total
// (prefixes clipped to it; with J.colex the prefixes are those numbered next ...
// among the side-`side` prefixes with last column vlast of a whole rank space,
// see split_block, and side 1 reads the matrix with its columns reversed),
// n_prefix, the slot count cap and, for FP32-bulk, tau and
// the segment of J.fb_entries (defer_cap entries from gwave * defer_cap).  Adds the
// round's terms to (hi, lo, ab); FP32-bulk queues its flagged minors in the
// wave's segment of J.fb_entries (nfb, gcount; gcount wave-uniform on return).
// Returns the number of prefixes taken; `minors` the round's minor count.
template <int M, bool F32, int BS>
__device__ __forceinline__ int shared_round(const FloatJob& J, const unsigned long long* bt,
                                            const typename std::conditional<F32, float, double>::type* src,
                                            unsigned long long next, unsigned long long pi1, int side, int vlast,
                                            const RoundLds& W, int lane, unsigned long long gwave, double& hi,
                                            double& lo, double& ab,
                                            unsigned long long& nfb, int& gcount, unsigned& minors) {
    using T = typename std::conditional<F32, float, double>::type;
    using TV = typename std::conditional<F32, float4, double2>::type;
    static_assert(sizeof(TV) == kSlotBytes, "slot size");
    constexpr int P = M - 2;
    constexpr int ST = F32 ? SharedLayout<M>::s32 : SharedLayout<M>::s64;
    const int n = J.n;
    const unsigned long long qend = J.q_begin + J.count;
    const T tau = (T)J.tau;
    PairHdr* hdr = W.hdr;
    unsigned* incl = W.incl;
    unsigned* cincl = W.cincl;
    float* ratios = W.ratios;
    uint4* wcols = W.wcols;
    TV* tv = reinterpret_cast<TV*>(W.tv);
    (void)ratios;
    (void)wcols;
    (void)gwave;
    (void)tau;

    // ---------------- the round's prefixes: lane l takes prefix next + l
    const unsigned long long pi = next + lane;
    const bool have = pi < pi1;
    int c[P];
    if (J.colex) split_unrank<P>(have ? pi : next, n, side, vlast, bt, BS, c);
    else unrank_prefix<P>(have ? pi : next, n, J.n_prefix, bt, BS, c);
    const int r = n - 1 - c[P - 1];
    // projected-column slots: lanes take prefixes while the slots last
    // (lane 0 always fits: cap >= n - m + 2 >= r)
    const unsigned rs = wave_scan_u32(have ? (unsigned)r : 0u, lane);
    const bool take = have && rs <= (unsigned)J.cap;
    const int ntake = __popcll(__ballot(take));
    const unsigned ncols = __shfl(rs, ntake - 1, kWave);
    const unsigned cnt = take ? (unsigned)(r * (r - 1) / 2) : 0u;
    // the prefix's pairs inside [q_begin, q_begin + count) (all of them over a
    // whole rank space)
    unsigned lo_c = 0, hi_c = cnt;
    if (!J.colex) {
        // dictionary rank of the prefix's first sequence (c, c_{m-3}+1,
        // c_{m-3}+2): the sequences after it number sum_k C(n-1-c_k, m-k)
        unsigned long long after = bt[(r - 1) * BS + 2] + bt[(r - 2) * BS + 1];
#pragma unroll
        for (int k = 0; k < P; ++k) after += bt[(n - 1 - c[k]) * BS + (M - k)];
        const unsigned long long base = J.total - 1 - after;
        if (base < J.q_begin) {
            const unsigned long long d = J.q_begin - base;
            lo_c = d < cnt ? (unsigned)d : cnt;
        }
        if (base + cnt > qend) {
            const unsigned long long d = qend > base ? qend - base : 0ull;
            hi_c = d < cnt ? (unsigned)d : cnt;
        }
        if (hi_c < lo_c) hi_c = lo_c;
    }
    // from here on c holds the matrix's columns: side 1 reads column c as n-1-c
#pragma unroll
    for (int k = 0; k < P; ++k) c[k] = side ? n - 1 - c[k] : c[k];
    const unsigned cc = hi_c - lo_c;
    const unsigned ccincl = wave_scan_u32(cc, lane);
    const unsigned Tr = __shfl(ccincl, kWave - 1, kWave);

    // ---------------- phase A: the prefix's m-2 elimination steps
    T pz0[P], pz1[P];          // the prefix's projection rows, kept for the exchange below
    unsigned long long prel;   // and its row order
    {
        T L[M][P];
        unsigned long long rel = 0;
#pragma unroll
        for (int q = 0; q < M; ++q) rel |= (unsigned long long)q << (4 * q);
        double prod = 1.0;
        bool neg = false;
        float ratio = 1.0f;
        left_steps<M, P, 0, T, F32>(L, src, ST, c, prod, neg, ratio, rel);
        // z_t = -l_{m-2+t} L11^{-1}: rows m-2, m-1 of L^{-1} in the lane's row order
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            T s0 = -L[P][k], s1 = -L[P + 1][k];
#pragma unroll
            for (int i = k + 1; i < P; ++i) {
                s0 = fma_t(-pz0[i], L[i][k], s0);
                s1 = fma_t(-pz1[i], L[i][k], s1);
            }
            pz0[k] = s0;
            pz1[k] = s1;
        }
        prel = rel;
        // sign: the lane's exchanges and the prefix's share of (-1)^(r+s) in
        // its side's coordinates (whose column sum has the parity of
        // side * P(n-1) + sum c); on side 1 a term of the reversed matrix is
        // (-1)^(m(m-1)/2 + m(n+1)) times the matrix's own
        int ps = M * (M + 1) / 2 + P + (side ? M * (M - 1) / 2 + M * (n + 1) + P * (n - 1) : 0);
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
                // the matrix's columns; a side-1 minor's are stored in
                // descending order, marked by bit 31 of the first word
                uint4 w = make_uint4(side ? kColsDescending : 0u, 0u, 0u, 0u);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const unsigned v = (unsigned)c[k] << (kColBits * (k % 3));
                    if (k / 3 == 0) w.x |= v;
                    else if (k / 3 == 1) w.y |= v;
                    else if (k / 3 == 2) w.z |= v;
                    else w.w |= v;
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
        // prefix owning column g0: the first s with cincl[s] > g0 (the last
        // taken prefix for a lane without columns)
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
        T z0[P], z1[P];
        int off[M];
        float pratio = 1.0f;   // FP32-bulk: prefix s's capped ratio product
        // the projection rows of prefix s, from its owner lane (every lane
        // takes part in the exchange)
        auto fetch = [&]() {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                z0[i] = __shfl(pz0[i], s, kWave);
                z1[i] = __shfl(pz1[i], s, kWave);
            }
            const unsigned long long rl = __shfl(prel, s, kWave);
#pragma unroll
            for (int i = 0; i < M; ++i) off[i] = (int)((rl >> (4 * i)) & 15ull);
            if constexpr (F32) pratio = ratios[s];
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
                // slot g holds column c_{m-3} + 1 + (g - sbeg) = n - send + g
                // (the matrix's column n-1-(n-send+g) on side 1)
                const T* colp = src + (side ? (int)send - (int)g - 1 : n - (int)send + (int)g) * ST;
                T t0, t1;
                project<M, P, T>(z0, z1, off, colp, t0, t1);
                // (-1)^j folded in for the j-th column after the prefix
                if ((g - sbeg) & 1u) {
                    t0 = -t0;
                    t1 = -t1;
                }
                TV v;
                v.x = t0;
                v.y = t1;
                if constexpr (F32) {
                    // a minor whose first column after the prefix is this one
                    // has the capped ratio product
                    // rho = h * min(|det| s_b / p_a, 1), h = pratio * min(p_a s_a, 1),
                    // with p_a = max(|t0|, |t1|) its step m-2 pivot and s_a, s_b
                    // the reciprocal column scales; rho < tau exactly when
                    // h < tau or |det| s_b < tau p_a / h: that threshold is
                    // stored with the column
                    const float pa = fmaxf(fabsf(t0), fabsf(t1));
                    const float sa = colp[M];
                    const float h2 = pratio * fminf(pa * sa, 1.f);
                    v.z = !(h2 >= (float)tau)
                              ? __builtin_inff()
                              : ((float)tau > 0.f ? (float)tau * pa * __builtin_amdgcn_rcpf(h2) : 0.f);
                    v.w = sa;
                }
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
        int ia = 0, ib = 1;
        if (active) {
            const unsigned excl = s > 0 ? incl[s - 1] : 0u;
            unrank_pair(g0 - excl + h.lo, hr, ia, ib);
        }
        const unsigned kend = active ? gend - g0 : 0u;
        // FP32-bulk: column a carries the threshold of its minors (.z)
        TV ta = tv[toff + ia];
        // runs of up to kRun terms are added plainly and each run is then
        // folded into the compensated pair, outside the inner loop: the
        // plain sums add at most gamma_(kRun-1) sum |det| of error
        constexpr unsigned kRun = 16;
        if constexpr (!F32) {
            // each lane walks exactly its share; both columns are read
            // every step (no loop-carried column, no copies)
            for (unsigned k = 0; k < kend;) {
              const unsigned kr = min(kend, k + kRun);
              double run = 0.0;
              for (; k < kr; ++k) {
                const TV ta2 = tv[toff + ia];
                const TV tb = tv[toff + ib];
                const T d = fma_t(ta2.x, tb.y, -(ta2.y * tb.x));
                run = fma((double)d, h.prodS, run);
                ab = fma(fabs((double)d), fabs(h.prodS), ab);
                if (++ib >= hr) {
                    ++ia;
                    ib = ia + 1;
                    if (ib >= hr) {
                        s = min(s + 1, ntake - 1);
                        h = hdr[s];
                        hr = (int)(h.rt & kRMask);
                        toff = (int)(h.rt >> kRBits);
                        ia = 0;
                        ib = 1;
                    }
                }
              }
              double sum, err;
              two_sum(hi, run, sum, err);
              hi = sum;
              lo += err;
            }
        }
        if constexpr (F32) {
            // as above, each lane walks its share; the flagged-minor count
            // stays exact on the lanes still walking (every ballot of a step
            // is seen by all of them) and is made wave-uniform after the loop
            for (unsigned k = 0; k < kend;) {
              const unsigned kr = min(kend, k + kRun);
              double run = 0.0;
              for (; k < kr; ++k) {
                const TV tb = tv[toff + ib];
                const T d = fma_t(ta.x, tb.y, -(ta.y * tb.x));
                const bool flag = fabsf(d) * tb.w < ta.z;
                const unsigned long long fm = __ballot(flag);
                if (fm) {
                    const int pos = gcount + (int)__builtin_amdgcn_mbcnt_hi(
                                                 (unsigned)(fm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                    if (flag && pos < J.defer_cap) {
                        const int ca = side ? hr - 1 - ia : n - hr + ia;
                        const int cbb = side ? hr - 1 - ib : n - hr + ib;
                        const uint4 pw = wcols[s];
                        unsigned w[4] = {pw.x, pw.y, pw.z, pw.w};
                        w[P / 3] |= (unsigned)ca << (kColBits * (P % 3));
                        w[(P + 1) / 3] |= (unsigned)cbb << (kColBits * ((P + 1) % 3));
                        unsigned* ent = J.fb_entries + ((size_t)gwave * J.defer_cap + pos) * 4;
                        ent[0] = w[0];
                        ent[1] = w[1];
                        ent[2] = w[2];
                        ent[3] = w[3];
                        nfb += 1;
                    }
                    gcount += __popcll(fm);
                }
                // a queued minor adds an exact 0
                const double dd = (double)(flag ? 0.f : d);
                run = fma(dd, h.prodS, run);
                ab = fma(fabs(dd), fabs(h.prodS), ab);
                // next pair; past the prefix's last pair, the next prefix
                if (++ib >= hr) {
                    ++ia;
                    ib = ia + 1;
                    if (ib >= hr) {
                        s = min(s + 1, ntake - 1);
                        h = hdr[s];
                        hr = (int)(h.rt & kRMask);
                        toff = (int)(h.rt >> kRBits);
                        ia = 0;
                        ib = 1;
                    }
                    ta = tv[toff + ia];
                }
              }
              double sum, err;
              two_sum(hi, run, sum, err);
              hi = sum;
              lo += err;
            }
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) gcount = max(gcount, __shfl_xor(gcount, o, kWave));
        }
    }
    minors = Tr;
    return ntake;
}

}  // namespace radic
