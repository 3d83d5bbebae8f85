// Group-shared exact elimination modulo a prime (the minors sharing their first
// m-3 columns), for the batched exact chunks and the single-matrix exact kernel.
//
// The same fraction-free steps as the prefix-shared form (shared_int.h), one
// step fewer: per group (m-3 columns; the sequences that begin with them are
// consecutive in the dictionary order of Section 3) a lane eliminates the
// m x (m-3) block and forms the three rows W (3 x m) of the fraction-free
// elimination operator that produce rows m-3 .. m-1.  A later column c is
// projected to u_c = W x_c mod p, with the factor (-1)^j of the j-th column
// after the group folded in.  For a minor with later columns a < b < c,
//     det = u_c . (u_a x u_b) / (P_{m-4} prod_{k<m-3} P_k)   (mod p),
// P_k = u_0 ... u_k the running pivot products (one more factor P_{m-4} than
// for prefixes of m-2 columns, since three rows below the block were scaled by
// each step): the last three elimination steps of the minor reduce to that
// 3 x 3 determinant.  The cross product of a pair, already multiplied by the
// group's signed inverse of that denominator, serves every third column after
// it.  Per minor this costs one dot product, against one
// elimination of an m x (m-3) block per group: the groups hold C(r, 3) minors
// (r later columns) where prefixes of m-2 columns hold C(r, 2), which pays from
// about m = 7 on for the narrow matrices of a batch.
#pragma once

#include "shared_int.h"

namespace radic {

// Number of the group (first m-3 columns, dictionary order) of the sequence of
// rank q; bt[x*stride + y] = C(x, y).
template <int M>
__device__ unsigned long long group_of_rank(unsigned long long q, int n, const unsigned long long* bt, int stride) {
    constexpr int P = M - 3;
    int c[M];
    unrank_strided<M>(q, n, bt, stride, c);
    unsigned long long g = 0;
    int prev = -1;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        // the P-subsets of [0, n-3) that agree before position k and hold v < c_k there
        for (int v = prev + 1; v < c[k]; ++v) g += bt[(n - 4 - v) * stride + (P - 1 - k)];
        prev = c[k];
    }
    return g;
}

// A projected later column: the three residues of u_c (each below 2^31).
__device__ __forceinline__ uint4 pack_u3(double a, double b, double c) {
    return make_uint4((unsigned)a, (unsigned)b, (unsigned)c, 0u);
}

// The signed minors mod p of the ranks [R0, R1) of one matrix whose residues
// mod p are staged column-major in cr (stride IntLayout<M>::st), summed into
// this lane's `acc`.  `next` is the group holding R0 and `rbase` the rank of its
// first sequence; groups [next, pi1) are visited in rounds of up to 64 (one per
// lane, while their later columns fit the cap projected-column slots of tv);
// n_group = C(n-3, m-3) numbers all groups.  incl holds 2 x 64 scans (minors,
// then projected columns).  bt[x*bstride + y] = C(x, y) for y < M.  Wave-uniform
// control flow outside the lanes' own walks.
template <int M>
__device__ void int_group_range(const double* cr, int n, const unsigned long long* bt, int bstride,
                                unsigned long long next, unsigned long long pi1, unsigned long long n_group,
                                unsigned long long rbase, unsigned long long R0, unsigned long long R1, double p,
                                double pinv, int cap, IntSlot* slot, unsigned* incl, uint4* tv, int lane,
                                double& acc) {
    static_assert(M >= 4, "a group leaves three later columns");
    constexpr int P = M - 3;
    constexpr int ST = IntLayout<M>::st;
    while (next < pi1 && rbase < R1) {
        // lane l takes group next + l if it starts before R1 and its later
        // columns still fit the projected-column slots (lane 0 always does)
        const unsigned long long gi = next + lane;
        const bool inb = gi < pi1;
        int c[P];
        unrank_prefix<P>(inb ? gi : next, n - 1, n_group, bt, bstride, c);
        const int r = n - 1 - c[P - 1];   // columns after the group, >= 3
        const unsigned cfull = inb ? (unsigned)r * (unsigned)(r - 1) * (unsigned)(r - 2) / 6u : 0u;
        const unsigned cscan = wave_scan_u32(cfull, lane);
        const unsigned long long base = rbase + (cscan - cfull);
        const bool have = inb && base < R1;
        const unsigned rs = wave_scan_u32(have ? (unsigned)r : 0u, lane);
        const bool take = have && rs <= (unsigned)cap;
        const int ntake = __popcll(__ballot(take));
        const unsigned round_total = __shfl(cscan, ntake - 1, kWave);
        const unsigned cnt = take ? cfull : 0u;
        unsigned lo_c = 0, hi_c = cnt;
        if (base < R0) {
            const unsigned long long d = R0 - base;
            lo_c = d < cnt ? (unsigned)d : cnt;
        }
        if (base + cnt > R1) {
            const unsigned long long d = R1 > base ? R1 - base : 0ull;
            hi_c = d < cnt ? (unsigned)d : cnt;
        }
        if (hi_c < lo_c) hi_c = lo_c;
        const unsigned cc = hi_c - lo_c;
        const unsigned ccincl = wave_scan_u32(cc, lane);
        const unsigned Tr = __shfl(ccincl, kWave - 1, kWave);

        // ---------------- phase A: the group's m-3 fraction-free steps
        unsigned* cincl = incl + kPrefixBlock;   // projected columns, inclusive scan
        const unsigned ncols = __shfl(rs, ntake - 1, kWave);
        double pw0[M], pw1[M], pw2[M];   // the group's rows of W, kept for the exchange below
        unsigned long long prel;         // and its row order
        {
            double L[M][P];
            double u[P];
            unsigned long long rel = 0;
#pragma unroll
            for (int q = 0; q < M; ++q) rel |= (unsigned long long)q << (4 * q);
            double Pk = 1.0, D = 1.0;
            bool zero = false, neg = false;
            int_left_steps<M, P, 0>(L, u, cr, ST, c, p, pinv, Pk, D, zero, neg, rel);
            // W rows m-3 .. m-1 of the elimination operator, by the backward
            // recurrence w <- w E_k (E_k: rows > k scaled by u_k, minus
            // multiples of row k)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                pw0[j] = (j == P) ? 1.0 : 0.0;
                pw1[j] = (j == P + 1) ? 1.0 : 0.0;
                pw2[j] = (j == P + 2) ? 1.0 : 0.0;
            }
// (lazy residues: each entry below 2.01 p in magnitude)
#pragma unroll
            for (int k = P - 1; k >= 0; --k) {
                double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
                for (int i = k + 1; i < M; ++i) {
                    d0 += mulmod_lazy(pw0[i], L[i][k], p, pinv);
                    d1 += mulmod_lazy(pw1[i], L[i][k], p, pinv);
                    d2 += mulmod_lazy(pw2[i], L[i][k], p, pinv);
                }
                d0 = reduce_lazy(d0, p, pinv);
                d1 = reduce_lazy(d1, p, pinv);
                d2 = reduce_lazy(d2, p, pinv);
#pragma unroll
                for (int j = k + 1; j < M; ++j) {
                    pw0[j] = mulmod_lazy(pw0[j], u[k], p, pinv);
                    pw1[j] = mulmod_lazy(pw1[j], u[k], p, pinv);
                    pw2[j] = mulmod_lazy(pw2[j], u[k], p, pinv);
                }
                pw0[k] -= d0;   // was 0: the unit rows sit at m-3 .. m-1
                pw1[k] -= d1;
                pw2[k] -= d2;
            }
            prel = rel;
            // the minor's denominator: step k scales the m-1-k rows below its
            // pivot by u_k and the eliminated block keeps u_k on its diagonal,
            // so det = det(3 x 3) / prod_k u_k^(m-2-k) = det(3 x 3) / (D P_{m-4})
            // with D = prod_{k<m-3} P_k.  Their inverses for every group of the
            // round: Montgomery's batch inversion over the wave (prefix
            // products, one inverse, suffix products)
            const double Dz = (take && !zero) ? mulmod(D, Pk, p, pinv) : 1.0;
            double pre = Dz;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const double v = __shfl_up(pre, off, kWave);
                if (lane >= off) pre = mulmod(pre, v, p, pinv);
            }
            double suf = Dz;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const double v = __shfl_down(suf, off, kWave);
                if (lane + off < kWave) suf = mulmod(suf, v, p, pinv);
            }
            const double total = __shfl(pre, kWave - 1, kWave);
            const double tinv = invmod(total, p, pinv);
            const double before = __shfl_up(pre, 1, kWave);
            const double after = __shfl_down(suf, 1, kWave);
            double inv = tinv;
            if (lane > 0) inv = mulmod(inv, before, p, pinv);
            if (lane < kWave - 1) inv = mulmod(inv, after, p, pinv);
            // sign: the group's row exchanges and its share of (-1)^(r+s); the
            // three later columns add 3 (n - r) + 3 + their offsets, the offsets
            // folded into the projected columns
            int ps = M * (M + 1) / 2 + P + 1 + (n - r);
#pragma unroll
            for (int k = 0; k < P; ++k) ps += c[k];
            const bool sg = neg ^ ((ps & 1) != 0);
            double F = zero ? 0.0 : inv;
            if (sg && F != 0.0) F = p - F;
            if (take) {
                IntSlot sl;
                sl.F = F;
                sl.r = r;
                sl.toff = (int)rs - r;
                sl.lo = lo_c;
                sl.pad = 0;
                slot[lane] = sl;
                incl[lane] = ccincl;
                cincl[lane] = rs;
            }
        }
        wave_lds_sync();

        // ---------------- projection: the round's columns split evenly over the lanes
        {
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
            double w0[M], w1[M], w2[M];
            int off[M];
            // W of group s, from its owner lane (every lane takes part)
            auto fetch = [&]() {
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    w0[i] = __shfl(pw0[i], s, kWave);
                    w1[i] = __shfl(pw1[i], s, kWave);
                    w2[i] = __shfl(pw2[i], s, kWave);
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
                    const double* colp = cr + (n - (int)send + (int)g) * ST;
                    double x[M];
#pragma unroll
                    for (int i = 0; i < M; ++i) x[i] = colp[off[i]];
                    double t0 = dot_mod<M>(w0, x, p, pinv);
                    double t1 = dot_mod<M>(w1, x, p, pinv);
                    double t2 = dot_mod<M>(w2, x, p, pinv);
                    // (-1)^j for the j-th column after the group
                    if ((g - sbeg) & 1u) {
                        t0 = t0 != 0.0 ? p - t0 : 0.0;
                        t1 = t1 != 0.0 ? p - t1 : 0.0;
                        t2 = t2 != 0.0 ? p - t2 : 0.0;
                    }
                    tv[g] = pack_u3(t0, t1, t2);
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
            IntSlot h = slot[s];
            // the lane's first triple: its number among the group's C(r, 3)
            // triples, unranked as three columns out of r
            int ia = 0, ib = 1, ic = 2;
            if (active) {
                const unsigned excl = s > 0 ? incl[s - 1] : 0u;
                int t3[3];
                unrank_prefix<3>(g0 - excl + h.lo, h.r + 2, bt[h.r * bstride + 3], bt, bstride, t3);
                ia = t3[0];
                ib = t3[1];
                ic = t3[2];
            }
            double wx, wy, wz;   // F (u_a x u_b), lazy residues below 2.01 p
            auto pair = [&]() {
                const uint4 qa = tv[h.toff + ia], qb = tv[h.toff + ib];
                const double ax = (double)qa.x, ay = (double)qa.y, az = (double)qa.z;
                const double bx = (double)qb.x, by = (double)qb.y, bz = (double)qb.z;
                wx = mulmod_lazy(h.F, mulmod_lazy(ay, bz, p, pinv) - mulmod_lazy(az, by, p, pinv), p, pinv);
                wy = mulmod_lazy(h.F, mulmod_lazy(az, bx, p, pinv) - mulmod_lazy(ax, bz, p, pinv), p, pinv);
                wz = mulmod_lazy(h.F, mulmod_lazy(ax, by, p, pinv) - mulmod_lazy(ay, bx, p, pinv), p, pinv);
            };
            pair();
            // each minor's three lazy products (below 6.1 p together) summed
            // exactly, reduced every kAccRun steps
            double run = 0.0;
            for (unsigned k0 = 0; k0 < chunk; k0 += kAccRun) {
                const unsigned k1 = min(chunk, k0 + kAccRun);
                for (unsigned k = k0; k < k1; ++k) {
                    const bool valid = g0 + k < gend;
                    const uint4 qc = tv[h.toff + ic];
                    const double t = mulmod_lazy(wx, (double)qc.x, p, pinv) + mulmod_lazy(wy, (double)qc.y, p, pinv) +
                                     mulmod_lazy(wz, (double)qc.z, p, pinv);
                    if (valid) run += t;
                    // next triple: c, then b, then a, then the next group
                    if (++ic >= h.r) {
                        if (++ib >= h.r - 1) {
                            if (++ia >= h.r - 2) {
                                s = min(s + 1, ntake - 1);
                                h = slot[s];
                                ia = 0;
                            }
                            ib = ia + 1;
                        }
                        ic = ib + 1;
                        pair();
                    }
                }
                run = reduce_lazy(run, p, pinv);
            }
            acc = addmod(acc, canon(run, p, pinv), p);
        }
        rbase += round_total;
        next += (unsigned long long)ntake;
        wave_lds_sync();
    }
}

}  // namespace radic
