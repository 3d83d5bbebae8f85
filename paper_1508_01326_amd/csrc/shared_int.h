// Prefix-shared exact elimination modulo a prime, shared by the single-matrix
// and batched exact kernels.
//
// The minors with equal first m-2 columns (a prefix; consecutive in the
// dictionary order of Section 3) share the first m-2 steps of their
// fraction-free elimination modulo p: every step k multiplies the rows below
// the pivot by the pivot u_k and subtracts multiples of the pivot row, and its
// pivot (the first nonzero entry of column k) and multipliers depend on the
// first k+1 columns only.  Per prefix a lane eliminates the m x (m-2) block
// (column by column, keeping only the multipliers) and forms the two rows W
// (2 x m) of the fraction-free elimination operator that produce rows m-2,
// m-1; the round's later columns are then split over the lanes, which fetch W
// from the owner lane and write t_c = W x_c mod p to LDS.  For a minor with
// later columns a < b,
//     det = (t_a0 t_b1 - t_a1 t_b0) / prod_{k<m-2} P_k   (mod p),
// P_k = u_0 ... u_k the running pivot products (the last two elimination steps
// of the minor, written out), with the sign of the prefix's row exchanges.  The
// denominators of the 64 prefixes of a round are inverted together (one Fermat
// inverse per round, Montgomery's batch trick over the wave).  A prefix whose
// block has a zero pivot column mod p makes all its minors 0 mod p.
#pragma once

#include "modp.h"
#include "prefix.h"

namespace radic {

struct IntSlot {
    double F;      // signed 1 / prod P_k mod p (0 if the prefix block is singular mod p)
    int r;         // columns after the prefix
    int toff;      // first projected-column slot
    unsigned lo;   // first pair inside the call's rank range
    int pad;
};

// sum_j w_j x_j mod p in [0, p), for |w_j|, |x_j| <= 4.1 p: the lazy products
// (each below 2.01 p) summed exactly (below 2^36) and reduced once
template <int M>
__device__ __forceinline__ double dot_mod(const double (&w)[M], const double (&x)[M], double p, double pinv) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) s += mulmod_lazy(w[j], x[j], p, pinv);
    return canon(s, p, pinv);
}

// Accumulated lazy terms (each below 6.1 p) are reduced after at most this
// many steps of a lane, so the running sum stays an exact double (< 2^51).
constexpr unsigned kAccRun = 1u << 16;

// Step K of the prefix's fraction-free elimination, column by column
// (left-looking).  Column c_K is read in the lane's current row order `rel` (4
// bits per position), the earlier steps are applied to it (x_i <- u_k x_i -
// L_ik x_k for i > k, k = 0, 1, ...), its pivot is the first row >= K with a
// nonzero entry, and an exchange swaps the two rows of L and of the column and
// is recorded in rel, so that later columns are read already exchanged.  L_iK
// keeps the column's entries below the pivot (the step's multipliers).  Every
// residue sees the same operations as in the row-by-row form.  The updates use
// lazy products (values below 4.1 p in magnitude, same residues); the column is
// brought to [0, p) before its pivot test, so pivots, multipliers and the zero
// test are those of canonical residues.
template <int M, int P, int K>
__device__ __forceinline__ void int_left_steps(double (&L)[M][P], double (&u)[P], const double* cr, int stride,
                                               const int (&c)[P], double p, double pinv, double& Pk, double& D,
                                               bool& zero, bool& neg, unsigned long long& rel) {
    if constexpr (K < P) {
        const double* colp = cr + c[K] * stride;
        double x[M];
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] = colp[(int)((rel >> (4 * i)) & 15ull)];
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int i = k + 1; i < M; ++i) {
                x[i] = mulmod_lazy(u[k], x[i], p, pinv) - mulmod_lazy(L[i][k], x[k], p, pinv);
                // an empty register constraint: keeps the compiler's instruction
                // combining from folding the whole chain of reductions (whose
                // compile time otherwise explodes from m = 8); no code
                asm volatile("" : "+v"(x[i]));
            }
        }
        if constexpr (K > 0) {
#pragma unroll
            for (int i = K; i < M; ++i) x[i] = canon(x[i], p, pinv);
        }
        unsigned best = 0;
#pragma unroll
        for (int i = K; i < M; ++i) best = max(best, x[i] != 0.0 ? (unsigned)(15 - i) : 0u);
        const bool col_zero = (best == 0u);
        const int pr = col_zero ? K : 15 - (int)best;
        zero |= col_zero;
        neg ^= (pr != K);
        if (__ballot(pr != K)) {
            const unsigned long long d = ((rel >> (4 * K)) ^ (rel >> (4 * pr))) & 15ull;
            rel ^= (d << (4 * K)) | (d << (4 * pr));
#pragma unroll
            for (int i = K + 1; i < M; ++i) {
                const bool e = (pr == i);
                if (__ballot(e)) {
                    {
                        const double v0 = x[K], v1 = x[i];
                        x[K] = e ? v1 : v0;
                        x[i] = e ? v0 : v1;
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const double v0 = L[K][k], v1 = L[i][k];
                        L[K][k] = e ? v1 : v0;
                        L[i][k] = e ? v0 : v1;
                    }
                }
            }
        }
        const double uk = col_zero ? 1.0 : x[K];
        u[K] = uk;
        Pk = mulmod(Pk, uk, p, pinv);
        D = mulmod(D, Pk, p, pinv);
#pragma unroll
        for (int i = K + 1; i < M; ++i) L[i][K] = x[i];
        int_left_steps<M, P, K + 1>(L, u, cr, stride, c, p, pinv, Pk, D, zero, neg, rel);
    }
}

// The signed minors mod p of the ranks [R0, R1) of one matrix whose residues
// mod p are staged column-major in cr (stride IntLayout<M>::st), summed into
// this lane's `acc`.  `next` is the prefix holding R0 and `rbase` the rank of its
// first sequence; prefixes [next, pi1) are visited in rounds of up to 64 (one
// per lane; while their later columns fit the cap projected-column slots);
// n_prefix = C(n-2, m-2) numbers all prefixes.  incl holds 2 x 64 scans (pairs,
// then projected columns).  bt[x*bstride + y] = C(x, y) for y < M.  Wave-uniform
// control flow outside the lanes' own walks.  COLEX: next and pi1 number the
// side-`side` prefixes with last column vlast of a two-sided block (see
// split_block; side 1 reads the matrix with its columns reversed) and the
// whole rank space is summed, so no pair is clipped and rbase, R0, R1 are not
// used.
template <int M, bool COLEX = false>
__device__ void int_prefix_range(const double* cr, int n, const unsigned long long* bt, int bstride,
                                 unsigned long long next, unsigned long long pi1, unsigned long long n_prefix,
                                 unsigned long long rbase,
                                 unsigned long long R0, unsigned long long R1, double p, double pinv, int cap,
                                 IntSlot* slot, unsigned* incl, double2* tv, int lane, double& acc, int side = 0,
                                 int vlast = 0) {
    constexpr int P = M - 2;
    constexpr int ST = IntLayout<M>::st;
    if (!COLEX) side = 0;
    while (next < pi1 && (COLEX || rbase < R1)) {
        // lane l takes prefix next + l if it starts before R1 and its later
        // columns still fit the projected-column slots (lane 0 always does)
        const unsigned long long pi = next + lane;
        const bool inb = pi < pi1;
        int c[P];
        if (COLEX) split_unrank<P>(inb ? pi : next, n, side, vlast, bt, bstride, c);
        else unrank_prefix<P>(inb ? pi : next, n, n_prefix, bt, bstride, c);
        const int r = n - 1 - c[P - 1];
        // from here on c holds the matrix's columns: side 1 reads column c as n-1-c
#pragma unroll
        for (int k = 0; k < P; ++k) c[k] = side ? n - 1 - c[k] : c[k];
        const unsigned cfull = inb ? (unsigned)(r * (r - 1) / 2) : 0u;
        const unsigned cscan = wave_scan_u32(cfull, lane);
        const unsigned long long base = rbase + (cscan - cfull);
        const bool have = inb && (COLEX || base < R1);
        const unsigned rs = wave_scan_u32(have ? (unsigned)r : 0u, lane);
        const bool take = have && rs <= (unsigned)cap;
        const int ntake = __popcll(__ballot(take));
        const unsigned round_total = __shfl(cscan, ntake - 1, kWave);
        const unsigned cnt = take ? cfull : 0u;
        unsigned lo_c = 0, hi_c = cnt;
        if (!COLEX) {
            if (base < R0) {
                const unsigned long long d = R0 - base;
                lo_c = d < cnt ? (unsigned)d : cnt;
            }
            if (base + cnt > R1) {
                const unsigned long long d = R1 > base ? R1 - base : 0ull;
                hi_c = d < cnt ? (unsigned)d : cnt;
            }
            if (hi_c < lo_c) hi_c = lo_c;
        }
        const unsigned cc = hi_c - lo_c;
        const unsigned ccincl = wave_scan_u32(cc, lane);
        const unsigned Tr = __shfl(ccincl, kWave - 1, kWave);

        // ---------------- phase A: the prefix's m-2 fraction-free steps
        unsigned* cincl = incl + kPrefixBlock;   // projected columns, inclusive scan
        const unsigned ncols = __shfl(rs, ntake - 1, kWave);
        double pw0[M], pw1[M];         // the prefix's rows of W, kept for the exchange below
        unsigned long long prel;       // and its row order
        {
            double L[M][P];
            double u[P];
            unsigned long long rel = 0;
#pragma unroll
            for (int q = 0; q < M; ++q) rel |= (unsigned long long)q << (4 * q);
            double Pk = 1.0, D = 1.0;
            bool zero = false, neg = false;
            int_left_steps<M, P, 0>(L, u, cr, ST, c, p, pinv, Pk, D, zero, neg, rel);
            // W rows m-2, m-1 of the elimination operator, by the backward
            // recurrence w <- w E_k (E_k: rows > k scaled by u_k, minus
            // multiples of row k)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                pw0[j] = (j == P) ? 1.0 : 0.0;
                pw1[j] = (j == P + 1) ? 1.0 : 0.0;
            }
// (lazy residues: each entry below 2.01 p in magnitude)
#pragma unroll
            for (int k = P - 1; k >= 0; --k) {
                double d0 = 0.0, d1 = 0.0;
#pragma unroll
                for (int i = k + 1; i < M; ++i) {
                    d0 += mulmod_lazy(pw0[i], L[i][k], p, pinv);
                    d1 += mulmod_lazy(pw1[i], L[i][k], p, pinv);
                }
                d0 = reduce_lazy(d0, p, pinv);
                d1 = reduce_lazy(d1, p, pinv);
#pragma unroll
                for (int j = k + 1; j < M; ++j) {
                    pw0[j] = mulmod_lazy(pw0[j], u[k], p, pinv);
                    pw1[j] = mulmod_lazy(pw1[j], u[k], p, pinv);
                }
                pw0[k] -= d0;   // was 0: the unit rows sit at m-2, m-1
                pw1[k] -= d1;
            }
            prel = rel;
            // 1 / D for every prefix of the round: Montgomery's batch inversion
            // over the wave (prefix products, one inverse, suffix products)
            const double Dz = (take && !zero) ? D : 1.0;
            double pre = Dz;   // inclusive prefix product
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const double v = __shfl_up(pre, off, kWave);
                if (lane >= off) pre = mulmod(pre, v, p, pinv);
            }
            double suf = Dz;   // inclusive suffix product
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
            // sign: prefix row exchanges and the prefix's share of (-1)^(r+s) in
            // its side's coordinates (column sum of the parity of side * P(n-1)
            // + sum c; on side 1 a term of the reversed matrix is
            // (-1)^(m(m-1)/2 + m(n+1)) times the matrix's own); the pair (a, b)
            // adds 2 (n - r + 1) + its offsets
            int ps = M * (M + 1) / 2 + P + (side ? M * (M - 1) / 2 + M * (n + 1) + P * (n - 1) : 0);
#pragma unroll
            for (int k = 0; k < P; ++k) ps += c[k];
            const bool sg = neg ^ ((ps & 1) != 0);
            double F = zero ? 0.0 : inv;
            if (sg && F != 0.0) F = p - F;
            const int toff = (int)rs - r;
            if (take) {
                IntSlot sl;
                sl.F = F;
                sl.r = r;
                sl.toff = toff;
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
            double w0[M], w1[M];
            int off[M];
            // W of prefix s, from its owner lane (every lane takes part)
            auto fetch = [&]() {
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    w0[i] = __shfl(pw0[i], s, kWave);
                    w1[i] = __shfl(pw1[i], s, kWave);
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
                        send = cincl[s];
                    }
                    fetch();
                }
                if (act) {
                    // slot g holds column c_{m-3} + 1 + (g - start of s) = n - send + g
                    // of its side (the matrix's n-1-(n-send+g) on side 1)
                    const double* colp = cr + (side ? (int)send - (int)g - 1 : n - (int)send + (int)g) * ST;
                    double x[M];
#pragma unroll
                    for (int i = 0; i < M; ++i) x[i] = colp[off[i]];
                    tv[g] = make_double2(dot_mod<M>(w0, x, p, pinv), dot_mod<M>(w1, x, p, pinv));
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
            int ia = 0, ib = 1;
            if (active) unrank_pair(g0 - (s > 0 ? incl[s - 1] : 0u) + h.lo, h.r, ia, ib);
            double2 ta = tv[h.toff + ia];
            // lazy terms (below 2.01 p) summed exactly, reduced every kAccRun steps
            double run = 0.0;
            for (unsigned k0 = 0; k0 < chunk; k0 += kAccRun) {
                const unsigned k1 = min(chunk, k0 + kAccRun);
                for (unsigned k = k0; k < k1; ++k) {
                    const bool valid = g0 + k < gend;
                    const double2 tb = tv[h.toff + ib];
                    const double cross = mulmod_lazy(ta.x, tb.y, p, pinv) - mulmod_lazy(ta.y, tb.x, p, pinv);
                    const double term = mulmod_lazy(h.F, cross, p, pinv);
                    if (valid) run += ((ia + ib) & 1) ? -term : term;
                    if (++ib >= h.r) {
                        ++ia;
                        ib = ia + 1;
                        if (ib >= h.r) {
                            s = min(s + 1, ntake - 1);
                            h = slot[s];
                            ia = 0;
                            ib = 1;
                        }
                        ta = tv[h.toff + ia];
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
