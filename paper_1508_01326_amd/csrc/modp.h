// Modular arithmetic on exact doubles and fraction-free elimination modulo a
// 31-bit prime, shared by the single-matrix and batched exact kernels.
#pragma once

#include "enumerate.h"

namespace radic {

// Prime set of the exact path (per translation unit, uploaded by the host), and
// for Garner's recombination the inverse of p_0 p_1 ... p_{i-1} modulo p_i.
static __device__ double g_prime[RADIC_MAX_PRIMES];
static __device__ double g_prime_inv[RADIC_MAX_PRIMES];
static __device__ unsigned long long g_garner_inv[RADIC_MAX_PRIMES];

static inline unsigned long long host_powmod(unsigned long long b, unsigned long long e, unsigned long long p) {
    unsigned long long r = 1 % p;
    b %= p;
    for (; e; e >>= 1) {
        if (e & 1ull) r = r * b % p;   // operands below 2^31: exact in 64 bits
        b = b * b % p;
    }
    return r;
}

static inline hipError_t upload_prime_table(const unsigned* primes, int count) {
    double pd[RADIC_MAX_PRIMES] = {0}, pi[RADIC_MAX_PRIMES] = {0};
    unsigned long long gi[RADIC_MAX_PRIMES] = {0};
    for (int i = 0; i < count && i < RADIC_MAX_PRIMES; ++i) {
        pd[i] = (double)primes[i];
        pi[i] = 1.0 / pd[i];
        const unsigned long long p = primes[i];
        unsigned long long prod = 1 % p;
        for (int j = 0; j < i; ++j) prod = prod * (primes[j] % p) % p;
        gi[i] = host_powmod(prod, p - 2, p);   // Fermat: the primes are distinct
    }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_prime), pd, sizeof(pd));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_prime_inv), pi, sizeof(pi));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_garner_inv), gi, sizeof(gi));
    return e;
}

template <int M> struct IntLayout {
    static constexpr int g64 = (((M + 1) / 2) % 2 == 0) ? (M + 1) / 2 + 1 : (M + 1) / 2;
    static constexpr int st = 2 * g64;   // doubles per column
};

// ---------------------------------------------------------------- modular arithmetic on exact doubles
__device__ __forceinline__ double mod_fix(double r, double p) {
    r = r < 0.0 ? r + p : r;
    return r >= p ? r - p : r;
}

// a*b mod p for 0 <= a, b < p < 2^31: h + l = a*b exactly (FMA split); q is
// floor(a*b/p) up to +-1, so h - q p + l lies in [-p, 2p) and is exact.
__device__ __forceinline__ double mulmod(double a, double b, double p, double pinv) {
    const double h = a * b;
    const double l = __builtin_fma(a, b, -h);
    const double q = __builtin_floor(h * pinv);
    const double r = __builtin_fma(-q, p, h) + l;
    return mod_fix(r, p);
}

// a*b up to a multiple of p, without the range fix: for integers |a|, |b| <=
// 4.1 p (p < 2^31) the quotient estimate q is off by at most one, h - q p and
// then h - q p + l are exact, so r = a b - q p with |r| < 2.01 p.  Sums and
// differences of two such results may be fed back in.
__device__ __forceinline__ double mulmod_lazy(double a, double b, double p, double pinv) {
    const double h = a * b;
    const double l = __builtin_fma(a, b, -h);
    const double q = __builtin_floor(h * pinv);
    return __builtin_fma(-q, p, h) + l;
}

// An integer |x| < 2^52 reduced to [-p, 2p) (same residue), and to [0, p).
__device__ __forceinline__ double reduce_lazy(double x, double p, double pinv) {
    return __builtin_fma(-__builtin_floor(x * pinv), p, x);
}
__device__ __forceinline__ double canon(double x, double p, double pinv) { return mod_fix(reduce_lazy(x, p, pinv), p); }

__device__ __forceinline__ double addmod(double a, double b, double p) {
    const double r = a + b;
    return r >= p ? r - p : r;
}

__device__ __forceinline__ double submod(double a, double b, double p) {
    const double r = a - b;
    return r < 0.0 ? r + p : r;
}

// x^(p-2) mod p (Fermat), x != 0
__device__ double invmod(double x, double p, double pinv) {
    unsigned long long e = (unsigned long long)p - 2ull;
    double r = 1.0, b = x;
    while (e) {
        if (e & 1ull) r = mulmod(r, b, p, pinv);
        b = mulmod(b, b, p, pinv);
        e >>= 1;
    }
    return r;
}

// ---------------------------------------------------------------- per-lane elimination mod p
template <int M, int K>
__device__ __forceinline__ void exchange_rows_int(double (&a)[M][M], int p) {
#pragma unroll
    for (int i = K + 1; i < M; ++i) {
        const bool c = (p == i);
        if (__ballot(c)) {
#pragma unroll
            for (int j = K; j < M; ++j) {
                const double x = a[K][j], y = a[i][j];
                a[K][j] = c ? y : x;
                a[i][j] = c ? x : y;
            }
        }
    }
}

template <int M, int K>
__device__ __forceinline__ void elim_steps_mod(double (&a)[M][M], double p, double pinv, double& N, double& P,
                                               double& D, bool& zero, bool& neg) {
    if constexpr (K < M) {
        // pivot: first row i >= K whose entry in column K is nonzero mod p
        unsigned best = 0;
#pragma unroll
        for (int i = K; i < M; ++i) best = max(best, a[i][K] != 0.0 ? (unsigned)(15 - i) : 0u);
        const bool col_zero = (best == 0u);
        const int piv_row = col_zero ? K : 15 - (int)best;
        zero |= col_zero;
        if constexpr (K < M - 1) {
            neg ^= (piv_row != K);
            exchange_rows_int<M, K>(a, piv_row);
        }
        const double u = col_zero ? 1.0 : a[K][K];
        N = mulmod(N, u, p, pinv);
        if constexpr (K < M - 1) {
            P = mulmod(P, u, p, pinv);
            D = mulmod(D, P, p, pinv);
#pragma unroll
            for (int i = K + 1; i < M; ++i) {
                const double l = a[i][K];
#pragma unroll
                for (int j = K + 1; j < M; ++j)
                    a[i][j] = submod(mulmod(u, a[i][j], p, pinv), mulmod(l, a[K][j], p, pinv), p);
            }
            elim_steps_mod<M, K + 1>(a, p, pinv, N, P, D, zero, neg);
        }
    }
}

// fraction (n1/d1) += (n2/d2)
__device__ __forceinline__ void frac_add(double& n1, double& d1, double n2, double d2, double p, double pinv) {
    n1 = addmod(mulmod(n1, d2, p, pinv), mulmod(n2, d1, p, pinv), p);
    d1 = mulmod(d1, d2, p, pinv);
}

// ---------------------------------------------------------------- Chinese remaindering (one wave)
// Multi-limb integers across a wave: lane l holds 32-bit limb l (little-endian).
// Carries between limbs by lookahead on the wave's ballots: with bit l of g set
// where limb l produces a carry by itself and bit l of q where it passes an
// incoming one on, the carries into the limbs are those of the binary sum
// (g | q) + g.  The same rule gives borrows.
__device__ __forceinline__ unsigned long long carries_in(unsigned long long g, unsigned long long q) {
    const unsigned long long x = g | q;
    return (x + g) ^ x ^ g;
}

// s * mult + add for mult, add < 2^31; the result must fit in the wave's limbs.
__device__ __forceinline__ unsigned limbs_mul_add(unsigned s, unsigned mult, unsigned add, int lane) {
    const unsigned long long prod = (unsigned long long)s * mult;
    const unsigned hi_below = __shfl_up((unsigned)(prod >> 32), 1, kWave);
    const unsigned long long sum = (prod & 0xffffffffull) + (lane == 0 ? add : hi_below);   // < 2^33
    const unsigned c_below = __shfl_up((unsigned)(sum >> 32), 1, kWave);
    const unsigned long long y = (sum & 0xffffffffull) + (lane == 0 ? 0u : c_below);          // <= 2^32
    const unsigned long long cin = carries_in(__ballot((y >> 32) != 0), __ballot(y == 0xffffffffull));
    return (unsigned)y + (unsigned)((cin >> lane) & 1ull);
}

// a - b for a >= b.
__device__ __forceinline__ unsigned limbs_sub(unsigned a, unsigned b, int lane) {
    const unsigned long long bin = carries_in(__ballot(a < b), __ballot(a == b));
    return a - b - (unsigned)((bin >> lane) & 1ull);
}

// The integer in (-P/2, P/2], P = p_0 p_1 ... p_{k-1} (the first k primes of
// the uploaded set), with residue r (exact double in [0, p_i)) on lane i < k.
// Garner's mixed-radix digits, v_i = (r_i - sum_{j<i} v_j p_0...p_{j-1})
// (p_0...p_{i-1})^-1 mod p_i, are found one per step, lane i keeping its
// running sum; then S = v_0 + v_1 p_0 + v_2 p_0 p_1 + ... (Horner) and P as
// limbs, and S - P when 2S > P.  Called by every lane of a wave with the same k
// (1 <= k <= RADIC_MAX_PRIMES); returns sign (-1, 0, 1), the number of
// significant limbs, and limb `lane` of the magnitude.
__device__ inline void wave_crt(double r, int k, int lane, int& sign, int& len, unsigned& limb) {
    const bool own = lane < k;
    const int li = own ? lane : 0;
    const double p = g_prime[li], pinv = g_prime_inv[li];
    double t = 0.0, w = 1.0, v = 0.0;   // running sum mod p_lane; p_0...p_{j-1} mod p_lane; digit
    for (int j = 0; j < k; ++j) {
        if (lane == j) v = mulmod(submod(r, t, p), (double)g_garner_inv[j], p, pinv);
        const double vj = __shfl(v, j, kWave);
        if (own && lane > j) {
            t = addmod(t, mulmod(canon(vj, p, pinv), w, p, pinv), p);
            w = mulmod(w, canon(g_prime[j], p, pinv), p, pinv);
        }
    }
    unsigned s = 0, pm = lane == 0 ? 1u : 0u;
    for (int i = k - 1; i >= 0; --i) s = limbs_mul_add(s, (unsigned)g_prime[i], (unsigned)__shfl(v, i, kWave), lane);
    for (int i = 0; i < k; ++i) pm = limbs_mul_add(pm, (unsigned)g_prime[i], 0u, lane);
    // compare 2S with P (P is odd, so they differ)
    const unsigned s_below = __shfl_up(s, 1, kWave);
    const unsigned s2 = (s << 1) | (lane == 0 ? 0u : s_below >> 31);
    const unsigned long long diff = __ballot(s2 != pm);
    bool above = false;
    if (diff) {
        const int top = 63 - __builtin_clzll(diff);
        above = __shfl(s2, top, kWave) > __shfl(pm, top, kWave);
    }
    const unsigned mag = above ? limbs_sub(pm, s, lane) : s;
    const unsigned long long nz = __ballot(mag != 0u);
    len = nz ? 64 - __builtin_clzll(nz) : 0;
    sign = len == 0 ? 0 : (above ? -1 : 1);
    limb = mag;
}

}  // namespace radic
