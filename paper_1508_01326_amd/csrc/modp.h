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

// Chinese remaindering of residues res[i] mod pr[i] (the first k primes of the
// uploaded set, whose Garner inverses are in g_garner_inv),
// Garner's mixed-radix form: S = v_0 + v_1 p_0 + v_2 p_0 p_1 + ..., then the
// representative in (-P/2, P/2], P = prod p_i, written as sign (-1, 0, 1) and
// little-endian 32-bit limbs mag[0..len-1] (mag holds at least k + 1 limbs).
__device__ inline void crt_to_limbs(const unsigned long long* res, const unsigned long long* pr, int k, int& sign,
                                    int& len_out, unsigned* mag) {
    unsigned long long v[RADIC_MAX_PRIMES];
    for (int i = 0; i < k; ++i) {
        // value of the digits found so far mod p_i, times the uploaded inverse of
        // the product of the earlier primes (pr is the uploaded prime set)
        unsigned long long t = 0;
        for (int j = i - 1; j >= 0; --j) t = (t * (pr[j] % pr[i]) + v[j]) % pr[i];
        const unsigned long long diff = (res[i] % pr[i] + pr[i] - t) % pr[i];
        v[i] = i == 0 ? res[0] % pr[0] : (diff * g_garner_inv[i]) % pr[i];
    }
    // S = v_{k-1}; S = S * p_i + v_i (Horner, 32-bit limbs); P = prod p_i
    unsigned S[RADIC_MAX_PRIMES + 1] = {0}, Pm[RADIC_MAX_PRIMES + 1] = {0};
    int len = 0, plen = 1;
    Pm[0] = 1;
    for (int i = k - 1; i >= 0; --i) {
        unsigned long long carry = v[i];
        for (int l = 0; l < len; ++l) {
            const unsigned long long cur = (unsigned long long)S[l] * pr[i] + carry;
            S[l] = (unsigned)cur;
            carry = cur >> 32;
        }
        while (carry) {
            S[len++] = (unsigned)carry;
            carry >>= 32;
        }
    }
    for (int i = 0; i < k; ++i) {
        unsigned long long carry = 0;
        for (int l = 0; l < plen; ++l) {
            const unsigned long long cur = (unsigned long long)Pm[l] * pr[i] + carry;
            Pm[l] = (unsigned)cur;
            carry = cur >> 32;
        }
        while (carry) {
            Pm[plen++] = (unsigned)carry;
            carry >>= 32;
        }
    }
    // compare 2S with P
    unsigned S2[RADIC_MAX_PRIMES + 2] = {0};
    int s2len = len;
    {
        unsigned carry = 0;
        for (int l = 0; l < len; ++l) {
            S2[l] = (S[l] << 1) | carry;
            carry = S[l] >> 31;
        }
        if (carry) S2[s2len++] = carry;
    }
    int cmp = 0;
    if (s2len != plen) cmp = s2len > plen ? 1 : -1;
    else
        for (int l = plen - 1; l >= 0 && cmp == 0; --l)
            if (S2[l] != Pm[l]) cmp = S2[l] > Pm[l] ? 1 : -1;
    sign = len == 0 ? 0 : 1;
    if (cmp > 0) {   // S > P/2: the value is S - P < 0; magnitude P - S
        long long borrow = 0;
        for (int l = 0; l < plen; ++l) {
            long long cur = (long long)Pm[l] - (l < len ? (long long)S[l] : 0) - borrow;
            borrow = cur < 0;
            S[l] = (unsigned)(cur + (borrow ? (1ll << 32) : 0));
        }
        len = plen;
        sign = -1;
    }
    while (len > 0 && S[len - 1] == 0) --len;
    if (len == 0) sign = 0;
    len_out = len;
    for (int l = 0; l < len; ++l) mag[l] = S[l];
}

}  // namespace radic
