// Enumeration of the prefix-shared kernels' two-sided blocks over a whole rank
// space (see split_shape in radic_internal.h): the prefix counts and the
// unranking of one prefix, shared by the kernels and the host (the launchers
// size their grids with it, and the host-side helpers exported for testing
// call it on a host binomial table).
#pragma once

#include "radic_internal.h"

namespace radic {

// Two-sided blocks (see split_shape).  The side-s prefixes with last column v
// number sum_{i >= imin} C(a, i) C(b, m-3-i): i of their first m-3 columns lie
// below a, the others in [a, v).  They are ordered by i, then by the columns
// in [a, v) (colex), then by those below a (colex), and cut into runs of
// colex_run(r, K) prefixes.  Blocks go over v upwards, side 0 before side 1
// for each v (both sides of a v have r = n-1-v later columns), so the heaviest
// come first and no block spans two values of v or two sides.
// bt[x*stride + y] = C(x, y) for y <= m-3.
template <int P>
__host__ __device__ inline unsigned long long split_count(int n, int side, int v, const unsigned long long* bt,
                                                          int stride) {
    int a, b, imin;
    bool on;
    split_shape(P, n, side, v, a, b, imin, on);
    unsigned long long N = 0;
    if (on)
        for (int i = imin; i <= P - 1; ++i) N += bt[a * stride + i] * bt[b * stride + (P - 1 - i)];
    return N;
}

// Largest x in [deg-1, lim-1] with C(x, deg) <= t (deg >= 1, t < C(lim, deg)).
__host__ __device__ inline int colex_digit(unsigned long long t, int deg, int lim, const unsigned long long* bt,
                                           int stride) {
    if (deg == 1) return (int)t;
    int lo = deg - 1, h = lim - 1;
    while (lo < h) {
        const int mid = (lo + h + 1) >> 1;
        if (bt[mid * stride + deg] <= t) lo = mid;
        else h = mid - 1;
    }
    return lo;
}

// The j-th side-s prefix with last column v (j < split_count) to its columns
// c_0 < ... < c_{m-3} = v, in the coordinates of its side.
template <int P>
__host__ __device__ inline void split_unrank(unsigned long long j, int n, int side, int v,
                                             const unsigned long long* bt, int stride, int (&c)[P]) {
    int a, b, imin;
    bool on;
    split_shape(P, n, side, v, a, b, imin, on);
    int i = imin;
    for (; i < P - 1; ++i) {
        const unsigned long long t = bt[a * stride + i] * bt[b * stride + (P - 1 - i)];
        if (j < t) break;
        j -= t;
    }
    // j = hi * C(a, i) + lo: hi numbers the columns in [a, v), lo those below a
    const unsigned long long A = bt[a * stride + i];
    unsigned long long hi, lo;
    if ((j >> 32) == 0 && (A >> 32) == 0) {
        hi = (unsigned)j / (unsigned)A;
        lo = (unsigned)j - (unsigned)hi * (unsigned)A;
    } else {
        hi = j / A;
        lo = j - hi * A;
    }
    int hlim = b, llim = a;
#pragma unroll
    for (int k = P - 2; k >= 0; --k) {
        const bool high = k >= i;
        const int deg = high ? k - i + 1 : k + 1;
        const unsigned long long t = high ? hi : lo;
        const int x = colex_digit(t, deg, high ? hlim : llim, bt, stride);
        const unsigned long long rest = t - (deg == 1 ? (unsigned long long)x : bt[x * stride + deg]);
        if (high) {
            hi = rest;
            hlim = x;
            c[k] = a + x;
        } else {
            lo = rest;
            llim = x;
            c[k] = x;
        }
    }
    c[P - 1] = v;
}

// Blocks of about K minors (colex_run(r, K) prefixes each) that the side-s
// prefixes with last column v are cut into.
template <int P>
__host__ __device__ inline unsigned long long split_blocks_at(int n, int side, int v, unsigned K,
                                                              const unsigned long long* bt, int stride) {
    const unsigned long long cnt = split_count<P>(n, side, v, bt, stride);
    const unsigned long long k = (unsigned long long)colex_run(n - 1 - v, K);
    return (cnt + k - 1) / k;
}

}  // namespace radic
