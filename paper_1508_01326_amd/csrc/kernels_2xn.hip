// Radic determinant of a 2 x n matrix in O(n) (the two-row special case that
// the paper's introduction cites as prior work).
//
// With u_j = (-1)^j a_1j and v_j = (-1)^j a_2j (1-based j), the signed minors of
// eq. (1) with r = 3 sum to
//     det(A) = - sum_{j<k} (u_j v_k - u_k v_j) = - sum_k (U_{k-1} v_k - V_{k-1} u_k),
// U, V the prefix sums of u, v.  A run of columns is summarised by the triple
// (U, V, C) of its sums and its own cross sum C; two adjacent runs combine as
//     (U1, V1, C1) + (U2, V2, C2) = (U1 + U2, V1 + V2, C1 + C2 + U1 V2 - V1 U2),
// an associative operation, so the columns are reduced by threads, then
// workgroups, then one finishing workgroup, always in column order (bitwise
// reproducible).  Every quantity is a double-double (TwoSum / FMA products).
// B carries the same recurrence on |u|, |v| with all signs positive: an upper
// bound on sum_{j<k} |u_j v_k - u_k v_j| >= sum |det(A_J)|.
#include "radic_internal.h"

namespace radic {

struct DD {
    double h, l;
};

__device__ __forceinline__ DD dd(double x) { return DD{x, 0.0}; }

__device__ __forceinline__ DD dd_plus(DD a, DD b) {
    double s, e;
    two_sum(a.h, b.h, s, e);
    e += a.l + b.l;
    const double h = s + e;
    return DD{h, e - (h - s)};
}

__device__ __forceinline__ DD dd_mul(DD a, DD b) {
    const double p = a.h * b.h;
    const double e = __builtin_fma(a.h, b.h, -p) + (a.h * b.l + a.l * b.h);
    const double h = p + e;
    return DD{h, e - (h - p)};
}

__device__ __forceinline__ DD dd_neg(DD a) { return DD{-a.h, -a.l}; }

struct Run {
    DD U, V, C;    // signed sums and cross sum
    DD Ua, Va, B;  // absolute sums and bound
};

__device__ __forceinline__ Run run_combine(const Run& x, const Run& y) {
    Run r;
    r.U = dd_plus(x.U, y.U);
    r.V = dd_plus(x.V, y.V);
    r.C = dd_plus(dd_plus(x.C, y.C), dd_plus(dd_mul(x.U, y.V), dd_neg(dd_mul(x.V, y.U))));
    r.Ua = dd_plus(x.Ua, y.Ua);
    r.Va = dd_plus(x.Va, y.Va);
    r.B = dd_plus(dd_plus(x.B, y.B), dd_plus(dd_mul(x.Ua, y.Va), dd_mul(x.Va, y.Ua)));
    return r;
}

__device__ __forceinline__ Run run_zero() {
    Run r;
    r.U = r.V = r.C = r.Ua = r.Va = r.B = dd(0.0);
    return r;
}

// Fixed-order tree over the workgroup's runs (run i of thread i), result in s[0].
__device__ void tree_combine(Run* s) {
    for (int w = 1; w < (int)blockDim.x; w <<= 1) {
        __syncthreads();
        const int i = threadIdx.x;
        if ((i % (2 * w)) == 0 && i + w < (int)blockDim.x) s[i] = run_combine(s[i], s[i + w]);
    }
    __syncthreads();
}

// Pass 1: workgroup g reduces columns [g * per_group, (g + 1) * per_group).
__global__ __launch_bounds__(256) void k_2xn_runs(const double* A, long long lda, long long n, long long per_group,
                                                  Run* runs, int* nonfinite) {
    __shared__ Run s[256];
    const long long g0 = (long long)blockIdx.x * per_group;
    const long long g1 = g0 + per_group < n ? g0 + per_group : n;
    const long long per_thread = (per_group + blockDim.x - 1) / blockDim.x;
    const long long t0 = g0 + (long long)threadIdx.x * per_thread;
    const long long t1 = t0 + per_thread < g1 ? t0 + per_thread : g1;
    Run r = run_zero();
    int bad = 0;
    for (long long j = t0; j < t1; ++j) {
        const double sg = (j & 1) ? 1.0 : -1.0;   // (-1)^(j+1) for the 0-based column j
        const double a1 = A[j], a2 = A[lda + j];
        bad |= (!isfinite(a1) || !isfinite(a2)) ? 1 : 0;
        const double u = sg * a1, v = sg * a2;
        // appending column j: C += U v - V u, B += Ua |v| + Va |u|
        r.C = dd_plus(r.C, dd_plus(dd_mul(r.U, dd(v)), dd_neg(dd_mul(r.V, dd(u)))));
        r.B = dd_plus(r.B, dd_plus(dd_mul(r.Ua, dd(fabs(v))), dd_mul(r.Va, dd(fabs(u)))));
        r.U = dd_plus(r.U, dd(u));
        r.V = dd_plus(r.V, dd(v));
        r.Ua = dd_plus(r.Ua, dd(fabs(u)));
        r.Va = dd_plus(r.Va, dd(fabs(v)));
    }
    s[threadIdx.x] = r;
    if (bad) atomicOr(nonfinite, 1);
    tree_combine(s);
    if (threadIdx.x == 0) runs[blockIdx.x] = s[0];
}

// Pass 2: one workgroup combines the G runs in order and writes the result.
__global__ __launch_bounds__(256) void k_2xn_finish(const Run* runs, int G, const int* nonfinite, long long n,
                                                    radic_f64_result* out) {
    __shared__ Run s[256];
    const int per = (G + blockDim.x - 1) / blockDim.x;
    Run r = run_zero();
    for (int i = threadIdx.x * per; i < (int)((threadIdx.x + 1) * per) && i < G; ++i) r = run_combine(r, runs[i]);
    s[threadIdx.x] = r;
    tree_combine(s);
    if (threadIdx.x == 0) {
        const Run t = s[0];
        radic_f64_result o;
        o.hi = -t.C.h;            // (-1)^r with r = 1 + 2
        o.lo = -t.C.l;
        o.value = o.hi + o.lo;
        o.abs_sum = t.B.h + t.B.l;
        o.n_subsets = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
        o.n_fallback = 0;
        o.status = *nonfinite ? RADIC_ENONFINITE : RADIC_OK;
        o.reserved = 0;
        if (*nonfinite) o.value = __builtin_nan("");
        *out = o;
    }
}

__global__ void k_2xn_clear(int* flag) { *flag = 0; }

size_t run_bytes() { return sizeof(Run); }

hipError_t launch_2xn(const double* A, long long lda, long long n, int G, void* runs, void* flag,
                      radic_f64_result* out, hipStream_t s) {
    const long long per_group = (n + G - 1) / G;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_2xn_clear, dim3(1), dim3(1), 0, s, static_cast<int*>(flag));
    hipLaunchKernelGGL(k_2xn_runs, dim3(G), dim3(256), 0, s, A, lda, n, per_group, static_cast<Run*>(runs),
                       static_cast<int*>(flag));
    hipLaunchKernelGGL(k_2xn_finish, dim3(1), dim3(256), 0, s, static_cast<const Run*>(runs), G,
                       static_cast<const int*>(flag), n, out);
    return hipGetLastError();
}

}  // namespace radic
