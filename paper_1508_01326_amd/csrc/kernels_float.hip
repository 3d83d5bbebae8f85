// Floating-point Radic determinant kernels for gfx950.
//
// One lane owns a chunk of `spl` consecutive dictionary ranks (the granularity
// scheme of Section 5).  Consecutive lanes of a wave own consecutive chunks, so
// the 64 minors a wave factors at any moment lie in a short stretch of the
// dictionary order and share their leading columns; the pivot row of the first
// LU steps is then usually the same in every lane, and row exchanges are done by
// a scalar branch over the distinct pivot rows present in the wave ("waterfall")
// instead of per-lane select chains.  Per subset a lane:
//   1. holds its ascending sequence as M column indices (unranked once per chunk
//      with the combinatorial addition of Section 4, then advanced with the
//      dictionary successor of Section 5);
//   2. gathers the M columns of the minor from LDS, where the workgroup staged A
//      column-major once (the EREW replication of A in Section 6 becomes one
//      staging per workgroup);
//   3. factors the minor by LU with partial pivoting in registers;
//   4. applies (-1)^(r+s) and the row-exchange parity (Definition 3, eq. (1));
//   5. accumulates the signed term with TwoSum into a double-double and |det|.
// Partials are combined wave -> workgroup -> grid in a fixed order (the tree sum
// of Section 6), so results are bitwise reproducible for a given launch shape.
#include <type_traits>

#include "lu_float.h"

namespace radic {

// Per-wave copy of the columns the lanes gather from, rows in the wave's order.
template <int M, bool F32> __host__ __device__ int wave_copy_bytes(int n) {
    return F32 ? align16(n * Layout<M>::st32 * 4) : align16(n * Layout<M>::st64 * 8);
}

// LDS per workgroup: binomial table, master copies of A (double; float for F32),
// then per wave: its row-ordered copy and, with QUEUE (FP32 export), its
// fallback region.
template <int M, bool F32, bool QUEUE> __host__ __device__ int lds_bytes(int n, int waves) {
    int b = binom_bytes<M>(n) + align16(n * Layout<M>::st64 * 8);
    if (F32) b += align16(n * Layout<M>::st32 * 4);
    b += waves * (wave_copy_bytes<M, F32>(n) + (QUEUE ? fallback_wave_bytes<M>() : 0));
    return b;
}

// Rewrite the wave's copy with rows in the order `perm` (copy row r = master row
// perm[r]); the column-scale slot of the float layout is row independent.
template <int M, typename T>
__device__ void write_wave_copy(T* dst, const T* master, int stride, int n, unsigned long long perm, int lane,
                                bool scale_slot) {
    wave_lds_sync();
    for (int e = lane; e < n * M; e += kWave) {
        const int j = e / M, r = e - j * M;
        const int src = (int)((perm >> (4 * r)) & 15ull);
        dst[j * stride + r] = master[j * stride + src];
    }
    if (scale_slot)
        for (int j = lane; j < n; j += kWave) dst[j * stride + M] = master[j * stride + M];
    wave_lds_sync();
}

// ---------------------------------------------------------------- staging
// Stage A column-major into LDS (double copy; for F32 also the row-scaled float
// copy and the per-column scale).  Returns the workgroup-wide non-finite flag.
// F32: rows scaled by 2^-e_i; WITH_F32: also write the float copy and its
// reciprocal column scales.
template <int M, bool F32, bool WITH_F32 = F32>
__device__ int stage_matrix(const FloatJob& J, double* cd, float* cf, int* rowexp) {
    constexpr int ST64 = Layout<M>::st64, ST32 = Layout<M>::st32;
    const int n = J.n;
    int bad = 0;
    if (F32) {
        // e_i: exponent of the row maximum, max|a_ij| = f 2^e_i with f in [0.5, 1)
        if (threadIdx.x < M) {
            const double* row = J.A + (long long)threadIdx.x * J.lda;
            double mx = 0.0;
            for (int j = 0; j < n; ++j) mx = fmax(mx, fabs(row[j]));
            int e = 0;
            if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
            rowexp[threadIdx.x] = e;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < M * n; e += blockDim.x) {
        int i = e / n, j = e - i * n;
        double v = J.A[(long long)i * J.lda + j];
        bad |= !isfinite(v);
        if (F32) v = ldexp(v, -rowexp[i]);   // exact power-of-two scaling
        cd[j * ST64 + i] = v;
        if (WITH_F32) cf[j * ST32 + i] = (float)v;
    }
    bad = __syncthreads_or(bad);
    if (WITH_F32) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) s = fmaxf(s, fabsf(cf[j * ST32 + i]));
            cf[j * ST32 + M] = s > 0.f ? 1.0f / s : 0.f;   // reciprocal column scale 1/s_j
        }
        __syncthreads();
    }
    return bad;
}

// Refactor queued minors in double with the whole wave on one minor at a time
// (LDS-resident, few registers); used when exporting FP32-bulk terms, where each
// term must land at its own rank.  Lane 0 accumulates the terms.
template <int M, bool EXPORT>
__device__ void flush_fallback(const FloatJob& J, const double* cd, const unsigned* queue, int count, double* W,
                               int lane, double& hi, double& lo, double& ab, int scale_exp) {
    for (int e = 0; e < count; ++e) {
        int c[M];
        unpack_cols<M>(queue + 4 * e, c);
        const unsigned off = queue[4 * e + 3];
        const double d = coop_det_f64<M>(cd, c, W, lane);
        const double term = radic_sign_odd<M>(c) ? -d : d;
        if (lane == 0) {
            double s, err;
            two_sum(hi, term, s, err);
            hi = s;
            lo += err;
            ab += fabs(d);
            if (EXPORT) J.terms[off] = ldexp(term, scale_exp);
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------- main kernel
template <int M, bool F32, bool EXPORT, bool DEFER>
__global__ __launch_bounds__(kMaxBlock) void k_radic_float(FloatJob J) {
    using T = typename std::conditional<F32, float, double>::type;
    constexpr int ST64 = Layout<M>::st64, ST32 = Layout<M>::st32;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rowexp[RADIC_MAX_M];
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];

    const int n = J.n;
    const int waves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;

    unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
    double* cd = reinterpret_cast<double*>(smem + binom_bytes<M>(n));
    float* cf = reinterpret_cast<float*>(smem + binom_bytes<M>(n) + align16(n * ST64 * 8));
    constexpr bool QUEUE = F32 && !DEFER;
    unsigned char* wr = smem + binom_bytes<M>(n) + align16(n * ST64 * 8) + (F32 ? align16(n * ST32 * 4) : 0) +
                        wave * (wave_copy_bytes<M, F32>(n) + (QUEUE ? fallback_wave_bytes<M>() : 0));
    T* wcopy = reinterpret_cast<T*>(wr);
    unsigned char* fb = wr + wave_copy_bytes<M, F32>(n);
    unsigned* queue = reinterpret_cast<unsigned*>(fb);
    double* W = reinterpret_cast<double*>(fb + kFallbackCap * 16);

    stage_binomials<M>(bt, n);
    const int bad = stage_matrix<M, F32>(J, cd, cf, rowexp);
    if (!EXPORT && blockIdx.x == 0 && threadIdx.x == 0) {
        J.header->nonfinite = bad;
        int se = 0;
        if (F32)
            for (int i = 0; i < M; ++i) se += rowexp[i];
        J.header->scale_exp = se;
    }

    // exported terms are returned in the units of A (row scaling undone)
    int scale_exp = 0;
    if (F32 && EXPORT)
        for (int i = 0; i < M; ++i) scale_exp += rowexp[i];
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    int qcount = 0;   // wave-uniform length of the LDS queue (export)
    int gcount = 0;   // wave-uniform number of flagged minors (deferred refactorisation)
    const T* master = F32 ? reinterpret_cast<const T*>(cf) : reinterpret_cast<const T*>(cd);
    const int colstride = F32 ? ST32 : ST64;
    const T tau = (T)J.tau;
    // the wave's row order (4 bits per position, identity to start) and its parity
    unsigned long long perm = 0;
#pragma unroll
    for (int r = 0; r < M; ++r) perm |= (unsigned long long)r << (4 * r);
    int perm_odd = 0;
    write_wave_copy<M, T>(wcopy, master, colstride, n, perm, lane, F32);
    const T* colbase = wcopy;

    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const unsigned long long nwaves = (unsigned long long)gridDim.x * waves;
    bool overflow = false;   // wave-uniform: more flagged minors than the segment holds
    for (unsigned long long wc = gwave * kWave; wc < J.chunks && !overflow; wc += nwaves * kWave) {
        const unsigned long long chunk = wc + lane;
        const bool vchunk = chunk < J.chunks;
        const unsigned long long off0 = vchunk ? chunk * (unsigned long long)J.spl : J.count - 1;
        const unsigned long long left = J.count - off0;
        const int cnt = vchunk ? (int)(left < (unsigned long long)J.spl ? left : (unsigned long long)J.spl) : 0;
        int col[M];
        unrank<M>(J.q_begin + off0, n, bt, col);
        for (int s = 0; s < J.spl; ++s) {
            const bool valid = s < cnt;
            T a[M][M];
            gather<M, T>(a, colbase, colstride, col);
            T sc[M];
            if (F32) {
#pragma unroll
                for (int j = 0; j < M; ++j) sc[j] = colbase[col[j] * colstride + M];
            }
            // the minor was gathered with rows in the wave's order: det(P A_J) = sgn(P) det(A_J)
            bool neg = radic_sign_odd<M>(col) ^ (perm_odd != 0);
            bool flag = false;
            const unsigned long long perm_before = perm;
            const T det = lu_det<M, T, F32>(a, neg, flag, sc, tau, perm, perm_odd);
            flag = flag && valid;
            if (valid && !flag) {
                const double d = (double)det;
                const double term = neg ? -d : d;
                double sum, err;
                two_sum(hi, term, sum, err);
                hi = sum;
                lo += err;
                ab += fabs(d);
                if (EXPORT) {
                    J.terms[off0 + s] = F32 ? ldexp(term, scale_exp) : term;
                }
            }
            if (EXPORT && valid && J.cols) {
#pragma unroll
                for (int j = 0; j < M; ++j) J.cols[(off0 + s) * M + j] = (unsigned char)(col[j] + 1);
            }
            if (DEFER) {
                const unsigned long long fm = __ballot(flag);
                if (fm) {
                    // append to this wave's global segment; once it would overflow,
                    // the wave stops: the refactorisation kernel then redoes its
                    // whole workgroup in double
                    const int pos = gcount + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                    if (flag && pos < kDeferCap) {
                        unsigned w[3];
                        pack_cols<M>(col, w);
                        unsigned* ent = J.fb_entries + ((size_t)gwave * kDeferCap + pos) * 4;
                        ent[0] = w[0];
                        ent[1] = w[1];
                        ent[2] = w[2];
                        ent[3] = 0u;
                        nfb += 1;
                    }
                    gcount += __popcll(fm);
                    if (gcount > kDeferCap) {
                        overflow = true;
                        break;
                    }
                }
            }
            if (QUEUE) {
                const unsigned long long fm = __ballot(flag);
                if (fm) {
                    if (flag) {
                        const int pos = qcount + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                        unsigned w[3];
                        pack_cols<M>(col, w);
                        queue[4 * pos + 0] = w[0];
                        queue[4 * pos + 1] = w[1];
                        queue[4 * pos + 2] = w[2];
                        queue[4 * pos + 3] = (unsigned)(off0 + s);
                        nfb += 1;
                    }
                    qcount += __popcll(fm);
                    if (qcount > kFallbackCap - kWave) {
                        wave_lds_sync();
                        flush_fallback<M, EXPORT>(J, cd, queue, qcount, W, lane, hi, lo, ab, scale_exp);
                        qcount = 0;
                    }
                }
            }
            if (perm != perm_before) write_wave_copy<M, T>(wcopy, master, colstride, n, perm, lane, false);
            successor<M>(col, n);
        }
    }
    if (QUEUE && qcount > 0) {
        wave_lds_sync();
        flush_fallback<M, EXPORT>(J, cd, queue, qcount, W, lane, hi, lo, ab, scale_exp);
    }
    if (EXPORT) return;
    if (DEFER && lane == 0) J.fb_count[gwave] = (unsigned)gcount;   // above kDeferCap: overflowed

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

// Redo in double every rank a wave of the float launch was given (same chunk
// mapping), rows in natural order from the row-scaled double copy cd.  Counts
// the valid ranks in nvalid.
template <int M>
__device__ void redo_wave_f64(const FloatJob& J, const unsigned long long* bt, const double* cd,
                              unsigned long long gwave, unsigned long long nwaves, int lane, double& hi, double& lo,
                              double& ab, unsigned long long& nvalid) {
    constexpr int ST64 = Layout<M>::st64;
    const double none[M] = {};
    for (unsigned long long wc = gwave * kWave; wc < J.chunks; wc += nwaves * kWave) {
        const unsigned long long chunk = wc + lane;
        const bool vchunk = chunk < J.chunks;
        const unsigned long long off0 = vchunk ? chunk * (unsigned long long)J.spl : J.count - 1;
        const unsigned long long left = J.count - off0;
        const int cnt = vchunk ? (int)(left < (unsigned long long)J.spl ? left : (unsigned long long)J.spl) : 0;
        int col[M];
        unrank<M>(J.q_begin + off0, J.n, bt, col);
        for (int s = 0; s < J.spl; ++s) {
            double a[M][M];
            gather<M, double>(a, cd, ST64, col);
            bool neg = radic_sign_odd<M>(col);
            bool flag = false;
            unsigned long long perm = 0;   // row order is not tracked here
            int perm_odd = 0;
            const double d = lu_det<M, double, false>(a, neg, flag, none, 0.0, perm, perm_odd);
            if (s < cnt) {
                const double term = neg ? -d : d;
                double sum, err;
                two_sum(hi, term, sum, err);
                hi = sum;
                lo += err;
                ab += fabs(d);
                nvalid += 1;
            }
            successor<M>(col, J.n);
        }
    }
}

// Deferred refactorisation: every wave of the float launch queued its flagged
// minors in a global segment; here one wave per segment refactors them in
// double, one minor per lane, and each workgroup writes the partial of its
// segments.  A workgroup with an overflowed segment instead redoes all of its
// ranks in double and clears the float partial it replaces.  Segments are read
// in wave order, so the sum is reproducible.
template <int M>
__global__ __launch_bounds__(kMaxBlock) void k_refactor_deferred(FloatJob J) {
    constexpr int ST64 = Layout<M>::st64;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rowexp[RADIC_MAX_M];
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];
    __shared__ int any, over;
    const int waves = blockDim.x / kWave, wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const int count = (int)J.fb_count[gwave];
    if (threadIdx.x == 0) any = over = 0;
    __syncthreads();
    if (lane == 0 && count > 0) atomicOr(&any, 1);
    if (lane == 0 && count > kDeferCap) atomicOr(&over, 1);
    __syncthreads();
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    if (any) {
        unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
        double* cd = reinterpret_cast<double*>(smem + binom_bytes<M>(J.n));
        if (over) stage_binomials<M>(bt, J.n);
        (void)stage_matrix<M, true, false>(J, cd, nullptr, rowexp);
        if (over)
            redo_wave_f64<M>(J, bt, cd, gwave, (unsigned long long)gridDim.x * waves, lane, hi, lo, ab, nfb);
        else
            refactor_queue_f64<M>(cd, J.fb_entries + gwave * kDeferCap * 4, count, lane, hi, lo, ab,
                                  [](int, double) {});
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
        double h = red[0], l = red[1], a2 = red[2];
        unsigned long long nf = redn[0];
        for (int w = 1; w < waves; ++w) {
            dd_add(h, l, red[4 * w + 0], red[4 * w + 1]);
            a2 += red[4 * w + 2];
            nf += redn[w];
        }
        J.fb_partials[blockIdx.x] = Partial{h, l, a2, nf};
        if (over) J.partials[blockIdx.x] = Partial{0.0, 0.0, 0.0, 0ull};
    }
}

// Fixed-order reduction of the workgroup partials into the result record.
__global__ __launch_bounds__(256) void k_finalize_float(const Partial* parts, const Partial* fb_parts, int G,
                                                        const DetHeader* h, radic_f64_result* out,
                                                        unsigned long long count, int use_scale) {
    __shared__ double sh[256], sl[256], sa[256];
    __shared__ unsigned long long sn[256];
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nf = 0;
    for (int i = threadIdx.x; i < G; i += blockDim.x) {
        Partial p = parts[i];
        dd_add(hi, lo, p.hi, p.lo);
        ab += p.abs;
        nf += p.nfb;
        if (fb_parts) {
            const Partial q = fb_parts[i];
            dd_add(hi, lo, q.hi, q.lo);
            ab += q.abs;
            nf += q.nfb;
        }
    }
    sh[threadIdx.x] = hi;
    sl[threadIdx.x] = lo;
    sa[threadIdx.x] = ab;
    sn[threadIdx.x] = nf;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double a = sh[threadIdx.x], b = sl[threadIdx.x];
            dd_add(a, b, sh[threadIdx.x + w], sl[threadIdx.x + w]);
            sh[threadIdx.x] = a;
            sl[threadIdx.x] = b;
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sn[threadIdx.x] += sn[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int e = use_scale ? h->scale_exp : 0;
        radic_f64_result r;
        r.hi = ldexp(sh[0], e);
        r.lo = ldexp(sl[0], e);
        r.abs_sum = ldexp(sa[0], e);
        r.value = r.hi + r.lo;
        r.n_subsets = count;
        r.n_fallback = sn[0];
        r.status = h->nonfinite ? RADIC_ENONFINITE : RADIC_OK;
        r.reserved = 0;
        if (h->nonfinite) r.value = __builtin_nan("");
        *out = r;
    }
}

__global__ void k_write_zero_result(radic_f64_result* out) {
    radic_f64_result r{};
    r.status = RADIC_OK;
    *out = r;
}

// ---------------------------------------------------------------- host launchers
template <int M, bool F32, bool EXPORT>
static hipError_t launch_m(const FloatJob& J, int grid, int block, hipStream_t s) {
    constexpr bool DEFER = F32 && !EXPORT;
    const int lds = lds_bytes<M, F32, F32 && !DEFER>(J.n, block / kWave);
    (void)hipGetLastError();   // clear an error left by an earlier, unrelated call
    hipLaunchKernelGGL((k_radic_float<M, F32, EXPORT, DEFER>), dim3(grid), dim3(block), lds, s, J);
    return hipGetLastError();
}

template <bool F32, bool EXPORT>
static hipError_t launch_dispatch(int m, const FloatJob& J, int grid, int block, hipStream_t s) {
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return launch_m<MM, F32, EXPORT>(J, grid, block, s);
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int M>
static hipError_t launch_refactor_m(const FloatJob& J, int grid, int block, hipStream_t s) {
    const int lds = binom_bytes<M>(J.n) + align16(J.n * Layout<M>::st64 * 8);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_refactor_deferred<M>, dim3(grid), dim3(block), lds, s, J);
    return hipGetLastError();
}

hipError_t launch_refactor(int m, const FloatJob& J, int grid, int block, hipStream_t s) {
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return launch_refactor_m<MM>(J, grid, block, s);
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
}

int float_lds_bytes(int m, int n, int prec, int waves) {
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return prec == RADIC_FP32_BULK ? lds_bytes<MM, true, true>(n, waves) : lds_bytes<MM, false, false>(n, waves);
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return 1 << 30;
    }
}

hipError_t launch_float(int m, int prec, bool export_terms, const FloatJob& J, int grid, int block, hipStream_t s) {
    if (prec == RADIC_FP32_BULK)
        return export_terms ? launch_dispatch<true, true>(m, J, grid, block, s)
                            : launch_dispatch<true, false>(m, J, grid, block, s);
    return export_terms ? launch_dispatch<false, true>(m, J, grid, block, s)
                        : launch_dispatch<false, false>(m, J, grid, block, s);
}

hipError_t launch_finalize_float(const Partial* parts, const Partial* fb_parts, int G, const DetHeader* h,
                                 radic_f64_result* out, unsigned long long count, int use_scale, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_finalize_float, dim3(1), dim3(256), 0, s, parts, fb_parts, G, h, out, count, use_scale);
    return hipGetLastError();
}

hipError_t launch_zero_result(radic_f64_result* out, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_write_zero_result, dim3(1), dim3(1), 0, s, out);
    return hipGetLastError();
}

hipError_t upload_binomials_float(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

}  // namespace radic
