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

#include "prefix.h"
#include "stage.h"

namespace radic {

// LDS per workgroup: binomial table, master copies of A (double; float for F32),
// then per wave: its row-ordered copy and, with QUEUE (FP32 export), its
// fallback region.
template <int M, bool F32, bool QUEUE> __host__ __device__ int lds_bytes(int n, int waves) {
    int b = binom_bytes<M>(n) + align16(n * Layout<M>::st64 * 8);
    if (F32) b += align16(n * Layout<M>::st32 * 4);
    b += waves * (wave_copy_bytes<M, F32>(n) + (QUEUE ? fallback_wave_bytes<M>() : 0));
    return b;
}

// Refactor queued minors in double with the whole wave on one minor at a time
// (LDS-resident, few registers); used when exporting FP32-bulk terms, where each
// term must land at its own rank.  The queue holds rank offsets, unranked here.
// Lane 0 accumulates the terms.
template <int M, bool EXPORT>
__device__ void flush_fallback(const FloatJob& J, const unsigned long long* bt, const double* cd,
                               const unsigned* queue, int count, double* W, int lane, double& hi, double& lo,
                               double& ab, int scale_exp) {
    for (int e = 0; e < count; ++e) {
        const unsigned off = queue[e];
        int c[M];
        unrank<M>(J.q_begin + off, J.n, bt, c);
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
    double* W = reinterpret_cast<double*>(fb + kFallbackCap * 4);

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
                    if (flag && pos < J.defer_cap) {
                        unsigned w[4];
                        pack_cols<M>(col, w);
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
            if (QUEUE) {
                const unsigned long long fm = __ballot(flag);
                if (fm) {
                    if (flag) {
                        const int pos = qcount + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
                        queue[pos] = (unsigned)(off0 + s);
                        nfb += 1;
                    }
                    qcount += __popcll(fm);
                    if (qcount > kFallbackCap - kWave) {
                        wave_lds_sync();
                        flush_fallback<M, EXPORT>(J, bt, cd, queue, qcount, W, lane, hi, lo, ab, scale_exp);
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
        flush_fallback<M, EXPORT>(J, bt, cd, queue, qcount, W, lane, hi, lo, ab, scale_exp);
    }
    if (EXPORT) return;
    if (DEFER && lane == 0) J.fb_count[gwave] = (unsigned)gcount;   // above J.defer_cap: overflowed

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

// Deferred refactorisation.  Every wave of the float launch queued its flagged
// minors in a global segment.  Workgroup j of this kernel takes the segments of
// `R` consecutive float workgroups (R * waves <= 64 segments), concatenates them
// and refactors the entries in double, one per lane, so that lanes stay busy
// even though each segment holds only a few minors.  A float workgroup with an
// overflowed segment is instead redone in double as a whole (its waves' rank
// chunks, by the waves of this workgroup), and its float partial is cleared.
// The entry-to-lane mapping is fixed, so the sum is reproducible.
template <int M>
__global__ __launch_bounds__(kMaxBlock) void k_refactor_deferred(FloatJob J, int G, int R) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rowexp[RADIC_MAX_M];
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];
    __shared__ unsigned segoff[65];
    __shared__ unsigned long long overmask;   // bit b: float workgroup fb0 + b overflowed
    const int waves = blockDim.x / kWave, wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int fb0 = blockIdx.x * R;
    const int nb = min(R, G - fb0);
    const int nseg = nb * waves;
    if (threadIdx.x < 64) {
        // wave 0: per-segment counts, the overflow mask and the exclusive prefix
        // of the counts of segments in non-overflowed workgroups
        const unsigned c = threadIdx.x < nseg ? J.fb_count[(size_t)fb0 * waves + threadIdx.x] : 0u;
        const unsigned long long ov = __ballot(c > (unsigned)J.defer_cap);
        unsigned long long om = 0;
        for (int b = 0; b < nb; ++b)
            if ((ov >> (b * waves)) & ((1ull << waves) - 1ull)) om |= 1ull << b;
        const bool mine_over = threadIdx.x < nseg && ((om >> (threadIdx.x / waves)) & 1ull);
        unsigned v = mine_over ? 0u : c;
        // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const unsigned u = __shfl_up(v, off, kWave);
            if (lane >= off) v += u;
        }
        segoff[threadIdx.x + 1] = v;
        if (threadIdx.x == 0) {
            segoff[0] = 0;
            overmask = om;
        }
    }
    __syncthreads();
    const unsigned E = segoff[nseg];
    const unsigned long long om = overmask;
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    if (E > 0 || om) {
        unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
        double* cd = reinterpret_cast<double*>(smem + binom_bytes<M>(J.n));
        if (om) stage_binomials<M>(bt, J.n);
        (void)stage_matrix<M, true, false>(J, cd, nullptr, rowexp);
        for (int b = 0; b < nb; ++b) {
            if (!((om >> b) & 1ull)) continue;
            const unsigned long long gw = (unsigned long long)(fb0 + b) * waves + wave;
            const unsigned long long nw = (unsigned long long)G * waves;
            if (J.mapping == 0) {
                redo_wave_f64<M>(J, bt, cd, gw, nw, lane, hi, lo, ab, nfb);
            } else if (J.mapping == 1) {
                if constexpr (M >= 3) {
                    // the blocks of m-2 column prefixes this wave of the float launch was given
                    const unsigned long long nblk =
                        J.colex ? J.colex_blocks : (J.p_end - J.p_begin + kPrefixBlock - 1) / kPrefixBlock;
                    // a two-sided block prefix by prefix (in its side's
                    // coordinates), a dictionary block whole
                    for (unsigned long long blk = gw; blk < nblk; blk += nw) {
                        unsigned long long t0 = 0;
                        int segs = 1, side = 0, vlast = 0;
                        if (J.colex) split_block<M - 2>(blk, J.n, bt, M, J.colex_pairs, lane, side, vlast, t0, segs);
                        for (int sgm = 0; sgm < segs; ++sgm) {
                            unsigned long long r0, r1;
                            if (J.colex) split_prefix_ranks<M>(J, bt, side, vlast, t0 + (unsigned long long)sgm, r0, r1);
                            else prefix_block_ranks<M>(J, bt, blk, r0, r1);
                            redo_ranks_f64<M>(J, bt, cd, r0, r1, lane, hi, lo, ab, nfb, side);
                        }
                    }
                }
            } else {
                if constexpr (M >= 4) {
                    // the blocks of m-3 column prefixes
                    const unsigned long long nblk = (J.p_end - J.p_begin + kGroupBlock - 1) / kGroupBlock;
                    for (unsigned long long blk = gw; blk < nblk; blk += nw) {
                        unsigned long long r0, r1;
                        prefix_block_ranks<M, FloatJob, 3, kGroupBlock>(J, bt, blk, r0, r1);
                        redo_ranks_f64<M>(J, bt, cd, r0, r1, lane, hi, lo, ab, nfb);
                    }
                }
            }
            if (threadIdx.x == 0) J.partials[fb0 + b] = Partial{0.0, 0.0, 0.0, 0ull};
        }
        for (unsigned base = (unsigned)wave * kWave; base < E; base += blockDim.x) {
            const unsigned e = base + lane;
            const bool valid = e < E;
            const unsigned ee = valid ? e : base;
            // segment holding entry ee: the last t with segoff[t] <= ee
            int lo_s = 0, hi_s = nseg - 1;
            while (lo_s < hi_s) {
                const int mid = (lo_s + hi_s + 1) >> 1;
                if (segoff[mid] <= ee) lo_s = mid;
                else hi_s = mid - 1;
            }
            const unsigned pos = ee - segoff[lo_s];
            const unsigned* ent = J.fb_entries + (((size_t)fb0 * waves + lo_s) * J.defer_cap + pos) * 4;
            double ad;
            const double term = refactor_entry_f64<M>(cd, ent, ad);
            if (valid) {
                double sum, err;
                two_sum(hi, term, sum, err);
                hi = sum;
                lo += err;
                ab += ad;
            }
        }
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
    }
}

// Fixed-order reduction of the workgroup partials (and of the refactorisation
// partials) into the result record.  Each thread loads its partials in batches
// of eight so that the loads overlap, then waves reduce by butterfly and wave
// results are combined in wave order.
__device__ __forceinline__ void add_partials(const Partial* parts, int G, double& hi, double& lo, double& ab,
                                             unsigned long long& nf) {
    constexpr int U = 8;
    for (int base = threadIdx.x; base < G; base += U * blockDim.x) {
        Partial p[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int i = base + k * blockDim.x;
            p[k] = i < G ? parts[i] : Partial{0.0, 0.0, 0.0, 0ull};
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            dd_add(hi, lo, p[k].hi, p[k].lo);
            ab += p[k].abs;
            nf += p[k].nfb;
        }
    }
}

// use_scale: bit 0 scales by 2^(sum of the row exponents) (FP32-bulk), bit 1
// reports every minor as done in double (an FP32-bulk call over too few minors
// for a float sum, run by the double kernel).
__global__ __launch_bounds__(512) void k_finalize_float(const Partial* parts, int G, const Partial* fb_parts, int G2,
                                                         const DetHeader* h, radic_f64_result* out,
                                                         unsigned long long count, int use_scale) {
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];
    const int waves = blockDim.x / kWave, wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nf = 0;
    add_partials(parts, G, hi, lo, ab, nf);
    if (fb_parts) add_partials(fb_parts, G2, hi, lo, ab, nf);
    wave_reduce_partial(hi, lo, ab, nf);
    if (lane == 0) {
        red[4 * wave + 0] = hi;
        red[4 * wave + 1] = lo;
        red[4 * wave + 2] = ab;
        redn[wave] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sh = red[0], sl = red[1], sa = red[2];
        unsigned long long sn = redn[0];
        for (int w = 1; w < waves; ++w) {
            dd_add(sh, sl, red[4 * w + 0], red[4 * w + 1]);
            sa += red[4 * w + 2];
            sn += redn[w];
        }
        const int e = (use_scale & 1) ? h->scale_exp : 0;
        radic_f64_result r;
        r.hi = ldexp(sh, e);
        r.lo = ldexp(sl, e);
        r.abs_sum = ldexp(sa, e);
        r.value = r.hi + r.lo;
        r.n_subsets = count;
        r.n_fallback = (use_scale & 2) ? count : sn;   // bit 1: every minor was done in double
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
    return launch_timed(k_radic_float<M, F32, EXPORT, DEFER>, dim3(grid), dim3(block), lds, s, J);
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

// Float workgroups per refactorisation workgroup: at most four (more workgroups
// spread the few flagged minors over more of the chip), and no more than keep
// the segments of one refactorisation workgroup within one wave's scan (64).
int refactor_group(int block) {
    const int r = kWave / (block / kWave);
    return r < 4 ? r : 4;
}

int refactor_grid(int grid, int block) {
    const int R = refactor_group(block);
    return (grid + R - 1) / R;
}

template <int M>
static hipError_t launch_refactor_m(const FloatJob& J, int grid, int block, hipStream_t s) {
    const int lds = binom_bytes<M>(J.n) + align16(J.n * Layout<M>::st64 * 8);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_refactor_deferred<M>, dim3(refactor_grid(grid, block)), dim3(block), lds, s, J, grid,
                       refactor_group(block));
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

hipError_t launch_finalize_float(const Partial* parts, int G, const Partial* fb_parts, int G2, const DetHeader* h,
                                 radic_f64_result* out, unsigned long long count, int use_scale, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_finalize_float, dim3(1), dim3(512), 0, s, parts, G, fb_parts, G2, h, out, count,
                       use_scale);
    return hipGetLastError();
}

hipError_t launch_zero_result(radic_f64_result* out, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_write_zero_result, dim3(1), dim3(1), 0, s, out);
    return hipGetLastError();
}

hipError_t upload_binomials_float(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

}  // namespace radic
