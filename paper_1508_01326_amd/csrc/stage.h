// Staging of a float64 matrix into LDS for the floating-point kernels, and the
// per-wave row-ordered copy the lanes gather minors from.
#pragma once

#include "lu_float.h"

namespace radic {

// Per-wave copy of the columns the lanes gather from, rows in the wave's order.
template <int M, bool F32> __host__ __device__ int wave_copy_bytes(int n) {
    return F32 ? align16(n * Layout<M>::st32 * 4) : align16(n * Layout<M>::st64 * 8);
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
// F32: rows scaled by 2^-e_i, e_i the exponent of the row maximum
// (max_j |a_ij| = f 2^e_i with f in [0.5, 1)); WITH_F32: also write the float
// copy and its reciprocal column scales.  Each wave loads whole rows (coalesced)
// and takes the row maximum by a butterfly.  Column strides ST64 (doubles) and
// ST32 (floats, the scale in slot M).
template <int M, bool F32, bool WITH_F32 = F32, int ST64 = Layout<M>::st64, int ST32 = Layout<M>::st32>
__device__ int stage_matrix(const FloatJob& J, double* cd, float* cf, int* rowexp) {
    static_assert(ST64 >= M && ST32 >= M + 1, "column strides");
    const int n = J.n;
    const int waves = blockDim.x / kWave, wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int bad = 0;
    for (int i = wave; i < M; i += waves) {
        const double* row = J.A + (long long)i * J.lda;
        double mx = 0.0;
        for (int j = lane; j < n; j += kWave) {
            const double v = row[j];
            bad |= !isfinite(v);
            mx = fmax(mx, fabs(v));
            cd[j * ST64 + i] = v;
        }
        if (F32) {
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, shfl_xor_d(mx, off));
            if (lane == 0) {
                int e = 0;
                if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
                rowexp[i] = e;
            }
        }
    }
    bad = __syncthreads_or(bad);
    if (F32) {
        for (int e = threadIdx.x; e < M * n; e += blockDim.x) {
            const int j = e / M, i = e - j * M;
            const double v = ldexp(cd[j * ST64 + i], -rowexp[i]);   // exact power-of-two scaling
            cd[j * ST64 + i] = v;
            if (WITH_F32) cf[j * ST32 + i] = (float)v;
        }
        __syncthreads();
    }
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

}  // namespace radic
