// Exact Radic determinant of an int32 matrix by modular arithmetic.
//
// The exact result S = sum_J (-1)^(r+s) det(A_J) (Definition 3, eq. (1)) is an
// integer with |S| <= sum_J prod_{j in J} ||a_j||_2 = e_m(||a_1||, ..., ||a_n||)
// (Hadamard's inequality per minor).  For k primes p_i < 2^31 whose product
// exceeds twice that bound, S is recovered from S mod p_i by the Chinese
// remainder theorem (Garner's mixed-radix form) in the symmetric range.
//
// Per lane and prime, each minor is eliminated fraction-free modulo p
// (Bareiss-type row updates row_i <- u_kk row_i - a_ik row_k, pivot = first row
// with a nonzero entry mod p).  The divisions that make Bareiss's recurrence
// exact are not done per step; since every update scales the rows below by the
// pivot, det(A_J) = prod_k u_kk / prod_{k<M-1} u_kk^(M-1-k) mod p, and the lane
// keeps its running sum as one fraction num/den, so a single modular inverse per
// workgroup replaces all per-minor divisions.  Residues are held in doubles
// (exact below 2^53) and multiplied with an error-free product and a floor-based
// reduction (double products of 31-bit operands are split with an FMA).
#include "shared_int.h"

namespace radic {

struct IntHeader {
    int n_primes;       // primes needed for the bound
    int status;         // RADIC_OK or RADIC_EOVERFLOW (bound needs more than the prime set)
    double bound_log2;  // log2 of the bound on |S|
};

struct IntResult {
    int status;
    int sign;
    int mag_len;
    int n_primes;
    unsigned mag[RADIC_MAX_PRIMES + 1];
    unsigned residue[RADIC_MAX_PRIMES];
};

struct IntJob {
    const int* A;
    long long lda;
    int m, n;
    unsigned long long count;
    unsigned long long chunks;
    int spl;
    int grid_x;
    double* partials;    // [prime][grid_x] residues
    IntHeader* header;
};

template <int M> __host__ __device__ int int_lds_bytes(int n) {
    return binom_bytes<M>(n) + align16(n * IntLayout<M>::st * 8);
}

// ---------------------------------------------------------------- bound and prime count
__global__ __launch_bounds__(256) void k_int_bound(const int* A, int m, int n, long long lda, IntHeader* h,
                                                   int prime_count) {
    __shared__ double norms[RADIC_MAX_N];
    __shared__ double lg[RADIC_MAX_PRIMES];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double a[RADIC_MAX_M];
#pragma unroll
        for (int i = 0; i < RADIC_MAX_M; ++i) a[i] = i < m ? (double)A[(long long)i * lda + j] : 0.0;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < RADIC_MAX_M; ++i) s = __builtin_fma(a[i], a[i], s);
        norms[j] = sqrt(s) * (1.0 + 1e-12);   // rounded up
    }
    if ((int)threadIdx.x < prime_count) lg[threadIdx.x] = log2(g_prime[threadIdx.x]);
    __syncthreads();
    if (threadIdx.x == 0) {
        // e_m of the column norms by the recurrence e_k += x e_{k-1} (all terms
        // >= 0), held in registers: the k loop is unrolled to the largest m with
        // no test of k against m (e_k for k > m never enters e_m), the column
        // loop by four so that the norms' LDS reads overlap
        double e[RADIC_MAX_M + 1];
        e[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= RADIC_MAX_M; ++k) e[k] = 0.0;
        auto step = [&](double x) {
#pragma unroll
            for (int k = RADIC_MAX_M; k >= 1; --k) e[k] = __builtin_fma(x, e[k - 1], e[k]);
        };
        int j = 0;
        for (; j + 4 <= n; j += 4) {
            const double x0 = norms[j], x1 = norms[j + 1], x2 = norms[j + 2], x3 = norms[j + 3];
            step(x0);
            step(x1);
            step(x2);
            step(x3);
        }
        for (; j < n; ++j) step(norms[j]);
        double em = 0.0;
#pragma unroll
        for (int k = 0; k <= RADIC_MAX_M; ++k) em = k == m ? e[k] : em;
        const double bound = em * (1.0 + 1e-9) + 1.0;
        const double need = log2(bound) + 1.0 + 1e-6;   // product of primes > 2 * bound
        double have = 0.0;
        int k = 0;
        while (k < prime_count && have <= need) have += lg[k++];
        h->bound_log2 = log2(bound);
        h->n_primes = k;
        h->status = have > need ? RADIC_OK : RADIC_EOVERFLOW;
    }
}

template <int M>
__global__ __launch_bounds__(kMaxBlock) void k_radic_int(IntJob J) {
    constexpr int ST = IntLayout<M>::st;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2 * 16];
    const int n = J.n;
    const int waves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    // primes beyond the bound kernel's count have nothing to do (see above)
    if ((int)blockIdx.y >= J.header->n_primes || J.header->status != RADIC_OK) return;
    const double p = g_prime[blockIdx.y];
    const double pinv = g_prime_inv[blockIdx.y];

    unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
    double* cr = reinterpret_cast<double*>(smem + binom_bytes<M>(n));
    stage_binomials<M>(bt, n);
    for (int e = threadIdx.x; e < M * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        const double v = (double)J.A[(long long)i * J.lda + j];
        const double q = __builtin_floor(v * pinv);
        cr[j * ST + i] = mod_fix(__builtin_fma(-q, p, v), p);   // exact residue in [0, p)
    }
    __syncthreads();

    double num = 0.0, den = 1.0;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const unsigned long long nwaves = (unsigned long long)gridDim.x * waves;
    for (unsigned long long wc = gwave * kWave; wc < J.chunks; wc += nwaves * kWave) {
        const unsigned long long chunk = wc + lane;
        const bool vchunk = chunk < J.chunks;
        const unsigned long long off0 = vchunk ? chunk * (unsigned long long)J.spl : J.count - 1;
        const unsigned long long left = J.count - off0;
        const int cnt = vchunk ? (int)(left < (unsigned long long)J.spl ? left : (unsigned long long)J.spl) : 0;
        int col[M];
        unrank<M>(off0, n, bt, col);
        for (int s = 0; s < J.spl; ++s) {
            double a[M][M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double* src = cr + col[j] * ST;
#pragma unroll
                for (int i = 0; i + 1 < M; i += 2) {
                    const double2 v = *reinterpret_cast<const double2*>(src + i);
                    a[i][j] = v.x;
                    a[i + 1][j] = v.y;
                }
                if (M & 1) a[M - 1][j] = src[M - 1];
            }
            double N = 1.0, P = 1.0, D = 1.0;
            bool zero = false;
            bool neg = radic_sign_odd<M>(col);
            elim_steps_mod<M, 0>(a, p, pinv, N, P, D, zero, neg);
            if (s < cnt && !zero) {
                const double t = neg ? (N == 0.0 ? 0.0 : p - N) : N;
                frac_add(num, den, t, D, p, pinv);
            }
            successor<M>(col, n);
        }
    }
    // fixed-order butterfly over the wave, then waves in order
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double n2 = shfl_xor_d(num, off), d2 = shfl_xor_d(den, off);
        frac_add(num, den, n2, d2, p, pinv);
    }
    if (lane == 0) {
        red[2 * wave] = num;
        red[2 * wave + 1] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double nn = red[0], dd = red[1];
        for (int w = 1; w < waves; ++w) frac_add(nn, dd, red[2 * w], red[2 * w + 1], p, pinv);
        J.partials[(long long)blockIdx.y * J.grid_x + blockIdx.x] = mulmod(nn, invmod(dd, p, pinv), p, pinv);
    }
}

// ---------------------------------------------------------------- prefix-shared exact kernel
struct IntSharedJob {
    const int* A;
    long long lda;
    int n;
    int cap;                      // projected-column slots per wave
    int grid_x;
    unsigned long long q_begin, count, total, n_prefix, p_begin, p_end;
    double* partials;             // [prime][grid_x] residues
    const IntHeader* header;      // the bound kernel's prime count and status
    int colex;                    // 1: two-sided blocks of the whole rank space (see split_block)
    unsigned colex_pairs;
    unsigned long long colex_blocks;
};

template <int M> __host__ __device__ int int_shared_lds_bytes(int n, int waves, int cap) {
    return binom_bytes<M>(n) + align16(n * IntLayout<M>::st * 8) +
           waves * (kPrefixBlock * (int)sizeof(IntSlot) + kPrefixBlock * 8 + align16(cap * 16));
}

template <int M>
__global__ __launch_bounds__(kMaxBlock) void k_radic_int_shared(IntSharedJob J) {
    constexpr int ST = IntLayout<M>::st;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    const int n = J.n;
    const int waves = blockDim.x / kWave, wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // the launch covers an upper bound on the primes: those the bound kernel
    // did not ask for (or every one, when it failed) have nothing to do
    if ((int)blockIdx.y >= J.header->n_primes || J.header->status != RADIC_OK) return;
    const double p = g_prime[blockIdx.y];
    const double pinv = g_prime_inv[blockIdx.y];

    unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
    double* cr = reinterpret_cast<double*>(smem + binom_bytes<M>(n));
    unsigned char* wr = smem + binom_bytes<M>(n) + align16(n * ST * 8) +
                        wave * (kPrefixBlock * (int)sizeof(IntSlot) + kPrefixBlock * 8 + align16(J.cap * 16));
    IntSlot* slot = reinterpret_cast<IntSlot*>(wr);
    unsigned* incl = reinterpret_cast<unsigned*>(wr + kPrefixBlock * sizeof(IntSlot));
    double2* tv = reinterpret_cast<double2*>(wr + kPrefixBlock * sizeof(IntSlot) + kPrefixBlock * 8);

    stage_binomials<M>(bt, n);
    for (int e = threadIdx.x; e < M * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        const double v = (double)J.A[(long long)i * J.lda + j];
        const double q = __builtin_floor(v * pinv);
        cr[j * ST + i] = mod_fix(__builtin_fma(-q, p, v), p);   // exact residue in [0, p)
    }
    __syncthreads();

    double acc = 0.0;   // this lane's sum of signed minors mod p
    const unsigned long long nblk = J.colex ? J.colex_blocks : (J.p_end - J.p_begin + kPrefixBlock - 1) / kPrefixBlock;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const unsigned long long nwaves = (unsigned long long)gridDim.x * waves;
    for (unsigned long long blk = gwave; blk < nblk; blk += nwaves) {
        unsigned long long next = J.p_begin + blk * kPrefixBlock;
        unsigned long long pi1 = next + kPrefixBlock < J.p_end ? next + kPrefixBlock : J.p_end;
        if (J.colex) {
            int cnt, side, vlast;
            split_block<M - 2>(blk, n, bt, M, J.colex_pairs, lane, side, vlast, next, cnt);
            pi1 = next + (unsigned long long)cnt;
            // two-sided blocks come heaviest first (prefixes with the most later columns)
            int_prefix_range<M, true>(cr, n, bt, M, next, pi1, J.n_prefix, 0ull, 0ull, J.total, p, pinv, J.cap,
                                      slot, incl, tv, lane, acc, side, vlast);
        } else {
            unsigned long long r0, r1;
            prefix_block_ranks<M>(J, bt, blk, r0, r1);
            const unsigned long long rbase = first_completion_rank<M>(next, J, bt);
            int_prefix_range<M>(cr, n, bt, M, next, pi1, J.n_prefix, rbase, r0, r1, p, pinv, J.cap, slot, incl, tv,
                                lane, acc);
        }
    }
    // fixed-order sum over the wave, then waves in order
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc = addmod(acc, __shfl_xor(acc, o, kWave), p);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < waves; ++w) t = addmod(t, red[w], p);
        J.partials[(long long)blockIdx.y * J.grid_x + blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------- CRT
// Sum the workgroup residues per prime (a wave per prime; the residues are
// below 2^31 and there are at most 8192 per prime, so the 64-bit integer sums
// are exact), then, on one wave, Garner's algorithm (mixed radix digits v_i
// with S = v_0 + v_1 p_0 + v_2 p_0 p_1 + ...) and the symmetric representative
// in (-P/2, P/2] as sign and 32-bit limbs.
// `launched`: the primes the modular kernel was launched for (an upper bound on
// the bound kernel's count; a larger count would leave residues missing).
__global__ __launch_bounds__(256) void k_int_finalize(const double* partials, int grid_x, int launched,
                                                      const IntHeader* h, IntResult* out) {
    __shared__ double res[RADIC_MAX_PRIMES];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave, waves = blockDim.x / kWave;
    const bool counted = h->n_primes <= launched;
    const int k = counted ? h->n_primes : 0;
    // one wave per prime: the workgroups' residues summed exactly in 64 bits,
    // four loads in flight per lane
    for (int t = wave; t < k; t += waves) {
        const double* row = partials + (long long)t * grid_x;
        unsigned long long s = 0;
        int b = lane;
        for (; b + 3 * kWave < grid_x; b += 4 * kWave)
            s += (unsigned long long)row[b] + (unsigned long long)row[b + kWave] +
                 (unsigned long long)row[b + 2 * kWave] + (unsigned long long)row[b + 3 * kWave];
        for (; b < grid_x; b += kWave) s += (unsigned long long)row[b];
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (lane == 0) res[t] = (double)(s % (unsigned long long)g_prime[t]);
    }
    __syncthreads();
    if (wave != 0) return;
    const int status = counted ? h->status : RADIC_EDEVICE;
    const bool ok = status == RADIC_OK && k > 0;
    const double r = lane < k ? res[lane] : 0.0;
    int sign = 0, len = 0;
    unsigned limb = 0;
    if (ok) wave_crt(r, k, lane, sign, len, limb);
    if (lane <= RADIC_MAX_PRIMES) out->mag[lane] = ok && lane < len ? limb : 0u;
    if (lane < RADIC_MAX_PRIMES) out->residue[lane] = ok && lane < k ? (unsigned)r : 0u;
    if (lane == 0) {
        out->status = status;
        out->sign = sign;
        out->mag_len = len;
        out->n_primes = k;
    }
}

// ---------------------------------------------------------------- host side
hipError_t upload_binomials_int(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

hipError_t upload_primes(const unsigned* primes, int count) { return upload_prime_table(primes, count); }

size_t int_header_bytes() { return 256; }
size_t int_partials_offset() { return 1024; }
size_t int_workspace_bytes() { return int_partials_offset() + sizeof(double) * (size_t)RADIC_MAX_PRIMES * kMaxGrid; }
size_t int_result_size() { return sizeof(IntResult); }

int int_lds(int m, int n) {
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return int_lds_bytes<MM>(n);
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return 1 << 30;
    }
}

hipError_t launch_int_bound(const int* A, int m, int n, long long lda, void* ws, int prime_count, hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_int_bound, dim3(1), dim3(256), 0, s, A, m, n, lda, reinterpret_cast<IntHeader*>(ws),
                       prime_count);
    return hipGetLastError();
}

hipError_t launch_int_main(const int* A, int m, int n, long long lda, unsigned long long count, int spl,
                           int grid_x, int n_primes, int block, void* ws, hipStream_t s) {
    IntJob J{};
    J.A = A;
    J.lda = lda;
    J.m = m;
    J.n = n;
    J.count = count;
    J.spl = spl;
    J.chunks = (count + spl - 1) / spl;
    J.grid_x = grid_x;
    J.partials = reinterpret_cast<double*>(static_cast<unsigned char*>(ws) + int_partials_offset());
    J.header = reinterpret_cast<IntHeader*>(ws);
    const int lds = int_lds(m, n);
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return launch_timed(k_radic_int<MM>, dim3(grid_x, n_primes), dim3(block), lds, s, J);
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
}

int int_shared_lds(int m, int n, int waves, int cap) {
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return int_shared_lds_bytes<MM>(n, waves, cap);
        RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10)
#undef RADIC_CASE
        default: return 1 << 30;
    }
}

hipError_t launch_int_shared(const int* A, int m, int n, long long lda, unsigned long long total,
                             unsigned long long n_prefix, unsigned colex_pairs, unsigned long long colex_blocks,
                             int cap, int grid_x, int n_primes, int block, void* ws, hipStream_t s) {
    IntSharedJob J{};
    J.A = A;
    J.lda = lda;
    J.n = n;
    J.cap = cap;
    J.grid_x = grid_x;
    J.q_begin = 0;
    J.count = total;
    J.total = total;
    J.n_prefix = n_prefix;
    J.p_begin = 0;
    J.p_end = n_prefix;
    J.colex = 1;
    J.colex_pairs = colex_pairs;
    J.colex_blocks = colex_blocks;
    J.partials = reinterpret_cast<double*>(static_cast<unsigned char*>(ws) + int_partials_offset());
    J.header = reinterpret_cast<const IntHeader*>(ws);
    const int lds = int_shared_lds(m, n, block / kWave, cap);
    switch (m) {
#define RADIC_CASE(MM) \
    case MM: return launch_timed(k_radic_int_shared<MM>, dim3(grid_x, n_primes), dim3(block), lds, s, J);
        RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_int_finalize(int grid_x, int launched, void* ws, void* out, hipStream_t s) {
    unsigned char* w = static_cast<unsigned char*>(ws);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_int_finalize, dim3(1), dim3(256), 0, s,
                       reinterpret_cast<const double*>(w + int_partials_offset()), grid_x, launched,
                       reinterpret_cast<const IntHeader*>(w), static_cast<IntResult*>(out));
    return hipGetLastError();
}

}  // namespace radic
