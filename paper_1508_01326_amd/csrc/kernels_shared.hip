// Prefix-shared floating-point Radic kernels (m >= 3) for gfx950.
//
// Gaussian elimination with partial pivoting chooses the pivot and the
// multipliers of step k from the first k+1 columns only.  In the dictionary
// order (Section 3) every minor with the same first m-2 columns (a prefix) is
// consecutive, and GEPP of all those minors performs the same first m-2 steps.
// Those steps are done once per prefix here; what is left of each minor is the
// last two steps on a 2 x 2 block.
//
// A wave takes a block of up to 64 prefixes and works in rounds.  Over a whole
// rank space each minor is shared either through its first m-2 columns or,
// when fewer columns follow those than precede its last m-2, through its last
// m-2 (the same scheme on the column-reversed matrix, see split_shape); blocks
// hold prefixes of one side with one last column and come heaviest first.  A
// rank range takes 64 consecutive prefixes in dictionary order.  A round:
//  A. Each lane takes one prefix and factors the m x (m-2) block of its columns
//     by LU with partial pivoting in registers, column by column (the first m-2
//     steps of every minor with that prefix).  From the multipliers it forms
//     the two rows of the projection onto the rows left after those steps,
//     W = rows m-2 and m-1 of L^{-1} P, with the signed product of the pivots.
//  P. The round's later columns (r per prefix) are split evenly over the lanes;
//     a lane fetches W of the prefix owning its column from the owner lane by a
//     cross-lane exchange and writes (-1)^j W x_c to the wave's LDS.
//  B. The wave's minors (the column pairs (a, b) after each prefix, in
//     dictionary order) are split evenly over the 64 lanes.  Each minor is
//     det(A_J) = (signed pivot product) * det([W x_a, W x_b]).  Its last two
//     elimination steps reduce to that 2 x 2 determinant: the pivot choice
//     between the two rows changes only the sign bookkeeping, which cancels.
//     The signed terms (-1)^(r+s) det(A_J) of eq. (1) are added in double in
//     runs of at most 16 per lane, each run folded into the lane's TwoSum pair.
// Every minor's determinant is still formed individually, so sum |det(A_J)| and
// the FP32-bulk conditioning test per minor are available.
//
// FP32-bulk runs both phases in float on the power-of-two row-scaled matrix.
// The capped pivot-ratio product of a minor is the prefix's product times the
// factors of the last two pivots.  Flagged minors are queued in the wave's
// segment of the workspace and refactored in double: up to m = 8 by the
// workgroup at its end (or by the wave between rounds once its segment is half
// full), beyond by the refactorisation kernel.  Up to m = 8 a round whose
// flagged minors would overflow the segment is done again in double by the same
// round code.
#include <type_traits>

#include "shared_round.h"

namespace radic {

template <int M, bool F32>
__global__ __launch_bounds__(kMaxBlock) void k_radic_shared(FloatJob J) {
    using T = typename std::conditional<F32, float, double>::type;
    constexpr int P = M - 2;
    constexpr int S64 = SharedLayout<M>::s64, S32 = SharedLayout<M>::s32;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rowexp[RADIC_MAX_M];
    __shared__ double red[4 * 16];
    __shared__ unsigned long long redn[16];
    __shared__ unsigned segn[16];   // FP32-bulk: flagged minors per wave

    const int n = J.n;
    const int waves = blockDim.x / kWave;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;

    constexpr int BS = M + 1;   // stride of the LDS binomial slice
    unsigned long long* bt = reinterpret_cast<unsigned long long*>(smem);
    double* cd = reinterpret_cast<double*>(smem + binom_bytes<BS>(n));
    float* cf = reinterpret_cast<float*>(smem + binom_bytes<BS>(n) + align16(n * S64 * 8));
    unsigned char* wr = smem + shared_common_bytes<M, F32>(n) + wave * shared_wave_bytes<M, F32>(J.cap);
    RoundLds W;
    W.hdr = reinterpret_cast<PairHdr*>(wr);
    W.incl = reinterpret_cast<unsigned*>(wr + kHdrBytes);   // pairs, inclusive scan over the lanes
    W.cincl = W.incl + kPrefixBlock;                         // columns, inclusive scan
    W.ratios = reinterpret_cast<float*>(wr + kHdrBytes + kScanBytes);
    W.wcols = reinterpret_cast<uint4*>(wr + kHdrBytes + kScanBytes + kPrefixBlock * 4);
    W.tv = wr + kHdrBytes + kScanBytes + (F32 ? kF32Extra : 0);   // projected-column slots

    stage_binomials<BS>(bt, n);
    const int bad = stage_matrix<M, F32, F32, S64, S32>(J, cd, cf, rowexp);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.header->nonfinite = bad;
        int se = 0;
        if (F32)
            for (int i = 0; i < M; ++i) se += rowexp[i];
        J.header->scale_exp = se;
    }

    const T* src = F32 ? reinterpret_cast<const T*>(cf) : reinterpret_cast<const T*>(cd);
    double hi = 0.0, lo = 0.0, ab = 0.0;
    unsigned long long nfb = 0;
    int gcount = 0;          // wave-uniform number of flagged minors (FP32-bulk)
    bool overflow = false;   // wave-uniform: more flagged minors than the segment holds
    const unsigned long long nblk = J.colex ? J.colex_blocks : (J.p_end - J.p_begin + kPrefixBlock - 1) / kPrefixBlock;
    const unsigned long long gwave = (unsigned long long)blockIdx.x * waves + wave;
    const unsigned long long nwaves = (unsigned long long)gridDim.x * waves;

    for (unsigned long long blk = gwave; blk < nblk && !overflow; blk += nwaves) {
        // two-sided blocks (whole rank space) hold prefixes of one side and
        // last column; otherwise 64 dictionary numbers from p_begin
        unsigned long long next, pi1;
        int side = 0, vlast = 0;
        if (J.colex) {
            int cnt;
            split_block<P>(blk, n, bt, BS, J.colex_pairs, lane, side, vlast, next, cnt);
            pi1 = next + (unsigned long long)cnt;
        } else {
            next = J.p_begin + blk * kPrefixBlock;
            const unsigned long long pe = next + kPrefixBlock;
            pi1 = pe < J.p_end ? pe : J.p_end;
        }
        // prefixes a round may take: halved while its flagged minors overflow
        // the segment (FP32-bulk up to m = 8)
        int limit = kPrefixBlock;
        while (next < pi1 && !overflow) {
            [[maybe_unused]] const double shi = hi, slo = lo, sab = ab;
            [[maybe_unused]] const unsigned long long snfb = nfb;
            [[maybe_unused]] const int sg = gcount;
            unsigned minors;
            const unsigned long long lend = next + (unsigned long long)limit;
            const int ntake = shared_round<M, F32, BS>(J, bt, src, next, lend < pi1 ? lend : pi1, side, vlast, W, lane,
                                                       gwave, hi, lo, ab, nfb, gcount, minors);
            if constexpr (F32 && shared_tail_refactor(M)) {
                if (gcount > J.defer_cap) {
                    // the round's flagged minors do not fit the segment: the
                    // round again over half as many prefixes, or, for a single
                    // prefix, its minors each in double by a lane group (and
                    // counted as refactored)
                    hi = shi;
                    lo = slo;
                    ab = sab;
                    nfb = snfb;
                    gcount = sg;
                    wave_lds_sync();
                    if (ntake > 1) {
                        limit = (ntake + 1) / 2;
                        continue;
                    }
                    redo_round_groups<M, BS, S64>(J, bt, cd, next, 1, side, vlast, lane, hi, lo, ab, nfb);
                }
            } else {
                // a full segment: the wave's blocks are redone in double (by the
                // refactorisation kernel), so the rest is not needed
                if (F32 && gcount > J.defer_cap) overflow = true;
            }
            next += (unsigned long long)ntake;
            wave_lds_sync();
            if constexpr (F32 && shared_tail_refactor(M)) {
                if (!overflow) relieve_segment<M, S64>(J, cd, gwave, gcount, lane, hi, lo, ab);
            }
        }
    }
    if constexpr (F32 && shared_tail_refactor(M)) {
        shared_fp32_tail<M, 2, kPrefixBlock, BS, S64>(J, bt, cd, gcount, gwave, nwaves, nblk, segn, hi, lo, ab, nfb);
    } else if (F32 && lane == 0) {
        J.fb_count[gwave] = (unsigned)gcount;   // above J.defer_cap: overflowed
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
        J.partials[blockIdx.x] = Partial{h, l, a2, nf};
    }
}

// ---------------------------------------------------------------- host side
hipError_t upload_binomials_shared(const unsigned long long* host_table) { return upload_binomial_table(host_table); }

int shared_lds(int m, int n, int prec, int waves, int cap) {
    switch (m) {
#define RADIC_CASE(MM)                                                                            \
    case MM:                                                                                      \
        return prec == RADIC_FP32_BULK ? shared_lds_bytes<MM, true>(n, waves, cap)                \
                                       : shared_lds_bytes<MM, false>(n, waves, cap);
        RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return 1 << 30;
    }
}

template <int M, bool F32>
static hipError_t launch_shared_m(const FloatJob& J, int grid, int block, int lds, hipStream_t s) {
    // beyond 64 KiB of dynamic LDS the kernel has to be allowed it first
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_radic_shared<M, F32>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return launch_timed(k_radic_shared<M, F32>, dim3(grid), dim3(block), lds, s, J);
}

hipError_t launch_shared(int m, int prec, const FloatJob& J, int grid, int block, hipStream_t s) {
    const int lds = shared_lds(m, J.n, prec, block / kWave, J.cap);
    switch (m) {
#define RADIC_CASE(MM)                                                                              \
    case MM:                                                                                        \
        return prec == RADIC_FP32_BULK ? launch_shared_m<MM, true>(J, grid, block, lds, s)          \
                                       : launch_shared_m<MM, false>(J, grid, block, lds, s);
        RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6) RADIC_CASE(7) RADIC_CASE(8)
        RADIC_CASE(9) RADIC_CASE(10) RADIC_CASE(11) RADIC_CASE(12)
#undef RADIC_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace radic
