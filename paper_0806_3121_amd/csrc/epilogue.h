// Optional extras of the product kernels' epilogue, shared by the binary64 /
// binary32 and low-precision matrix-core kernels:
//  * a one-shot flip of one accumulator bit before the store (a test hook
//    that models a fault inside the computation: the flipped value reaches C
//    and the partial sums alike);
//  * the fused checksum accumulation: binary64 column sums of the tile's rows
//    and row sums of its columns (the b = 1 relations of Eq. ABFT-GEMM),
//    written per tile row / tile column so that verification reads these
//    partials instead of C.
// Accumulator layout (every kernel here): value v of lane l in 16 x 16 tile
// (a, b) of a wave is row r0 + 16 a + rowof(l, v), column c0 + 16 b + l % 16.
#pragma once

#include "common.h"

namespace abft {

struct EpiArgs {
    double *pc;          // column partials: pc[tm * ldpc + col] = sum over the tile's rows (null: none)
    double *pr;          // row partials:    pr[tn * ldpr + row] = sum over the tile's columns
    int64_t ldpc, ldpr;
    int64_t fi, fj;      // accumulator flip at output element (fi, fj) of the launch
    int fbit;            // bit to flip; < 0: no flip
    // host side only: the launch's tile grid, filled in by the dispatcher
    int64_t tiles_m, tiles_n;
};

inline EpiArgs epi_none() {
    EpiArgs e{};
    e.fbit = -1;
    return e;
}

__device__ inline void flip_bit(double &x, int bit) {
    x = __longlong_as_double(__double_as_longlong(x) ^ (1ll << bit));
}
__device__ inline void flip_bit(float &x, int bit) { x = __uint_as_float(__float_as_uint(x) ^ (1u << bit)); }

// x * 2^e with one rounding (exact unless the result leaves the format's range)
__device__ inline float scale_pow2(float x, int e) { return __builtin_ldexpf(x, e); }
__device__ inline double scale_pow2(double x, int e) { return __builtin_ldexp(x, e); }

// Flip the armed accumulator bit if this lane holds element (fi, fj): the
// target's index in acc is found first, then one unrolled pass of selects, so
// no register array is indexed at run time.  r0, c0: the wave tile's origin.
template <int TM, int TN, typename V4, typename RowOf>
__device__ __attribute__((always_inline)) inline void epi_flip(V4 (&acc)[TM][TN], const EpiArgs &e, int64_t r0,
                                                               int64_t c0, int lane, RowOf rowof) {
    const int64_t dr = e.fi - r0, dc = e.fj - c0;
    int tgt = -1;
    if (dr >= 0 && dr < 16 * TM && dc >= 0 && dc < 16 * TN && dc % 16 == lane % 16) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (rowof(lane, v) == (int)(dr % 16)) tgt = (int)(dr / 16) * TN * 4 + (int)(dc / 16) * 4 + v;
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if ((a * TN + b) * 4 + v == tgt) {
                    auto x = acc[a][b][v];
                    flip_bit(x, e.fbit);
                    acc[a][b][v] = x;
                }
}

// The store loop with the fused checksum accumulation: each value times the
// exact power of two `scale` is stored to C (added to it with accumulate;
// rows < M and columns < N only) and added to its row's and column's
// binary64 sums; the wave sums are combined across lanes, then across waves in
// LDS (sh: WM*BN + WN*BM doubles of free LDS), and each tile writes its column
// partials pc[tm][.] and row partials pr[tn][.].  Every thread of the block
// calls this.  Row sums die with each row of tiles, so the extra registers are
// the TN column sums and four row sums.
template <int TM, int TN, int WM, int WN, int BM, int BN, typename V4, typename TC, typename RowOf>
__device__ __attribute__((always_inline)) inline void epi_store_fused(const V4 (&acc)[TM][TN], const EpiArgs &e,
                                                                      double *sh, int64_t row0, int64_t col0,
                                                                      int64_t tm, int64_t tn, int64_t M, int64_t N,
                                                                      int wm, int wn, int lane, int shift, TC *C,
                                                                      int64_t ldc, bool accumulate, RowOf rowof) {
    const int wr0 = wm * (BM / WM), wc0 = wn * (BN / WN);
    const int64_t rl = M - row0 - wr0, cl = N - col0 - wc0;
    const int rlim = (int)(rl < BM ? rl : BM), clim = (int)(cl < BN ? cl : BN);
    double cs[TN];
#pragma unroll
    for (int b = 0; b < TN; ++b) cs[b] = 0.0;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
        double rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < TN; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * a + rowof(lane, v), c = 16 * b + lane % 16;
                const bool in = r < rlim && c < clim;
                const TC y = scale_pow2(acc[a][b][v], shift);
                if (in) {
                    TC *dst = C + (row0 + wr0 + r) * ldc + col0 + wc0 + c;
                    *dst = accumulate ? *dst + y : y;
                }
                const double x = in ? (double)y : 0.0;
                cs[b] += x;
                rs[v] += x;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double s = rs[v];
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 4);
            s += __shfl_xor(s, 8);
            if (lane % 16 == 0) sh[WM * BN + wn * BM + wr0 + 16 * a + rowof(lane, v)] = s;
        }
        // keep the scheduler from hoisting the next rows' conversions (register pressure)
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
        double s = cs[b];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (lane < 16) sh[wm * BN + wc0 + 16 * b + lane] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < BN; t += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < WM; ++w) s += sh[w * BN + t];
        if (col0 + t < N) e.pc[tm * e.ldpc + col0 + t] = s;
    }
    for (int t = threadIdx.x; t < BM; t += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < WN; ++w) s += sh[WM * BN + w * BM + t];
        if (row0 + t < M) e.pr[tn * e.ldpr + row0 + t] = s;
    }
}

}  // namespace abft
