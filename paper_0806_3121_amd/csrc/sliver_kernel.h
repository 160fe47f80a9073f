// Carried checksum blocks of C_f computed as skinny products with binary64
// accumulation (the "sliver" path, used when a checksum block is thinner than
// a matrix-core tile):
//   carried row block    C_f[m + r, j] = sum_l (C_C^T A)[r, l] B_f[l, j]   (r < br, j < N)
//   carried column block C_f[i, n + c] = sum_l A_f[i, l] (B C_R)[l, c]     (i < rows, c < bc)
// Both have the form out[u, s] = sum_l X[u, l] Y[s, l] with many rows u (a
// whole operand, streamed once from HBM) and few rows s (the checksum rows,
// L2-resident).  One wave owns one u at a time; lanes stride k with 16-byte
// loads; the few partial sums are folded with wavefront shuffles.
#pragma once

#include "common.h"

namespace abft {

constexpr int kSliverThreads = 256;
constexpr int kSliverR = 8;   // few rows per pass

// out = v, or out += v (accumulate: the sum is taken in binary64 and rounded once)
template <typename T> __device__ inline void store_out(T *p, double v, bool accumulate);
template <> __device__ inline void store_out<double>(double *p, double v, bool accumulate) {
    *p = accumulate ? *p + v : v;
}
template <> __device__ inline void store_out<float>(float *p, double v, bool accumulate) {
    *p = (float)(accumulate ? (double)*p + v : v);
}

// X: U rows of type TX (ldx); Y: R rows of type TY (ldy), R <= kSliverR per launch.
// out[u*ou + s*os] = scale * sum_l X[u,l] Y[s,l], scale = 2^-(e[0] + e[1]) when
// the device scale exponents e are given (FP8), else 1.  K is a multiple of
// both vector widths.
template <typename TX, typename TY, typename TC>
__global__ __launch_bounds__(kSliverThreads) void k_sliver(const TX *__restrict__ X, int64_t ldx, int64_t U,
                                                          const TY *__restrict__ Y, int64_t ldy, int R, int64_t K,
                                                          TC *__restrict__ out, int64_t ou, int64_t os,
                                                          const int *__restrict__ scale_exp, int accumulate) {
    const double scale = scale_exp ? ldexp(1.0, -(scale_exp[0] + scale_exp[1])) : 1.0;
    constexpr int VX = vec16<TX>::N, VY = vec16<TY>::N;
    constexpr int V = VX > VY ? VX : VY;             // k per lane per step
    const int lane = threadIdx.x % 64;
    const int64_t wave = ((int64_t)blockIdx.x * kSliverThreads + threadIdx.x) / 64;
    const int64_t nwaves = (int64_t)gridDim.x * kSliverThreads / 64;
    constexpr int UNR = V >= 16 ? 1 : (V >= 8 ? 2 : 4);   // 16-byte loads in flight per lane and operand row
    for (int64_t u = wave; u < U; u += nwaves) {
        double acc[kSliverR];
#pragma unroll
        for (int s = 0; s < kSliverR; ++s) acc[s] = 0.0;
        const TX *xr = X + u * ldx;
        int64_t k0 = (int64_t)lane * V;
        for (; k0 + (UNR - 1) * 64 * V < K; k0 += UNR * 64 * V) {
            double xv[UNR][V];
#pragma unroll
            for (int w = 0; w < UNR; ++w)
#pragma unroll
                for (int q = 0; q < V; q += VX) vec16<TX>::load(xr + k0 + w * 64 * V + q, xv[w] + q);
#pragma unroll
            for (int s = 0; s < kSliverR; ++s) {
                if (s < R) {
                    double yv[UNR][V];
#pragma unroll
                    for (int w = 0; w < UNR; ++w)
#pragma unroll
                        for (int q = 0; q < V; q += VY) vec16<TY>::load(Y + s * ldy + k0 + w * 64 * V + q, yv[w] + q);
#pragma unroll
                    for (int w = 0; w < UNR; ++w)
#pragma unroll
                        for (int q = 0; q < V; ++q) acc[s] = fma(xv[w][q], yv[w][q], acc[s]);
                }
            }
        }
        for (; k0 < K; k0 += 64 * V) {
            double xv[V];
#pragma unroll
            for (int q = 0; q < V; q += VX) vec16<TX>::load(xr + k0 + q, xv + q);
#pragma unroll
            for (int s = 0; s < kSliverR; ++s) {
                if (s < R) {
                    double yv[V];
#pragma unroll
                    for (int q = 0; q < V; q += VY) vec16<TY>::load(Y + s * ldy + k0 + q, yv + q);
#pragma unroll
                    for (int q = 0; q < V; ++q) acc[s] = fma(xv[q], yv[q], acc[s]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kSliverR; ++s) {
            double v = acc[s];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && s < R) store_out<TC>(out + u * ou + s * os, scale * v, accumulate != 0);
        }
    }
}

// One checksum row (R = 1): a wave takes NR rows of X together, so that each
// chunk of Y is read once for NR rows and NR 16-byte loads of X are in flight
// per lane (kept raw until summed).  Per row the same sums in the same order
// as k_sliver: each lane over its chunks in increasing k, then the butterfly.
template <typename TX, typename TY, typename TC, int NR, int UK>
__global__ __launch_bounds__(kSliverThreads) void k_sliver1(const TX *__restrict__ X, int64_t ldx, int64_t U,
                                                           const TY *__restrict__ Y, int64_t K, TC *__restrict__ out,
                                                           int64_t ou, const int *__restrict__ scale_exp,
                                                           int accumulate) {
    const double scale = scale_exp ? ldexp(1.0, -(scale_exp[0] + scale_exp[1])) : 1.0;
    constexpr int VX = vec16<TX>::N, VY = vec16<TY>::N;
    constexpr int V = VX > VY ? VX : VY;             // k per lane per step
    const int lane = threadIdx.x % 64;
    const int64_t wave = ((int64_t)blockIdx.x * kSliverThreads + threadIdx.x) / 64;
    const int64_t nwaves = (int64_t)gridDim.x * kSliverThreads / 64;
    for (int64_t u0 = wave * NR; u0 < U; u0 += nwaves * NR) {
        double acc[NR];
        const TX *xr[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            acc[r] = 0.0;
            xr[r] = X + min(u0 + r, U - 1) * ldx;      // rows past U re-read the last (not stored)
        }
        // UK chunks of k per lane in flight (a chunk at or past K is clamped to
        // the lane's first and not summed)
        for (int64_t k0 = (int64_t)lane * V; k0 < K; k0 += UK * 64 * V) {
            v4u32 xw[UK][NR][V / VX], yw[UK][V / VY];
#pragma unroll
            for (int c = 0; c < UK; ++c) {
                const int64_t kc = k0 + c * 64 * V < K ? k0 + c * 64 * V : k0;
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int q = 0; q < V / VX; ++q) xw[c][r][q] = *(const v4u32 *)(xr[r] + kc + q * VX);
#pragma unroll
                for (int q = 0; q < V / VY; ++q) yw[c][q] = *(const v4u32 *)(Y + kc + q * VY);
            }
#pragma unroll
            for (int c = 0; c < UK; ++c) {
                if (k0 + c * 64 * V >= K) break;
                double yv[V];
#pragma unroll
                for (int q = 0; q < V / VY; ++q) vec16<TY>::widen(yw[c][q], yv + q * VY);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    double xv[V];
#pragma unroll
                    for (int q = 0; q < V / VX; ++q) vec16<TX>::widen(xw[c][r][q], xv + q * VX);
#pragma unroll
                    for (int q = 0; q < V; ++q) acc[r] = fma(xv[q], yv[q], acc[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v = acc[r];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && u0 + r < U) store_out<TC>(out + (u0 + r) * ou, scale * v, accumulate != 0);
        }
    }
}
// k_sliver1 serves one checksum row over enough operand rows to fill the device.
inline bool sliver_multirow(int64_t R, int64_t U) { return R == 1 && U >= 16384; }
constexpr int kSliverRows = 4;        // rows of X per wave in k_sliver1
constexpr int kSliverChunks = 2;      // chunks of k per lane in flight in k_sliver1

template <typename TX, typename TY, typename TC>
inline int sliver(const TX *X, int64_t ldx, int64_t U, const TY *Y, int64_t ldy, int64_t R, int64_t K, TC *out,
                  int64_t ou, int64_t os, const int *scale_exp, hipStream_t s, bool accumulate = false) {
    const int64_t waves_per_block = kSliverThreads / 64;
    if (sliver_multirow(R, U)) {
        const int64_t waves = (U + kSliverRows - 1) / kSliverRows;
        const unsigned blocks = (unsigned)std::min<int64_t>((waves + waves_per_block - 1) / waves_per_block, 4096);
        k_sliver1<TX, TY, TC, kSliverRows, kSliverChunks><<<blocks, kSliverThreads, 0, s>>>(X, ldx, U, Y, K, out, ou, scale_exp,
                                                                            accumulate ? 1 : 0);
        ABFT_LAUNCHED();
        return ABFT_OK;
    }
    unsigned blocks = (unsigned)std::min<int64_t>((U + waves_per_block - 1) / waves_per_block, 4096);
    for (int64_t r0 = 0; r0 < R; r0 += kSliverR) {
        int rr = (int)std::min<int64_t>(kSliverR, R - r0);
        k_sliver<TX, TY, TC><<<blocks, kSliverThreads, 0, s>>>(X, ldx, U, Y + r0 * ldy, ldy, rr, K, out + r0 * os, ou,
                                                               os, scale_exp, accumulate ? 1 : 0);
    }
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// Carried row block: C_f[m + r, 0:N) = sum_l Acs[r, l] Bt[j, l] (checksum rows Acs, br x K; the
// operands may start at a k offset, K is the panel depth).
template <typename TA, typename TB, typename TC>
inline int launch_sliver_rows(const Geom &g, const TA *Acs, int64_t ldacs, const TB *Bt, int64_t ldb, TC *C,
                              int64_t ldc, int64_t K, bool accumulate, hipStream_t s) {
    return sliver<TB, TA, TC>(Bt, ldb, g.N, Acs, ldacs, g.br, K, C + g.m * ldc, 1, ldc, nullptr, s, accumulate);
}
// Carried column block: C_f[0:rows, n + c) = sum_l A[i, l] Bcs[c, l] (checksum columns Bcs, bc x K).
template <typename TA, typename TB, typename TC>
inline int launch_sliver_cols(const Geom &g, int64_t rows, const TA *A, int64_t lda, const TB *Bcs, int64_t ldbcs,
                              TC *C, int64_t ldc, int64_t K, bool accumulate, hipStream_t s) {
    return sliver<TA, TB, TC>(A, lda, rows, Bcs, ldbcs, g.bc, K, C + g.n, ldc, 1, nullptr, s, accumulate);
}

}  // namespace abft
