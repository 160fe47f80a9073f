// Peak probes: what the matrix cores and HBM deliver on this device, measured
// with the same instructions the product and the streaming passes use, so that
// the benchmark reports each kernel's fraction of the datasheet peak and of the
// measured one.  Nothing here is part of the protected product.
//
// MFMA loop: every wave runs `iters` rounds of 8 (binary64: 16) independent matrix-core
// instructions on register operands (no memory traffic), enough independent
// accumulators to cover the instruction latency; 4 waves per block, 2 blocks
// per CU.  HBM stream: a read-only pass over a caller buffer, one block per
// 16 KB chunk (four 16-byte non-temporal loads per lane, all in flight), the
// fastest of the read patterns measured here (grid-stride loops, chunked loops,
// 1 to 8 loads per lane, 1024 to 10^6 blocks); the loaded words are folded
// and stored only when the fold hits a constant, so the loads stay.
#include "common.h"

namespace abft {
namespace {

// Independent accumulators per wave (each chain's next instruction comes
// after all the others: the latency is covered).
template <int DT> constexpr int chains_of() { return DT == ABFT_F64 ? 16 : 8; }
constexpr int kProbeThreads = 256;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f_p __attribute__((ext_vector_type(4)));

template <int DT>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int64_t iters, double *sink) {
    constexpr int kChains = chains_of<DT>();
    const int lane = threadIdx.x % 64;
    double out = 0.0;
    if constexpr (DT == ABFT_F64) {
        v4d acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = v4d{(double)c, 0.0, 0.0, 0.0};
        const double a = 1.0 + lane * 0x1p-20, b = 1.0 - lane * 0x1p-21;
        // accumulators tied in place (from the builtin, the compiler copied all
        // of them to the accumulation registers and back on every iteration)
        asm volatile("s_nop 7" ::: "memory");
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                asm volatile("v_mfma_f64_16x16x4_f64 %0, %1, %2, %0" : "+v"(acc[c]) : "v"(a), "v"(b));
        }
        asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
        for (int c = 0; c < kChains; ++c) out += acc[c][0] + acc[c][3];
    } else if constexpr (DT == ABFT_F32) {
        v4f_p acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = v4f_p{0.f, 0.f, 0.f, 0.f};
        const float a = 1.0f + lane * 0x1p-20f, b = 1.0f - lane * 0x1p-21f;
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
        for (int c = 0; c < kChains; ++c) out += (double)acc[c][0] + (double)acc[c][3];
    } else {
        // bfloat16, the 16x16x32 instruction of the low-precision product.  Written
        // as one instruction per chain with its accumulator tied in place: from the
        // builtin, the compiler moved the accumulators between registers on every
        // iteration of this operand-only loop (as many moves as instructions).
        v4f_p acc[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = v4f_p{(float)c, 0.f, 0.f, 0.f};
        // operands: bfloat16 bit patterns of values near 1 (lane-dependent)
        v4u32 x, y;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            x[q] = 0x3F803F80u + (uint32_t)((lane + q) & 7) * 0x00010001u;
            y[q] = 0x3F803F80u + (uint32_t)((lane + 2 * q) & 7) * 0x00010001u;
        }
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %2, %0" : "+v"(acc[c]) : "v"(x), "v"(y));
        }
        // the results of the last instructions settle before ordinary code reads them
        asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
#pragma unroll
        for (int c = 0; c < kChains; ++c) out += (double)acc[c][0] + (double)acc[c][3];
    }
    // one value per block keeps the chains live
    __shared__ double sh[kProbeThreads / 64];
    if (lane == 0) sh[threadIdx.x / 64] = out;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kProbeThreads / 64; ++w) s += sh[w];
        sink[blockIdx.x] = s;
    }
}

// Flops of one instruction of each probe (2 x the multiply-adds of its output tile).
constexpr double kFlopsPerInst[3] = {2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32};

constexpr int kStreamLoads = 4;                       // 16-byte loads per lane: 16 KB per block
__global__ __launch_bounds__(kProbeThreads) void k_probe_stream(const v4u32 *__restrict__ x, int64_t n16,
                                                                double *sink) {
    const int64_t t0 = (int64_t)blockIdx.x * (kProbeThreads * kStreamLoads) + threadIdx.x;
    v4u32 v[kStreamLoads];
#pragma unroll
    for (int u = 0; u < kStreamLoads; ++u) {
        const int64_t t = t0 + (int64_t)u * kProbeThreads;
        v[u] = t < n16 ? __builtin_nontemporal_load(x + t) : v4u32{0u, 0u, 0u, 0u};
    }
    uint32_t acc = 0;
#pragma unroll
    for (int u = 0; u < kStreamLoads; ++u) acc ^= v[u][0] ^ v[u][1] ^ v[u][2] ^ v[u][3];
    if (acc == 0x9E3779B9u) sink[0] = (double)acc;
}

}  // namespace
}  // namespace abft

using namespace abft;

extern "C" {

int abft_probe_mfma(int32_t dtype, int64_t iters, double *sink, int64_t sink_len, double *flops, void *stream) {
    if (iters < 1 || !sink || !flops) return ABFT_E_ARG;
    if (dtype != ABFT_F64 && dtype != ABFT_F32 && dtype != ABFT_BF16) return ABFT_E_UNSUPPORTED;
    const int64_t blocks = 256 * 2;                      // two blocks of four waves per CU: two waves per SIMD
    if (sink_len < blocks) return ABFT_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    switch (dtype) {
    case ABFT_F64: k_probe_mfma<ABFT_F64><<<(unsigned)blocks, kProbeThreads, 0, s>>>(iters, sink); break;
    case ABFT_F32: k_probe_mfma<ABFT_F32><<<(unsigned)blocks, kProbeThreads, 0, s>>>(iters, sink); break;
    default: k_probe_mfma<ABFT_BF16><<<(unsigned)blocks, kProbeThreads, 0, s>>>(iters, sink); break;
    }
    ABFT_LAUNCHED();
    const int idx = dtype == ABFT_F64 ? 0 : (dtype == ABFT_F32 ? 1 : 2);
    const int chains = dtype == ABFT_F64 ? chains_of<ABFT_F64>() : chains_of<ABFT_F32>();
    *flops = (double)blocks * (kProbeThreads / 64) * (double)iters * chains * kFlopsPerInst[idx];
    return ABFT_OK;
}

int abft_probe_stream(const void *buf, size_t bytes, double *sink, int64_t sink_len, void *stream) {
    if (!buf || ((uintptr_t)buf & 15u) || bytes < 16 || !sink || sink_len < 1) return ABFT_E_ARG;
    const int64_t n16 = (int64_t)(bytes / 16), per = kProbeThreads * kStreamLoads;
    const int64_t blocks = (n16 + per - 1) / per;
    if (blocks > 0x7FFFFFFF) return ABFT_E_ARG;
    k_probe_stream<<<(unsigned)blocks, kProbeThreads, 0, (hipStream_t)stream>>>((const v4u32 *)buf, n16, sink);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

}  // extern "C"
