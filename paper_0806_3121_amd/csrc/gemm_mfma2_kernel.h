// binary64 / binary32 product kernel, direct-to-LDS variant (gfx950):
// BM x BN block of WM x WN waves (e.g. 256 x 128, eight waves of 64 x 64), v_mfma_f64_16x16x4_f64 or
// v_mfma_f32_16x16x4_f32.  K advances in slabs of 128 bytes per row (16
// binary64 or 32 binary32 values) that go global -> LDS directly
// (global_load_lds_dwordx4: lane L of a wave writes the 16 bytes at
// base + 16 L), through a ring of STAGES buffers: the loads of slab t + STAGES - 1
// are issued while slab t feeds the matrix cores, with no register staging
// and no LDS write instructions.  One barrier per slab; the wait before it
// only covers the slab about to be used, the later ones stay in flight.
//
// LDS layout per slab and operand: row r is 128 bytes = 8 chunks of 16
// bytes; chunk kc of row r is stored at slot kc ^ ((r >> 1) & 7), so the 16
// rows a quarter-wave reads at one chunk index fall on 16 distinct four-bank
// groups.  The swizzle is applied on the global side: the lane that writes
// slot s of row r fetches chunk s ^ ((r >> 1) & 7).
//
// Fragments as in gemm_mfma_kernel.h: inside a 16-deep k group each lane
// holds four consecutive k of its row (32 bytes for binary64, 16 for
// binary32) and feeds them to four MFMAs; A and B use the same k order.
// Rows beyond M (columns beyond N) load a clamped valid row and their results
// are not stored.  K must be a multiple of the slab; other K use the
// register-staged kernel of gemm_mfma_kernel.h.
#pragma once

#include "gemm_mfma_kernel.h"

namespace abft {

// s_waitcnt with vmcnt = N (N < 64) and no wait on the other counters.
template <int N> __device__ inline void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | 0x0F70);
}

// A barrier without the memory fence of __syncthreads, which would also wait
// for every load still in flight.
__device__ inline void bare_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One fragment (four consecutive k of row r from chunk kc0 on) of a swizzled slab.
__device__ inline v4d frag_at(const double *, const uint8_t *slab, int r, int kc0) {
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d lo = *(const v2d *)(slab + r * 128 + (((kc0) ^ ((r >> 1) & 7)) << 4));
    const v2d hi = *(const v2d *)(slab + r * 128 + (((kc0 + 1) ^ ((r >> 1) & 7)) << 4));
    return v4d{lo[0], lo[1], hi[0], hi[1]};
}
__device__ inline v4f frag_at(const float *, const uint8_t *slab, int r, int kc0) {
    return *(const v4f *)(slab + r * 128 + ((kc0 ^ ((r >> 1) & 7)) << 4));
}

template <typename E_, int STAGES_, int BM_ = 256, int BN_ = 128, int WM_ = 4, int WN_ = 2, int MINB_ = 1>
struct Mfma2Tile {
    typedef E_ E;
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, GROUP_M = 8, STAGES = STAGES_, MINB = MINB_;
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int SLAB = 128;                                  // bytes of k per row and slab
    static constexpr int BK = SLAB / (int)sizeof(E);                 // k per slab
    static constexpr int STAGE = (BM + BN) * SLAB;                   // bytes per slab of both operands
    static constexpr int HDR = 256;                                   // keeps every LDS base address non-zero
    static constexpr int LPA = BM * SLAB / 1024 / (WM * WN);         // 1 KB load instructions per wave, A
    static constexpr int LPB = BN * SLAB / 1024 / (WM * WN);         // and B
    static constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    static constexpr int CPF = 4 * (int)sizeof(E) / 16;              // 16-byte chunks per fragment (2 or 1)
    static_assert(LPA * 1024 * WM * WN == BM * SLAB && LPB * 1024 * WM * WN == BN * SLAB, "load split");
};

template <class T, bool FUSED>
__global__ __launch_bounds__(T::THREADS, T::MINB) void k_gemm_mfma2(const typename T::E *__restrict__ A, int64_t lda,
                                                             const typename T::E *__restrict__ Bt, int64_t ldb,
                                                             typename T::E *__restrict__ C, int64_t ldc, int64_t M,
                                                             int64_t N, int64_t K, int accumulate, EpiArgs epi) {
    typedef typename T::E E;
    typedef MfmaOps<E> Ops;
    constexpr int BM = T::BM, BN = T::BN, SLAB = T::SLAB, STAGE = T::STAGE, HDR = T::HDR;
    constexpr int LPA = T::LPA, LPB = T::LPB, TM = T::TM, TN = T::TN, CPF = T::CPF;
    constexpr int VEC = 16 / (int)sizeof(E);
    __shared__ __attribute__((aligned(16))) uint8_t lds[HDR + T::STAGES * STAGE];

    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int64_t tm, tn;
    tile_of<T::GROUP_M>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = tm * BM, col0 = tn * BN;

    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wm = wave / T::WN, wn = wave % T::WN;

    // global sources of this lane's chunks per slab (swizzled on the global side)
    const E *srcA[LPA];
    const E *srcB[LPB];
#pragma unroll
    for (int q = 0; q < LPA; ++q) {
        const int c = (wave * LPA + q) * 64 + lane, r = c / 8, slot = c % 8;
        const int64_t ga = row0 + r < M ? row0 + r : M - 1;
        srcA[q] = A + ga * lda + (slot ^ ((r >> 1) & 7)) * VEC;
    }
#pragma unroll
    for (int q = 0; q < LPB; ++q) {
        const int c = (wave * LPB + q) * 64 + lane, r = c / 8, slot = c % 8;
        const int64_t gb = col0 + r < N ? col0 + r : N - 1;
        srcB[q] = Bt + gb * ldb + (slot ^ ((r >> 1) & 7)) * VEC;
    }
    auto issue = [&](int buf, int64_t k0) {
        uint8_t *a = lds + HDR + buf * STAGE + wave * LPA * 1024;
        uint8_t *b = lds + HDR + buf * STAGE + BM * SLAB + wave * LPB * 1024;
#pragma unroll
        for (int q = 0; q < LPA; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(srcA[q] + k0), (void *)(a + q * 1024), 16, 0, 0);
#pragma unroll
        for (int q = 0; q < LPB; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(srcB[q] + k0), (void *)(b + q * 1024), 16, 0, 0);
    };

    typename Ops::acc acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = typename Ops::acc{};

    const int lr = lane % 16, lq = lane / 16;
    const int arow = wm * (BM / T::WM) + lr, brow = wn * (BN / T::WN) + lr;

    const int64_t nk = K / T::BK;
#pragma unroll
    for (int s = 0; s < T::STAGES - 1; ++s)
        if (s < nk) issue(s, s * T::BK);
    for (int64_t kt = 0; kt < nk; ++kt) {
        // slab kt has landed once at most the later slabs already issued are outstanding
        if (kt + T::STAGES - 2 < nk) wait_vm<(T::STAGES - 2) * (LPA + LPB)>();
        else wait_vm<0>();
        bare_barrier();
        if (kt + T::STAGES - 1 < nk) issue((int)((kt + T::STAGES - 1) % T::STAGES), (kt + T::STAGES - 1) * T::BK);
        const uint8_t *As = lds + HDR + (kt % T::STAGES) * STAGE;
        const uint8_t *Bs = As + BM * SLAB;
#pragma unroll
        for (int kg = 0; kg < T::BK; kg += 16) {
            typename Ops::frag fa[TM], fb[TN];
            const int kc0 = kg * (int)sizeof(E) / 16 + lq * CPF;      // first chunk of this lane's fragment
#pragma unroll
            for (int a = 0; a < TM; ++a) fa[a] = frag_at((const E *)nullptr, As, arow + 16 * a, kc0);
#pragma unroll
            for (int b = 0; b < TN; ++b) fb[b] = frag_at((const E *)nullptr, Bs, brow + 16 * b, kc0);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b) acc[a][b] = Ops::mfma(fa[a][q], fb[b][q], acc[a][b]);
        }
    }

    // epilogue extras (uniform branches): the accumulator flip hook, then the
    // store with the fused partial sums; LDS is free once every wave is past the loop
    auto rowof = [](int l, int v) { return Ops::crow(l, v); };
    if (epi.fbit >= 0 && epi.fi >= row0 && epi.fi < row0 + BM && epi.fj >= col0 && epi.fj < col0 + BN)
        epi_flip(acc, epi, row0 + wm * (BM / T::WM), col0 + wn * (BN / T::WN), lane, rowof);
    if constexpr (FUSED) {
        __syncthreads();
        epi_store_fused<TM, TN, T::WM, T::WN, BM, BN>(acc, epi, (double *)(lds + HDR), row0, col0, tm, tn, M, N, wm,
                                                     wn, lane, 0, C, ldc, accumulate != 0, rowof);
        return;
    }
    const int ccol = lane % 16;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int64_t gc = col0 + wn * (BN / T::WN) + b * 16 + ccol;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gr = row0 + wm * (BM / T::WM) + a * 16 + Ops::crow(lane, v);
                if (gr < M && gc < N) C[gr * ldc + gc] = accumulate ? C[gr * ldc + gc] + acc[a][b][v] : acc[a][b][v];
            }
        }
    }
}

template <class T>
inline int launch_gemm_mfma2(const typename T::E *A, int64_t lda, const typename T::E *Bt, int64_t ldb,
                             typename T::E *C, int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s,
                             bool accumulate = false, EpiArgs *epi = nullptr) {
    if (K % T::BK) return ABFT_E_ARG;
    const int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
    if (tiles > INT32_MAX) return ABFT_E_ARG;
    EpiArgs e = epi ? *epi : epi_none();
    if (epi) {
        epi->tiles_m = (M + T::BM - 1) / T::BM;
        epi->tiles_n = (N + T::BN - 1) / T::BN;
    }
    if (e.pc)
        k_gemm_mfma2<T, true><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, accumulate, e);
    else
        k_gemm_mfma2<T, false><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, accumulate, e);
    return ABFT_OK;
}

}  // namespace abft
