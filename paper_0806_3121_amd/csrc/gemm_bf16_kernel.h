// bfloat16 x bfloat16 -> binary32 product on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), templated on the tile shape.  A is row-major and
// B column-major (Bt row-major), both k-contiguous, so every operand fragment
// is one 16-byte LDS read: lane l of a 16 x 32 block holds row l % 16,
// k = 8 * (l / 16) .. +7 (both operands); accumulator value v of lane l is
// C[4 * (l / 16) + v][l % 16] (measured on gfx950).
//
// Block tile BM x BN, WM x WN waves; K advances in BK-wide slabs through a
// double-buffered LDS (one barrier per slab, the next slab's global loads in
// flight while the current one feeds the matrix cores).  LDS rows are padded
// by 16 bytes: with BK = 64 the 16 rows a quarter-wave reads fall on 16
// disjoint 4-bank groups.
#pragma once

#include "gemm_mfma_kernel.h"

namespace abft {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <int BM_, int BN_, int BK_, int WM_, int WN_, int GROUP_M_ = 8, int MINB_ = 1>
struct Bf16Tile {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, GROUP_M = GROUP_M_, MINB = MINB_;
    static constexpr int VEC = 8;                           // bfloat16 per 16-byte load
    static constexpr int LDSROW = BK + VEC;                 // elements per LDS row
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    static constexpr int VPR = BK / VEC;
    static constexpr int ROWS_PER_PASS = THREADS / VPR;
    static constexpr int PASSES_A = BM / ROWS_PER_PASS, PASSES_B = BN / ROWS_PER_PASS;
    static constexpr int BUF = (BM + BN) * LDSROW;
    static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "wave tile");
    static_assert(BK % 32 == 0, "k group");
    static_assert(THREADS % VPR == 0 && BM % ROWS_PER_PASS == 0 && BN % ROWS_PER_PASS == 0, "load split");
};

template <class T>
__global__ __launch_bounds__(T::THREADS, T::MINB) void k_gemm_bf16(const uint16_t *__restrict__ A, int64_t lda,
                                                             const uint16_t *__restrict__ Bt, int64_t ldb,
                                                             float *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                                             int64_t K) {
    __shared__ uint16_t lds[2 * T::BUF];

    const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
    int64_t tm, tn;
    tile_of<T::GROUP_M>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = tm * T::BM, col0 = tn * T::BN;

    const int tid = threadIdx.x;
    const int lane = tid % 64, wave = tid / 64;
    const int wm = wave / T::WN, wn = wave % T::WN;

    const int lr = tid / T::VPR, lv = tid % T::VPR;
    v4u ra[T::PASSES_A], rb[T::PASSES_B];
    const uint16_t *pa[T::PASSES_A];
    const uint16_t *pb[T::PASSES_B];
    bool oka[T::PASSES_A], okb[T::PASSES_B];
#pragma unroll
    for (int p = 0; p < T::PASSES_A; ++p) {
        int64_t gr = row0 + lr + p * T::ROWS_PER_PASS;
        oka[p] = gr < M;
        pa[p] = A + (oka[p] ? gr : M - 1) * lda + T::VEC * lv;
    }
#pragma unroll
    for (int p = 0; p < T::PASSES_B; ++p) {
        int64_t gc = col0 + lr + p * T::ROWS_PER_PASS;
        okb[p] = gc < N;
        pb[p] = Bt + (okb[p] ? gc : N - 1) * ldb + T::VEC * lv;
    }
    const v4u zero = {0u, 0u, 0u, 0u};
    bool kin = true;
    auto load_slab = [&](int64_t k0) {
        kin = k0 + T::VEC * lv < K;
        int64_t ko = kin ? k0 : K - T::VEC - T::VEC * lv;
#pragma unroll
        for (int p = 0; p < T::PASSES_A; ++p) ra[p] = *(const v4u *)(pa[p] + ko);
#pragma unroll
        for (int p = 0; p < T::PASSES_B; ++p) rb[p] = *(const v4u *)(pb[p] + ko);
    };
    auto store_slab = [&](int buf) {
        uint16_t *As = lds + buf * T::BUF;
        uint16_t *Bs = As + T::BM * T::LDSROW;
#pragma unroll
        for (int p = 0; p < T::PASSES_A; ++p)
            *(v4u *)(As + (lr + p * T::ROWS_PER_PASS) * T::LDSROW + T::VEC * lv) = (oka[p] && kin) ? ra[p] : zero;
#pragma unroll
        for (int p = 0; p < T::PASSES_B; ++p)
            *(v4u *)(Bs + (lr + p * T::ROWS_PER_PASS) * T::LDSROW + T::VEC * lv) = (okb[p] && kin) ? rb[p] : zero;
    };

    v4f acc[T::TM][T::TN];
#pragma unroll
    for (int a = 0; a < T::TM; ++a)
#pragma unroll
        for (int b = 0; b < T::TN; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    const int lrow = lane % 16, lk = 8 * (lane / 16);
    const int a_off = (wm * (T::BM / T::WM) + lrow) * T::LDSROW + lk;
    const int b_off = T::BM * T::LDSROW + (wn * (T::BN / T::WN) + lrow) * T::LDSROW + lk;

    const int64_t nk = (K + T::BK - 1) / T::BK;
    load_slab(0);
    store_slab(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const bool more = kt + 1 < nk;
        if (more) load_slab((kt + 1) * T::BK);
        const uint16_t *Aw = lds + (kt & 1) * T::BUF + a_off;
        const uint16_t *Bw = lds + (kt & 1) * T::BUF + b_off;
#pragma unroll
        for (int kg = 0; kg < T::BK; kg += 32) {
            v8bf fa[T::TM], fb[T::TN];
#pragma unroll
            for (int a = 0; a < T::TM; ++a) fa[a] = *(const v8bf *)(Aw + a * 16 * T::LDSROW + kg);
#pragma unroll
            for (int b = 0; b < T::TN; ++b) fb[b] = *(const v8bf *)(Bw + b * 16 * T::LDSROW + kg);
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
#pragma unroll
                for (int b = 0; b < T::TN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        if (more) store_slab((kt + 1) & 1);
        __syncthreads();
    }

    const int ccol = lane % 16;
#pragma unroll
    for (int a = 0; a < T::TM; ++a) {
#pragma unroll
        for (int b = 0; b < T::TN; ++b) {
            int64_t gc = col0 + wn * (T::BN / T::WN) + b * 16 + ccol;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t gr = row0 + wm * (T::BM / T::WM) + a * 16 + 4 * (lane / 16) + v;
                if (gr < M && gc < N) C[gr * ldc + gc] = acc[a][b][v];
            }
        }
    }
}

template <class T>
inline int launch_gemm_bf16_tile(const uint16_t *A, int64_t lda, const uint16_t *Bt, int64_t ldb, float *C,
                                 int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s) {
    int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
    if (tiles > INT32_MAX) return ABFT_E_ARG;
    k_gemm_bf16<T><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K);
    return ABFT_OK;
}

}  // namespace abft
