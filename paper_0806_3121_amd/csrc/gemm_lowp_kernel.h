// Low-precision products with binary32 accumulation on the gfx950 matrix
// cores, templated on the element type and the tile shape:
//   bfloat16: v_mfma_f32_16x16x32_bf16 (16 x 16 x 32 per instruction)
//   FP8 E4M3 (OCP e4m3fn): v_mfma_f32_16x16x32_fp8_fp8
// A is row-major and B column-major (Bt row-major), both k-contiguous.  Each
// lane reads one 16-byte fragment of its row per 64-byte k group: lane l of a
// 16-row block holds row l % 16 and the 16 bytes at k-byte offset
// 16 * (l / 16); bfloat16 feeds it to one MFMA (8 values), FP8 to two MFMAs
// (8 values each).  A and B use the same k mapping, so every product is
// formed exactly once.  Accumulator value v of lane l is
// C[4 * (l / 16) + v][l % 16] (measured on gfx950).  FP8 products are scaled
// back by 2^-(eA + eB), read from the device (the per-tensor scales of the
// quantizer), in the epilogue: an exact power-of-two scaling.
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

// Each Ops feeds one MFMA group from CPM 16-byte chunks per lane (mfma_chunks).
struct Bf16Ops {
    typedef uint16_t E;
    static constexpr int KG = 32;       // k per fragment read across the wave's four lane groups
    static constexpr int CPM = 1;
    static constexpr int MT = 16;       // output tile of one instruction: MT x MT
    __device__ static void mfma(const v4u &a, const v4u &b, v4f &c) {
        v8bf x, y;
        __builtin_memcpy(&x, &a, 16);
        __builtin_memcpy(&y, &b, 16);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
    __device__ static void mfma_chunks(const v4u *a, const v4u *b, v4f &c) { mfma(a[0], b[0], c); }
};
struct Fp8Ops {
    typedef uint8_t E;
    static constexpr int KG = 64;
    static constexpr int CPM = 1;
    static constexpr int MT = 16;
    __device__ static void mfma(const v4u &a, const v4u &b, v4f &c) {
        long a0 = (long)(((uint64_t)a[1] << 32) | a[0]), a1 = (long)(((uint64_t)a[3] << 32) | a[2]);
        long b0 = (long)(((uint64_t)b[1] << 32) | b[0]), b1 = (long)(((uint64_t)b[3] << 32) | b[2]);
        c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, c, 0, 0, 0);
    }
    __device__ static void mfma_chunks(const v4u *a, const v4u *b, v4f &c) { mfma(a[0], b[0], c); }
};

// FP8 E4M3 through v_mfma_scale_f32_32x32x64_f8f6f4 (unit E8M0 scales): a 32 x 32
// output tile over 64 k per instruction.  Lane l holds row (column) l % 32 and
// 32 bytes of k, lanes 32-63 the second half of the 64; accumulator value v of
// lane l is row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32 (measured on
// gfx950 with integer-valued data, whose products and sums are exact).
typedef float v16f __attribute__((ext_vector_type(16)));
struct Fp8x64Ops {
    typedef uint8_t E;
    static constexpr int CPM = 2;
    static constexpr int MT = 32;
    typedef int v8i __attribute__((ext_vector_type(8)));
    __device__ static void mfma(const v8i &a, const v8i &b, v16f &c) {
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    }
};

template <class Ops_, int BM_, int BN_, int BK_, int WM_, int WN_, int GROUP_M_ = 8, int MINB_ = 1>
struct LowpTile {
    typedef Ops_ Ops;
    typedef typename Ops::E E;
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, GROUP_M = GROUP_M_, MINB = MINB_;
    static constexpr int VEC = 16 / (int)sizeof(E);        // elements per 16-byte load
    static constexpr int LDSROW = BK + VEC;                 // elements per LDS row (16-byte skew)
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    static constexpr int VPR = BK / VEC;
    static constexpr int ROWS_PER_PASS = THREADS / VPR;
    static constexpr int PASSES_A = BM / ROWS_PER_PASS, PASSES_B = BN / ROWS_PER_PASS;
    static constexpr int BUF = (BM + BN) * LDSROW;
    static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "wave tile");
    static_assert(BK % Ops::KG == 0, "k group");
    static_assert(THREADS % VPR == 0 && BM % ROWS_PER_PASS == 0 && BN % ROWS_PER_PASS == 0, "load split");
};

// One BM x BN tile of C at (row0, col0): the whole k loop and the epilogue.
// lds holds 2 * T::BUF elements; the function ends with a barrier, so a
// persistent caller may reuse lds for its next tile.
template <class T, bool FUSED>
__device__ inline void lowp_tile(const typename T::E *__restrict__ A, int64_t lda, const typename T::E *__restrict__ Bt,
                                 int64_t ldb, float *__restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                 int sh, int64_t row0, int64_t col0, typename T::E *lds, const EpiArgs &epi,
                                 int64_t tm, int64_t tn) {
    typedef typename T::E E;
    const int tid = threadIdx.x;
    const int lane = tid % 64, wave = tid / 64;
    const int wm = wave / T::WN, wn = wave % T::WN;

    const int lr = tid / T::VPR, lv = tid % T::VPR;
    v4u ra[T::PASSES_A], rb[T::PASSES_B];
    const E *pa[T::PASSES_A];
    const E *pb[T::PASSES_B];
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
        E *As = lds + buf * T::BUF;
        E *Bs = As + T::BM * T::LDSROW;
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

    const int lrow = lane % 16, lk = T::VEC * (lane / 16);
    const int a_off = (wm * (T::BM / T::WM) + lrow) * T::LDSROW + lk;
    const int b_off = T::BM * T::LDSROW + (wn * (T::BN / T::WN) + lrow) * T::LDSROW + lk;

    const int64_t nk = (K + T::BK - 1) / T::BK;
    load_slab(0);
    store_slab(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const bool more = kt + 1 < nk;
        if (more) load_slab((kt + 1) * T::BK);
        const E *Aw = lds + (kt & 1) * T::BUF + a_off;
        const E *Bw = lds + (kt & 1) * T::BUF + b_off;
#pragma unroll
        for (int kg = 0; kg < T::BK; kg += T::Ops::KG) {
            v4u fa[T::TM], fb[T::TN];
#pragma unroll
            for (int a = 0; a < T::TM; ++a) fa[a] = *(const v4u *)(Aw + a * 16 * T::LDSROW + kg);
#pragma unroll
            for (int b = 0; b < T::TN; ++b) fb[b] = *(const v4u *)(Bw + b * 16 * T::LDSROW + kg);
#pragma unroll
            for (int a = 0; a < T::TM; ++a)
#pragma unroll
                for (int b = 0; b < T::TN; ++b) T::Ops::mfma(fa[a], fb[b], acc[a][b]);
        }
        if (more) store_slab((kt + 1) & 1);
        __syncthreads();
    }

    // epilogue extras (uniform branches): the accumulator flip hook, then the
    // store with the fused partial sums
    auto rowof = [](int l, int v) { return 4 * (l / 16) + v; };
    if (epi.fbit >= 0 && epi.fi >= row0 && epi.fi < row0 + T::BM && epi.fj >= col0 && epi.fj < col0 + T::BN)
        epi_flip(acc, epi, row0 + wm * (T::BM / T::WM), col0 + wn * (T::BN / T::WN), lane, rowof);
    if constexpr (FUSED) {
        epi_store_fused<T::TM, T::TN, T::WM, T::WN, T::BM, T::BN>(
            acc, epi, (double *)lds, row0, col0, tm, tn, M, N, wm, wn, lane, sh, C, ldc, false, rowof);
        return;
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
                if (gr < M && gc < N) C[gr * ldc + gc] = __builtin_ldexpf(acc[a][b][v], sh);
            }
        }
    }
}

template <class T, bool FUSED>
__global__ __launch_bounds__(T::THREADS, T::MINB) void k_gemm_lowp(const typename T::E *__restrict__ A, int64_t lda,
                                                             const typename T::E *__restrict__ Bt, int64_t ldb,
                                                             float *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                                             int64_t K, const int *__restrict__ scale_exp,
                                                             EpiArgs epi) {
    __shared__ __attribute__((aligned(16))) typename T::E lds[2 * T::BUF];
    const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
    int64_t tm, tn;
    tile_of<T::GROUP_M>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int sh = scale_exp ? -(scale_exp[0] + scale_exp[1]) : 0;      // scale back by 2^sh with ldexp
    lowp_tile<T, FUSED>(A, lda, Bt, ldb, C, ldc, M, N, K, sh, tm * T::BM, tn * T::BN, lds, epi, tm, tn);
}

template <class T>
inline int launch_gemm_lowp_tile(const typename T::E *A, int64_t lda, const typename T::E *Bt, int64_t ldb, float *C,
                                 int64_t ldc, int64_t M, int64_t N, int64_t K, const int *scale_exp, hipStream_t s,
                                 EpiArgs *epi = nullptr) {
    int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
    if (tiles > INT32_MAX) return ABFT_E_ARG;
    EpiArgs e = epi ? *epi : epi_none();
    if (epi) {
        epi->tiles_m = (M + T::BM - 1) / T::BM;
        epi->tiles_n = (N + T::BN - 1) / T::BN;
    }
    if (e.pc)
        k_gemm_lowp<T, true><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, scale_exp, e);
    else
        k_gemm_lowp<T, false><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, scale_exp, e);
    return ABFT_OK;
}

}  // namespace abft
