// binary64 / binary32 product kernel on the gfx950 matrix cores
// (v_mfma_f64_16x16x4_f64, v_mfma_f32_16x16x4_f32), templated on the element
// type and the tile shape.  A is row-major (k contiguous) and B is stored
// column-major (its transpose Bt row-major, k contiguous), so both operands
// stream k-contiguous rows.
//
// Block tile BM x BN, WM x WN waves, each wave owning (BM/WM) x (BN/WN) as
// 16 x 16 MFMA tiles.  K advances in BK-wide slabs through a double-buffered
// LDS: while the matrix cores consume slab t from one buffer, slab t+1 (loaded
// into registers at the top of the iteration) is written to the other, so one
// barrier per slab suffices.  Loads are branch-free: out-of-range rows and
// k are clamped to a valid address and the value is replaced by zero.
//
// Inside a 16-wide k group each lane reads four consecutive k of its row (one
// LDS read) and feeds them to four MFMAs; A and B use the same k permutation,
// so every product a_il * b_lj is formed exactly once.
//
// MFMA 16x16x4 lane layout (lane l of 64), both types: A operand
// A[l % 16][l / 16], B operand B[l / 16][l % 16].  Accumulator value v of lane
// l is C[l / 16 + 4 * v][l % 16] for f64 and C[4 * (l / 16) + v][l % 16] for
// f32 (measured on gfx950).
#pragma once

#include "common.h"
#include "epilogue.h"

namespace abft {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename E> struct MfmaOps;
template <> struct MfmaOps<double> {
    typedef double vec16 __attribute__((ext_vector_type(2)));   // one 16-byte global load
    typedef v4d frag;                                            // four consecutive k of one row
    typedef v4d acc;
    __device__ static acc mfma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int crow(int lane, int v) { return lane / 16 + 4 * v; }
};
template <> struct MfmaOps<float> {
    typedef float vec16 __attribute__((ext_vector_type(4)));
    typedef v4f frag;
    typedef v4f acc;
    __device__ static acc mfma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int crow(int lane, int v) { return 4 * (lane / 16) + v; }
};

template <typename E_, int BM_, int BN_, int BK_, int WM_, int WN_, int GROUP_M_ = 8, int MINB_ = 1>
struct MfmaTile {
    typedef E_ E;
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, GROUP_M = GROUP_M_, MINB = MINB_;
    static constexpr int VEC = 16 / (int)sizeof(E);        // elements per 16-byte load
    static constexpr int PAD = VEC;                         // 16-byte row skew against bank conflicts
    static constexpr int LDSROW = BK + PAD;                 // elements per LDS row
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    static constexpr int VPR = BK / VEC;                    // 16-byte vectors per tile row
    static constexpr int ROWS_PER_PASS = THREADS / VPR;
    static constexpr int PASSES_A = BM / ROWS_PER_PASS, PASSES_B = BN / ROWS_PER_PASS;
    static constexpr int BUF = (BM + BN) * LDSROW;          // elements per LDS buffer
    static constexpr size_t LDS_BYTES = 2 * BUF * sizeof(E);
    static_assert(BM % (WM * 16) == 0 && BN % (WN * 16) == 0, "wave tile");
    static_assert(BK % 16 == 0, "k group");
    static_assert(THREADS % VPR == 0 && BM % ROWS_PER_PASS == 0 && BN % ROWS_PER_PASS == 0, "load split");
};

// Map the linear workgroup id to a C tile: ids are first spread back from the
// round-robin XCD dispatch (workgroup w runs on XCD w mod 8) so each XCD owns a
// contiguous range, then ranges are walked in GROUP_M-row bands so that the
// tiles an XCD runs together share A rows and B columns in its L2.
template <int GROUP_M>
__device__ inline void tile_of(int64_t wg, int64_t nwg, int64_t tiles_m, int64_t tiles_n, int64_t &tm, int64_t &tn) {
    const int64_t nxcd = 8;
    int64_t id = wg;
    if (nwg % nxcd == 0) id = (wg % nxcd) * (nwg / nxcd) + wg / nxcd;
    int64_t band = id / (GROUP_M * tiles_n);
    int64_t first_m = band * GROUP_M;
    int64_t gm = tiles_m - first_m < GROUP_M ? tiles_m - first_m : GROUP_M;
    int64_t in = id - band * GROUP_M * tiles_n;
    tm = first_m + in % gm;
    tn = in / gm;
}

template <class T, bool FUSED>
__global__ __launch_bounds__(T::THREADS, T::MINB) void k_gemm_mfma(const typename T::E *__restrict__ A, int64_t lda,
                                                             const typename T::E *__restrict__ Bt, int64_t ldb,
                                                             typename T::E *__restrict__ C, int64_t ldc, int64_t M,
                                                             int64_t N, int64_t K, int accumulate, EpiArgs epi) {
    typedef typename T::E E;
    typedef MfmaOps<E> Ops;
    typedef typename Ops::vec16 v16;
    __shared__ __attribute__((aligned(16))) E lds[2 * T::BUF];

    const int64_t tiles_m = (M + T::BM - 1) / T::BM, tiles_n = (N + T::BN - 1) / T::BN;
    int64_t tm, tn;
    tile_of<T::GROUP_M>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = tm * T::BM, col0 = tn * T::BN;

    const int tid = threadIdx.x;
    const int lane = tid % 64, wave = tid / 64;
    const int wm = wave / T::WN, wn = wave % T::WN;

    // global -> register staging; thread loads vector lv of tile rows lr + p*ROWS_PER_PASS
    const int lr = tid / T::VPR, lv = tid % T::VPR;
    v16 ra[T::PASSES_A], rb[T::PASSES_B];
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
    const v16 zero = {};
    bool kin = true;
    // Raw loads only: the zero mask is applied when the slab is written to LDS,
    // after the matrix-core work, so the loads stay in flight meanwhile.
    auto load_slab = [&](int64_t k0) {
        // k0 + VEC*lv and K are multiples of VEC, so a vector is either wholly in or out
        kin = k0 + T::VEC * lv < K;
        int64_t ko = kin ? k0 : K - T::VEC - T::VEC * lv;   // clamp to a valid in-row address
#pragma unroll
        for (int p = 0; p < T::PASSES_A; ++p) ra[p] = *(const v16 *)(pa[p] + ko);
#pragma unroll
        for (int p = 0; p < T::PASSES_B; ++p) rb[p] = *(const v16 *)(pb[p] + ko);
    };
    auto store_slab = [&](int buf) {
        E *As = lds + buf * T::BUF;
        E *Bs = As + T::BM * T::LDSROW;
#pragma unroll
        for (int p = 0; p < T::PASSES_A; ++p)
            *(v16 *)(As + (lr + p * T::ROWS_PER_PASS) * T::LDSROW + T::VEC * lv) = (oka[p] && kin) ? ra[p] : zero;
#pragma unroll
        for (int p = 0; p < T::PASSES_B; ++p)
            *(v16 *)(Bs + (lr + p * T::ROWS_PER_PASS) * T::LDSROW + T::VEC * lv) = (okb[p] && kin) ? rb[p] : zero;
    };

    typename Ops::acc acc[T::TM][T::TN];
#pragma unroll
    for (int a = 0; a < T::TM; ++a)
#pragma unroll
        for (int b = 0; b < T::TN; ++b) acc[a][b] = typename Ops::acc{};

    const int lrow = lane % 16, lk = 4 * (lane / 16);
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
        for (int kg = 0; kg < T::BK; kg += 16) {
            typename Ops::frag fa[T::TM], fb[T::TN];
#pragma unroll
            for (int a = 0; a < T::TM; ++a) fa[a] = *(const typename Ops::frag *)(Aw + a * 16 * T::LDSROW + kg);
#pragma unroll
            for (int b = 0; b < T::TN; ++b) fb[b] = *(const typename Ops::frag *)(Bw + b * 16 * T::LDSROW + kg);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int a = 0; a < T::TM; ++a)
#pragma unroll
                    for (int b = 0; b < T::TN; ++b)
                        acc[a][b] = Ops::mfma(fa[a][q], fb[b][q], acc[a][b]);
        }
        if (more) store_slab((kt + 1) & 1);
        __syncthreads();
    }

    // epilogue extras (uniform branches): the accumulator flip hook, then the
    // store with the fused partial sums
    auto rowof = [](int l, int v) { return Ops::crow(l, v); };
    if (epi.fbit >= 0 && epi.fi >= row0 && epi.fi < row0 + T::BM && epi.fj >= col0 && epi.fj < col0 + T::BN)
        epi_flip(acc, epi, row0 + wm * (T::BM / T::WM), col0 + wn * (T::BN / T::WN), lane, rowof);
    if constexpr (FUSED) {
        epi_store_fused<T::TM, T::TN, T::WM, T::WN, T::BM, T::BN>(
            acc, epi, (double *)lds, row0, col0, tm, tn, M, N, wm, wn, lane, 0, C, ldc, accumulate != 0, rowof);
        return;
    }

    // epilogue: lane holds row Ops::crow(lane, v), column lane % 16 of each 16 x 16 tile
    const int ccol = lane % 16;
#pragma unroll
    for (int a = 0; a < T::TM; ++a) {
#pragma unroll
        for (int b = 0; b < T::TN; ++b) {
            int64_t gc = col0 + wn * (T::BN / T::WN) + b * 16 + ccol;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t gr = row0 + wm * (T::BM / T::WM) + a * 16 + Ops::crow(lane, v);
                if (gr < M && gc < N) C[gr * ldc + gc] = accumulate ? C[gr * ldc + gc] + acc[a][b][v] : acc[a][b][v];
            }
        }
    }
}

template <class T>
inline int launch_gemm_tile(const typename T::E *A, int64_t lda, const typename T::E *Bt, int64_t ldb,
                            typename T::E *C, int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s,
                            bool accumulate = false, EpiArgs *epi = nullptr) {
    int64_t tiles = ((M + T::BM - 1) / T::BM) * ((N + T::BN - 1) / T::BN);
    if (tiles > INT32_MAX) return ABFT_E_ARG;
    EpiArgs e = epi ? *epi : epi_none();
    if (epi) {
        epi->tiles_m = (M + T::BM - 1) / T::BM;
        epi->tiles_n = (N + T::BN - 1) / T::BN;
    }
    if (e.pc)
        k_gemm_mfma<T, true><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, accumulate, e);
    else
        k_gemm_mfma<T, false><<<(unsigned)tiles, T::THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, accumulate, e);
    return ABFT_OK;
}

}  // namespace abft
