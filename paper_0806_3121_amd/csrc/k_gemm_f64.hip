// Protected product C_f = A_f B_f in binary64 on the gfx950 matrix cores
// (v_mfma_f64_16x16x4_f64).  A_f is row-major (k contiguous) and B_f is
// column-major (k contiguous), so both operands stream k-contiguous rows.
//
// Block tile BM x BN with 256 threads (4 waves in a 2 x 2 grid, 64 x 64 per
// wave = 4 x 4 MFMA tiles of 16 x 16).  K advances in BK-wide slabs staged in
// LDS; the next slab is loaded into registers while the current one feeds the
// matrix cores.  Inside a 16-wide k group each lane reads four consecutive k
// of its row (one 32-byte LDS read) and feeds them to four MFMAs; A and B use
// the same k permutation, so every product a_il * b_lj is formed exactly once.
//
// MFMA 16x16x4 f64 operand layout (lane l of 64): A[l % 16][l / 16],
// B[l / 16][l % 16]; the 4 accumulator values of lane l are
// C[l / 16 + 4 * v][l % 16], v = 0..3.
#include "common.h"

namespace abft {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

namespace f64gemm {
constexpr int BM = 128, BN = 128, BK = 32, PAD = 2;
constexpr int LDSROW = BK + PAD;               // doubles per LDS row
constexpr int THREADS = 256;
constexpr int WM = 2, WN = 2;                  // wave grid
constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
constexpr int VPR = BK / 2;                    // 16-byte vectors per tile row
constexpr int ROWS_PER_PASS = THREADS / VPR;   // tile rows loaded per pass
constexpr int PASSES_A = BM / ROWS_PER_PASS, PASSES_B = BN / ROWS_PER_PASS;
constexpr int GROUP_M = 8;                     // tile-row grouping for L2 reuse
}  // namespace f64gemm

// Map the linear workgroup id to a C tile: ids are first spread back from the
// round-robin XCD dispatch (workgroup w runs on XCD w mod 8) so each XCD owns a
// contiguous range, then ranges are walked in GROUP_M-row bands so that the
// tiles an XCD runs together share A rows and B columns in its L2.
__device__ inline void tile_of(int64_t wg, int64_t nwg, int64_t tiles_m, int64_t tiles_n, int64_t &tm, int64_t &tn) {
    const int64_t nxcd = 8;
    int64_t id = wg;
    if (nwg % nxcd == 0) id = (wg % nxcd) * (nwg / nxcd) + wg / nxcd;
    const int64_t G = f64gemm::GROUP_M;
    int64_t band = id / (G * tiles_n);
    int64_t first_m = band * G;
    int64_t gm = min(tiles_m - first_m, G);
    int64_t in = id - band * G * tiles_n;
    tm = first_m + in % gm;
    tn = in / gm;
}

__global__ __launch_bounds__(f64gemm::THREADS, 1) void k_gemm_f64(const double *__restrict__ A, int64_t lda,
                                                                  const double *__restrict__ Bt, int64_t ldb,
                                                                  double *__restrict__ C, int64_t ldc, int64_t M,
                                                                  int64_t N, int64_t K) {
    using namespace f64gemm;
    __shared__ double As[BM * LDSROW];
    __shared__ double Bs[BN * LDSROW];

    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int64_t tm, tn;
    tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = tm * BM, col0 = tn * BN;

    const int tid = threadIdx.x;
    const int lane = tid % 64, wave = tid / 64;
    const int wm = wave / WN, wn = wave % WN;

    // global -> register staging: thread loads vector v of tile rows rr + p*ROWS_PER_PASS
    const int lr = tid / VPR, lv = tid % VPR;
    v2d ra[PASSES_A], rb[PASSES_B];

    auto load_tiles = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < PASSES_A; ++p) {
            int64_t gr = row0 + lr + p * ROWS_PER_PASS, gk = k0 + 2 * lv;
            if (gr < M && gk < K) ra[p] = *(const v2d *)(A + gr * lda + gk);
            else ra[p] = v2d{0.0, 0.0};
        }
#pragma unroll
        for (int p = 0; p < PASSES_B; ++p) {
            int64_t gc = col0 + lr + p * ROWS_PER_PASS, gk = k0 + 2 * lv;
            if (gc < N && gk < K) rb[p] = *(const v2d *)(Bt + gc * ldb + gk);
            else rb[p] = v2d{0.0, 0.0};
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int p = 0; p < PASSES_A; ++p) *(v2d *)(As + (lr + p * ROWS_PER_PASS) * LDSROW + 2 * lv) = ra[p];
#pragma unroll
        for (int p = 0; p < PASSES_B; ++p) *(v2d *)(Bs + (lr + p * ROWS_PER_PASS) * LDSROW + 2 * lv) = rb[p];
    };

    v4d acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

    const int lrow = lane % 16, lk = 4 * (lane / 16);
    const double *Aw = As + (wm * (BM / WM) + lrow) * LDSROW + lk;
    const double *Bw = Bs + (wn * (BN / WN) + lrow) * LDSROW + lk;

    const int64_t nk = (K + BK - 1) / BK;
    load_tiles(0);
    store_tiles();
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
        for (int kg = 0; kg < BK; kg += 16) {
            v4d fa[TM], fb[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) fa[a] = *(const v4d *)(Aw + a * 16 * LDSROW + kg);
#pragma unroll
            for (int b = 0; b < TN; ++b) fb[b] = *(const v4d *)(Bw + b * 16 * LDSROW + kg);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a][q], fb[b][q], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store_tiles();
            __syncthreads();
        }
    }

    // epilogue: lane holds C[lane/16 + 4*v][lane % 16] of each 16 x 16 tile
    const int crow = lane / 16, ccol = lane % 16;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            int64_t gc = col0 + wn * (BN / WN) + b * 16 + ccol;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t gr = row0 + wm * (BM / WM) + a * 16 + crow + 4 * v;
                if (gr < M && gc < N) C[gr * ldc + gc] = acc[a][b][v];
            }
        }
    }
}

int launch_gemm_f64(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc, int64_t M,
                    int64_t N, int64_t K, hipStream_t s) {
    using namespace f64gemm;
    int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    if (tiles > INT32_MAX) return ABFT_E_ARG;
    k_gemm_f64<<<(unsigned)tiles, THREADS, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_gemm(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, uint32_t flags, hipStream_t s) {
    Geom g = geom_of(p);
    int64_t M = (flags & ABFT_PLAIN) ? g.m : g.M;
    int64_t N = (flags & ABFT_PLAIN) ? g.n : g.N;
    switch (p->dtype) {
    case ABFT_F64:
        return launch_gemm_f64((const double *)A_f, p->lda, (const double *)B_f, p->ldb, (double *)C_f, p->ldc, M, N,
                               g.k, s);
    default:
        return ABFT_E_UNSUPPORTED;
    }
}

}  // namespace abft
