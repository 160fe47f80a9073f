// Protected product C_f = A_f B_f (Eq. ABFT-GEMM) dispatch.
//
// The data part and any thick checksum block (b > kSliverMaxB) run on the
// matrix cores (gemm_f64_kernel.h).  A thin checksum block (b <= kSliverMaxB,
// e.g. the classic b = 1) would occupy a whole row or column of tiles for a
// few useful rows, so it is computed instead by the skinny-product kernel
// (k_sliver.hip), which streams the other operand once.
#include "gemm_f64_kernel.h"

namespace abft {

int launch_sliver_rows_f64(const Geom &g, const double *Acs, int64_t ldacs, const double *Bt, int64_t ldb, double *C,
                           int64_t ldc, hipStream_t s);
int launch_sliver_cols_f64(const Geom &g, int64_t rows, const double *A, int64_t lda, const double *Bcs, int64_t ldbcs,
                           double *C, int64_t ldc, hipStream_t s);

constexpr int64_t kSliverMaxB = 8;

// Tile candidates: per-tile efficiency measured on MI355X at 8192^3 / 9216^2 x 8192,
// and resident blocks per CU (LDS- and register-limited).
using F64_256x128 = F64Tile<256, 128, 16, 4, 2>;
using F64_128x128 = F64Tile<128, 128, 16, 2, 2>;
using F64_128x96 = F64Tile<128, 96, 16, 2, 2, 8, 2>;
using F64_96x96 = F64Tile<96, 96, 16, 2, 2, 8, 2>;

struct TileChoice { int id; int bm, bn, per_cu; double eff; };
static const TileChoice kF64Tiles[] = {
    {0, 256, 128, 1, 0.818}, {1, 128, 128, 2, 0.787}, {2, 128, 96, 2, 0.80}, {3, 96, 96, 2, 0.76},
};

// Estimated time ~ rounds of resident blocks x time per round (tile flops x
// blocks per CU / efficiency); the smallest wins.  256 CUs.
static int choose_f64_tile(int64_t M, int64_t N) {
    double best = 0;
    int pick = 0;
    for (const TileChoice &t : kF64Tiles) {
        int64_t tiles = ((M + t.bm - 1) / t.bm) * ((N + t.bn - 1) / t.bn);
        int64_t slots = 256 * t.per_cu;
        double rounds = (double)((tiles + slots - 1) / slots);
        double cost = rounds * (double)t.bm * t.bn * t.per_cu / t.eff;
        if (best == 0 || cost < best) { best = cost; pick = t.id; }
    }
    return pick;
}

static int gemm_f64_main(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc,
                         int64_t M, int64_t N, int64_t K, hipStream_t s) {
    switch (choose_f64_tile(M, N)) {
    case 0: return launch_gemm_f64_tile<F64_256x128>(A, lda, Bt, ldb, C, ldc, M, N, K, s);
    case 1: return launch_gemm_f64_tile<F64_128x128>(A, lda, Bt, ldb, C, ldc, M, N, K, s);
    case 2: return launch_gemm_f64_tile<F64_128x96>(A, lda, Bt, ldb, C, ldc, M, N, K, s);
    default: return launch_gemm_f64_tile<F64_96x96>(A, lda, Bt, ldb, C, ldc, M, N, K, s);
    }
}

int launch_gemm(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, uint32_t flags, hipStream_t s) {
    Geom g = geom_of(p);
    const bool plain = flags & ABFT_PLAIN;
    const bool thin_r = !plain && g.S * g.br <= kSliverMaxB;
    const bool thin_c = !plain && g.S * g.bc <= kSliverMaxB;
    int64_t Mm = (plain || thin_r) ? g.m : g.M;
    int64_t Nm = (plain || thin_c) ? g.n : g.N;
    int st;
    switch (p->dtype) {
    case ABFT_F64: {
        const double *A = (const double *)A_f, *Bt = (const double *)B_f;
        double *C = (double *)C_f;
        st = gemm_f64_main(A, p->lda, Bt, p->ldb, C, p->ldc, Mm, Nm, g.k, s);
        if (st) return st;
        ABFT_LAUNCHED();
        // carried row block over all N columns (corner included), then the
        // carried column block over the rows the main product covered
        if (thin_r && (st = launch_sliver_rows_f64(g, A + g.m * p->lda, p->lda, Bt, p->ldb, C, p->ldc, s))) return st;
        if (thin_c && (st = launch_sliver_cols_f64(g, Mm, A, p->lda, Bt + g.n * p->ldb, p->ldb, C, p->ldc, s)))
            return st;
        return ABFT_OK;
    }
    default:
        return ABFT_E_UNSUPPORTED;
    }
}

}  // namespace abft
