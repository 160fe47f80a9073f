// Protected product C_f = A_f B_f (Eq. ABFT-GEMM) dispatch.
//
// The data part and any thick checksum block (b > kSliverMaxB) run on the
// matrix cores (gemm_mfma2_kernel.h / gemm_mfma_kernel.h for binary64 and
// binary32, gemm_lowp2_kernel.h / gemm_lowp_kernel.h for bfloat16 and FP8).
// A thin checksum block (b <= kSliverMaxB, e.g. the classic b = 1) would
// occupy a whole row or column of tiles for a few useful rows, so it is
// computed instead by the skinny-product kernel (sliver_kernel.h), which
// streams the other operand once with binary64 accumulation.  The tile pick
// lives in one function per element type, used by the launch and by
// abft_describe_gemm alike.
#include "gemm_lowp2_kernel.h"
#include "gemm_lowp_kernel.h"
#include "gemm_mfma2_kernel.h"
#include "gemm_mfma_kernel.h"
#include "sliver_kernel.h"

#include <cstdio>

namespace abft {

constexpr int64_t kSliverMaxB = 8;

struct TileChoice { int id; int bm, bn, per_cu; double eff; };

// Estimated time ~ rounds of resident blocks x time per round (tile flops x
// blocks per CU / per-tile efficiency); the smallest wins.  256 CUs.  Returns
// the index of the pick in tab.
static int choose_tile(const TileChoice *tab, int n, int64_t M, int64_t N) {
    double best = 0;
    int pick = 0;
    for (int q = 0; q < n; ++q) {
        const TileChoice &t = tab[q];
        int64_t tiles = ((M + t.bm - 1) / t.bm) * ((N + t.bn - 1) / t.bn);
        int64_t slots = 256 * t.per_cu;
        double rounds = (double)((tiles + slots - 1) / slots);
        double cost = rounds * (double)t.bm * t.bn * t.per_cu / t.eff;
        if (best == 0 || cost < best) { best = cost; pick = q; }
    }
    return pick;
}

// binary64 / binary32 direct-to-LDS candidates (K a multiple of the 128-byte slab); per-tile
// efficiencies measured on MI355X at 8192^3 and 9216^2 x 8192 (binary64).  A 256 x 128 binary64
// tile (0.85) is never cheaper than 128 x 128 at two blocks per CU and is not offered.
static const TileChoice kF64DirectTiles[] = {
    {1, 128, 128, 2, 0.87}, {2, 128, 96, 2, 0.89}, {3, 96, 96, 2, 0.88},
};
static const TileChoice kF32DirectTiles[] = {
    {0, 256, 128, 1, 0.85}, {1, 128, 128, 2, 0.84},
};

// binary64 candidates of the register-staged kernel (any even K); efficiencies measured on MI355X at
// 8192^3 and 9216^2 x 8192.
static const TileChoice kF64Tiles[] = {
    {0, 256, 128, 1, 0.818}, {1, 128, 128, 2, 0.787}, {2, 128, 96, 2, 0.80}, {3, 96, 96, 2, 0.76},
};
// binary32 candidates (same shapes; the f32 matrix core is twice as fast per instruction).
static const TileChoice kF32Tiles[] = {
    {0, 256, 128, 1, 0.80}, {1, 128, 128, 2, 0.78},
};

// The data-part kernel and tile for an M x N x K product of element type E.
struct MainPick {
    bool direct;            // direct-to-LDS kernel (else register-staged / padded-LDS)
    const TileChoice *t;
};
static MainPick pick_main(const double *, int64_t M, int64_t N, int64_t K) {
    if (K % 16 == 0) return {true, &kF64DirectTiles[choose_tile(kF64DirectTiles, 3, M, N)]};
    return {false, &kF64Tiles[choose_tile(kF64Tiles, 4, M, N)]};
}
static MainPick pick_main(const float *, int64_t M, int64_t N, int64_t K) {
    if (K % 32 == 0) return {true, &kF32DirectTiles[choose_tile(kF32DirectTiles, 2, M, N)]};
    return {false, &kF32Tiles[choose_tile(kF32Tiles, 2, M, N)]};
}

static int gemm_main(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc, int64_t M,
                     int64_t N, int64_t K, hipStream_t s, bool acc = false, EpiArgs *e = nullptr) {
    const MainPick pk = pick_main(A, M, N, K);
    if (pk.direct) {
        switch (pk.t->id) {
        case 1:
            return launch_gemm_mfma2<Mfma2Tile<double, 2, 128, 128, 2, 2, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s,
                                                                             acc, e);
        case 2:
            return launch_gemm_mfma2<Mfma2Tile<double, 2, 128, 96, 2, 2, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc,
                                                                            e);
        default:
            return launch_gemm_mfma2<Mfma2Tile<double, 2, 96, 96, 2, 2, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc,
                                                                           e);
        }
    }
    switch (pk.t->id) {
    case 0: return launch_gemm_tile<MfmaTile<double, 256, 128, 16, 4, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc, e);
    case 1: return launch_gemm_tile<MfmaTile<double, 128, 128, 16, 2, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc, e);
    case 2:
        return launch_gemm_tile<MfmaTile<double, 128, 96, 16, 2, 2, 8, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc,
                                                                          e);
    default:
        return launch_gemm_tile<MfmaTile<double, 96, 96, 16, 2, 2, 8, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc, e);
    }
}

static int gemm_main(const float *A, int64_t lda, const float *Bt, int64_t ldb, float *C, int64_t ldc, int64_t M,
                     int64_t N, int64_t K, hipStream_t s, bool acc = false, EpiArgs *e = nullptr) {
    const MainPick pk = pick_main(A, M, N, K);
    if (pk.direct) {
        switch (pk.t->id) {
        case 0: return launch_gemm_mfma2<Mfma2Tile<float, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc, e);
        default:
            return launch_gemm_mfma2<Mfma2Tile<float, 2, 128, 128, 2, 2, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc,
                                                                            e);
        }
    }
    switch (pk.t->id) {
    case 0: return launch_gemm_tile<MfmaTile<float, 256, 128, 32, 4, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc, e);
    default: return launch_gemm_tile<MfmaTile<float, 128, 128, 32, 2, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K, s, acc, e);
    }
}

// C_f = (acc ? C_f : 0) + A_f[:, k0:k0+K) B_f[k0:k0+K, :)  (the whole product: k0 = 0, K = k).
template <typename E>
static int protected_product(const abft_problem *p, const Geom &g, const E *A, const E *Bt, E *C, bool plain,
                             hipStream_t s, int64_t k0 = 0, int64_t K = -1, bool acc = false,
                             EpiArgs *e = nullptr) {
    if (K < 0) K = g.k;
    const bool thin_r = !plain && g.S * g.br <= kSliverMaxB;
    const bool thin_c = !plain && g.S * g.bc <= kSliverMaxB;
    int64_t Mm = (plain || thin_r) ? g.m : g.M;
    int64_t Nm = (plain || thin_c) ? g.n : g.N;
    const E *Ak = A + k0, *Bk = Bt + k0;
    int st = gemm_main(Ak, p->lda, Bk, p->ldb, C, p->ldc, Mm, Nm, K, s, acc, e);
    if (st) return st;
    ABFT_LAUNCHED();
    // carried row block over all N columns (corner included), then the carried
    // column block over the rows the main product covered
    if (thin_r && (st = launch_sliver_rows<E, E, E>(g, Ak + g.m * p->lda, p->lda, Bk, p->ldb, C, p->ldc, K, acc, s)))
        return st;
    if (thin_c &&
        (st = launch_sliver_cols<E, E, E>(g, Mm, Ak, p->lda, Bk + g.n * p->ldb, p->ldb, C, p->ldc, K, acc, s)))
        return st;
    return ABFT_OK;
}

// bfloat16 / FP8 candidates.  When k is a multiple of the 128-byte slab the
// direct-to-LDS kernel runs (measured at 16384^3: bfloat16 53%, FP8 through
// the 32x32x64 instruction 49%); otherwise the padded-LDS kernel, on a 256 x 256
// or 128 x 128 tile (bfloat16 41% / 30% at 16384^3).
static const TileChoice kLowpTiles[] = {
    {0, 256, 256, 1, 0.411}, {1, 128, 128, 2, 0.303},
};
static const TileChoice kLowpDirectTile = {0, 256, 256, 1, 0.49};
static MainPick pick_main_lowp(int64_t elem_size, int64_t M, int64_t N, int64_t K) {
    if (K % (128 / elem_size) == 0 && M * N >= (int64_t)256 * 256 * 256) return {true, &kLowpDirectTile};
    return {false, &kLowpTiles[choose_tile(kLowpTiles, 2, M, N)]};
}
template <class Ops, class Ops2>
static int gemm_main_lowp(const typename Ops::E *A, int64_t lda, const typename Ops::E *Bt, int64_t ldb, float *C,
                          int64_t ldc, int64_t M, int64_t N, int64_t K, const int *scale_exp, hipStream_t s,
                          EpiArgs *e = nullptr) {
    const MainPick pk = pick_main_lowp((int64_t)sizeof(typename Ops::E), M, N, K);
    if (pk.direct) return launch_gemm_lowp2<Ops2, 4>(A, lda, Bt, ldb, C, ldc, M, N, K, scale_exp, s, e);
    switch (pk.t->id) {
    case 0:
        return launch_gemm_lowp_tile<LowpTile<Ops, 256, 256, 128 / sizeof(typename Ops::E), 4, 2>>(
            A, lda, Bt, ldb, C, ldc, M, N, K, scale_exp, s, e);
    default:
        return launch_gemm_lowp_tile<LowpTile<Ops, 128, 128, 64, 2, 2, 8, 2>>(A, lda, Bt, ldb, C, ldc, M, N, K,
                                                                              scale_exp, s, e);
    }
}

// Low-precision operands: the data part on the matrix cores, every carried
// block from the binary32 checksum rows in the workspace (Acs: br x k,
// Bcs: bc x k) with binary64 accumulation; FP8 results are scaled back by
// 2^-(eA + eB) on the device.
template <class Ops, class Ops2>
static int protected_product_lowp(const abft_problem *p, const Geom &g, const typename Ops::E *A,
                                  const typename Ops::E *Bt, float *C, const float *Acs, const float *Bcs,
                                  const int *scale_exp, bool plain, hipStream_t s, EpiArgs *e = nullptr) {
    typedef typename Ops::E E;
    int st = gemm_main_lowp<Ops, Ops2>(A, p->lda, Bt, p->ldb, C, p->ldc, g.m, g.n, g.k, scale_exp, s, e);
    if (st) return st;
    ABFT_LAUNCHED();
    if (plain) return ABFT_OK;
    float *Crow = C + g.m * p->ldc;
    // C_f[m + r, j], j < n
    if ((st = sliver<E, float, float>(Bt, p->ldb, g.n, Acs, g.k, g.br, g.k, Crow, 1, p->ldc, scale_exp, s))) return st;
    // corner C_f[m + r, n + c]
    if ((st = sliver<float, float, float>(Bcs, g.k, g.bc, Acs, g.k, g.br, g.k, Crow + g.n, 1, p->ldc, scale_exp, s)))
        return st;
    // C_f[i, n + c], i < m
    return sliver<E, float, float>(A, p->lda, g.m, Bcs, g.k, g.bc, g.k, C + g.n, p->ldc, 1, scale_exp, s);
}

int launch_skinny_f64(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K, hipStream_t s) {
    int st = sliver<double, double, double>(A, lda, M, Bt, ldb, N, K, C, ldc, 1, nullptr, s);
    if (st) return st;
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_gemm_f64(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc, int64_t M,
                    int64_t N, int64_t K, hipStream_t s) {
    int st = gemm_main(A, lda, Bt, ldb, C, ldc, M, N, K, s);
    if (st) return st;
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_skinny_f32(const float *A, int64_t lda, const float *Bt, int64_t ldb, float *C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K, hipStream_t s) {
    int st = sliver<float, float, float>(A, lda, M, Bt, ldb, N, K, C, ldc, 1, nullptr, s);
    if (st) return st;
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_gemm_f32(const float *A, int64_t lda, const float *Bt, int64_t ldb, float *C, int64_t ldc, int64_t M,
                    int64_t N, int64_t K, hipStream_t s) {
    int st = gemm_main(A, lda, Bt, ldb, C, ldc, M, N, K, s);
    if (st) return st;
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_gemm_panel(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, int64_t k0, int64_t k1,
                      uint32_t flags, hipStream_t s) {
    Geom g = geom_of(p);
    const bool plain = flags & ABFT_PLAIN, acc = flags & ABFT_ACCUMULATE;
    switch (p->dtype) {
    case ABFT_F64:
        return protected_product<double>(p, g, (const double *)A_f, (const double *)B_f, (double *)C_f, plain, s, k0,
                                         k1 - k0, acc);
    case ABFT_F32:
        return protected_product<float>(p, g, (const float *)A_f, (const float *)B_f, (float *)C_f, plain, s, k0,
                                        k1 - k0, acc);
    default:
        return ABFT_E_UNSUPPORTED;
    }
}

// The kernels and tiles launch_gemm runs for p and flags, as text (a
// diagnostic: tests check that every tile is exercised, benchmarks report it).
int describe_gemm(const abft_problem *p, uint32_t flags, char *buf, size_t len) {
    const Geom g = geom_of(p);
    const bool plain = flags & ABFT_PLAIN;
    const bool lowp = p->dtype == ABFT_BF16 || p->dtype == ABFT_FP8_E4M3;
    static const char *const kDt[] = {"f64", "f32", "bf16", "fp8"};
    bool thin_r, thin_c;
    int64_t Mm, Nm;
    MainPick pk;
    const char *kname;
    if (lowp) {
        thin_r = thin_c = !plain;             // every carried block from the workspace checksum rows
        Mm = g.m;
        Nm = g.n;
        pk = pick_main_lowp(p->dtype == ABFT_BF16 ? 2 : 1, Mm, Nm, g.k);
        kname = pk.direct ? "k_gemm_lowp2" : "k_gemm_lowp";
    } else {
        thin_r = !plain && g.S * g.br <= kSliverMaxB;
        thin_c = !plain && g.S * g.bc <= kSliverMaxB;
        Mm = (plain || thin_r) ? g.m : g.M;
        Nm = (plain || thin_c) ? g.n : g.N;
        pk = p->dtype == ABFT_F64 ? pick_main((const double *)nullptr, Mm, Nm, g.k)
                                  : pick_main((const float *)nullptr, Mm, Nm, g.k);
        kname = pk.direct ? "k_gemm_mfma2" : "k_gemm_mfma";
    }
    // the carried blocks' kernels: rows over the N columns (lowp: n), columns over the data rows
    const char *sr = sliver_multirow(g.br, lowp ? g.n : g.N) ? " + k_sliver1 carried rows" : " + k_sliver carried rows";
    const char *sc = sliver_multirow(g.bc, Mm) ? " + k_sliver1 carried columns" : " + k_sliver carried columns";
    const int n = snprintf(buf, len, "%s %s %dx%d on %lldx%lld k=%lld%s%s%s", kname, kDt[p->dtype], pk.t->bm,
                           pk.t->bn, (long long)Mm, (long long)Nm, (long long)g.k, thin_r ? sr : "",
                           (lowp && !plain) ? " + k_sliver corner" : "", thin_c ? sc : "");
    return (n < 0 || (size_t)n >= len) ? ABFT_E_ARG : ABFT_OK;
}

// Owner tag of the fused partial sums (the stateless stand-in for "the last
// product on this workspace"): a 64-bit mix of the problem, its tile grid and
// C_f, never 0 (0 marks "no valid partials").
static uint64_t mix64(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    return h ^ (h >> 29);
}

uint64_t fused_key(const abft_problem *p, const void *C_f, int64_t *tiles_m, int64_t *tiles_n) {
    const Geom g = geom_of(p);
    const bool lowp = p->dtype == ABFT_BF16 || p->dtype == ABFT_FP8_E4M3;
    // b = 1: the carried row and column are slivers, the main product covers m x n
    const MainPick pk = lowp ? pick_main_lowp(p->dtype == ABFT_BF16 ? 2 : 1, g.m, g.n, g.k)
                             : (p->dtype == ABFT_F64 ? pick_main((const double *)nullptr, g.m, g.n, g.k)
                                                     : pick_main((const float *)nullptr, g.m, g.n, g.k));
    *tiles_m = (g.m + pk.t->bm - 1) / pk.t->bm;
    *tiles_n = (g.n + pk.t->bn - 1) / pk.t->bn;
    uint64_t h = 0x6A09E667F3BCC908ull;
    for (uint64_t v : {(uint64_t)p->dtype, (uint64_t)g.m, (uint64_t)g.n, (uint64_t)g.k, (uint64_t)g.br,
                       (uint64_t)g.bc, (uint64_t)p->ldc, (uint64_t)(uintptr_t)C_f, (uint64_t)*tiles_m,
                       (uint64_t)*tiles_n})
        h = mix64(h, v);
    return h ? h : 1;
}

__global__ void k_store_tag(uint64_t *dst, uint64_t v) { *dst = v; }

static int product_with_extras(const abft_problem *p, const Geom &g, const void *A_f, const void *B_f, void *C_f,
                               bool plain, void *ws, const float *Acs, const float *Bcs, const int *scale,
                               EpiArgs *e, hipStream_t s) {
    switch (p->dtype) {
    case ABFT_F64:
        return protected_product<double>(p, g, (const double *)A_f, (const double *)B_f, (double *)C_f, plain, s, 0,
                                         -1, false, e);
    case ABFT_F32:
        return protected_product<float>(p, g, (const float *)A_f, (const float *)B_f, (float *)C_f, plain, s, 0, -1,
                                        false, e);
    case ABFT_BF16:
        return protected_product_lowp<Bf16Ops, Bf16Ops>(p, g, (const uint16_t *)A_f, (const uint16_t *)B_f,
                                                        (float *)C_f, Acs, Bcs, nullptr, plain, s, e);
    case ABFT_FP8_E4M3:
        return protected_product_lowp<Fp8Ops, Fp8x64Ops>(p, g, (const uint8_t *)A_f, (const uint8_t *)B_f,
                                                         (float *)C_f, Acs, Bcs, scale, plain, s, e);
    default:
        return ABFT_E_UNSUPPORTED;
    }
}

int launch_gemm(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, uint32_t flags, void *ws,
                const abft_fault *fault, hipStream_t s) {
    Geom g = geom_of(p);
    const bool plain = flags & ABFT_PLAIN, fused = flags & ABFT_FUSED;
    // epilogue extras: the test-only accumulator flip and the fused partial sums
    EpiArgs e = epi_none();
    if (fault) {
        e.fi = fault->i; e.fj = fault->j; e.fbit = fault->bit;
    }
    WsLayout L = ws_layout(p);
    if (fused) {
        e.pc = (double *)((char *)ws + L.fused_c);
        e.pr = (double *)((char *)ws + L.fused_r);
        e.ldpc = g.n;
        e.ldpr = g.m;
    }
    const char *wsc = (const char *)ws;
    const bool lowp = p->dtype == ABFT_BF16 || p->dtype == ABFT_FP8_E4M3;
    const float *Acs = (lowp && ws) ? (const float *)(wsc + L.acs) : nullptr;
    const float *Bcs = (lowp && ws) ? (const float *)(wsc + L.bcs) : nullptr;
    const int *scale = (p->dtype == ABFT_FP8_E4M3 && ws) ? (const int *)(wsc + L.scale) : nullptr;
    int st = product_with_extras(p, g, A_f, B_f, C_f, plain, ws, Acs, Bcs, scale, (fault || fused) ? &e : nullptr, s);
    if (st) return st;
    if (ws) {
        // record in ws who owns the fused partials now: this product (fused) or nobody
        uint64_t key = 0;
        if (fused) {
            int64_t tm = 0, tn = 0;
            key = fused_key(p, C_f, &tm, &tn);
            if (tm != e.tiles_m || tn != e.tiles_n) key = 0;   // a grid the fused verification would not read
        }
        k_store_tag<<<1, 1, 0, s>>>((uint64_t *)((char *)ws + L.fused_tag), key);
        ABFT_LAUNCHED();
    }
    return ABFT_OK;
}

}  // namespace abft
