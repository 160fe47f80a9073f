// libabft C ABI: argument checks, workspace layout, host-side classification
// and dispatch to the gfx950 kernels.  See include/abft.h for the contract.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace abft {

static thread_local int g_last_hip_error = 0;
void set_hip_error(hipError_t e) { g_last_hip_error = (int)e; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t group_partitions(int64_t G, int64_t b, int64_t cols) {
    // Enough independent sums to fill 256 CUs with ~2K threads each; each
    // partition sums a contiguous run of groups in ascending order.
    const int64_t target = int64_t(1) << 19;
    int64_t rel = b * cols;
    int64_t P = (target + rel - 1) / rel;
    if (P > G) P = G;
    if (P < 1) P = 1;
    return P;
}

bool rows_fused(const abft_problem *p) {
    const int64_t vpe = 16 / (int64_t)dtype_size(p->dtype);
    return (p->tau_mode == ABFT_TAU_DET || p->tau_mode == ABFT_TAU_STAT) && (p->k / vpe) % 64 == 0;
}

WsLayout ws_layout(const abft_problem *p) {
    Geom g = geom_of(p);
    WsLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.na = take(sizeof(double) * g.M);
    L.na_abs = take(sizeof(double) * g.br);
    L.nb = take(sizeof(double) * g.N);
    L.nb_abs = take(sizeof(double) * g.bc);
    L.qr = take(sizeof(double) * g.M);
    L.qc = take(sizeof(double) * g.N);
    L.nv = take(sizeof(double) * g.br);
    L.nw = take(sizeof(double) * g.bc);
    L.grpA = take(sizeof(double) * g.br * g.k);
    L.grpB = take(sizeof(double) * g.bc * g.k);
    L.acs = take(cs_in_ws(p->dtype) ? sizeof(float) * g.br * g.k : 8);
    L.bcs = take(cs_in_ws(p->dtype) ? sizeof(float) * g.bc * g.k : 8);
    L.scale = take(16);
    // partial sums: encode A (2 stats), encode B (2 stats), verify columns (1);
    // encode threads own 16 bytes of a row each
    int64_t vpe = 16 / (int64_t)dtype_size(p->dtype);
    int64_t pa = group_partitions(g.Gr, g.br, g.k / vpe);
    int64_t pb = group_partitions(g.Gc, g.bc, g.k / vpe);
    int64_t pc = std::max(group_partitions(g.Gr, g.br, g.N), group_partitions(g.Gr, g.br, (g.N + 1) / 2));
    pc = std::max(pc, group_partitions(g.Gr, g.br, (g.N + 3) / 4));
    size_t need = 0;
    if (pa > 1) need = std::max(need, (size_t)(pa * g.br * g.k * 2));
    if (pb > 1) need = std::max(need, (size_t)(pb * g.bc * g.k * 2));
    if (pc > 1) need = std::max(need, (size_t)(pc * g.br * g.N));
    L.partial_bytes = sizeof(double) * need;
    L.partial = take(L.partial_bytes > 0 ? L.partial_bytes : 8);
    // fused row statistics: the larger operand's data rows plus its checksum and group rows, k / 64 slots each
    L.rowpart = take(rows_fused(p) ? sizeof(double) * (std::max(g.m, g.n) + 2 * std::max(g.br, g.bc)) * (g.k / 64) : 8);
    // one-pass re-read verification (b = 1): column sums per kVerifyPartRows-row tile, row sums per 128-column
    // (binary64 C) or 256-column (binary32 C) tile
    const bool b1 = g.br == 1 && g.bc == 1;
    const int64_t vw = 64 * (16 / (p->dtype == ABFT_F64 ? 8 : 4));
    L.vpart_c = take(b1 ? sizeof(double) * ((g.m + kVerifyPartRows - 1) / kVerifyPartRows) * g.n : 8);
    L.vpart_r = take(b1 ? sizeof(double) * ((g.n + vw - 1) / vw) * g.m : 8);
    L.report = take(sizeof(abft_report));
    // fused partials (b = 1 only): column sums per tile row, row sums per tile column
    const bool fused = g.br == 1 && g.bc == 1;
    const int64_t tm = (g.m + kMinTileEdge - 1) / kMinTileEdge, tn = (g.n + kMinTileEdge - 1) / kMinTileEdge;
    L.fused_c = take(fused ? sizeof(double) * tm * g.n : 8);
    L.fused_r = take(fused ? sizeof(double) * tn * g.m : 8);
    L.fused_tag = take(sizeof(uint64_t));
    L.chain_a = take(sizeof(double) * g.br);
    L.chain_w = take(sizeof(double) * g.N);
    L.chain_cs = take(p->dtype == ABFT_F64 || p->dtype == ABFT_F32 ? dtype_size(p->dtype) * g.br * g.k : 8);
    L.total = off;
    return L;
}

static double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

TauCoef tau_coef(const abft_problem *p) {
    Geom g = geom_of(p);
    TauCoef t;
    t.mode = p->tau_mode;
    t.cst = 0.0;
    t.lambda = p->lambda > 0 ? p->lambda : 10.0;
    const double u64 = std::ldexp(1.0, -53);
    const double u32 = std::ldexp(1.0, -24);
    if (p->tau_mode == ABFT_TAU_DET) {
        double kappa = p->kappa >= 1.0 ? p->kappa : 1.0 + std::ldexp(1.0, -20);
        double u_acc = p->dtype == ABFT_F64 ? u64 : u32;
        double u_st = p->dtype == ABFT_F64 ? 0.0 : u32;
        t.cc = kappa * (2 * gamma_n((double)g.k, u_acc) + 2 * gamma_n((double)(g.Gr + g.S), u64) + u_st);
        t.cr = kappa * (2 * gamma_n((double)g.k, u_acc) + 2 * gamma_n((double)(g.Gc + g.S), u64) + u_st);
    } else if (p->tau_mode == ABFT_TAU_STAT) {
        // sigma^2 = (u^2/3)(T/2 + s) Q.  T = accumulation steps: k for binary32
        // (one rounding per product bounds every matrix-core order) and k/4 for
        // bfloat16 / FP8 (measured: the bfloat16 matrix core rounds no more
        // often than once per 4 products).  s = 2 covers the binary32 storage
        // of the checksum row and of the carried total.  FP8 adds the narrow
        // product-sum window of its matrix core, a per-product error of u_w =
        // 2^-15 (measured rms 2^-16.3): s += (u_w / u)^2.
        double u = p->dtype == ABFT_F64 ? u64 : u32;
        double T = (p->dtype == ABFT_BF16 || p->dtype == ABFT_FP8_E4M3) ? (double)g.k / 4.0 : (double)g.k;
        double sst = 2.0;
        if (p->dtype == ABFT_FP8_E4M3) sst += std::ldexp(1.0, 2 * (24 - 15));
        t.cc = t.cr = t.lambda * t.lambda * (u * u / 3.0) * (T / 2.0 + sst);
        // The stored total of a relation (the carried checksum entry) is rounded
        // once to the element type: error up to u |tot|.  For data of one sign
        // the total is far larger than the root-sum-square of its products that
        // Q measures, so its rounding enters with its own magnitude, read from
        // C_f at verification.
        t.cst = t.lambda * t.lambda * (u * u / 3.0);
    } else {
        t.cc = t.cr = 0.0;
    }
    return t;
}

// ------------------------------------------------------------------ checks
static int check_problem(const abft_problem *p) {
    if (!p) return ABFT_E_ARG;
    if (p->dtype < ABFT_F64 || p->dtype > ABFT_FP8_E4M3) return ABFT_E_ARG;
    if (p->m < 1 || p->n < 1 || p->k < 1 || p->br < 1 || p->bc < 1) return ABFT_E_ARG;
    if (p->br > p->m || p->bc > p->n) return ABFT_E_ARG;
    if (p->m % p->br || p->n % p->bc) return ABFT_E_ARG;
    if (p->tau_mode < ABFT_TAU_DET || p->tau_mode > ABFT_TAU_EXACT) return ABFT_E_ARG;
    return ABFT_OK;
}

static bool aligned16(const void *q) { return ((uintptr_t)q & 15u) == 0; }

// A workspace must be present and at least the problem's workspace size.
static int check_ws(const abft_problem *p, const void *ws, size_t ws_bytes) {
    if (!ws || ws_bytes < ws_layout(p).total) return ABFT_E_WORKSPACE;
    return ABFT_OK;
}

static int check_operands(const abft_problem *p, const void *A_f, const void *B_f) {
    size_t es = dtype_size(p->dtype);
    if (!A_f || !B_f) return ABFT_E_ARG;
    if (p->lda < p->k || p->ldb < p->k) return ABFT_E_ARG;
    if ((p->lda * es) % 16 || (p->ldb * es) % 16 || (p->k * es) % 16) return ABFT_E_ARG;
    if (!aligned16(A_f) || !aligned16(B_f)) return ABFT_E_ARG;
    return ABFT_OK;
}

static int check_c(const abft_problem *p, const void *C_f, bool plain) {
    Geom g = geom_of(p);
    if (!C_f) return ABFT_E_ARG;
    if (p->ldc < (plain ? g.n : g.N)) return ABFT_E_ARG;
    if (((uintptr_t)C_f % c_size(p->dtype)) != 0) return ABFT_E_ARG;
    return ABFT_OK;
}

static int check_rect(const Geom &g, const abft_rect &e) {
    if (e.h < 1 || e.w < 1 || e.i0 < 0 || e.j0 < 0) return ABFT_E_ARG;
    if (e.i0 + e.h > g.M || e.j0 + e.w > g.N) return ABFT_E_ARG;
    return ABFT_OK;
}

// ------------------------------------------------------------------ classification (host)
static bool col_erased_h(const abft_rect *kn, int nk, int64_t r, int64_t j, int64_t br) {
    for (int q = 0; q < nk; ++q) {
        const abft_rect &e = kn[q];
        if (j < e.j0 || j >= e.j0 + e.w) continue;
        if (e.h >= br) return true;
        int64_t off = ((r - e.i0) % br + br) % br;
        if (off < e.h) return true;
    }
    return false;
}
static bool row_erased_h(const abft_rect *kn, int nk, int64_t i, int64_t c, int64_t bc) {
    for (int q = 0; q < nk; ++q) {
        const abft_rect &e = kn[q];
        if (i < e.i0 || i >= e.i0 + e.h) continue;
        if (e.w >= bc) return true;
        int64_t off = ((c - e.j0) % bc + bc) % bc;
        if (off < e.w) return true;
    }
    return false;
}

static int classify(const abft_problem *p, const abft_report *rep, const abft_rect *kn, int nk, abft_location *out) {
    Geom g = geom_of(p);
    out->cls = ABFT_CLS_MULTI;
    out->dir = ABFT_DIR_COL;
    out->i = out->j = -1;
    int64_t nc = rep->n_flag_c, nr = rep->n_flag_r;
    if (nc == 0 && nr == 0) { out->cls = ABFT_CLS_CLEAN; return ABFT_OK; }
    // A carried entry is "stored total" of its relation: its residual sign is
    // negative; a data entry is a summand.  Split parts all count as totals.
    auto is_data_row = [&](int64_t i) { return i < g.m; };
    auto is_data_col = [&](int64_t j) { return j < g.n; };
    auto kind = [&](int64_t i, int64_t j) {
        return (is_data_row(i) && is_data_col(j)) ? ABFT_CLS_DATA : ABFT_CLS_CHECKSUM;
    };
    if (nc == 1 && nr == 1) {
        const abft_flag &fc = rep->flag_c[0], &fr = rep->flag_r[0];
        int64_t r = fc.a, j = fc.b, i = fr.a, c = fr.b;
        int64_t ri = is_data_row(i) ? i % g.br : (i - g.m) % g.br;
        int64_t cj = is_data_col(j) ? j % g.bc : (j - g.n) % g.bc;
        if (ri != r || cj != c) return ABFT_OK;  // MULTI
        if (std::isfinite(fc.d) && std::isfinite(fr.d)) {
            // Both residual sums contain the bad value, so each is also off by
            // up to gamma_{G+S+1} |delta| (large after an exponent-bit flip).
            const double u64 = std::ldexp(1.0, -53);
            double big = std::max(std::fabs(fc.d), std::fabs(fr.d));
            double tol = fc.tau + fr.tau + (gamma_n((double)(g.Gr + g.S + 1), u64) + gamma_n((double)(g.Gc + g.S + 1), u64)) * big;
            double sc = is_data_row(i) ? 1.0 : -1.0, sr = is_data_col(j) ? 1.0 : -1.0;
            if (!(std::fabs(sc * fc.d - sr * fr.d) <= tol)) return ABFT_OK;  // MULTI
        }
        out->cls = kind(i, j); out->i = i; out->j = j; out->dir = ABFT_DIR_COL;
        return ABFT_OK;
    }
    if (nk > 0 && nc == 0 && nr == 1) {
        const abft_flag &fr = rep->flag_r[0];
        int64_t i = fr.a, c = fr.b, found = -1, cnt = 0;
        int64_t r = is_data_row(i) ? i % g.br : (i - g.m) % g.br;
        for (int64_t j = c; j < g.N; j += g.bc)
            if (col_erased_h(kn, nk, r, j, g.br)) { found = j; ++cnt; }
        if (cnt != 1) return ABFT_OK;
        out->cls = kind(i, found); out->i = i; out->j = found; out->dir = ABFT_DIR_ROW;
        return ABFT_OK;
    }
    if (nk > 0 && nc == 1 && nr == 0) {
        const abft_flag &fc = rep->flag_c[0];
        int64_t r = fc.a, j = fc.b, found = -1, cnt = 0;
        int64_t c = is_data_col(j) ? j % g.bc : (j - g.n) % g.bc;
        for (int64_t i = r; i < g.M; i += g.br)
            if (row_erased_h(kn, nk, i, c, g.bc)) { found = i; ++cnt; }
        if (cnt != 1) return ABFT_OK;
        out->cls = kind(found, j); out->i = found; out->j = j; out->dir = ABFT_DIR_COL;
        return ABFT_OK;
    }
    return ABFT_OK;  // MULTI
}

// ------------------------------------------------------------------ static scratch (abft_verify_noalloc)
// Device scratch for callers that cannot allocate: every GPU the library runs
// on holds its own copy of this array until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address): the device address is taken once per
// device with hipGetSymbolAddress, with that device current, and cached here.
// The cache only ever holds the one address of each device, so concurrent
// first calls store the same value.
static __device__ __align__(256) uint8_t scratch[ABFT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::atomic<char *> g_scratch_ptr[kMaxDevices];

static int scratch_ptr(char **out) {
    int dev = -1;
    ABFT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return ABFT_E_ARG;
    char *ptr = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!ptr) {
        void *addr = nullptr;
        ABFT_HIP(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
        ptr = (char *)addr;
        g_scratch_ptr[dev].store(ptr, std::memory_order_release);
    }
    *out = ptr;
    return ABFT_OK;
}

static int to_erasures(const Geom &g, const abft_rect *known, int n_known, Erasures *er) {
    if (n_known < 0 || n_known > 4 || (n_known > 0 && !known)) return ABFT_E_ARG;
    er->n = n_known;
    for (int q = 0; q < n_known; ++q) {
        if (check_rect(g, known[q])) return ABFT_E_ARG;
        er->i0[q] = known[q].i0; er->j0[q] = known[q].j0; er->h[q] = known[q].h; er->w[q] = known[q].w;
    }
    return ABFT_OK;
}

}  // namespace abft

using namespace abft;

extern "C" {

size_t abft_workspace_size(const abft_problem *p) {
    if (check_problem(p) != ABFT_OK) return 0;
    return ws_layout(p).total;
}

int abft_encode(const abft_problem *p, void *A_f, void *B_f, void *ws, size_t ws_bytes, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_operands(p, A_f, B_f))) return st;
    if ((st = check_ws(p, ws, ws_bytes))) return st;
    return launch_encode(p, A_f, B_f, (char *)ws, (hipStream_t)stream);
}

int abft_encode_chained(const abft_problem *p, const void *A_f, void *B_f, void *ws, size_t ws_bytes,
                        const abft_problem *prev, const void *ws_prev, size_t ws_prev_bytes, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_problem(prev))) return st;
    if ((p->dtype != ABFT_F64 && p->dtype != ABFT_F32) || prev->dtype != p->dtype) return ABFT_E_UNSUPPORTED;
    if (p->tau_mode != prev->tau_mode) return ABFT_E_ARG;
    if (p->tau_mode != ABFT_TAU_DET && p->tau_mode != ABFT_TAU_EXACT) return ABFT_E_UNSUPPORTED;
    if (p->m != prev->m || p->br != prev->br || p->k != prev->n || p->lda != prev->ldc) return ABFT_E_ARG;
    if ((st = check_operands(p, A_f, B_f))) return st;
    if ((st = check_ws(p, ws, ws_bytes)) || (st = check_ws(prev, ws_prev, ws_prev_bytes))) return st;
    const double cc_prev = p->tau_mode == ABFT_TAU_DET ? tau_coef(prev).cc : 0.0;
    return launch_encode_chained(p, A_f, B_f, (char *)ws, prev, (const char *)ws_prev, cc_prev, (hipStream_t)stream);
}

int abft_quantize(const abft_problem *p, int which, const float *X, int64_t ldx, void *dst, void *ws, size_t ws_bytes,
                  void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if (!cs_in_ws(p->dtype)) return ABFT_E_ARG;
    if (which != 0 && which != 1) return ABFT_E_ARG;
    if (!X || !dst || ((uintptr_t)X & 15u) || ((uintptr_t)dst & 15u)) return ABFT_E_ARG;
    if (ldx < p->k || (ldx * 4) % 16) return ABFT_E_ARG;
    int64_t ldd = which == 0 ? p->lda : p->ldb;
    size_t es = dtype_size(p->dtype);
    if (ldd < p->k || (ldd * es) % 16 || (p->k * es) % 16) return ABFT_E_ARG;
    if ((st = check_ws(p, ws, ws_bytes))) return st;
    return launch_quantize(p, which, X, ldx, dst, (char *)ws, (hipStream_t)stream);
}

int abft_quantize_encode(const abft_problem *p, const float *A32, int64_t lda32, const float *B32, int64_t ldb32,
                         void *A_f, void *B_f, void *ws, size_t ws_bytes, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if (!cs_in_ws(p->dtype)) return ABFT_E_UNSUPPORTED;
    if (!A32 || !B32 || ((uintptr_t)A32 & 15u) || ((uintptr_t)B32 & 15u)) return ABFT_E_ARG;
    if (lda32 < p->k || ldb32 < p->k || lda32 % 4 || ldb32 % 4) return ABFT_E_ARG;
    if ((st = check_operands(p, A_f, B_f))) return st;
    const size_t es = dtype_size(p->dtype);
    if ((p->k * es) % 16) return ABFT_E_ARG;
    if ((st = check_ws(p, ws, ws_bytes))) return st;
    return launch_quantize_encode(p, A32, lda32, B32, ldb32, A_f, B_f, (char *)ws, (hipStream_t)stream);
}

int abft_gemm_fault(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, void *ws, size_t ws_bytes,
                    uint32_t flags, const abft_fault *fault, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if (flags & ~(ABFT_PLAIN | ABFT_FUSED)) return ABFT_E_ARG;
    if (flags & ABFT_FUSED) {
        if (flags & ABFT_PLAIN) return ABFT_E_ARG;
        if (p->br != 1 || p->bc != 1) return ABFT_E_UNSUPPORTED;
        if (!ws) return ABFT_E_WORKSPACE;
    }
    if (fault) {
        if (fault->i < 0 || fault->i >= p->m || fault->j < 0 || fault->j >= p->n) return ABFT_E_ARG;
        if (fault->bit < 0 || fault->bit >= (p->dtype == ABFT_F64 ? 64 : 32)) return ABFT_E_ARG;
    }
    if ((st = check_operands(p, A_f, B_f))) return st;
    if ((st = check_c(p, C_f, flags & ABFT_PLAIN))) return st;
    if (!ws && (p->dtype == ABFT_FP8_E4M3 || (p->dtype == ABFT_BF16 && !(flags & ABFT_PLAIN)))) return ABFT_E_WORKSPACE;
    if (ws && (st = check_ws(p, ws, ws_bytes))) return st;
    return launch_gemm(p, A_f, B_f, C_f, flags, ws, fault, (hipStream_t)stream);
}

int abft_gemm(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, void *ws, size_t ws_bytes,
              uint32_t flags, void *stream) {
    return abft_gemm_fault(p, A_f, B_f, C_f, ws, ws_bytes, flags, nullptr, stream);
}

int abft_describe_gemm(const abft_problem *p, uint32_t flags, char *buf, size_t len) {
    int st = check_problem(p);
    if (st) return st;
    if (!buf || len == 0) return ABFT_E_ARG;
    buf[0] = 0;
    if (flags & ~(ABFT_PLAIN | ABFT_FUSED)) return ABFT_E_ARG;
    return describe_gemm(p, flags, buf, len);
}

int abft_gemm_panel(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, int64_t k0, int64_t k1,
                    uint32_t flags, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if (flags & ~(ABFT_PLAIN | ABFT_ACCUMULATE)) return ABFT_E_ARG;
    if (p->dtype != ABFT_F64 && p->dtype != ABFT_F32) return ABFT_E_UNSUPPORTED;
    if ((st = check_operands(p, A_f, B_f))) return st;
    if ((st = check_c(p, C_f, flags & ABFT_PLAIN))) return st;
    const int64_t align = 16 / (int64_t)dtype_size(p->dtype);
    if (k0 < 0 || k1 <= k0 || k1 > p->k || k0 % align || k1 % align) return ABFT_E_ARG;
    return launch_gemm_panel(p, A_f, B_f, C_f, k0, k1, flags, (hipStream_t)stream);
}

int abft_verify_fused(const abft_problem *p, const void *C_f, void *ws, size_t ws_bytes, abft_report *host_out,
                      void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    if ((st = check_ws(p, ws, ws_bytes))) return st;
    if (p->br != 1 || p->bc != 1) return ABFT_E_UNSUPPORTED;
    int64_t tm = 0, tn = 0;
    const uint64_t key = fused_key(p, C_f, &tm, &tn);
    if ((st = launch_verify_fused(p, C_f, (char *)ws, tm, tn, key, (hipStream_t)stream))) return st;
    if (host_out) {
        WsLayout L = ws_layout(p);
        ABFT_HIP(hipMemcpyAsync(host_out, (char *)ws + L.report, sizeof(abft_report), hipMemcpyDeviceToHost,
                                (hipStream_t)stream));
    }
    return ABFT_OK;
}

int abft_verify(const abft_problem *p, const void *C_f, const abft_rect *known, int n_known, void *ws,
                size_t ws_bytes, abft_report *host_out, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    if ((st = check_ws(p, ws, ws_bytes))) return st;
    Geom g = geom_of(p);
    Erasures er;
    if ((st = to_erasures(g, known, n_known, &er))) return st;
    if ((st = launch_verify(p, C_f, er, (char *)ws, (hipStream_t)stream))) return st;
    if (host_out) {
        WsLayout L = ws_layout(p);
        ABFT_HIP(hipMemcpyAsync(host_out, (char *)ws + L.report, sizeof(abft_report), hipMemcpyDeviceToHost,
                                (hipStream_t)stream));
    }
    return ABFT_OK;
}

int abft_verify_noalloc(const abft_problem *p, const void *C_f, const abft_rect *known, int n_known,
                        const void *ws, size_t ws_bytes, abft_report *host_out, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    if ((st = check_ws(p, ws, ws_bytes))) return st;
    if (!host_out) return ABFT_E_ARG;
    Geom g = geom_of(p);
    Erasures er;
    if ((st = to_erasures(g, known, n_known, &er))) return st;
    if (verify_scratch_layout(p, C_f, nullptr, nullptr) > ABFT_NOALLOC_SCRATCH_BYTES) return ABFT_E_WORKSPACE;
    char *base = nullptr;
    if ((st = scratch_ptr(&base))) return st;
    VerifyScratch sc;
    verify_scratch_layout(p, C_f, base, &sc);
    if ((st = launch_verify_scratch(p, C_f, er, (const char *)ws, sc, (hipStream_t)stream))) return st;
    ABFT_HIP(hipMemcpyAsync(host_out, sc.rep, sizeof(abft_report), hipMemcpyDeviceToHost, (hipStream_t)stream));
    return ABFT_OK;
}

int abft_classify(const abft_problem *p, const abft_report *report, const abft_rect *known, int n_known,
                  abft_location *out) {
    int st = check_problem(p);
    if (st) return st;
    if (!report || !out) return ABFT_E_ARG;
    Geom g = geom_of(p);
    Erasures er;
    if ((st = to_erasures(g, known, n_known, &er))) return st;
    // The device writes flags in arrival order; classify a sorted copy so the
    // outcome does not depend on it.
    abft_report rep = *report;
    int64_t kc = std::min<int64_t>(rep.n_flag_c, ABFT_MAX_FLAGS), kr = std::min<int64_t>(rep.n_flag_r, ABFT_MAX_FLAGS);
    auto less = [](const abft_flag &x, const abft_flag &y) { return x.a < y.a || (x.a == y.a && x.b < y.b); };
    std::sort(rep.flag_c, rep.flag_c + kc, less);
    std::sort(rep.flag_r, rep.flag_r + kr, less);
    return classify(p, &rep, known, n_known, out);
}

int abft_correct(const abft_problem *p, void *C_f, const abft_location *loc, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    if (!loc) return ABFT_E_ARG;
    if (loc->cls == ABFT_CLS_CLEAN) return ABFT_OK;
    if (loc->cls == ABFT_CLS_MULTI) return ABFT_E_UNCORRECTABLE;
    if (loc->cls != ABFT_CLS_DATA && loc->cls != ABFT_CLS_CHECKSUM) return ABFT_E_ARG;
    Geom g = geom_of(p);
    if (loc->i < 0 || loc->i >= g.M || loc->j < 0 || loc->j >= g.N) return ABFT_E_ARG;
    if (loc->dir != ABFT_DIR_COL && loc->dir != ABFT_DIR_ROW) return ABFT_E_ARG;
    return launch_correct(p, C_f, loc->i, loc->j, loc->dir, (hipStream_t)stream);
}

int abft_recover_block(const abft_problem *p, void *C_f, abft_rect e, int use_rows, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    Geom g = geom_of(p);
    if ((st = check_rect(g, e))) return st;
    if (!use_rows && e.h > g.br) return ABFT_E_UNRECOVERABLE;
    if (use_rows && e.w > g.bc) return ABFT_E_UNRECOVERABLE;
    return launch_recover(p, C_f, e, use_rows, (hipStream_t)stream);
}

int abft_inject_flip(const abft_problem *p, void *C_f, int64_t i, int64_t j, int bit, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    Geom g = geom_of(p);
    if (i < 0 || i >= g.M || j < 0 || j >= g.N) return ABFT_E_ARG;
    if (bit < 0 || bit >= (int)(8 * c_size(p->dtype))) return ABFT_E_ARG;
    return launch_inject_flip(p, C_f, i, j, bit, (hipStream_t)stream);
}

int abft_inject_erase(const abft_problem *p, void *C_f, abft_rect e, int nan_fill, void *stream) {
    int st = check_problem(p);
    if (st) return st;
    if ((st = check_c(p, C_f, false))) return st;
    Geom g = geom_of(p);
    if ((st = check_rect(g, e))) return st;
    return launch_inject_erase(p, C_f, e, nan_fill, (hipStream_t)stream);
}

int abft_fill_uniform(int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed,
                      int32_t stream_id, void *dst, void *stream) {
    if (dtype != ABFT_F64 && dtype != ABFT_F32) return ABFT_E_ARG;
    if (rows < 1 || cols < 1 || !dst) return ABFT_E_ARG;
    if (ld < (transpose ? rows : cols)) return ABFT_E_ARG;
    return launch_fill_uniform(dtype, rows, cols, ld, transpose, seed, stream_id, dst, (hipStream_t)stream);
}

int abft_fill_normal(int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed, double frac, float scale,
                     float *dst, void *stream) {
    if (rows < 1 || cols < 1 || !dst || ((uintptr_t)dst & 3u)) return ABFT_E_ARG;
    if (ld < (transpose ? rows : cols)) return ABFT_E_ARG;
    if (!(frac >= 0.0 && frac <= 1.0) || !std::isfinite(scale)) return ABFT_E_ARG;
    return launch_fill_normal(rows, cols, ld, transpose, seed, frac, scale, dst, (hipStream_t)stream);
}

int abft_last_hip_error(void) { return g_last_hip_error; }

const char *abft_status_string(int s) {
    switch (s) {
    case ABFT_OK: return "ok";
    case ABFT_FAULT_DETECTED: return "fault detected";
    case ABFT_E_ARG: return "invalid argument";
    case ABFT_E_HIP: return "HIP runtime error";
    case ABFT_E_UNCORRECTABLE: return "uncorrectable: the failed relations do not name one element";
    case ABFT_E_UNRECOVERABLE: return "unrecoverable: more unknowns than checksum relations";
    case ABFT_E_WORKSPACE: return "workspace missing or too small";
    case ABFT_E_UNSUPPORTED: return "unsupported combination";
    case ABFT_E_STALE: return "the fused partial sums in the workspace belong to another product";
    default: return "unknown status";
    }
}

}  // extern "C"
