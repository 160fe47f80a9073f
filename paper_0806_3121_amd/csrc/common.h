// Internal declarations shared by the libabft HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abft.h"

namespace abft {

// ------------------------------------------------------------------ types
struct bf16 { uint16_t bits; };

__host__ __device__ inline float bf16_to_f32(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Round-to-nearest-even binary32 -> bfloat16 bits (NaN stays NaN).
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    // branch-free (a select, not a divergent branch per element): NaN keeps its
    // sign and top payload bits and is made quiet
    const uint32_t rounded = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    const uint32_t quiet = (u >> 16) | 0x40u;
    return (uint16_t)((u & 0x7FFFFFFFu) > 0x7F800000u ? quiet : rounded);
}

// OCP FP8 E4M3 (e4m3fn): bias 7, 3 fraction bits, largest finite 448, no
// infinities, S.1111.111 is NaN.  Every E4M3 value is a binary32 value, so the
// gfx950 conversion instructions (which decode the OCP format) are exact:
// e4m3_to_f64 converts byte 0 of c; e4m3x4_to_f64 the four bytes of a dword,
// byte 0 first, two per instruction.  Checked against the format's definition
// for all 256 codes in every byte position on gfx950.
typedef float v2f32 __attribute__((ext_vector_type(2)));
__device__ inline double e4m3_to_f64(uint32_t c) { return (double)__builtin_amdgcn_cvt_f32_fp8((int)c, 0); }
__device__ inline void e4m3x4_to_f64(uint32_t w, double *o) {
    const v2f32 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false), hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    o[0] = lo[0];
    o[1] = lo[1];
    o[2] = hi[0];
    o[3] = hi[1];
}

// binary32 -> E4M3, round to nearest, ties to even fraction; |x| >= 464 (the
// midpoint above 448 and beyond) saturates to +-448; NaN -> 0x7F.
__host__ __device__ inline uint8_t f32_to_e4m3_rne(float x) {
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    uint32_t a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return 0x7F;
    float ax;
    __builtin_memcpy(&ax, &a, 4);
    if (ax >= 464.0f) return sign | 0x7E;
    if (ax < 0x1p-6f) {                                   // subnormal grid: multiples of 2^-9
        float q = __builtin_rintf(ax * 512.0f);          // exact scaling, ties to even
        return sign | (uint8_t)q;                         // q == 8 is 2^-6, code 0x08
    }
    uint32_t r = (a + 0x7FFFFu + ((a >> 20) & 1u)) & 0xFFF00000u;   // round the fraction at bit 20
    int E = (int)(r >> 23) - 127;
    uint32_t code = ((uint32_t)(E + 7) << 3) | ((r >> 20) & 7u);
    if (code > 0x7Eu) code = 0x7E;
    return sign | (uint8_t)code;
}

template <typename T> struct elem;
template <> struct elem<double> {
    __device__ static double load(const double *p) { return *p; }
};
template <> struct elem<float> {
    __device__ static double load(const float *p) { return (double)*p; }
};
template <> struct elem<uint16_t> {   // bfloat16 storage
    __device__ static double load(const uint16_t *p) { return (double)bf16_to_f32(*p); }
};
template <> struct elem<uint8_t> {    // FP8 E4M3 storage (values in the scaled domain)
    __device__ static double load(const uint8_t *p) { return e4m3_to_f64(*p); }
};

// One 16-byte load of N elements, widened to binary64 (16-byte aligned address).
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
template <typename T> struct vec16;
template <> struct vec16<double> {
    static constexpr int N = 2;
    __device__ static void load(const double *p, double *o) {
        typedef double v2 __attribute__((ext_vector_type(2)));
        v2 v = *(const v2 *)p;
        o[0] = v[0]; o[1] = v[1];
    }
    // the same N values from a chunk already loaded as raw words
    __device__ static void widen(const v4u32 &w, double *o) {
        o[0] = __hiloint2double((int)w[1], (int)w[0]);
        o[1] = __hiloint2double((int)w[3], (int)w[2]);
    }
};
template <> struct vec16<float> {
    static constexpr int N = 4;
    __device__ static void load(const float *p, double *o) {
        typedef float v4 __attribute__((ext_vector_type(4)));
        v4 v = *(const v4 *)p;
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
    __device__ static void widen(const v4u32 &w, double *o) {
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = (double)__uint_as_float(w[q]);
    }
};
template <> struct vec16<uint16_t> {                 // bfloat16
    static constexpr int N = 8;
    __device__ static void load(const uint16_t *p, double *o) {
        typedef uint32_t v4u __attribute__((ext_vector_type(4)));
        v4u v = *(const v4u *)p;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (double)bf16_to_f32((uint16_t)(v[q] & 0xFFFFu));
            o[2 * q + 1] = (double)bf16_to_f32((uint16_t)(v[q] >> 16));
        }
    }
    __device__ static void widen(const v4u32 &w, double *o) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (double)bf16_to_f32((uint16_t)(w[q] & 0xFFFFu));
            o[2 * q + 1] = (double)bf16_to_f32((uint16_t)(w[q] >> 16));
        }
    }
};

template <> struct vec16<uint8_t> {                  // FP8 E4M3
    static constexpr int N = 16;
    __device__ static void load(const uint8_t *p, double *o) {
        v4u32 v = *(const v4u32 *)p;
#pragma unroll
        for (int w = 0; w < 4; ++w) e4m3x4_to_f64(v[w], o + 4 * w);
    }
    __device__ static void widen(const v4u32 &w, double *o) {
#pragma unroll
        for (int q = 0; q < 4; ++q) e4m3x4_to_f64(w[q], o + 4 * q);
    }
};


inline size_t dtype_size(int dt) {
    switch (dt) {
    case ABFT_F64: return 8;
    case ABFT_F32: return 4;
    case ABFT_BF16: return 2;
    case ABFT_FP8_E4M3: return 1;
    default: return 0;
    }
}
inline size_t c_size(int dt) { return dt == ABFT_F64 ? 8 : 4; }
// Low-precision inputs keep their checksum rows in binary32 in the workspace;
// F64 and F32 keep them in the extra rows of A_f / B_f.
inline bool cs_in_ws(int dt) { return dt == ABFT_BF16 || dt == ABFT_FP8_E4M3; }

// ------------------------------------------------------------------ geometry
struct Geom {
    int64_t m, n, k, br, bc;
    int64_t S;           // entries per carried checksum (1: every carried value is one entry of C_f)
    int64_t M, N;        // encoded sizes m + br, n + bc
    int64_t Gr, Gc;      // m / br, n / bc
};
inline Geom geom_of(const abft_problem *p) {
    Geom g;
    g.m = p->m; g.n = p->n; g.k = p->k; g.br = p->br; g.bc = p->bc;
    g.S = 1;
    g.M = g.m + g.S * g.br;
    g.N = g.n + g.S * g.bc;
    g.Gr = g.m / g.br;
    g.Gc = g.n / g.bc;
    return g;
}

// Up to 4 known erased rectangles, passed to kernels by value.
struct Erasures {
    int n;
    int64_t i0[4], j0[4], h[4], w[4];
};

// Does column relation (r, j) (members: rows i == r mod br, column j) hold an erased element?
__device__ inline bool col_rel_erased(const Erasures &e, int64_t r, int64_t j, int64_t br) {
    for (int q = 0; q < e.n; ++q) {
        if (j < e.j0[q] || j >= e.j0[q] + e.w[q]) continue;
        if (e.h[q] >= br) return true;
        int64_t off = ((r - e.i0[q]) % br + br) % br;   // first row >= i0 with residue r is i0 + off
        if (off < e.h[q]) return true;
    }
    return false;
}
__device__ inline bool row_rel_erased(const Erasures &e, int64_t i, int64_t c, int64_t bc) {
    for (int q = 0; q < e.n; ++q) {
        if (i < e.i0[q] || i >= e.i0[q] + e.h[q]) continue;
        if (e.w[q] >= bc) return true;
        int64_t off = ((c - e.j0[q]) % bc + bc) % bc;
        if (off < e.w[q]) return true;
    }
    return false;
}

// ------------------------------------------------------------------ workspace
// All offsets in bytes from ws, 256-byte aligned.
struct WsLayout {
    size_t na, na_abs, nb, nb_abs;   // det statistics (double)
    size_t qr, qc, nv, nw;           // stat statistics (double)
    size_t grpA, grpB;               // per-residue group sums of |A| (or A^2) and of |B| (double, br*k / bc*k)
    size_t acs, bcs;                 // binary32 checksum rows of low-precision operands (float, br*k / bc*k)
    size_t scale;                    // FP8 per-tensor scale exponents and amax scratch (4 x int32)
    size_t partial;                  // two-level reduction partials (double)
    size_t fused_c, fused_r;         // product-epilogue partial sums for b = 1 (double)
    size_t chain_a, chain_w;         // chained products: inherited threshold term chain_a[r] chain_w[j]
    size_t chain_cs;                 // chained products: the recomputed checksum rows (discarded; br x k elements)
    size_t rowpart;                  // fused row statistics: per-row partial sums
    size_t vpart_c, vpart_r;         // one-pass re-read verification for b = 1: tile partial sums (double)
    size_t fused_tag;                // owner of the fused partials: fused_key() of the last fused product, else 0
    size_t report;                   // abft_report
    size_t total;
    size_t partial_bytes;
};
WsLayout ws_layout(const abft_problem *p);

// Det or statistical thresholds with k / (16 / size) a multiple of 64: the
// encode pass also produces the row statistics (rows_fused), from per-row
// partials in ws.
bool rows_fused(const abft_problem *p);

// Number of partitions used for the row-group sums of a (G groups, b residues, cols) sum.
int64_t group_partitions(int64_t G, int64_t b, int64_t cols);

// ------------------------------------------------------------------ error plumbing
void set_hip_error(hipError_t e);
#define ABFT_HIP(call)                                        \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) { ::abft::set_hip_error(e_); return ABFT_E_HIP; } \
    } while (0)
#define ABFT_LAUNCHED()                                       \
    do {                                                      \
        hipError_t e_ = hipGetLastError();                    \
        if (e_ != hipSuccess) { ::abft::set_hip_error(e_); return ABFT_E_HIP; } \
    } while (0)

// ------------------------------------------------------------------ launchers (return abft_status)
int launch_encode(const abft_problem *p, void *A_f, void *B_f, char *ws, hipStream_t s);
// Binary64 matrix-core product C = A B^T-stored (A: M x K rows, Bt: N x K rows), all M x N entries.
int launch_gemm_f64(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc, int64_t M,
                    int64_t N, int64_t K, hipStream_t s);
// Binary64 skinny product (N <= a few columns, e.g. a matrix-vector product):
// streams A once, binary64 accumulation.  Same layouts as launch_gemm_f64.
int launch_skinny_f64(const double *A, int64_t lda, const double *Bt, int64_t ldb, double *C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K, hipStream_t s);
// The same in binary32: the matrix-core product accumulates in binary32; the
// skinny product accumulates in binary64 and rounds each entry once.
int launch_gemm_f32(const float *A, int64_t lda, const float *Bt, int64_t ldb, float *C, int64_t ldc, int64_t M,
                    int64_t N, int64_t K, hipStream_t s);
int launch_skinny_f32(const float *A, int64_t lda, const float *Bt, int64_t ldb, float *C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K, hipStream_t s);
int launch_gemm_panel(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, int64_t k0, int64_t k1,
                      uint32_t flags, hipStream_t s);
int describe_gemm(const abft_problem *p, uint32_t flags, char *buf, size_t len);
// fault: a test-only accumulator flip (null: none).
int launch_gemm(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, uint32_t flags, void *ws,
                const abft_fault *fault, hipStream_t s);
int launch_verify(const abft_problem *p, const void *C_f, const Erasures &er, char *ws, hipStream_t s);
// The verification's scratch (everything it writes): the device report, the
// tile partial sums of the one-pass b = 1 check and the two-level reduction
// partials.  launch_verify takes them from ws; launch_verify_scratch from
// anywhere, reading only the threshold statistics from ws.
struct VerifyScratch {
    abft_report *rep;
    double *vpart_c, *vpart_r, *partial;
};
int launch_verify_scratch(const abft_problem *p, const void *C_f, const Erasures &er, const char *ws,
                          const VerifyScratch &sc, hipStream_t s);
size_t verify_scratch_layout(const abft_problem *p, const void *C_f, char *base, VerifyScratch *sc);
int launch_encode_chained(const abft_problem *p, const void *A_f, void *B_f, char *ws, const abft_problem *prev,
                          const char *ws_prev, double cc_prev, hipStream_t s);
int launch_verify_fused(const abft_problem *p, const void *C_f, char *ws, int64_t tiles_m, int64_t tiles_n,
                        uint64_t key, hipStream_t s);
// The tile grid of the fused partials an ABFT_FUSED product of p writes, and
// the owner tag it stores in ws: a nonzero hash of the problem, the tile grid
// and C_f.
uint64_t fused_key(const abft_problem *p, const void *C_f, int64_t *tiles_m, int64_t *tiles_n);
// Smallest tile edge of every product kernel: bounds the tile rows / columns of the fused partials.
constexpr int64_t kMinTileEdge = 96;
// Row tile of the one-pass b = 1 re-read verification (column sums per tile of this many rows); its row
// sums are per tile of 64 16-byte vectors (128 binary64 or 256 binary32 columns).
constexpr int64_t kVerifyPartRows = 128;
int launch_correct(const abft_problem *p, void *C_f, int64_t i, int64_t j, int dir, hipStream_t s);
int launch_recover(const abft_problem *p, void *C_f, abft_rect e, int use_rows, hipStream_t s);
int launch_inject_flip(const abft_problem *p, void *C_f, int64_t i, int64_t j, int bit, hipStream_t s);
int launch_inject_erase(const abft_problem *p, void *C_f, abft_rect e, int nan_fill, hipStream_t s);
int launch_fill_uniform(int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed,
                        int32_t stream_id, void *dst, hipStream_t s);
int launch_fill_normal(int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed, double frac,
                       float scale, float *dst, hipStream_t s);
int launch_quantize_encode(const abft_problem *p, const float *A32, int64_t lda32, const float *B32, int64_t ldb32,
                           void *A_f, void *B_f, char *ws, hipStream_t s);
int launch_quantize(const abft_problem *p, int which, const float *X, int64_t ldx, void *dst, char *ws, hipStream_t s);

// Threshold coefficients shared by encode (statistics) and verify.
struct TauCoef {
    int mode;
    double cc, cr;       // det: tau_c = cc*na_abs[r]*nb[j], tau_r = cr*na[i]*nb_abs[c];
                         // stat: tau = sqrt(cc * Q + cst * tot^2), cc = lambda^2 (u^2/3)(T/2 + s)
    double cst;          // stat: lambda^2 u^2 / 3, the binary32 storage of the relation's stored total tot
    double lambda;
};
TauCoef tau_coef(const abft_problem *p);

}  // namespace abft
