// Correction of one located element, rebuild of an erased rectangle (both the
// unit-weight single-checksum recovery of Sec. 2.1 applied to a relation of
// C_f), the test-only fault injectors and the synthetic-input generator.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace abft {

constexpr int kThreads = 256;

template <typename T> __device__ inline void store_c(T *p, double v);
template <> __device__ inline void store_c<double>(double *p, double v) { *p = v; }
template <> __device__ inline void store_c<float>(float *p, double v) { *p = (float)v; }

// Relation through (i, j).  Column direction: members are rows g*br + r
// (g < Gr, summands) and m + s*br + r (s < S, totals) of column j, r = i mod br.
// Row direction: columns h*bc + c (summands) and n + s*bc + c (totals) of row i.
// The element is solved from the others:  summand = sum(totals) - sum(other summands),
// total = sum(summands) - sum(other totals).  Member t of the relation, t < Gr + S.
struct Rel {
    int64_t base, step_data, step_tot, first_tot, n_data, n_tot, self;
    bool self_is_total;
};

__device__ inline Rel make_rel(const Geom &g, int64_t ldc, int64_t i, int64_t j, int dir) {
    Rel R;
    if (dir == ABFT_DIR_COL) {
        int64_t r = i % g.br;
        R.base = r * ldc + j;               // data member g at base + g*step_data
        R.step_data = g.br * ldc;
        R.first_tot = (g.m + r) * ldc + j;  // total s at first_tot + s*step_tot
        R.step_tot = g.br * ldc;
        R.n_data = g.Gr; R.n_tot = g.S;
        R.self_is_total = i >= g.m;
        R.self = R.self_is_total ? (i - g.m) / g.br : i / g.br;
    } else {
        int64_t c = j % g.bc;
        R.base = i * ldc + c;
        R.step_data = g.bc;
        R.first_tot = i * ldc + g.n + c;
        R.step_tot = g.bc;
        R.n_data = g.Gc; R.n_tot = g.S;
        R.self_is_total = j >= g.n;
        R.self = R.self_is_total ? (j - g.n) / g.bc : j / g.bc;
    }
    return R;
}

// Signed contribution of member t (data members first, then totals) to the
// solved value; the element itself contributes 0.
template <typename T>
__device__ inline double member_term(const T *C, const Rel &R, int64_t t) {
    if (t < R.n_data) {
        if (!R.self_is_total && t == R.self) return 0.0;
        double v = elem<T>::load(C + R.base + t * R.step_data);
        return R.self_is_total ? v : -v;
    }
    int64_t s = t - R.n_data;
    if (R.self_is_total && s == R.self) return 0.0;
    double v = elem<T>::load(C + R.first_tot + s * R.step_tot);
    return R.self_is_total ? -v : v;
}

// One block rebuilds one element: threads take members t = tid, tid+256, ...,
// then a fixed-order tree combines them.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_correct(T *C, Geom g, int64_t ldc, int64_t i, int64_t j, int dir) {
    __shared__ double sh[kThreads];
    Rel R = make_rel(g, ldc, i, j, dir);
    int64_t nmem = R.n_data + R.n_tot;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < nmem; t += kThreads) s += member_term<T>(C, R, t);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) store_c<T>(C + i * ldc + j, sh[0]);
}

// One thread per erased element; its relation has no other erased member
// (h <= br for columns, w <= bc for rows), so in-place writes do not race
// with the reads of other threads.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_recover(T *C, Geom g, int64_t ldc, abft_rect e, int dir) {
    const int64_t total = e.h * e.w;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t a = t / e.w, b = t - a * e.w;
        int64_t i = e.i0 + a, j = e.j0 + b;
        Rel R = make_rel(g, ldc, i, j, dir);
        double s = 0.0;
        for (int64_t q = 0; q < R.n_data + R.n_tot; ++q) s += member_term<T>(C, R, q);
        store_c<T>(C + i * ldc + j, s);
    }
}

template <typename T>
static int correct_typed(const abft_problem *p, T *C, int64_t i, int64_t j, int dir, hipStream_t s) {
    Geom g = geom_of(p);
    k_correct<T><<<1, kThreads, 0, s>>>(C, g, p->ldc, i, j, dir);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_correct(const abft_problem *p, void *C_f, int64_t i, int64_t j, int dir, hipStream_t s) {
    if (p->dtype == ABFT_F64) return correct_typed<double>(p, (double *)C_f, i, j, dir, s);
    return correct_typed<float>(p, (float *)C_f, i, j, dir, s);
}

int launch_recover(const abft_problem *p, void *C_f, abft_rect e, int use_rows, hipStream_t s) {
    Geom g = geom_of(p);
    unsigned blocks = (unsigned)std::min<int64_t>((e.h * e.w + kThreads - 1) / kThreads, 65536);
    int dir = use_rows ? ABFT_DIR_ROW : ABFT_DIR_COL;
    if (p->dtype == ABFT_F64)
        k_recover<double><<<blocks, kThreads, 0, s>>>((double *)C_f, g, p->ldc, e, dir);
    else
        k_recover<float><<<blocks, kThreads, 0, s>>>((float *)C_f, g, p->ldc, e, dir);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// ------------------------------------------------------------------ injectors (test only)
__global__ void k_flip64(uint64_t *p, int bit) { *p ^= (1ull << bit); }
__global__ void k_flip32(uint32_t *p, int bit) { *p ^= (1u << bit); }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_rect(T *C, int64_t ldc, abft_rect e, T v) {
    const int64_t total = e.h * e.w;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t a = t / e.w, b = t - a * e.w;
        C[(e.i0 + a) * ldc + e.j0 + b] = v;
    }
}

int launch_inject_flip(const abft_problem *p, void *C_f, int64_t i, int64_t j, int bit, hipStream_t s) {
    if (p->dtype == ABFT_F64)
        k_flip64<<<1, 1, 0, s>>>((uint64_t *)C_f + i * p->ldc + j, bit);
    else
        k_flip32<<<1, 1, 0, s>>>((uint32_t *)C_f + i * p->ldc + j, bit);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_inject_erase(const abft_problem *p, void *C_f, abft_rect e, int nan_fill, hipStream_t s) {
    unsigned blocks = (unsigned)std::min<int64_t>((e.h * e.w + kThreads - 1) / kThreads, 65536);
    if (p->dtype == ABFT_F64)
        k_fill_rect<double><<<blocks, kThreads, 0, s>>>((double *)C_f, p->ldc, e, nan_fill ? (double)NAN : 0.0);
    else
        k_fill_rect<float><<<blocks, kThreads, 0, s>>>((float *)C_f, p->ldc, e, nan_fill ? (float)NAN : 0.0f);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// ------------------------------------------------------------------ synthetic inputs
// splitmix64 (Steele, Lea, Flood 2014) used counter-based: element idx of
// stream (seed, sid) is mix64(key + (idx+1)*gamma), key = mix64(seed*256 + sid).
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T> __device__ inline T uniform_from(uint64_t x);
template <> __device__ inline double uniform_from<double>(uint64_t x) { return (double)(x >> 11) * 0x1p-52 - 1.0; }
template <> __device__ inline float uniform_from<float>(uint64_t x) { return (float)((double)(x >> 40) * 0x1p-23 - 1.0); }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_uniform(T *dst, int64_t rows, int64_t cols, int64_t ld, int transpose,
                                                           uint64_t key) {
    const int64_t total = rows * cols;
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t r, c;
        if (transpose) { c = t / rows; r = t - c * rows; }   // walk the stored (column) order
        else { r = t / cols; c = t - r * cols; }
        uint64_t idx = (uint64_t)r * (uint64_t)cols + (uint64_t)c;
        T v = uniform_from<T>(mix64(key + (idx + 1) * gamma));
        if (transpose) dst[c * ld + r] = v;
        else dst[r * ld + c] = v;
    }
}

int launch_fill_uniform(int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed,
                        int32_t stream_id, void *dst, hipStream_t s) {
    uint64_t key = mix64(seed * 256ull + (uint64_t)stream_id);
    unsigned blocks = (unsigned)std::min<int64_t>((rows * cols + kThreads - 1) / kThreads, 65536);
    if (dtype == ABFT_F64)
        k_fill_uniform<double><<<blocks, kThreads, 0, s>>>((double *)dst, rows, cols, ld, transpose, key);
    else
        k_fill_uniform<float><<<blocks, kThreads, 0, s>>>((float *)dst, rows, cols, ld, transpose, key);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// Heavy-tailed binary32 inputs: N(0,1) by Box-Muller in binary64 from the
// seed's streams A (u1 in (0, 1]) and B (u2 in [0, 1)) at the element's
// row-major index, rounded to binary32; with probability frac (stream 6, the
// outlier mask) the value is multiplied by fl32(scale).  The recipe of the host
// generator; the device's log and cos may differ from the host library's in
// the last bit, so a value can differ from the host's by one rounding (the
// sets serve runs that need no oracle).
__global__ __launch_bounds__(kThreads) void k_fill_normal(float *dst, int64_t rows, int64_t cols, int64_t ld,
                                                          int transpose, uint64_t key1, uint64_t key2, uint64_t keyo,
                                                          double frac, float scale) {
    const int64_t total = rows * cols;
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t r, c;
        if (transpose) { c = t / rows; r = t - c * rows; }
        else { r = t / cols; c = t - r * cols; }
        const uint64_t idx = (uint64_t)r * (uint64_t)cols + (uint64_t)c;
        const uint64_t step = (idx + 1) * gamma;
        const double u1 = ((double)(mix64(key1 + step) >> 11) + 1.0) * 0x1p-53;
        const double u2 = (double)(mix64(key2 + step) >> 11) * 0x1p-53;
        float z = (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
        if ((double)(mix64(keyo + step) >> 11) * 0x1p-53 < frac) z = z * scale;
        if (transpose) dst[c * ld + r] = z;
        else dst[r * ld + c] = z;
    }
}

int launch_fill_normal(int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed, double frac,
                       float scale, float *dst, hipStream_t s) {
    const uint64_t k1 = mix64(seed * 256ull + 0), k2 = mix64(seed * 256ull + 1), ko = mix64(seed * 256ull + 6);
    const unsigned blocks = (unsigned)std::min<int64_t>((rows * cols + kThreads - 1) / kThreads, 65536);
    k_fill_normal<<<blocks, kThreads, 0, s>>>(dst, rows, cols, ld, transpose, k1, k2, ko, frac, scale);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// ------------------------------------------------------------------ 2-D block-cyclic layout (Sec. 4.1)
// One dimension of n indices over Pn processes with blocks of nb: global
// index i is local index ((i/nb) div Pn) nb + i mod nb of process (i/nb) mod Pn;
// its stacked position is process * (n / Pn) + local index.
__device__ inline int64_t bc_stacked(int64_t i, int64_t nb, int64_t Pn, int64_t ln) {
    const int64_t I = i / nb;
    return (I % Pn) * ln + (I / Pn) * nb + (i - I * nb);
}
__device__ inline int64_t bc_global(int64_t r, int64_t nb, int64_t Pn, int64_t ln) {
    const int64_t p = r / ln, li = r - p * ln, lI = li / nb;
    return (lI * Pn + p) * nb + (li - lI * nb);
}

// Copy with the stacked <-> global permutation: destination element (r, c)
// takes the source element its index maps to.  stack: destination stacked.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_block_cyclic(const T *__restrict__ src, int64_t lds, T *__restrict__ dst,
                                                          int64_t ldd, int64_t rows, int64_t cols, int64_t nb,
                                                          int64_t P, int64_t Q, int stack) {
    const int64_t lm = rows / P, ln = cols / Q, total = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        const int64_t r = t / cols, c = t - r * cols;
        const int64_t i = stack ? bc_global(r, nb, P, lm) : bc_stacked(r, nb, P, lm);
        const int64_t j = stack ? bc_global(c, nb, Q, ln) : bc_stacked(c, nb, Q, ln);
        dst[r * ldd + c] = src[i * lds + j];
    }
}

static int block_cyclic_copy(const void *src, int64_t lds, void *dst, int64_t ldd, int64_t rows, int64_t cols,
                             int32_t es, int64_t nb, int32_t P, int32_t Q, bool stack, hipStream_t s) {
    if (!src || !dst || rows < 1 || cols < 1 || nb < 1 || P < 1 || Q < 1) return ABFT_E_ARG;
    if (es != 1 && es != 2 && es != 4 && es != 8) return ABFT_E_ARG;
    // a dimension over one process is not permuted; over several, every process gets whole blocks alike
    if ((P > 1 && rows % (nb * P)) || (Q > 1 && cols % (nb * Q)) || lds < cols || ldd < cols) return ABFT_E_ARG;
    if ((uintptr_t)src % es || (uintptr_t)dst % es) return ABFT_E_ARG;
    const unsigned grid = (unsigned)std::min<int64_t>((rows * cols + kThreads - 1) / kThreads, 65536);
    switch (es) {
    case 1: k_block_cyclic<uint8_t><<<grid, kThreads, 0, s>>>((const uint8_t *)src, lds, (uint8_t *)dst, ldd, rows, cols, nb, P, Q, stack); break;
    case 2: k_block_cyclic<uint16_t><<<grid, kThreads, 0, s>>>((const uint16_t *)src, lds, (uint16_t *)dst, ldd, rows, cols, nb, P, Q, stack); break;
    case 4: k_block_cyclic<uint32_t><<<grid, kThreads, 0, s>>>((const uint32_t *)src, lds, (uint32_t *)dst, ldd, rows, cols, nb, P, Q, stack); break;
    case 8: k_block_cyclic<uint64_t><<<grid, kThreads, 0, s>>>((const uint64_t *)src, lds, (uint64_t *)dst, ldd, rows, cols, nb, P, Q, stack); break;
    default: return ABFT_E_ARG;
    }
    ABFT_LAUNCHED();
    return ABFT_OK;
}

}  // namespace abft

extern "C" int abft_block_cyclic_stack(const void *G, int64_t ldg, int64_t rows, int64_t cols, int32_t elem_size,
                                       int64_t nb, int32_t P, int32_t Q, void *S, int64_t lds, void *stream) {
    return abft::block_cyclic_copy(G, ldg, S, lds, rows, cols, elem_size, nb, P, Q, true, (hipStream_t)stream);
}

extern "C" int abft_block_cyclic_unstack(const void *S, int64_t lds, int64_t rows, int64_t cols, int32_t elem_size,
                                         int64_t nb, int32_t P, int32_t Q, void *G, int64_t ldg, void *stream) {
    return abft::block_cyclic_copy(S, lds, G, ldg, rows, cols, elem_size, nb, P, Q, false, (hipStream_t)stream);
}
