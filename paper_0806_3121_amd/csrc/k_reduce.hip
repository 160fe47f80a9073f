// Encode (checksum rows/columns + threshold statistics) and verify (relation
// residuals, thresholds, flags) for gfx950.  Both are HBM-bound row-group
// sums: every element is read once per pass, lanes walk contiguous columns,
// sums are binary64, and the per-block maxima/counts are folded with
// wavefront shuffles before one atomic per block.
#include <cmath>

#include "common.h"

namespace abft {

constexpr int kThreads = 256;
constexpr int kWave = 64;

// ------------------------------------------------------------------ block reductions
__device__ inline double wave_max(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
__device__ inline double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Fold one value per thread into the report: max ratio and excluded count.
__device__ inline void fold_block(double ratio, unsigned long long excl, double *rep_ratio, int64_t *rep_excl) {
    __shared__ double s_r[kThreads / kWave];
    __shared__ unsigned long long s_e[kThreads / kWave];
    ratio = wave_max(ratio);
    excl = wave_sum_u64(excl);
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) { s_r[w] = ratio; s_e[w] = excl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = s_r[0];
        unsigned long long e = s_e[0];
        for (int q = 1; q < kThreads / kWave; ++q) { r = fmax(r, s_r[q]); e += s_e[q]; }
        if (r > 0) {
            unsigned long long bits;
            __builtin_memcpy(&bits, &r, 8);
            atomicMax((unsigned long long *)rep_ratio, bits);   // ordering of non-negative doubles = ordering of their bits
        }
        if (e) atomicAdd((unsigned long long *)rep_excl, e);
    }
}

// Record a relation residual; returns the ratio |d|/tau for the block maximum (0 if not finite).
__device__ inline double record(abft_report *rep, bool col, int64_t a, int64_t b, double d, double tau) {
    if (!(fabs(d) <= tau)) {
        unsigned long long *cnt = (unsigned long long *)(col ? &rep->n_flag_c : &rep->n_flag_r);
        unsigned long long q = atomicAdd(cnt, 1ull);
        if (q < ABFT_MAX_FLAGS) {
            abft_flag *f = col ? &rep->flag_c[q] : &rep->flag_r[q];
            f->a = a; f->b = b; f->d = d; f->tau = tau;
        }
        if (!isfinite(d)) atomicAdd((unsigned long long *)&rep->n_nonfinite, 1ull);
    }
    if (isfinite(d) && tau > 0) return fabs(d) / tau;
    return 0.0;
}

__global__ void k_report_init(abft_report *rep) {
    uint64_t *w = (uint64_t *)rep;
    const int nw = sizeof(abft_report) / 8;
    for (int q = threadIdx.x; q < nw; q += blockDim.x) w[q] = 0;
}

// ------------------------------------------------------------------ store helpers
template <typename T> __device__ inline void store_checksum(T *row0, int64_t stride_s, int64_t l, double s, int S);
template <> __device__ inline void store_checksum<double>(double *row0, int64_t, int64_t l, double s, int) { row0[l] = s; }
template <> __device__ inline void store_checksum<float>(float *row0, int64_t, int64_t l, double s, int) { row0[l] = (float)s; }
template <> __device__ inline void store_checksum<uint16_t>(uint16_t *row0, int64_t stride_s, int64_t l, double s, int S) {
    // binary32 checksum split into S bfloat16 parts whose sum is exact (S = 3)
    float c = (float)s;
    for (int q = 0; q < S; ++q) {
        uint16_t h = f32_to_bf16_rne(c);
        row0[q * stride_s + l] = h;
        c = c - bf16_to_f32(h);
    }
}

// ------------------------------------------------------------------ encode
// Operand X (rows >= R + S*b, row-major, ld): the checksum rows
// X[R + s*b + r, l] receive sum_{g<G} X[g*b + r, l] (s = split part), and
// grp[r*k + l] = sum_g |X[g*b + r, l]| (det statistics).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_encode_direct(T *X, int64_t ld, int64_t R, int64_t b, int64_t G,
                                                            int64_t k, int S, double *grp) {
    const int64_t total = b * k;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / k, l = t - r * k;
        double s = 0.0, sa = 0.0;
        const T *p = X + r * ld + l;
        for (int64_t g = 0; g < G; ++g) {
            double v = elem<T>::load(p + g * b * ld);
            s += v;
            sa += fabs(v);
        }
        store_checksum<T>(X + (R + r) * ld, b * ld, l, s, S);
        grp[t] = sa;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_encode_partial(const T *X, int64_t ld, int64_t b, int64_t G, int64_t k,
                                                             int64_t P, int64_t chunk, double *part) {
    const int64_t rel = b * k, total = P * rel;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t p = t / rel, q = t - p * rel;
        int64_t r = q / k, l = q - r * k;
        int64_t g0 = p * chunk, g1 = min(G, g0 + chunk);
        double s = 0.0, sa = 0.0;
        const T *src = X + r * ld + l;
        for (int64_t g = g0; g < g1; ++g) {
            double v = elem<T>::load(src + g * b * ld);
            s += v;
            sa += fabs(v);
        }
        part[(2 * p) * rel + q] = s;
        part[(2 * p + 1) * rel + q] = sa;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_encode_finish(T *X, int64_t ld, int64_t R, int64_t b, int64_t k, int S,
                                                            int64_t P, const double *part, double *grp) {
    const int64_t rel = b * k;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < rel; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / k, l = t - r * k;
        double s = 0.0, sa = 0.0;
        for (int64_t p = 0; p < P; ++p) {
            s += part[(2 * p) * rel + t];
            sa += part[(2 * p + 1) * rel + t];
        }
        store_checksum<T>(X + (R + r) * ld, b * ld, l, s, S);
        grp[t] = sa;
    }
}

// out[i] = || X[i, 0:k] ||_2, one block per row (grid-stride over rows).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_row_norms(const T *X, int64_t ld, int64_t rows, int64_t k, double *out) {
    __shared__ double sh[kThreads / kWave];
    for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
        const T *row = X + i * ld;
        double s = 0.0;
        for (int64_t l = threadIdx.x; l < k; l += kThreads) {
            double v = elem<T>::load(row + l);
            s += v * v;
        }
        s = wave_sum(s);
        if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < kThreads / kWave; ++q) t += sh[q];
            out[i] = sqrt(t);
        }
        __syncthreads();
    }
}

template <typename T>
static int encode_operand(T *X, int64_t ld, int64_t R, int64_t b, int64_t k, int S, int64_t rows_total,
                          double *grp, double *norms_rows, double *norms_grp, double *part, hipStream_t s) {
    int64_t G = R / b;
    int64_t P = group_partitions(G, b, k);
    auto blocks = [](int64_t work) { return (unsigned)std::min<int64_t>((work + kThreads - 1) / kThreads, 65536); };
    if (P == 1) {
        k_encode_direct<T><<<blocks(b * k), kThreads, 0, s>>>(X, ld, R, b, G, k, S, grp);
    } else {
        int64_t chunk = (G + P - 1) / P;
        P = (G + chunk - 1) / chunk;
        k_encode_partial<T><<<blocks(P * b * k), kThreads, 0, s>>>(X, ld, b, G, k, P, chunk, part);
        k_encode_finish<T><<<blocks(b * k), kThreads, 0, s>>>(X, ld, R, b, k, S, P, part, grp);
    }
    ABFT_LAUNCHED();
    k_row_norms<T><<<(unsigned)std::min<int64_t>(rows_total, 65536), kThreads, 0, s>>>(X, ld, rows_total, k, norms_rows);
    k_row_norms<double><<<(unsigned)std::min<int64_t>(b, 65536), kThreads, 0, s>>>(grp, k, b, k, norms_grp);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_encode(const abft_problem *p, void *A_f, void *B_f, char *ws, hipStream_t s) {
    Geom g = geom_of(p);
    WsLayout L = ws_layout(p);
    double *part = (double *)(ws + L.partial);
    int st;
    switch (p->dtype) {
    case ABFT_F64:
        st = encode_operand<double>((double *)A_f, p->lda, g.m, g.br, g.k, (int)g.S, g.M, (double *)(ws + L.grpA),
                                    (double *)(ws + L.na), (double *)(ws + L.na_abs), part, s);
        if (st) return st;
        return encode_operand<double>((double *)B_f, p->ldb, g.n, g.bc, g.k, (int)g.S, g.N, (double *)(ws + L.grpB),
                                      (double *)(ws + L.nb), (double *)(ws + L.nb_abs), part, s);
    default:
        return ABFT_E_UNSUPPORTED;
    }
}

// ------------------------------------------------------------------ verify
struct VerifyArgs {
    int64_t m, n, br, bc, S, Gr, Gc, M, N, ldc;
    int mode;
    double cc, cr;
    const double *na, *na_abs, *nb, *nb_abs;
    abft_report *rep;
    Erasures er;
};

__device__ inline double tau_col(const VerifyArgs &a, int64_t r, int64_t j) {
    return a.mode == ABFT_TAU_DET ? a.cc * a.na_abs[r] * a.nb[j] : 0.0;
}
__device__ inline double tau_row(const VerifyArgs &a, int64_t i, int64_t c) {
    return a.mode == ABFT_TAU_DET ? a.cr * a.na[i] * a.nb_abs[c] : 0.0;
}

// Column relation (r, j): sum_{g<Gr} C[g*br + r, j] - sum_{s<S} C[m + s*br + r, j]
template <typename T>
__device__ inline void finish_col(const VerifyArgs &a, const T *C, int64_t r, int64_t j, double s, double &ratio,
                                  unsigned long long &excl) {
    double tot = 0.0;
    for (int64_t q = 0; q < a.S; ++q) tot += elem<T>::load(C + (a.m + q * a.br + r) * a.ldc + j);
    if (col_rel_erased(a.er, r, j, a.br)) { excl++; return; }
    ratio = fmax(ratio, record(a.rep, true, r, j, s - tot, tau_col(a, r, j)));
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vcol_direct(const T *C, VerifyArgs a) {
    const int64_t total = a.br * a.N;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / a.N, j = t - r * a.N;
        const T *p = C + r * a.ldc + j;
        double s = 0.0;
        for (int64_t g = 0; g < a.Gr; ++g) s += elem<T>::load(p + g * a.br * a.ldc);
        finish_col<T>(a, C, r, j, s, ratio, excl);
    }
    fold_block(ratio, excl, &a.rep->max_ratio_c, &a.rep->n_excl_c);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vcol_partial(const T *C, VerifyArgs a, int64_t P, int64_t chunk, double *part) {
    const int64_t rel = a.br * a.N, total = P * rel;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t p = t / rel, q = t - p * rel;
        int64_t r = q / a.N, j = q - r * a.N;
        int64_t g0 = p * chunk, g1 = min(a.Gr, g0 + chunk);
        const T *src = C + r * a.ldc + j;
        double s = 0.0;
        for (int64_t g = g0; g < g1; ++g) s += elem<T>::load(src + g * a.br * a.ldc);
        part[t] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vcol_finish(const T *C, VerifyArgs a, int64_t P, const double *part) {
    const int64_t rel = a.br * a.N;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < rel; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / a.N, j = t - r * a.N;
        double s = 0.0;
        for (int64_t p = 0; p < P; ++p) s += part[p * rel + t];
        finish_col<T>(a, C, r, j, s, ratio, excl);
    }
    fold_block(ratio, excl, &a.rep->max_ratio_c, &a.rep->n_excl_c);
}

// Row relation (i, c): sum_{h<Gc} C[i, h*bc + c] - sum_{s<S} C[i, n + s*bc + c]
template <typename T>
__device__ inline void finish_row(const VerifyArgs &a, const T *C, int64_t i, int64_t c, double s, double &ratio,
                                  unsigned long long &excl) {
    double tot = 0.0;
    for (int64_t q = 0; q < a.S; ++q) tot += elem<T>::load(C + i * a.ldc + a.n + q * a.bc + c);
    if (row_rel_erased(a.er, i, c, a.bc)) { excl++; return; }
    ratio = fmax(ratio, record(a.rep, false, i, c, s - tot, tau_row(a, i, c)));
}

// One thread per row relation; lanes take consecutive c (coalesced when bc >= 64).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vrow_strided(const T *C, VerifyArgs a) {
    const int64_t total = a.M * a.bc;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t i = t / a.bc, c = t - i * a.bc;
        const T *p = C + i * a.ldc + c;
        double s = 0.0;
        for (int64_t h = 0; h < a.Gc; ++h) s += elem<T>::load(p + h * a.bc);
        finish_row<T>(a, C, i, c, s, ratio, excl);
    }
    fold_block(ratio, excl, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

// One block per row for bc dividing 256: thread t sums the columns j = t mod 256,
// all of residue t mod bc; a fixed-order tree then combines the 256/bc partial
// sums of each residue.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vrow_block(const T *C, VerifyArgs a) {
    __shared__ double sh[kThreads];
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t i = blockIdx.x; i < a.M; i += gridDim.x) {
        const T *row = C + i * a.ldc;
        double s0 = 0.0, s1 = 0.0;
        int64_t j = threadIdx.x;
        for (; j + kThreads < a.n; j += 2 * kThreads) {
            s0 += elem<T>::load(row + j);
            s1 += elem<T>::load(row + j + kThreads);
        }
        if (j < a.n) s0 += elem<T>::load(row + j);
        sh[threadIdx.x] = s0 + s1;
        __syncthreads();
        for (int w = kThreads / 2; w >= a.bc; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x < a.bc) finish_row<T>(a, C, i, threadIdx.x, sh[threadIdx.x], ratio, excl);
        __syncthreads();
    }
    fold_block(ratio, excl, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

template <typename T>
static int verify_typed(const abft_problem *p, const T *C, const Erasures &er, char *ws, hipStream_t s) {
    Geom g = geom_of(p);
    WsLayout L = ws_layout(p);
    TauCoef tc = tau_coef(p);
    VerifyArgs a;
    a.m = g.m; a.n = g.n; a.br = g.br; a.bc = g.bc; a.S = g.S; a.Gr = g.Gr; a.Gc = g.Gc; a.M = g.M; a.N = g.N;
    a.ldc = p->ldc;
    a.mode = tc.mode; a.cc = tc.cc; a.cr = tc.cr;
    a.na = (const double *)(ws + L.na); a.na_abs = (const double *)(ws + L.na_abs);
    a.nb = (const double *)(ws + L.nb); a.nb_abs = (const double *)(ws + L.nb_abs);
    a.rep = (abft_report *)(ws + L.report);
    a.er = er;
    k_report_init<<<1, kThreads, 0, s>>>(a.rep);
    auto blocks = [](int64_t work) { return (unsigned)std::min<int64_t>((work + kThreads - 1) / kThreads, 4096); };
    int64_t P = group_partitions(g.Gr, g.br, g.N);
    if (P == 1) {
        k_vcol_direct<T><<<blocks(g.br * g.N), kThreads, 0, s>>>(C, a);
    } else {
        int64_t chunk = (g.Gr + P - 1) / P;
        P = (g.Gr + chunk - 1) / chunk;
        double *part = (double *)(ws + L.partial);
        k_vcol_partial<T><<<blocks(P * g.br * g.N), kThreads, 0, s>>>(C, a, P, chunk, part);
        k_vcol_finish<T><<<blocks(g.br * g.N), kThreads, 0, s>>>(C, a, P, part);
    }
    if (g.bc < 64 && (kThreads % g.bc) == 0)
        k_vrow_block<T><<<(unsigned)std::min<int64_t>(g.M, 8192), kThreads, 0, s>>>(C, a);
    else
        k_vrow_strided<T><<<blocks(g.M * g.bc), kThreads, 0, s>>>(C, a);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_verify(const abft_problem *p, const void *C_f, const Erasures &er, char *ws, hipStream_t s) {
    if (p->dtype == ABFT_F64) return verify_typed<double>(p, (const double *)C_f, er, ws, s);
    return verify_typed<float>(p, (const float *)C_f, er, ws, s);
}

}  // namespace abft
