// Weighted f-checksums (Sec. 2.1) on the block product (Sec. 2.2), binary64 or
// binary32 operands and C_f: encoding, threshold statistics, verification of
// every column and row group, location from the weight ratios of a group, and
// the f x f recovery of lost blocks.  Every sum is accumulated in binary64 over
// the blocks in increasing order; a stored result is rounded once to the
// element type.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace abft {
namespace {

constexpr int kT = 256;
constexpr int kW = 64;
constexpr int FM = ABFT_WMAX;
constexpr int64_t kSkinnyN = 8;    // products with at most this many columns stream A_f once

struct WGeom {
    int64_t m, n, k, br, bc, Gr, Gc, M, N, lda, ldb, ldc;
    int fr, fc;
    int dtype;        // ABFT_F64 or ABFT_F32
    int64_t V;        // elements per 16-byte load: 2, 4
};

WGeom wgeom(const abft_wproblem *p) {
    WGeom g;
    g.m = p->p.m; g.n = p->p.n; g.k = p->p.k; g.br = p->p.br; g.bc = p->p.bc;
    g.fr = p->fr; g.fc = p->fc;
    g.Gr = g.m / g.br; g.Gc = g.n / g.bc;
    g.M = g.m + g.fr * g.br; g.N = g.n + g.fc * g.bc;
    g.lda = p->p.lda; g.ldb = p->p.ldb; g.ldc = p->p.ldc;
    g.dtype = p->p.dtype;
    g.V = g.dtype == ABFT_F64 ? 2 : 4;
    return g;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WLayout {
    size_t wr, wc, na, nb, s1, s2, part, report, total;
};

// Partitions of a (G blocks x rel relations) sum: independent sums enough to
// fill the chip; one partition sums a contiguous run of blocks in order.
int64_t parts(int64_t G, int64_t rel) {
    int64_t P = ((int64_t(1) << 19) + rel - 1) / rel;
    return std::max<int64_t>(1, std::min(P, G));
}

WLayout wlayout(const WGeom &g) {
    WLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += al256(bytes); return o; };
    L.wr = take(sizeof(double) * g.fr * g.Gr);
    L.wc = take(sizeof(double) * g.fc * g.Gc);
    L.na = take(sizeof(double) * g.M);
    L.nb = take(sizeof(double) * g.N);
    L.s1 = take(sizeof(double) * g.fr * g.br);
    L.s2 = take(sizeof(double) * g.fc * g.bc);
    int64_t kv = g.k / g.V;
    size_t pa = 0;
    int64_t P = parts(g.Gr, g.br * kv);
    if (P > 1) pa = std::max(pa, (size_t)(P * g.fr * g.br * g.k));
    P = parts(g.Gc, g.bc * kv);
    if (P > 1) pa = std::max(pa, (size_t)(P * g.fc * g.bc * g.k));
    P = parts(g.Gr, g.br * g.N);
    if (P > 1) pa = std::max(pa, (size_t)(P * g.fr * g.br * g.N));
    L.part = take(sizeof(double) * std::max<size_t>(pa, 1));
    L.report = take(sizeof(abft_wreport));
    L.total = off;
    return L;
}

// ------------------------------------------------------------------ wave helpers
__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = kW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wmax(double v) {
#pragma unroll
    for (int o = kW / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ inline unsigned long long wsum_u(unsigned long long v) {
#pragma unroll
    for (int o = kW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// One atomic per block for the max ratio (non-negative doubles order as their
// bits) and the exclusions; every thread of the block must call it.
__device__ inline void fold_block(double ratio, unsigned long long excl, double *rep_ratio, int64_t *rep_excl) {
    __shared__ double s_r[kT / kW];
    __shared__ unsigned long long s_e[kT / kW];
    ratio = wmax(ratio);
    excl = wsum_u(excl);
    const int lane = threadIdx.x % kW, w = threadIdx.x / kW;
    if (lane == 0) { s_r[w] = ratio; s_e[w] = excl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kT / kW; ++q) { ratio = fmax(ratio, s_r[q]); excl += s_e[q]; }
        if (ratio > 0) atomicMax((unsigned long long *)rep_ratio, (unsigned long long)__double_as_longlong(ratio));
        if (excl) atomicAdd((unsigned long long *)rep_excl, excl);
    }
}

__device__ inline bool fails(double d, double t) { return !(fabs(d) <= t); }

// Record a group if one of its relations fails; returns its largest finite |D|/tau.
template <int F>
__device__ inline double group(abft_wreport *rep, bool col, int64_t a, int64_t b, const double *d,
                               const double *t) {
    bool bad = false;
    double ratio = 0.0;
#pragma unroll
    for (int r = 0; r < F; ++r) {
        bad |= fails(d[r], t[r]);
        if (isfinite(d[r]) && t[r] > 0) ratio = fmax(ratio, fabs(d[r]) / t[r]);
    }
    if (bad) {
        unsigned long long q = atomicAdd((unsigned long long *)(col ? &rep->n_fail_c : &rep->n_fail_r), 1ull);
        if (q < ABFT_MAX_FLAGS) {
            abft_wgroup *gp = col ? &rep->col[q] : &rep->row[q];
            gp->a = a; gp->b = b;
#pragma unroll
            for (int r = 0; r < ABFT_WMAX; ++r) {
                gp->d[r] = r < F ? d[r] : 0.0;
                gp->tau[r] = r < F ? t[r] : 0.0;
            }
        }
    }
    return ratio;
}

// ------------------------------------------------------------------ encoding
// Elements are binary64 or binary32 (T); every sum is taken in binary64 and a
// stored result is rounded once to T.  V = elements per 16-byte load.
template <typename T> __device__ inline double ld(const T *p) { return (double)*p; }

// Checksum rows out[r*b + i, l] = sum_g W[r][g] X[g*b + i, l] for the blocks
// [g0, g1); X has rows of k elements (16-byte aligned, k a multiple of V).
// P == 1: outT is the checksum rows (row r*b + i, leading dimension ldo),
// rounded to T; P > 1: part is the binary64 partial buffer, partition p at
// p*rstride.
template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wenc(const T *__restrict__ X, int64_t ld_, int64_t b, int64_t G, int64_t k,
                                             const double *__restrict__ W, int64_t P, int64_t chunk,
                                             T *__restrict__ outT, double *__restrict__ part, int64_t ldo,
                                             int64_t rstride) {
    constexpr int V = vec16<T>::N;
    const int64_t kv = k / V, total = P * b * kv;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        const int64_t p = t / (b * kv), q = t - p * (b * kv);
        const int64_t i = q / kv, l = (q - i * kv) * V;
        const int64_t g0 = p * chunk, g1 = min(G, g0 + chunk);
        double s[F][V];
#pragma unroll
        for (int r = 0; r < F; ++r)
#pragma unroll
            for (int e = 0; e < V; ++e) s[r][e] = 0.0;
        for (int64_t g = g0; g < g1; ++g) {
            double v[V];
            vec16<T>::load(X + (g * b + i) * ld_ + l, v);
#pragma unroll
            for (int r = 0; r < F; ++r) {
                const double w = W[r * G + g];
#pragma unroll
                for (int e = 0; e < V; ++e) s[r][e] += w * v[e];
            }
        }
        if (P == 1) {
#pragma unroll
            for (int r = 0; r < F; ++r)
#pragma unroll
                for (int e = 0; e < V; ++e) outT[(r * b + i) * ldo + l + e] = (T)s[r][e];
        } else {
            double *o = part + p * rstride;
#pragma unroll
            for (int r = 0; r < F; ++r)
#pragma unroll
                for (int e = 0; e < V; ++e) o[(r * b + i) * k + l + e] = s[r][e];
        }
    }
}

// Sum the partitions in order: out[e] = sum_p part[p*rows*k + e], e over rows x k, rounded once to T.
template <typename T>
__global__ __launch_bounds__(kT) void k_wpart_sum(const double *__restrict__ part, int64_t P, int64_t rows, int64_t k,
                                                  T *__restrict__ out, int64_t ldo) {
    const int64_t total = rows * k;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        double s = 0.0;
        for (int64_t p = 0; p < P; ++p) s += part[p * total + t];
        const int64_t x = t / k, l = t - x * k;
        out[x * ldo + l] = (T)s;
    }
}

// ||X[x, :]||_2 for each of rows rows: one wave per row, binary64.
template <typename T>
__global__ __launch_bounds__(kT) void k_wnorm(const T *__restrict__ X, int64_t ld_, int64_t rows, int64_t k,
                                              double *__restrict__ out) {
    constexpr int V = vec16<T>::N;
    const int lane = threadIdx.x % kW;
    const int64_t w0 = ((int64_t)blockIdx.x * kT + threadIdx.x) / kW, nw = (int64_t)gridDim.x * kT / kW;
    for (int64_t x = w0; x < rows; x += nw) {
        const T *row = X + x * ld_;
        double s = 0.0;
        for (int64_t l = V * lane; l < k; l += V * kW) {
            double v[V];
            vec16<T>::load(row + l, v);
#pragma unroll
            for (int e = 0; e < V; ++e) s += v[e] * v[e];
        }
        s = wsum(s);
        if (lane == 0) out[x] = sqrt(s);
    }
}

// S[r*b + i] = sum_g |W[r][g]| nrm[g*b + i]
__global__ __launch_bounds__(kT) void k_wsumnorm(const double *__restrict__ W, int f, int64_t G, int64_t b,
                                                 const double *__restrict__ nrm, double *__restrict__ S) {
    const int64_t total = f * b;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        const int64_t r = t / b, i = t - r * b;
        double s = 0.0;
        for (int64_t g = 0; g < G; ++g) s += fabs(W[r * G + g]) * nrm[g * b + i];
        S[t] = s;
    }
}

// ------------------------------------------------------------------ verification
struct VArgs {
    const double *wr, *wc, *na, *nb, *s1, *s2;
    int64_t m, n, br, bc, Gr, Gc, M, N, ldc;
    double cc, cr;        // threshold coefficients (0 for exact)
    Erasures er;
    abft_wreport *rep;
};

__global__ void k_wreport_init(abft_wreport *rep) {
    if (threadIdx.x == 0) {
        rep->n_fail_c = rep->n_fail_r = rep->n_excl_c = rep->n_excl_r = 0;
        rep->max_ratio_c = rep->max_ratio_r = 0.0;
    }
}

// Column group (i, j): s[r] = sum_g wr[r][g] C[g*br + i, j] (given), then the checksum entries.
template <int F, typename T>
__device__ inline void col_finish(const VArgs &a, const T *C, int64_t i, int64_t j, const double *s, double &ratio,
                                  unsigned long long &excl) {
    if (col_rel_erased(a.er, i, j, a.br)) { excl++; return; }
    double d[F], t[F];
#pragma unroll
    for (int r = 0; r < F; ++r) {
        d[r] = s[r] - ld(C + (a.m + r * a.br + i) * a.ldc + j);
        t[r] = a.cc * a.s1[r * a.br + i] * a.nb[j];
    }
    ratio = fmax(ratio, group<F>(a.rep, true, i, j, d, t));
}

// Direct: one thread per (i, V consecutive columns), all Gr blocks; the block
// loop is unrolled so several rows are in flight.  vec: rows of C_f start on
// 16-byte boundaries (C aligned, ldc a multiple of V).
template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wvcol(const T *__restrict__ C, VArgs a, int vec) {
    constexpr int V = vec16<T>::N;
    const int64_t NP = (a.N + V - 1) / V, total = a.br * NP;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        const int64_t i = t / NP, j = (t - i * NP) * V;
        const int cnt = (int)min((int64_t)V, a.N - j);
        double s[F][V];
#pragma unroll
        for (int r = 0; r < F; ++r)
#pragma unroll
            for (int e = 0; e < V; ++e) s[r][e] = 0.0;
        const T *col = C + i * a.ldc + j;
        if (cnt == V && vec) {
#pragma unroll 4
            for (int64_t g = 0; g < a.Gr; ++g) {
                double v[V];
                vec16<T>::load(col + g * a.br * a.ldc, v);
#pragma unroll
                for (int r = 0; r < F; ++r)
#pragma unroll
                    for (int e = 0; e < V; ++e) s[r][e] += a.wr[r * a.Gr + g] * v[e];
            }
        } else {
#pragma unroll 4
            for (int64_t g = 0; g < a.Gr; ++g) {
                const T *e0 = col + g * a.br * a.ldc;
                double v[V];
#pragma unroll
                for (int e = 0; e < V; ++e) v[e] = e < cnt ? ld(e0 + e) : 0.0;
#pragma unroll
                for (int r = 0; r < F; ++r)
#pragma unroll
                    for (int e = 0; e < V; ++e) s[r][e] += a.wr[r * a.Gr + g] * v[e];
            }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (e < cnt) {
                double se[F];
#pragma unroll
                for (int r = 0; r < F; ++r) se[r] = s[r][e];
                col_finish<F, T>(a, C, i, j + e, se, ratio, excl);
            }
        }
    }
    fold_block(ratio, excl, &a.rep->max_ratio_c, &a.rep->n_excl_c);
}

// Partitioned: partial sums of a run of blocks per (p, i, j), then the finish.
template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wvcol_part(const T *__restrict__ C, VArgs a, int64_t P, int64_t chunk,
                                                   double *__restrict__ part) {
    const int64_t rel = a.br * a.N, total = P * rel;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        const int64_t p = t / rel, q = t - p * rel;
        const int64_t i = q / a.N, j = q - i * a.N;
        const int64_t g0 = p * chunk, g1 = min(a.Gr, g0 + chunk);
        double s[F];
#pragma unroll
        for (int r = 0; r < F; ++r) s[r] = 0.0;
        for (int64_t g = g0; g < g1; ++g) {
            const double v = ld(C + (g * a.br + i) * a.ldc + j);
#pragma unroll
            for (int r = 0; r < F; ++r) s[r] += a.wr[r * a.Gr + g] * v;
        }
#pragma unroll
        for (int r = 0; r < F; ++r) part[(p * F + r) * rel + q] = s[r];
    }
}
template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wvcol_fin(const T *__restrict__ C, VArgs a, int64_t P,
                                                  const double *__restrict__ part) {
    const int64_t rel = a.br * a.N;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < rel; t += (int64_t)gridDim.x * kT) {
        const int64_t i = t / a.N, j = t - i * a.N;
        double s[F];
#pragma unroll
        for (int r = 0; r < F; ++r) {
            s[r] = 0.0;
            for (int64_t p = 0; p < P; ++p) s[r] += part[(p * F + r) * rel + t];
        }
        col_finish<F, T>(a, C, i, j, s, ratio, excl);
    }
    fold_block(ratio, excl, &a.rep->max_ratio_c, &a.rep->n_excl_c);
}

template <int F, typename T>
__device__ inline void row_finish(const VArgs &a, const T *C, int64_t x, int64_t jj, const double *s,
                                  double &ratio, unsigned long long &excl) {
    if (row_rel_erased(a.er, x, jj, a.bc)) { excl++; return; }
    double d[F], t[F];
#pragma unroll
    for (int c = 0; c < F; ++c) {
        d[c] = s[c] - ld(C + x * a.ldc + a.n + c * a.bc + jj);
        t[c] = a.cr * a.na[x] * a.s2[c * a.bc + jj];
    }
    ratio = fmax(ratio, group<F>(a.rep, false, x, jj, d, t));
}

// Row groups, wide blocks (bc >= 64, a multiple of V): one thread per (x, V
// consecutive residues), consecutive threads read consecutive columns; the
// block loop is unrolled.
template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wvrow_thread(const T *__restrict__ C, VArgs a, int vec) {
    constexpr int V = vec16<T>::N;
    const int64_t BP = a.bc / V, total = a.M * BP;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        const int64_t x = t / BP, jj = (t - x * BP) * V;
        const T *row = C + x * a.ldc + jj;
        double s[F][V];
#pragma unroll
        for (int c = 0; c < F; ++c)
#pragma unroll
            for (int e = 0; e < V; ++e) s[c][e] = 0.0;
#pragma unroll 4
        for (int64_t h = 0; h < a.Gc; ++h) {
            double v[V];
            if (vec) {
                vec16<T>::load(row + h * a.bc, v);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) v[e] = ld(row + h * a.bc + e);
            }
#pragma unroll
            for (int c = 0; c < F; ++c)
#pragma unroll
                for (int e = 0; e < V; ++e) s[c][e] += a.wc[c * a.Gc + h] * v[e];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            double se[F];
#pragma unroll
            for (int c = 0; c < F; ++c) se[c] = s[c][e];
            row_finish<F, T>(a, C, x, jj + e, se, ratio, excl);
        }
    }
    fold_block(ratio, excl, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

// Row groups, narrow blocks: one wave per (x, jj), the lanes split the Gc
// blocks (lane l takes h = l, l + 64, ...), wave-tree sum.
template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wvrow_wave(const T *__restrict__ C, VArgs a) {
    const int lane = threadIdx.x % kW;
    const int64_t total = a.M * a.bc;
    const int64_t w0 = ((int64_t)blockIdx.x * kT + threadIdx.x) / kW, nw = (int64_t)gridDim.x * kT / kW;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = w0; t < total; t += nw) {
        const int64_t x = t / a.bc, jj = t - x * a.bc;
        const T *row = C + x * a.ldc + jj;
        double s[F];
#pragma unroll
        for (int c = 0; c < F; ++c) s[c] = 0.0;
        for (int64_t h = lane; h < a.Gc; h += kW) {
            const double v = ld(row + h * a.bc);
#pragma unroll
            for (int c = 0; c < F; ++c) s[c] += a.wc[c * a.Gc + h] * v;
        }
#pragma unroll
        for (int c = 0; c < F; ++c) s[c] = wsum(s[c]);
        if (lane == 0) row_finish<F, T>(a, C, x, jj, s, ratio, excl);
    }
    fold_block(ratio, excl, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

// ------------------------------------------------------------------ recovery
// Rebuild of lost members along lines (columns for the column direction,
// rows for the row direction).  Line pos in [lo, lo + len), residue i in
// [i0, i1): member g of its group is element g*b + i of the line (checksum
// block r is member G + r, at base + r*b + i).  Lost data members U (nu of
// them) are solved from the intact checksum relations R with the host's
// inverse Wi of W[R][U]; then the lost checksum members Lc are recomputed.
// Solved and recomputed values are binary64, rounded once when stored as T.
struct RArgs {
    const double *W;          // f x G weights
    int64_t G, b, base, ldc, lo, len, i0, i1;
    int f, nu, nl, dir;
    int U[FM], R[FM], Lc[FM];
    double Wi[FM * FM];
};

__device__ inline int64_t elem_at(const RArgs &a, int64_t pos, int64_t along) {
    return a.dir == ABFT_DIR_COL ? along * a.ldc + pos : pos * a.ldc + along;
}

template <int F, typename T>
__global__ __launch_bounds__(kT) void k_wrecover(T *__restrict__ C, RArgs a) {
    const int64_t nres = a.i1 - a.i0, total = nres * a.len;
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        // column direction: consecutive threads take consecutive columns; row direction: consecutive residues
        int64_t pos, i;
        if (a.dir == ABFT_DIR_COL) { i = a.i0 + t / a.len; pos = a.lo + t % a.len; }
        else { pos = a.lo + t / nres; i = a.i0 + t % nres; }
        double S[F];
#pragma unroll
        for (int r = 0; r < F; ++r) S[r] = 0.0;
        for (int64_t g = 0; g < a.G; ++g) {
            bool lost = false;
            for (int u = 0; u < a.nu; ++u) lost |= (a.U[u] == g);
            if (lost) continue;
            const double v = ld(C + elem_at(a, pos, g * a.b + i));
#pragma unroll
            for (int r = 0; r < F; ++r) S[r] += a.W[r * a.G + g] * v;
        }
        if (a.nu > 0) {
            double rhs[FM], x[FM];
            for (int q = 0; q < a.nu; ++q) {
                double acc = 0.0;
#pragma unroll
                for (int r = 0; r < F; ++r) acc = (r == a.R[q]) ? S[r] : acc;
                rhs[q] = ld(C + elem_at(a, pos, a.base + a.R[q] * a.b + i)) - acc;
            }
            for (int u = 0; u < a.nu; ++u) {
                double v = 0.0;
                for (int q = 0; q < a.nu; ++q) v += a.Wi[u * FM + q] * rhs[q];
                x[u] = v;
            }
            for (int u = 0; u < a.nu; ++u) {
                const T stored = (T)x[u];
                C[elem_at(a, pos, a.U[u] * a.b + i)] = stored;
#pragma unroll
                for (int r = 0; r < F; ++r) S[r] += a.W[r * a.G + a.U[u]] * (double)stored;
            }
        }
        for (int q = 0; q < a.nl; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < F; ++r) acc = (r == a.Lc[q]) ? S[r] : acc;
            C[elem_at(a, pos, a.base + a.Lc[q] * a.b + i)] = (T)acc;
        }
    }
}

unsigned grid(int64_t work) { return (unsigned)std::min<int64_t>(std::max<int64_t>((work + kT - 1) / kT, 1), 65536); }
// Verification grids: enough blocks to fill the chip (8 waves per SIMD), few
// enough that the one atomic per block stays cheap.
unsigned vgrid(int64_t work) { return std::min<unsigned>(grid(work), 2048); }

// Run STMT with the compile-time checksum count F = fv (1..ABFT_WMAX).
#define WSWITCH(fv, STMT)                                 \
    switch (fv) {                                         \
    case 1: { constexpr int F = 1; STMT; } break;         \
    case 2: { constexpr int F = 2; STMT; } break;         \
    case 3: { constexpr int F = 3; STMT; } break;         \
    default: { constexpr int F = 4; STMT; } break;        \
    }

// ------------------------------------------------------------------ host checks
int check_wproblem(const abft_wproblem *p) {
    if (!p) return ABFT_E_ARG;
    const abft_problem &q = p->p;
    if (q.dtype != ABFT_F64 && q.dtype != ABFT_F32) return ABFT_E_UNSUPPORTED;
    if (q.tau_mode != ABFT_TAU_DET && q.tau_mode != ABFT_TAU_EXACT) return ABFT_E_UNSUPPORTED;
    if (q.m < 1 || q.n < 1 || q.k < 1 || q.br < 1 || q.bc < 1) return ABFT_E_ARG;
    if (q.br > q.m || q.bc > q.n || q.m % q.br || q.n % q.bc) return ABFT_E_ARG;
    if (p->fr < 1 || p->fr > ABFT_WMAX || p->fc < 1 || p->fc > ABFT_WMAX) return ABFT_E_ARG;
    const int64_t V = q.dtype == ABFT_F64 ? 2 : 4;     // elements per 16-byte load
    if (q.k % V || q.lda < q.k || q.ldb < q.k || q.lda % V || q.ldb % V) return ABFT_E_ARG;
    if (q.ldc < q.n + p->fc * q.bc) return ABFT_E_ARG;
    if (!p->wr || !p->wc) return ABFT_E_ARG;
    const int64_t Gr = q.m / q.br, Gc = q.n / q.bc;
    for (int64_t e = 0; e < p->fr * Gr; ++e)
        if (!std::isfinite(p->wr[e])) return ABFT_E_ARG;
    for (int64_t e = 0; e < p->fc * Gc; ++e)
        if (!std::isfinite(p->wc[e])) return ABFT_E_ARG;
    return ABFT_OK;
}

bool aligned16(const void *x) { return ((uintptr_t)x & 15u) == 0; }

double gam(double n, double u = std::ldexp(1.0, -53)) { return n * u / (1.0 - n * u); }

// Inverse of the s x s matrix A (row-major, s <= 4) by Gauss-Jordan with
// partial pivoting; false if singular or its 1-norm condition number exceeds 1e12.
bool invert_small(int s, const double *A, double *Ainv) {
    double a[FM][2 * FM];
    for (int r = 0; r < s; ++r)
        for (int c = 0; c < 2 * s; ++c) a[r][c] = c < s ? A[r * s + c] : (c - s == r ? 1.0 : 0.0);
    for (int c = 0; c < s; ++c) {
        int piv = c;
        for (int r = c + 1; r < s; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return false;
        if (piv != c)
            for (int q = 0; q < 2 * s; ++q) std::swap(a[c][q], a[piv][q]);
        const double d = a[c][c];
        for (int q = 0; q < 2 * s; ++q) a[c][q] /= d;
        for (int r = 0; r < s; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f == 0.0) continue;
            for (int q = 0; q < 2 * s; ++q) a[r][q] -= f * a[c][q];
        }
    }
    double n1 = 0.0, ni = 0.0;
    for (int c = 0; c < s; ++c) {
        double cs = 0.0, ci = 0.0;
        for (int r = 0; r < s; ++r) {
            cs += std::fabs(A[r * s + c]);
            ci += std::fabs(a[r][s + c]);
        }
        n1 = std::max(n1, cs);
        ni = std::max(ni, ci);
    }
    if (!(n1 * ni <= 1e12)) return false;
    for (int r = 0; r < s; ++r)
        for (int c = 0; c < s; ++c) Ainv[r * FM + c] = a[r][s + c];
    return true;
}

// Fill RArgs for lost blocks `lost` (sorted, distinct) of one direction.
int recover_args(const abft_wproblem *p, const WGeom &g, const WLayout &L, char *ws, int dir,
                 const std::vector<int> &lost, RArgs &a) {
    const int f = dir == ABFT_DIR_COL ? g.fr : g.fc;
    const int64_t G = dir == ABFT_DIR_COL ? g.Gr : g.Gc;
    const double *Wh = dir == ABFT_DIR_COL ? p->wr : p->wc;
    a.W = (const double *)(ws + (dir == ABFT_DIR_COL ? L.wr : L.wc));
    a.G = G; a.b = dir == ABFT_DIR_COL ? g.br : g.bc; a.base = dir == ABFT_DIR_COL ? g.m : g.n;
    a.ldc = g.ldc; a.f = f; a.dir = dir;
    a.nu = a.nl = 0;
    for (int x : lost) {
        if (x < 0 || x >= G + f) return ABFT_E_ARG;
        if (x < G) a.U[a.nu++] = x;
        else a.Lc[a.nl++] = x - (int)G;
    }
    int nr = 0;
    for (int r = 0; r < f && nr < a.nu; ++r) {
        bool gone = false;
        for (int q = 0; q < a.nl; ++q) gone |= a.Lc[q] == r;
        if (!gone) a.R[nr++] = r;
    }
    if (nr < a.nu) return ABFT_E_UNRECOVERABLE;
    if (a.nu > 0) {
        double Ws[FM * FM];
        for (int q = 0; q < a.nu; ++q)
            for (int u = 0; u < a.nu; ++u) Ws[q * a.nu + u] = Wh[a.R[q] * G + a.U[u]];
        if (!invert_small(a.nu, Ws, a.Wi)) return ABFT_E_UNRECOVERABLE;
    }
    return ABFT_OK;
}

template <typename T>
int launch_recover(T *C, const RArgs &a, hipStream_t s) {
    const int64_t work = (a.i1 - a.i0) * a.len;
    if (work <= 0) return ABFT_OK;
    WSWITCH(a.f, (k_wrecover<F, T><<<grid(work), kT, 0, s>>>(C, a)));
    ABFT_LAUNCHED();
    return ABFT_OK;
}
int launch_recover_any(int dtype, void *C, const RArgs &a, hipStream_t s) {
    return dtype == ABFT_F64 ? launch_recover((double *)C, a, s) : launch_recover((float *)C, a, s);
}

// Weighted checksum rows of one operand (rows of A_f, or rows of B_f^T):
// out = X + G*b*ld, one pass (P == 1) or binary64 partial sums then their
// ordered sum; stored rounded once to T.
template <typename T>
int encode_side(const T *X, int64_t ld_, int64_t G, int64_t b, int64_t k, int f, const double *W, double *part,
                hipStream_t s) {
    T *out = const_cast<T *>(X) + G * b * ld_;
    const int64_t kv = k / vec16<T>::N;
    int64_t P = parts(G, b * kv);
    if (P == 1) {
        WSWITCH(f, (k_wenc<F, T><<<grid(b * kv), kT, 0, s>>>(X, ld_, b, G, k, W, 1, G, out, nullptr, ld_, 0)));
    } else {
        const int64_t chunk = (G + P - 1) / P;
        P = (G + chunk - 1) / chunk;
        WSWITCH(f, (k_wenc<F, T><<<grid(P * b * kv), kT, 0, s>>>(X, ld_, b, G, k, W, P, chunk, nullptr, part, ld_,
                                                                  f * b * k)));
        k_wpart_sum<T><<<grid(f * b * k), kT, 0, s>>>(part, P, f * b, k, out, ld_);
    }
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int to_werasures(const WGeom &g, const abft_rect *known, int n_known, Erasures *er) {
    if (n_known < 0 || n_known > 4 || (n_known > 0 && !known)) return ABFT_E_ARG;
    er->n = n_known;
    for (int q = 0; q < n_known; ++q) {
        const abft_rect &e = known[q];
        if (e.h < 1 || e.w < 1 || e.i0 < 0 || e.j0 < 0 || e.i0 + e.h > g.M || e.j0 + e.w > g.N) return ABFT_E_ARG;
        er->i0[q] = e.i0; er->j0[q] = e.j0; er->h[q] = e.h; er->w[q] = e.w;
    }
    return ABFT_OK;
}

// Location of one failed group (host): DATA with its member, CHECKSUM with
// its checksum index, or MULTI.
int fit_group(const abft_wgroup &gp, int f, int64_t G, const double *W, int64_t *q) {
    for (int r = 0; r < f; ++r)
        if (!std::isfinite(gp.d[r])) return ABFT_CLS_MULTI;
    int failed[FM], nf = 0;
    for (int r = 0; r < f; ++r)
        if (!(std::fabs(gp.d[r]) <= gp.tau[r])) failed[nf++] = r;
    if (nf == 1 && f >= 2) { *q = failed[0]; return ABFT_CLS_CHECKSUM; }
    if (nf < 2) return ABFT_CLS_MULTI;
    const double eps = 4.0 * (double)(G + 2) * std::ldexp(1.0, -53);
    int64_t found = -1, n_found = 0;
    for (int64_t g = 0; g < G; ++g) {
        double ww = 0.0, wd = 0.0;
        for (int r = 0; r < f; ++r) {
            ww += W[r * G + g] * W[r * G + g];
            wd += W[r * G + g] * gp.d[r];
        }
        const double delta = wd / ww;
        bool fit = true;
        for (int r = 0; r < f && fit; ++r) {
            const double e = W[r * G + g] * delta;
            fit = std::fabs(gp.d[r] - e) <= gp.tau[r] + eps * (std::fabs(gp.d[r]) + std::fabs(e));
        }
        if (fit) { found = g; ++n_found; }
    }
    if (n_found != 1) return ABFT_CLS_MULTI;
    *q = found;
    return ABFT_CLS_DATA;
}

}  // namespace
}  // namespace abft

using namespace abft;

extern "C" {

// A workspace must be present and at least the problem's workspace size.
static int check_wws(const abft_wproblem *p, const void *ws, size_t ws_bytes) {
    if (!ws || ws_bytes < wlayout(wgeom(p)).total) return ABFT_E_WORKSPACE;
    return ABFT_OK;
}

size_t abft_wworkspace_size(const abft_wproblem *p) {
    if (check_wproblem(p) != ABFT_OK) return 0;
    return wlayout(wgeom(p)).total;
}

int abft_wsetup(const abft_wproblem *p, void *ws, size_t ws_bytes) {
    int st = check_wproblem(p);
    if (st) return st;
    if ((st = check_wws(p, ws, ws_bytes))) return st;
    const WGeom g = wgeom(p);
    const WLayout L = wlayout(g);
    ABFT_HIP(hipMemcpy((char *)ws + L.wr, p->wr, sizeof(double) * g.fr * g.Gr, hipMemcpyHostToDevice));
    ABFT_HIP(hipMemcpy((char *)ws + L.wc, p->wc, sizeof(double) * g.fc * g.Gc, hipMemcpyHostToDevice));
    return ABFT_OK;
}

int abft_wencode(const abft_wproblem *p, void *A_f, void *B_f, void *ws, size_t ws_bytes, void *stream) {
    int st = check_wproblem(p);
    if (st) return st;
    if (!A_f || !B_f || !aligned16(A_f) || !aligned16(B_f)) return ABFT_E_ARG;
    if ((st = check_wws(p, ws, ws_bytes))) return st;
    const WGeom g = wgeom(p);
    const WLayout L = wlayout(g);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    double *part = (double *)(w + L.part);
    const double *wr = (const double *)(w + L.wr), *wc = (const double *)(w + L.wc);
    if (g.dtype == ABFT_F64) {
        if ((st = encode_side((const double *)A_f, g.lda, g.Gr, g.br, g.k, g.fr, wr, part, s))) return st;
        if ((st = encode_side((const double *)B_f, g.ldb, g.Gc, g.bc, g.k, g.fc, wc, part, s))) return st;
        k_wnorm<double><<<grid(g.M * kW), kT, 0, s>>>((const double *)A_f, g.lda, g.M, g.k, (double *)(w + L.na));
        k_wnorm<double><<<grid(g.N * kW), kT, 0, s>>>((const double *)B_f, g.ldb, g.N, g.k, (double *)(w + L.nb));
    } else {
        if ((st = encode_side((const float *)A_f, g.lda, g.Gr, g.br, g.k, g.fr, wr, part, s))) return st;
        if ((st = encode_side((const float *)B_f, g.ldb, g.Gc, g.bc, g.k, g.fc, wc, part, s))) return st;
        k_wnorm<float><<<grid(g.M * kW), kT, 0, s>>>((const float *)A_f, g.lda, g.M, g.k, (double *)(w + L.na));
        k_wnorm<float><<<grid(g.N * kW), kT, 0, s>>>((const float *)B_f, g.ldb, g.N, g.k, (double *)(w + L.nb));
    }
    k_wsumnorm<<<grid(g.fr * g.br), kT, 0, s>>>((const double *)(w + L.wr), g.fr, g.Gr, g.br,
                                                (const double *)(w + L.na), (double *)(w + L.s1));
    k_wsumnorm<<<grid(g.fc * g.bc), kT, 0, s>>>((const double *)(w + L.wc), g.fc, g.Gc, g.bc,
                                                (const double *)(w + L.nb), (double *)(w + L.s2));
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int abft_wgemm(const abft_wproblem *p, const void *A_f, const void *B_f, void *C_f, void *stream) {
    int st = check_wproblem(p);
    if (st) return st;
    const WGeom g = wgeom(p);
    if (!A_f || !B_f || !C_f || !aligned16(A_f) || !aligned16(B_f) || ((uintptr_t)C_f % (16 / g.V))) return ABFT_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    // a few columns (the matrix-vector case n = 1): stream A_f once instead of tiling the matrix cores
    if (g.dtype == ABFT_F32) {
        if (g.N <= kSkinnyN)
            return launch_skinny_f32((const float *)A_f, g.lda, (const float *)B_f, g.ldb, (float *)C_f, g.ldc, g.M,
                                     g.N, g.k, s);
        return launch_gemm_f32((const float *)A_f, g.lda, (const float *)B_f, g.ldb, (float *)C_f, g.ldc, g.M, g.N,
                               g.k, s);
    }
    if (g.N <= kSkinnyN)
        return launch_skinny_f64((const double *)A_f, g.lda, (const double *)B_f, g.ldb, (double *)C_f, g.ldc, g.M,
                                 g.N, g.k, s);
    return launch_gemm_f64((const double *)A_f, g.lda, (const double *)B_f, g.ldb, (double *)C_f, g.ldc, g.M, g.N,
                           g.k, s);
}

}  // extern "C"

namespace abft {
namespace {
// The verification kernels over C_f of element type T (16-byte loads when
// every row of C_f starts on a 16-byte boundary).
template <typename T>
void launch_wverify(const WGeom &g, const WLayout &L, char *w, const T *C, const VArgs &a, int vec, hipStream_t s) {
    constexpr int64_t V = vec16<T>::N;
    int64_t P = parts(g.Gr, g.br * g.N);
    if (P == 1) {
        WSWITCH(g.fr, (k_wvcol<F, T><<<vgrid(g.br * ((g.N + V - 1) / V)), kT, 0, s>>>(C, a, vec)));
    } else {
        const int64_t chunk = (g.Gr + P - 1) / P;
        P = (g.Gr + chunk - 1) / chunk;
        double *part = (double *)(w + L.part);
        WSWITCH(g.fr, (k_wvcol_part<F, T><<<grid(P * g.br * g.N), kT, 0, s>>>(C, a, P, chunk, part)));
        WSWITCH(g.fr, (k_wvcol_fin<F, T><<<vgrid(g.br * g.N), kT, 0, s>>>(C, a, P, part)));
    }
    if (g.bc >= kW && g.bc % V == 0) {
        WSWITCH(g.fc, (k_wvrow_thread<F, T><<<vgrid(g.M * (g.bc / V)), kT, 0, s>>>(C, a, vec)));
    } else {
        WSWITCH(g.fc, (k_wvrow_wave<F, T><<<vgrid(g.M * g.bc * kW), kT, 0, s>>>(C, a)));
    }
}
}  // namespace
}  // namespace abft

extern "C" {

int abft_wverify(const abft_wproblem *p, const void *C_f, const abft_rect *known, int n_known, void *ws,
                 size_t ws_bytes, abft_wreport *host_out, void *stream) {
    int st = check_wproblem(p);
    if (st) return st;
    const WGeom g = wgeom(p);
    const int64_t es = 16 / g.V;                       // element bytes
    if (!C_f || ((uintptr_t)C_f % es)) return ABFT_E_ARG;
    if ((st = check_wws(p, ws, ws_bytes))) return st;
    const WLayout L = wlayout(g);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    VArgs a;
    if ((st = to_werasures(g, known, n_known, &a.er))) return st;
    a.wr = (const double *)(w + L.wr); a.wc = (const double *)(w + L.wc);
    a.na = (const double *)(w + L.na); a.nb = (const double *)(w + L.nb);
    a.s1 = (const double *)(w + L.s1); a.s2 = (const double *)(w + L.s2);
    a.m = g.m; a.n = g.n; a.br = g.br; a.bc = g.bc; a.Gr = g.Gr; a.Gc = g.Gc; a.M = g.M; a.N = g.N; a.ldc = g.ldc;
    if (p->p.tau_mode == ABFT_TAU_DET) {
        // binary64: products accumulated in binary64, checksum rows the binary64 sums; binary32: products
        // accumulated in binary32 (u_acc = 2^-24) and checksum rows rounded once to binary32 (u_st = 2^-24)
        const double kappa = p->p.kappa >= 1.0 ? p->p.kappa : 1.0 + std::ldexp(1.0, -20);
        const double u_acc = std::ldexp(1.0, g.dtype == ABFT_F64 ? -53 : -24);
        const double u_st = g.dtype == ABFT_F64 ? 0.0 : std::ldexp(1.0, -24);
        a.cc = kappa * (2 * gam((double)g.k, u_acc) + u_st + 3 * gam((double)(g.Gr + 1)));
        a.cr = kappa * (2 * gam((double)g.k, u_acc) + u_st + 3 * gam((double)(g.Gc + 1)));
    } else {
        a.cc = a.cr = 0.0;
    }
    a.rep = (abft_wreport *)(w + L.report);
    k_wreport_init<<<1, kW, 0, s>>>(a.rep);
    const int vec = ((uintptr_t)C_f % 16 == 0) && (g.ldc % g.V == 0);
    if (g.dtype == ABFT_F64) launch_wverify(g, L, w, (const double *)C_f, a, vec, s);
    else launch_wverify(g, L, w, (const float *)C_f, a, vec, s);
    ABFT_LAUNCHED();
    if (host_out) ABFT_HIP(hipMemcpyAsync(host_out, a.rep, sizeof(abft_wreport), hipMemcpyDeviceToHost, s));
    return ABFT_OK;
}

int abft_wlocate(const abft_wproblem *p, const abft_wreport *rep, abft_location *out, int max_out, int *n_out) {
    int st = check_wproblem(p);
    if (st) return st;
    if (!rep || !n_out || max_out < 0 || (max_out > 0 && !out)) return ABFT_E_ARG;
    const WGeom g = wgeom(p);
    std::vector<abft_location> locs;
    bool multi = false;
    auto sorted = [](const abft_wgroup *gs, int64_t n) {
        std::vector<abft_wgroup> v(gs, gs + std::min<int64_t>(n, ABFT_MAX_FLAGS));
        std::sort(v.begin(), v.end(), [](const abft_wgroup &x, const abft_wgroup &y) {
            return x.a != y.a ? x.a < y.a : x.b < y.b;
        });
        return v;
    };
    if (g.fr >= 2 || g.fc >= 2) {
        const bool cols = g.fr >= 2;
        const int64_t nf = cols ? rep->n_fail_c : rep->n_fail_r;
        if (nf > ABFT_MAX_FLAGS) multi = true;
        for (const abft_wgroup &gp : sorted(cols ? rep->col : rep->row, nf)) {
            int64_t q = -1;
            const int cls = cols ? fit_group(gp, g.fr, g.Gr, p->wr, &q) : fit_group(gp, g.fc, g.Gc, p->wc, &q);
            abft_location L;
            L.cls = cls;
            L.dir = cols ? ABFT_DIR_COL : ABFT_DIR_ROW;
            if (cols) {
                L.j = gp.b;
                L.i = cls == ABFT_CLS_DATA ? q * g.br + gp.a : (cls == ABFT_CLS_CHECKSUM ? g.m + q * g.br + gp.a : -1);
            } else {
                L.i = gp.a;
                L.j = cls == ABFT_CLS_DATA ? q * g.bc + gp.b : (cls == ABFT_CLS_CHECKSUM ? g.n + q * g.bc + gp.b : -1);
            }
            multi |= cls == ABFT_CLS_MULTI;
            locs.push_back(L);
        }
    } else if (rep->n_fail_c || rep->n_fail_r) {
        // one checksum each way: one failed column group and one failed row group meet in one element
        abft_location L;
        L.cls = ABFT_CLS_MULTI; L.dir = ABFT_DIR_COL; L.i = L.j = -1;
        if (rep->n_fail_c == 1 && rep->n_fail_r == 1) {
            const int64_t i = rep->col[0].a, j = rep->col[0].b, x = rep->row[0].a, jj = rep->row[0].b;
            if (x % g.br == i && j % g.bc == jj) {
                L.cls = (x < g.m && j < g.n) ? ABFT_CLS_DATA : ABFT_CLS_CHECKSUM;
                L.i = x; L.j = j;
            }
        }
        multi = L.cls == ABFT_CLS_MULTI;
        locs.push_back(L);
    }
    *n_out = (int)locs.size();
    for (int q = 0; q < (int)locs.size() && q < max_out; ++q) out[q] = locs[q];
    return multi ? ABFT_E_UNCORRECTABLE : ABFT_OK;
}

int abft_wcorrect(const abft_wproblem *p, void *C_f, const abft_location *locs, int n, void *ws, size_t ws_bytes,
                  void *stream) {
    int st = check_wproblem(p);
    if (st) return st;
    if (!C_f || n < 0 || (n > 0 && !locs)) return ABFT_E_ARG;
    if ((st = check_wws(p, ws, ws_bytes))) return st;
    const WGeom g = wgeom(p);
    const WLayout L = wlayout(g);
    for (int q = 0; q < n; ++q) {
        if (locs[q].cls == ABFT_CLS_MULTI) return ABFT_E_UNCORRECTABLE;
        if (locs[q].cls == ABFT_CLS_CLEAN) continue;
        if (locs[q].i < 0 || locs[q].i >= g.M || locs[q].j < 0 || locs[q].j >= g.N) return ABFT_E_ARG;
        if (locs[q].dir != ABFT_DIR_COL && locs[q].dir != ABFT_DIR_ROW) return ABFT_E_ARG;
    }
    for (int q = 0; q < n; ++q) {
        const abft_location &l = locs[q];
        if (l.cls == ABFT_CLS_CLEAN) continue;
        RArgs a;
        const bool col = l.dir == ABFT_DIR_COL;
        const int64_t b = col ? g.br : g.bc, along = col ? l.i : l.j;
        if ((st = recover_args(p, g, L, (char *)ws, l.dir, {(int)(along / b)}, a))) return st;
        a.lo = col ? l.j : l.i;
        a.len = 1;
        a.i0 = along % b;
        a.i1 = a.i0 + 1;
        if ((st = launch_recover_any(g.dtype, C_f, a, (hipStream_t)stream))) return st;
    }
    return ABFT_OK;
}

int abft_wrecover(const abft_wproblem *p, void *C_f, int dir, const int32_t *blocks, int n_blocks, int64_t lo,
                  int64_t len, void *ws, size_t ws_bytes, void *stream) {
    int st = check_wproblem(p);
    if (st) return st;
    if (!C_f || n_blocks < 0 || (n_blocks > 0 && !blocks)) return ABFT_E_ARG;
    if (dir != ABFT_DIR_COL && dir != ABFT_DIR_ROW) return ABFT_E_ARG;
    if ((st = check_wws(p, ws, ws_bytes))) return st;
    const WGeom g = wgeom(p);
    const WLayout L = wlayout(g);
    const int64_t lines = dir == ABFT_DIR_COL ? g.N : g.M;
    if (lo < 0 || len < 0 || lo + len > lines) return ABFT_E_ARG;
    std::vector<int> lost(blocks, blocks + n_blocks);
    std::sort(lost.begin(), lost.end());
    lost.erase(std::unique(lost.begin(), lost.end()), lost.end());
    if ((int)lost.size() > (dir == ABFT_DIR_COL ? g.fr : g.fc) + (int)(dir == ABFT_DIR_COL ? g.Gr : g.Gc))
        return ABFT_E_ARG;
    RArgs a;
    if ((st = recover_args(p, g, L, (char *)ws, dir, lost, a))) return st;
    if (a.nu + a.nl > FM) return ABFT_E_UNRECOVERABLE;
    a.lo = lo;
    a.len = len;
    a.i0 = 0;
    a.i1 = dir == ABFT_DIR_COL ? g.br : g.bc;
    return launch_recover_any(g.dtype, C_f, a, (hipStream_t)stream);
}

}  // extern "C"
