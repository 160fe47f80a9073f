// Encode (checksum rows/columns + threshold statistics) and verify (relation
// residuals, thresholds, flags) for gfx950.  Both are HBM-bound row-group
// sums: every element is read once per pass, lanes walk contiguous columns,
// sums are binary64, and the per-block maxima/counts are folded with
// wavefront shuffles before one atomic per block.
#include <cmath>
#include <type_traits>

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

__global__ __launch_bounds__(kThreads) void k_fill_zero(double *x, int64_t n) {
    for (int64_t t = threadIdx.x; t < n; t += kThreads) x[t] = 0.0;
}

__global__ void k_report_init(abft_report *rep) {
    uint64_t *w = (uint64_t *)rep;
    const int nw = sizeof(abft_report) / 8;
    for (int q = threadIdx.x; q < nw; q += blockDim.x) w[q] = 0;
}

// Report of a fused verification: cleared, with status ABFT_E_STALE when the
// owner tag in ws does not name this problem and C_f (the verify kernels then
// record nothing).
__global__ void k_report_init_tag(abft_report *rep, const uint64_t *tag, uint64_t key) {
    uint64_t *w = (uint64_t *)rep;
    const int nw = sizeof(abft_report) / 8;
    for (int q = threadIdx.x; q < nw; q += blockDim.x) w[q] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && *tag != key) rep->status = ABFT_E_STALE;
}

// ------------------------------------------------------------------ encode
// Checksum rows of an operand X (R data rows, row-major, ld; the B operand is
// passed as its transpose, so both sides are the same row-group sum):
//   CS[r, l] = sum_{g<G} X[g*b + r, l]       (binary64 sum, rounded once to TC)
// and the per-residue statistic grp[r, l] of the threshold:
//   det:  sum_g |X[g*b + r, l]|               (row r of C_C^T |X|)
//   stat: sum_g X[g*b + r, l]^2 + CS[r, l]^2  (the squares of every member of the relation)
template <typename TC> __device__ inline void finish_encode(double sv, double ssv, bool stat, TC *cs, double *grp) {
    TC c = (TC)sv;
    *cs = c;
    *grp = stat ? ssv + (double)c * (double)c : ssv;
}

// Per-row statistics of the thresholds:
//   ROW_L2:  ||x||_2              ROW_W: sum_l x_l^2 w_l          ROW_L4SQ: ||x||_4^2
enum { ROW_L2 = 0, ROW_W = 1, ROW_L4SQ = 2 };
__device__ inline double row_term(int mode, double x, double w) {
    const double x2 = x * x;
    return mode == ROW_W ? x2 * w : (mode == ROW_L4SQ ? x2 * x2 : x2);
}

// Row partials of the fused row statistics: with rp set, a wave whose 64 lanes
// hold 64 consecutive vectors of one row also writes the sum of that 64-vector
// chunk's terms, rp[row * rps + chunk]: data row g*b + r and checksum row R + r
// (statistic rmode, weights rw for ROW_W), group-statistic row R + b + r
// (ROW_L2).  The host sets rp only when k / V is a multiple of 64, so every
// wave is whole and shares r.
__device__ inline void row_partial(double *rp, int64_t rps, int64_t row, int64_t chunk, double q2) {
    q2 = wave_sum(q2);
    if (threadIdx.x % kWave == 0) rp[row * rps + chunk] = q2;
}

// Where the encode pass takes an operand's values from: the stored operand,
// or binary32 values quantized to bfloat16 on the way (round to nearest even),
// which are written to the operand's storage and used as stored.  load(row, l0, v) fills the V values
// X[row, l0 .. l0+V) as binary64.
template <typename T> struct SrcStored {
    const T *X;
    int64_t ld;
    __device__ void load(int64_t row, int64_t l0, double *v) const { vec16<T>::load(X + row * ld + l0, v); }
};
struct SrcQuantBf16 {
    const float *X;
    int64_t ldx;
    uint16_t *Q;
    int64_t ldq;
    __device__ void load(int64_t row, int64_t l0, double *v) const {
        typedef float v4 __attribute__((ext_vector_type(4)));
        const v4 x0 = *(const v4 *)(X + row * ldx + l0), x1 = *(const v4 *)(X + row * ldx + l0 + 4);
        uint16_t h[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            h[q] = f32_to_bf16_rne(x0[q]);
            h[4 + q] = f32_to_bf16_rne(x1[q]);
        }
        v4u32 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = (uint32_t)h[2 * q] | ((uint32_t)h[2 * q + 1] << 16);
        *(v4u32 *)(Q + row * ldq + l0) = o;
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (double)bf16_to_f32(h[q]);
    }
};
// Each thread owns V = 16/sizeof(T) consecutive columns l (one 16-byte load per
// row); rows of X are 16-byte aligned and k is a multiple of V.  STAT: the
// statistical group statistic (sum of squares, else sum of magnitudes); RM:
// the row statistic of the fused row partials, kRowNone for none (rp unused).
constexpr int kRowNone = -1;
template <typename T, typename TC, class Src, bool STAT, int RM>
__global__ __launch_bounds__(kThreads) void k_encode_direct(Src src, int64_t b, int64_t G, int64_t k, TC *CS,
                                                            int64_t ldcs, double *grp, double *rp, int64_t rps,
                                                            const double *rw) {
    constexpr int V = vec16<T>::N;
    const int64_t kv = k / V, total = b * kv;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / kv, l0 = (t - r * kv) * V;
        const int64_t chunk = l0 / (kWave * V);
        double s[V], ss[V], wv[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            s[q] = ss[q] = 0.0;
            wv[q] = RM == ROW_W ? rw[l0 + q] : 0.0;
        }
        for (int64_t g = 0; g < G; ++g) {
            double v[V];
            src.load(g * b + r, l0, v);
            double q2 = 0.0;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                s[q] += v[q];
                ss[q] += STAT ? v[q] * v[q] : fabs(v[q]);
                if constexpr (RM != kRowNone) q2 += row_term(RM, v[q], wv[q]);
            }
            if constexpr (RM != kRowNone) row_partial(rp, rps, g * b + r, chunk, q2);
        }
        double c2 = 0.0, g2 = 0.0;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            finish_encode<TC>(s[q], ss[q], STAT, CS + r * ldcs + l0 + q, grp + r * k + l0 + q);
            if constexpr (RM != kRowNone) {
                const double c = (double)(TC)s[q], gv = STAT ? ss[q] + c * c : ss[q];
                c2 += row_term(RM, c, wv[q]);
                g2 += gv * gv;
            }
        }
        if constexpr (RM != kRowNone) {
            row_partial(rp, rps, G * b + r, chunk, c2);
            row_partial(rp, rps, G * b + b + r, chunk, g2);
        }
    }
}

template <typename T, class Src, bool STAT, int RM>
__global__ __launch_bounds__(kThreads) void k_encode_partial(Src src, int64_t b, int64_t G, int64_t k, int64_t P,
                                                             int64_t chunk, double *part, double *rp, int64_t rps,
                                                             const double *rw) {
    constexpr int V = vec16<T>::N;
    const int64_t kv = k / V, rel = b * k, total = P * b * kv;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t p = t / (b * kv), q = t - p * (b * kv);
        int64_t r = q / kv, l0 = (q - r * kv) * V;
        int64_t g0 = p * chunk, g1 = min(G, g0 + chunk);
        const int64_t lc = l0 / (kWave * V);
        double s[V], ss[V], wv[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            s[e] = ss[e] = 0.0;
            wv[e] = RM == ROW_W ? rw[l0 + e] : 0.0;
        }
        for (int64_t g = g0; g < g1; ++g) {
            double v[V];
            src.load(g * b + r, l0, v);
            double q2 = 0.0;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                s[e] += v[e];
                ss[e] += STAT ? v[e] * v[e] : fabs(v[e]);
                if constexpr (RM != kRowNone) q2 += row_term(RM, v[e], wv[e]);
            }
            if constexpr (RM != kRowNone) row_partial(rp, rps, g * b + r, lc, q2);
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            part[(2 * p) * rel + r * k + l0 + e] = s[e];
            part[(2 * p + 1) * rel + r * k + l0 + e] = ss[e];
        }
    }
}

template <typename TC>
__global__ __launch_bounds__(kThreads) void k_encode_finish(int64_t b, int64_t k, TC *CS, int64_t ldcs, bool stat,
                                                            int64_t P, const double *part, double *grp, double *rp,
                                                            int64_t rps, int64_t R, int rmode, const double *rw) {
    const int64_t rel = b * k;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < rel; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / k, l = t - r * k;
        // four independent running sums (partitions p mod 4) keep eight loads in flight
        double s4[4] = {0.0, 0.0, 0.0, 0.0}, ss4[4] = {0.0, 0.0, 0.0, 0.0};
        int64_t p = 0;
        for (; p + 3 < P; p += 4) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s4[q] += part[(2 * (p + q)) * rel + t];
                ss4[q] += part[(2 * (p + q) + 1) * rel + t];
            }
        }
        for (int q = 0; p < P; ++p, ++q) {
            s4[q] += part[(2 * p) * rel + t];
            ss4[q] += part[(2 * p + 1) * rel + t];
        }
        const double sv = (s4[0] + s4[1]) + (s4[2] + s4[3]), ssv = (ss4[0] + ss4[1]) + (ss4[2] + ss4[3]);
        finish_encode<TC>(sv, ssv, stat, CS + r * ldcs + l, grp + t);
        if (rp) {
            const double c = (double)(TC)sv, gv = stat ? ssv + c * c : ssv;
            row_partial(rp, rps, R + r, l / kWave, row_term(rmode, c, rmode == ROW_W ? rw[l] : 0.0));
            row_partial(rp, rps, R + b + r, l / kWave, gv * gv);
        }
    }
}

// The fused row statistics from their partials, each row summing its chunks in
// order: statistic rmode of the R data rows and b checksum rows (out[0 .. R + b);
// the square root of the sum except for ROW_W) and ||row||_2 of the b
// group-statistic rows (out_grp).
__global__ __launch_bounds__(kThreads) void k_rows_finish(const double *rp, int64_t rps, int64_t R, int64_t b,
                                                          int64_t n_data, int64_t n_tail, int rmode, double *out,
                                                          double *out_grp) {
    const int64_t rows = R + 2 * b;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kThreads) {
        const int64_t nc = i < R ? n_data : n_tail;
        double acc = 0.0;
        for (int64_t c = 0; c < nc; ++c) acc += rp[i * rps + c];
        if (i < R + b) out[i] = rmode == ROW_W ? acc : sqrt(acc);
        else out_grp[i - R - b] = sqrt(acc);
    }
}

// Per-row statistic of X[i, 0:k), one wave per row (grid-stride over rows),
// 16-byte loads, eight in flight per lane, kept as raw words until each is
// widened and summed in column order (the statistics are listed above the
// encode kernels).  With ROW_W the weights sit in LDS as binary32, permuted so
// that the lanes of a wave read consecutive words: lane L needs w[l0 + q] with
// l0 = 64 V c + V L (chunk c of 64 V columns), stored at 64 V c + 64 q + L.
constexpr int64_t kRowWMaxK = 16384;   // ROW_W keeps w (as binary32, 64 KB) in LDS up to this k
constexpr int kRowThreads = 512;       // 8 waves share one copy of w
// The rows of one block for a statistic fixed at compile time (WLDS: ROW_W
// with the weights in LDS, permuted as above).
template <typename T, int MODE, bool WLDS>
__device__ __attribute__((always_inline)) inline void row_stats_rows(const T *X, int64_t ld, int64_t rows, int64_t k,
                                                                     const double *w, const float *wsh, double *out) {
    constexpr int V = vec16<T>::N;
    constexpr int NW = kRowThreads / kWave;
    constexpr int64_t CH = (int64_t)kWave * V;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    auto term = [&](const double *v, int64_t l0, double &acc) {
        const float *wc = wsh + (l0 / CH) * CH + lane;  // this lane's weights of l0's chunk, stride kWave
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const double v2 = v[q] * v[q];
            if constexpr (MODE == ROW_W) acc += v2 * (WLDS ? (double)wc[q * kWave] : w[l0 + q]);
            else if constexpr (MODE == ROW_L4SQ) acc += v2 * v2;
            else acc += v2;
        }
    };
    for (int64_t i = (int64_t)blockIdx.x * NW + wave; i < rows; i += (int64_t)gridDim.x * NW) {
        const T *row = X + i * ld;
        double acc = 0.0;
        constexpr int64_t step = CH;
        int64_t l0 = (int64_t)lane * V;
        for (; l0 + 7 * step < k; l0 += 8 * step) {
            v4u32 raw[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) raw[u] = *(const v4u32 *)(row + l0 + u * step);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                double v[V];
                vec16<T>::widen(raw[u], v);
                term(v, l0 + u * step, acc);
            }
        }
        for (; l0 < k; l0 += step) {
            double v0[V];
            vec16<T>::load(row + l0, v0);
            term(v0, l0, acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) out[i] = MODE == ROW_W ? acc : sqrt(acc);
    }
}

template <typename T>
__global__ __launch_bounds__(kRowThreads) void k_row_stats(const T *X, int64_t ld, int64_t rows, int64_t k, int mode,
                                                           const double *w, double *out) {
    constexpr int64_t CH = (int64_t)kWave * vec16<T>::N;   // columns per chunk (one 16-byte load per lane)
    extern __shared__ float wsh[];                     // whole chunks of k when mode == ROW_W and k <= kRowWMaxK
    const bool wlds = mode == ROW_W && k <= kRowWMaxK;
    if (wlds) {
        for (int64_t l = threadIdx.x; l < k; l += kRowThreads) {
            const int64_t c = l / CH, e = l - c * CH;
            wsh[c * CH + (e % vec16<T>::N) * kWave + e / vec16<T>::N] = (float)w[l];
        }
        __syncthreads();
    }
    if (mode == ROW_W) {
        if (wlds) row_stats_rows<T, ROW_W, true>(X, ld, rows, k, w, wsh, out);
        else row_stats_rows<T, ROW_W, false>(X, ld, rows, k, w, wsh, out);
    } else if (mode == ROW_L4SQ) {
        row_stats_rows<T, ROW_L4SQ, false>(X, ld, rows, k, w, wsh, out);
    } else {
        row_stats_rows<T, ROW_L2, false>(X, ld, rows, k, w, wsh, out);
    }
}

// Row statistics launch: with LDS-staged weights a block serves many rows.
template <typename T>
static void row_stats(const T *X, int64_t ld, int64_t rows, int64_t k, int mode, const double *w, double *out,
                      hipStream_t s) {
    if (rows <= 0) return;
    constexpr int NW = kRowThreads / kWave;
    constexpr int64_t CH = (int64_t)kWave * vec16<T>::N;   // the permuted weights fill whole chunks
    static_assert(kRowWMaxK % CH == 0, "whole chunks within the LDS limit");
    size_t lds = (mode == ROW_W && k <= kRowWMaxK) ? sizeof(float) * (size_t)((k + CH - 1) / CH * CH) : 0;
    unsigned grid = (unsigned)std::min<int64_t>((rows + NW - 1) / NW, lds ? 512 : 65536);
    k_row_stats<T><<<grid, kRowThreads, lds, s>>>(X, ld, rows, k, mode, w, out);
}

static unsigned grid_for(int64_t work) { return (unsigned)std::min<int64_t>((work + kThreads - 1) / kThreads, 65536); }
static unsigned rows_grid(int64_t rows) { return (unsigned)std::min<int64_t>(std::max<int64_t>(rows, 1), 65536); }

// Pass 1 over one operand: checksum rows CS (ldcs) and grp; with rp (k / V a
// multiple of 64) also the row-statistic partials of the data and checksum rows
// (statistic rmode, weights rw) and of the group rows, finished into rows_out
// (R + b) and grp_out (b).
template <typename T, typename TC, class Src>
static void encode_pass1(Src src, int64_t R, int64_t b, int64_t k, TC *CS, int64_t ldcs, bool stat, double *grp,
                         double *part, hipStream_t s, double *rp = nullptr, int rmode = ROW_L2,
                         const double *rw = nullptr, double *rows_out = nullptr, double *grp_out = nullptr) {
    constexpr int V = vec16<T>::N;
    int64_t G = R / b;
    int64_t P = group_partitions(G, b, k / V);
    const int64_t rps = k / kWave;                 // partial slots per row (chunks of 64 columns at most)
    int64_t n_tail;
    int64_t chunk = 0;
    if (P > 1) {
        chunk = (G + P - 1) / P;
        P = (G + chunk - 1) / chunk;
    }
    // the statistic modes as template arguments (no per-element selects)
    auto pass = [&](auto st, auto rm) {
        constexpr bool ST = decltype(st)::value;
        constexpr int RM = decltype(rm)::value;
        if (P == 1)
            k_encode_direct<T, TC, Src, ST, RM><<<grid_for(b * k / V), kThreads, 0, s>>>(src, b, G, k, CS, ldcs, grp,
                                                                                         rp, rps, rw);
        else
            k_encode_partial<T, Src, ST, RM><<<grid_for(P * b * k / V), kThreads, 0, s>>>(src, b, G, k, P, chunk, part,
                                                                                          rp, rps, rw);
    };
    auto by_row = [&](auto st) {
        if (!rp) pass(st, std::integral_constant<int, kRowNone>{});
        else if (rmode == ROW_W) pass(st, std::integral_constant<int, ROW_W>{});
        else if (rmode == ROW_L4SQ) pass(st, std::integral_constant<int, ROW_L4SQ>{});
        else pass(st, std::integral_constant<int, ROW_L2>{});
    };
    if (stat) by_row(std::true_type{});
    else by_row(std::false_type{});
    if (P == 1) {
        n_tail = k / (kWave * V);
    } else {
        k_encode_finish<TC><<<grid_for(b * k), kThreads, 0, s>>>(b, k, CS, ldcs, stat, P, part, grp, rp, rps, R,
                                                                 rmode, rw);
        n_tail = k / kWave;
    }
    if (rp)
        k_rows_finish<<<grid_for(R + 2 * b), kThreads, 0, s>>>(rp, rps, R, b, k / (kWave * V), n_tail, rmode,
                                                               rows_out, grp_out);
}

// Pass 2 over one operand: a statistic per row of the data rows and of the
// checksum rows.  det: ||row||_2; stat with the other side thin (b_other == 1):
// sum_l row_l^2 w_l (w = the other side's grp); stat otherwise: ||row||_4^2.
template <typename T, typename TC>
static void encode_pass2(const T *X, int64_t ld, int64_t R, const TC *CS, int64_t ldcs, int64_t b, int64_t k,
                         bool stat, int64_t b_other, const double *w_other, double *out, hipStream_t s) {
    int mode = !stat ? ROW_L2 : (b_other == 1 ? ROW_W : ROW_L4SQ);
    row_stats<T>(X, ld, R, k, mode, w_other, out, s);
    row_stats<TC>(CS, ldcs, b, k, mode, w_other, out + R, s);
}

template <typename T, typename TC, class SrcA, class SrcB>
static int encode_typed(const abft_problem *p, SrcA srcA, SrcB srcB, T *A, T *Bt, TC *Acs, int64_t ldacs, TC *Bcs,
                        int64_t ldbcs, char *ws, hipStream_t s) {
    Geom g = geom_of(p);
    WsLayout L = ws_layout(p);
    double *part = (double *)(ws + L.partial);
    double *grpA = (double *)(ws + L.grpA), *grpB = (double *)(ws + L.grpB);
    const bool stat = p->tau_mode == ABFT_TAU_STAT;
    // row statistics (det: na, nb; stat: qr, qc) and the norms of the grp rows
    // (det: na_abs, nb_abs; stat: nv, nw)
    double *ra = (double *)(ws + (stat ? L.qr : L.na)), *rb = (double *)(ws + (stat ? L.qc : L.nb));
    double *ga = (double *)(ws + (stat ? L.nv : L.na_abs)), *gb = (double *)(ws + (stat ? L.nw : L.nb_abs));
    // det: ||row||_2; stat with the other side thin: sum_l row_l^2 w_l (w = the other side's grp); stat
    // otherwise: ||row||_4^2
    const int modeA = !stat ? ROW_L2 : (g.bc == 1 ? ROW_W : ROW_L4SQ);
    const int modeB = !stat ? ROW_L2 : (g.br == 1 ? ROW_W : ROW_L4SQ);
    // With rows_fused the encode pass produces the row statistics too (no second read of the operand),
    // except A's sum_l A_il^2 w_l, whose weights (B's grp) exist only after B's encode.
    double *rp = rows_fused(p) ? (double *)(ws + L.rowpart) : nullptr;
    const bool fuseA = rp && modeA != ROW_W, fuseB = rp != nullptr;
    encode_pass1<T, TC>(srcA, g.m, g.br, g.k, Acs, ldacs, stat, grpA, part, s, fuseA ? rp : nullptr, modeA, nullptr,
                        ra, ga);
    encode_pass1<T, TC>(srcB, g.n, g.bc, g.k, Bcs, ldbcs, stat, grpB, part, s, fuseB ? rp : nullptr, modeB, grpA, rb,
                        gb);
    if (!fuseA) {
        encode_pass2<T, TC>(A, p->lda, g.m, Acs, ldacs, g.br, g.k, stat, g.bc, grpB, ra, s);
        row_stats<double>(grpA, g.k, g.br, g.k, ROW_L2, nullptr, ga, s);
    }
    if (!fuseB) {
        encode_pass2<T, TC>(Bt, p->ldb, g.n, Bcs, ldbcs, g.bc, g.k, stat, g.br, grpA, rb, s);
        row_stats<double>(grpB, g.k, g.bc, g.k, ROW_L2, nullptr, gb, s);
    }
    // an operand encoded here carries no inherited residual
    k_fill_zero<<<1, kThreads, 0, s>>>((double *)(ws + L.chain_a), g.br);
    k_fill_zero<<<1, kThreads, 0, s>>>((double *)(ws + L.chain_w), g.N);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// Chained product (the result of a product fed to the next one, F64 or F32,
// det or exact): A_f is the previous C_f, whose carried rows are used as they are.
// Its checksum rows are recomputed only into scratch, for the group statistic;
// the row statistics are taken over the rows that enter the product (the
// carried ones).  B_f is encoded as usual.  The previous column relations hold
// up to their residual, at most tau_prev(r, l) = cc_prev na_abs_prev[r]
// nb_prev[l]; through the product it contributes at most
// sum_l tau_prev(r, l) |B_f[l, j]| to relation (r, j): stored as
// chain_a[r] = cc_prev na_abs_prev[r] and chain_w[j] = sum_l nb_prev[l] |B_f[l, j]|.
__global__ __launch_bounds__(kThreads) void k_chain_a(const double *na_abs_prev, double cc_prev, int64_t br,
                                                      double *chain_a) {
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < br; r += (int64_t)gridDim.x * kThreads)
        chain_a[r] = cc_prev * na_abs_prev[r];
}

// out[j] = sum_l w[l] |X[j, l]|: one wave per row, binary64.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_row_absdot(const T *X, int64_t ld, int64_t rows, int64_t k,
                                                         const double *w, double *out) {
    constexpr int V = vec16<T>::N;
    const int lane = threadIdx.x % kWave;
    const int64_t w0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kThreads / kWave;
    for (int64_t j = w0; j < rows; j += nw) {
        const T *row = X + j * ld;
        double acc = 0.0;
        for (int64_t l = V * lane; l < k; l += V * kWave) {
            double v[V];
            vec16<T>::load(row + l, v);
#pragma unroll
            for (int e = 0; e < V; ++e) acc += w[l + e] * fabs(v[e]);
        }
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) out[j] = acc;
    }
}

template <typename T>
static int encode_chained_typed(const abft_problem *p, const T *A, T *Bt, char *ws, const abft_problem *prev,
                                const char *ws_prev, double cc_prev, hipStream_t s) {
    Geom g = geom_of(p);
    WsLayout L = ws_layout(p), Lp = ws_layout(prev);
    double *part = (double *)(ws + L.partial);
    double *grpA = (double *)(ws + L.grpA), *grpB = (double *)(ws + L.grpB);
    T *cs = (T *)(ws + L.chain_cs);
    // the A side: group statistic (checksum rows into scratch), row norms of the rows that enter the product
    encode_pass1<T, T>(SrcStored<T>{A, p->lda}, g.m, g.br, g.k, cs, g.k, false, grpA, part, s);
    encode_pass2<T, T>(A, p->lda, g.m, A + g.m * p->lda, p->lda, g.br, g.k, false, g.bc, grpB, (double *)(ws + L.na),
                       s);
    // the B side as in a plain encode
    encode_pass1<T, T>(SrcStored<T>{Bt, p->ldb}, g.n, g.bc, g.k, Bt + g.n * p->ldb, p->ldb, false, grpB, part, s);
    encode_pass2<T, T>(Bt, p->ldb, g.n, Bt + g.n * p->ldb, p->ldb, g.bc, g.k, false, g.br, grpA,
                       (double *)(ws + L.nb), s);
    row_stats<double>(grpA, g.k, g.br, g.k, ROW_L2, nullptr, (double *)(ws + L.na_abs), s);
    row_stats<double>(grpB, g.k, g.bc, g.k, ROW_L2, nullptr, (double *)(ws + L.nb_abs), s);
    // the inherited term
    k_chain_a<<<1, kThreads, 0, s>>>((const double *)(ws_prev + Lp.na_abs), cc_prev, g.br, (double *)(ws + L.chain_a));
    k_row_absdot<T><<<(unsigned)std::min<int64_t>((g.N + 3) / 4, 65536), kThreads, 0, s>>>(
        Bt, p->ldb, g.N, g.k, (const double *)(ws_prev + Lp.nb), (double *)(ws + L.chain_w));
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_encode_chained(const abft_problem *p, const void *A_f, void *B_f, char *ws, const abft_problem *prev,
                          const char *ws_prev, double cc_prev, hipStream_t s) {
    if (p->dtype == ABFT_F32)
        return encode_chained_typed(p, (const float *)A_f, (float *)B_f, ws, prev, ws_prev, cc_prev, s);
    return encode_chained_typed(p, (const double *)A_f, (double *)B_f, ws, prev, ws_prev, cc_prev, s);
}

int launch_encode(const abft_problem *p, void *A_f, void *B_f, char *ws, hipStream_t s) {
    Geom g = geom_of(p);
    switch (p->dtype) {
    case ABFT_F64: {
        double *A = (double *)A_f, *Bt = (double *)B_f;
        return encode_typed<double, double>(p, SrcStored<double>{A, p->lda}, SrcStored<double>{Bt, p->ldb}, A, Bt,
                                            A + g.m * p->lda, p->lda, Bt + g.n * p->ldb, p->ldb, ws, s);
    }
    case ABFT_F32: {
        float *A = (float *)A_f, *Bt = (float *)B_f;
        return encode_typed<float, float>(p, SrcStored<float>{A, p->lda}, SrcStored<float>{Bt, p->ldb}, A, Bt,
                                          A + g.m * p->lda, p->lda, Bt + g.n * p->ldb, p->ldb, ws, s);
    }
    case ABFT_BF16: {
        // bfloat16 data, binary32 checksum rows in the workspace
        WsLayout L = ws_layout(p);
        uint16_t *A = (uint16_t *)A_f, *Bt = (uint16_t *)B_f;
        return encode_typed<uint16_t, float>(p, SrcStored<uint16_t>{A, p->lda}, SrcStored<uint16_t>{Bt, p->ldb}, A,
                                             Bt, (float *)(ws + L.acs), g.k, (float *)(ws + L.bcs), g.k, ws, s);
    }
    case ABFT_FP8_E4M3: {
        // E4M3 data (scaled domain), binary32 checksum rows in the workspace
        WsLayout L = ws_layout(p);
        uint8_t *A = (uint8_t *)A_f, *Bt = (uint8_t *)B_f;
        return encode_typed<uint8_t, float>(p, SrcStored<uint8_t>{A, p->lda}, SrcStored<uint8_t>{Bt, p->ldb}, A, Bt,
                                            (float *)(ws + L.acs), g.k, (float *)(ws + L.bcs), g.k, ws, s);
    }
    default:
        return ABFT_E_UNSUPPORTED;
    }
}

// ------------------------------------------------------------------ quantize
// binary32 -> bfloat16, round to nearest even; 8 values per thread and step.
__global__ __launch_bounds__(kThreads) void k_quantize_bf16(const float *X, int64_t ldx, int64_t rows, int64_t k,
                                                            uint16_t *Q, int64_t ldq) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const int64_t per_row = k / 8, total = rows * per_row;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t i = t / per_row, c = (t - i * per_row) * 8;
        v4 x0 = *(const v4 *)(X + i * ldx + c), x1 = *(const v4 *)(X + i * ldx + c + 4);
        v4u o;
        o[0] = f32_to_bf16_rne(x0[0]) | ((uint32_t)f32_to_bf16_rne(x0[1]) << 16);
        o[1] = f32_to_bf16_rne(x0[2]) | ((uint32_t)f32_to_bf16_rne(x0[3]) << 16);
        o[2] = f32_to_bf16_rne(x1[0]) | ((uint32_t)f32_to_bf16_rne(x1[1]) << 16);
        o[3] = f32_to_bf16_rne(x1[2]) | ((uint32_t)f32_to_bf16_rne(x1[3]) << 16);
        *(v4u *)(Q + i * ldq + c) = o;
    }
}

// FP8 per-tensor scaling, kept on the device (no host synchronisation):
// amax = max |x| over the finite entries (binary32 bit patterns of
// non-negative values order like unsigned integers), then the scale exponent
// e = the largest e with amax * 2^e <= 448 (0 when amax is 0), then x * 2^e
// (ldexp: exact wherever the result can round to a non-zero code, also where
// 2^e itself is beyond binary32) rounded to E4M3;
// NaN stays NaN and an infinity saturates to +-448 like any |x 2^e| >= 464.
// ws scale words: [0] = e_A, [1] = e_B, [2] = amax_A bits, [3] = amax_B bits.
__global__ void k_amax_init(int *scale, int which) { scale[2 + which] = 0; }

// 16-byte loads: rows of X are 16-byte aligned and k is a multiple of 4 (as for the quantizer).
// |x| for finite x, else 0 (NaN and infinities take no part in the scale)
__device__ inline float fin_abs(float x) {
    const float a = fabsf(x);
    return a <= 3.40282347e38f ? a : 0.0f;
}

__global__ __launch_bounds__(kThreads) void k_amax(const float *X, int64_t ldx, int64_t rows, int64_t k, int *scale,
                                                   int which) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __shared__ float sh[kThreads / kWave];
    float mx = 0.0f;
    const int64_t kv = k / 4, total = rows * kv;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t i = t / kv, l = (t - i * kv) * 4;
        const v4 x = *(const v4 *)(X + i * ldx + l);
        mx = fmaxf(mx, fmaxf(fmaxf(fin_abs(x[0]), fin_abs(x[1])), fmaxf(fin_abs(x[2]), fin_abs(x[3]))));
    }
    for (int off = kWave / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kWave));
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kThreads / kWave; ++q) mx = fmaxf(mx, sh[q]);
        atomicMax((unsigned int *)&scale[2 + which], __float_as_uint(mx));
    }
}

__global__ void k_scale_exp(int *scale, int which) {
    double amax = (double)__uint_as_float((unsigned int)scale[2 + which]);
    int e = 0;
    if (amax > 0.0 && amax <= 3.40282347e38) {        // finite by construction; both loops end within 160 steps
        while (ldexp(amax, e + 1) <= 448.0) ++e;
        while (ldexp(amax, e) > 448.0) --e;
    }
    scale[which] = e;
}

__global__ __launch_bounds__(kThreads) void k_quantize_fp8(const float *X, int64_t ldx, int64_t rows, int64_t k,
                                                           uint8_t *Q, int64_t ldq, const int *scale, int which) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const int e = scale[which];
    const int64_t per_row = k / 4, total = rows * per_row;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t i = t / per_row, c = (t - i * per_row) * 4;
        v4 x = *(const v4 *)(X + i * ldx + c);
        uint32_t o = (uint32_t)f32_to_e4m3_rne(__builtin_ldexpf(x[0], e)) |
                     ((uint32_t)f32_to_e4m3_rne(__builtin_ldexpf(x[1], e)) << 8) |
                     ((uint32_t)f32_to_e4m3_rne(__builtin_ldexpf(x[2], e)) << 16) |
                     ((uint32_t)f32_to_e4m3_rne(__builtin_ldexpf(x[3], e)) << 24);
        *(uint32_t *)(Q + i * ldq + c) = o;
    }
}

int launch_quantize(const abft_problem *p, int which, const float *X, int64_t ldx, void *dst, char *ws, hipStream_t s) {
    int64_t rows = which == 0 ? p->m : p->n;
    int64_t ldq = which == 0 ? p->lda : p->ldb;
    if (p->dtype == ABFT_BF16) {
        k_quantize_bf16<<<grid_for(rows * p->k / 8), kThreads, 0, s>>>(X, ldx, rows, p->k, (uint16_t *)dst, ldq);
        ABFT_LAUNCHED();
        return ABFT_OK;
    }
    if (p->dtype == ABFT_FP8_E4M3) {
        WsLayout L = ws_layout(p);
        int *scale = (int *)(ws + L.scale);
        k_amax_init<<<1, 1, 0, s>>>(scale, which);
        k_amax<<<(unsigned)std::min<int64_t>((rows * p->k / 4 + kThreads - 1) / kThreads, 4096), kThreads, 0, s>>>(
            X, ldx, rows, p->k, scale, which);
        k_scale_exp<<<1, 1, 0, s>>>(scale, which);
        k_quantize_fp8<<<grid_for(rows * p->k / 4), kThreads, 0, s>>>(X, ldx, rows, p->k, (uint8_t *)dst, ldq, scale,
                                                                      which);
        ABFT_LAUNCHED();
        return ABFT_OK;
    }
    return ABFT_E_UNSUPPORTED;
}

// Quantize both binary32 operands and encode them.  bfloat16: in the same
// pass (the values abft_quantize would store are written and the encode uses
// them as stored), so the result equals quantize + quantize + encode bit for
// bit.  FP8: the separate passes, which measured faster than one pass that
// rounds, decodes and sums 16 values per thread (absmax, quantize and encode
// per operand).
int launch_quantize_encode(const abft_problem *p, const float *A32, int64_t lda32, const float *B32, int64_t ldb32,
                           void *A_f, void *B_f, char *ws, hipStream_t s) {
    if (p->dtype == ABFT_BF16) {
        WsLayout L = ws_layout(p);
        uint16_t *A = (uint16_t *)A_f, *Bt = (uint16_t *)B_f;
        return encode_typed<uint16_t, float>(p, SrcQuantBf16{A32, lda32, A, p->lda}, SrcQuantBf16{B32, ldb32, Bt, p->ldb},
                                             A, Bt, (float *)(ws + L.acs), p->k, (float *)(ws + L.bcs), p->k, ws, s);
    }
    if (p->dtype == ABFT_FP8_E4M3) {
        int st = launch_quantize(p, 0, A32, lda32, A_f, ws, s);
        if (!st) st = launch_quantize(p, 1, B32, ldb32, B_f, ws, s);
        if (!st) st = launch_encode(p, A_f, B_f, ws, s);
        return st;
    }
    return ABFT_E_UNSUPPORTED;
}

// ------------------------------------------------------------------ verify
struct VerifyArgs {
    int64_t m, n, br, bc, S, Gr, Gc, M, N, ldc;
    int mode;
    double cc, cr;                  // det coefficients; stat: cc = lambda^2 (u^2/3)(T/2 + s)
    double cst;                     // stat: lambda^2 u^2 / 3 (the stored total's binary32 rounding)
    const double *na, *na_abs, *nb, *nb_abs;
    const double *chain_a, *chain_w; // det: inherited term of a chained product (zero otherwise)
    const double *qr, *qc, *nv, *nw;
    const int *scale_exp;           // FP8: statistics are in the scaled domain, C is not
    abft_report *rep;
    Erasures er;
    const uint64_t *tag;            // fused verification: the owner tag the product wrote into ws (null: none)
    uint64_t key;                   // and the value it must hold for this problem and C_f
};

// det:  tau_c = cc ||(C_C^T|A|)[r,:]||_2 ||B_f[:,j]||_2
// stat: tau_c = sqrt(s^2 cc Q_c[r,j] + cst tot^2),  Q_c = qc[j] (br = 1, exact) or nv[r] qc[j]
//       (Cauchy-Schwarz bound), s the FP8 result scale (Q is in the scaled domain), tot the
//       relation's stored total as read from C_f; a non-finite total adds no term (its
//       residual is then non-finite and the relation fails, as it must)
__device__ inline double tau_scale(const VerifyArgs &a) {
    return a.scale_exp ? ldexp(1.0, -(a.scale_exp[0] + a.scale_exp[1])) : 1.0;
}
__device__ inline double tau_col(const VerifyArgs &a, int64_t r, int64_t j, double tot) {
    if (a.mode == ABFT_TAU_DET) return tau_scale(a) * a.cc * a.na_abs[r] * a.nb[j] + a.chain_a[r] * a.chain_w[j];
    if (a.mode == ABFT_TAU_STAT) {
        const double sc = tau_scale(a), t = isfinite(tot) ? tot : 0.0;
        return sqrt(sc * sc * a.cc * (a.br == 1 ? a.qc[j] : a.nv[r] * a.qc[j]) + a.cst * t * t);
    }
    return 0.0;
}
__device__ inline double tau_row(const VerifyArgs &a, int64_t i, int64_t c, double tot) {
    if (a.mode == ABFT_TAU_DET) return tau_scale(a) * a.cr * a.na[i] * a.nb_abs[c];
    if (a.mode == ABFT_TAU_STAT) {
        const double sc = tau_scale(a), t = isfinite(tot) ? tot : 0.0;
        return sqrt(sc * sc * a.cr * (a.bc == 1 ? a.qr[i] : a.qr[i] * a.nw[c]) + a.cst * t * t);
    }
    return 0.0;
}

// Column relation (r, j): sum_{g<Gr} C[g*br + r, j] - sum_{s<S} C[m + s*br + r, j]
template <typename T>
__device__ inline void finish_col(const VerifyArgs &a, const T *C, int64_t r, int64_t j, double s, double &ratio,
                                  unsigned long long &excl) {
    double tot = 0.0;
    for (int64_t q = 0; q < a.S; ++q) tot += elem<T>::load(C + (a.m + q * a.br + r) * a.ldc + j);
    if (col_rel_erased(a.er, r, j, a.br)) { excl++; return; }
    ratio = fmax(ratio, record(a.rep, true, r, j, s - tot, tau_col(a, r, j, tot)));
}

// V consecutive elements of a C row: one 16-byte load (V > 1, aligned rows) or one element.
template <typename T, int V> __device__ inline void load_c(const T *p, double *v) {
    if constexpr (V == 1) v[0] = elem<T>::load(p);
    else vec16<T>::load(p, v);
}

// Column relations, one thread per residue r and V consecutive columns.  With
// V > 1 the rows of C are 16-byte aligned and ldc is a multiple of V, so the
// last vector of a row stays inside the row's ldc elements; columns >= N are
// read but not used.
template <typename T, int V>
__global__ __launch_bounds__(kThreads) void k_vcol_direct(const T *C, VerifyArgs a) {
    const int64_t nv = (a.N + V - 1) / V, total = a.br * nv;
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t r = t / nv, j0 = (t - r * nv) * V;
        const T *p = C + r * a.ldc + j0;
        double s[V], v[V];
#pragma unroll
        for (int q = 0; q < V; ++q) s[q] = 0.0;
        for (int64_t g = 0; g < a.Gr; ++g) {
            load_c<T, V>(p + g * a.br * a.ldc, v);
#pragma unroll
            for (int q = 0; q < V; ++q) s[q] += v[q];
        }
#pragma unroll
        for (int q = 0; q < V; ++q)
            if (j0 + q < a.N) finish_col<T>(a, C, r, j0 + q, s[q], ratio, excl);
    }
    fold_block(ratio, excl, &a.rep->max_ratio_c, &a.rep->n_excl_c);
}

template <typename T, int V>
__global__ __launch_bounds__(kThreads) void k_vcol_partial(const T *C, VerifyArgs a, int64_t P, int64_t chunk, double *part) {
    const int64_t nv = (a.N + V - 1) / V, rel = a.br * a.N, total = P * a.br * nv;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        int64_t p = t / (a.br * nv), q = t - p * (a.br * nv);
        int64_t r = q / nv, j0 = (q - r * nv) * V;
        int64_t g0 = p * chunk, g1 = min(a.Gr, g0 + chunk);
        const T *src = C + r * a.ldc + j0;
        double s[V], v[V];
#pragma unroll
        for (int e = 0; e < V; ++e) s[e] = 0.0;
        for (int64_t g = g0; g < g1; ++g) {
            load_c<T, V>(src + g * a.br * a.ldc, v);
#pragma unroll
            for (int e = 0; e < V; ++e) s[e] += v[e];
        }
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (j0 + e < a.N) part[p * rel + r * a.N + j0 + e] = s[e];
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
    ratio = fmax(ratio, record(a.rep, false, i, c, s - tot, tau_row(a, i, c, tot)));
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
// sums of each residue.  With V > 1 (bc == 1 and 16-byte aligned rows) thread t
// sums whole vectors t, t + 256, ... of the row.
template <typename T, int V>
__global__ __launch_bounds__(kThreads) void k_vrow_block(const T *C, VerifyArgs a) {
    __shared__ double sh[kThreads];
    double ratio = 0.0;
    unsigned long long excl = 0;
    for (int64_t i = blockIdx.x; i < a.M; i += gridDim.x) {
        const T *row = C + i * a.ldc;
        double s0 = 0.0, s1 = 0.0, v[V], w[V];
        int64_t j = (int64_t)threadIdx.x * V;
        for (; j + kThreads * V < a.n; j += 2 * kThreads * V) {
            load_c<T, V>(row + j, v);
            load_c<T, V>(row + j + kThreads * V, w);
#pragma unroll
            for (int q = 0; q < V; ++q) {
                if (j + q < a.n) s0 += v[q];
                if (j + kThreads * V + q < a.n) s1 += w[q];
            }
        }
        if (j < a.n) {
            load_c<T, V>(row + j, v);
#pragma unroll
            for (int q = 0; q < V; ++q)
                if (j + q < a.n) s0 += v[q];
        }
        sh[threadIdx.x] = s0 + s1;
        __syncthreads();
        for (int wd = kThreads / 2; wd >= a.bc; wd >>= 1) {
            if (threadIdx.x < wd) sh[threadIdx.x] += sh[threadIdx.x + wd];
            __syncthreads();
        }
        if (threadIdx.x < a.bc) finish_row<T>(a, C, i, threadIdx.x, sh[threadIdx.x], ratio, excl);
        __syncthreads();
    }
    fold_block(ratio, excl, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

// Erasure tests of the one-pass kernel: the residues of each known
// rectangle's first row (mod br) and first column (mod bc) are taken on the
// host, so a test is a few comparisons on kernel arguments (the same answer as
// col_rel_erased / row_rel_erased for 0 <= r < br and 0 <= c < bc).
struct ErasureRes {
    int n;
    int64_t i0[4], j0[4], h[4], w[4], ri[4], cj[4];
};
static ErasureRes erasure_res(const Erasures &e, int64_t br, int64_t bc) {
    ErasureRes x{};
    x.n = e.n;
    for (int q = 0; q < e.n && q < 4; ++q) {
        x.i0[q] = e.i0[q]; x.j0[q] = e.j0[q]; x.h[q] = e.h[q]; x.w[q] = e.w[q];
        x.ri[q] = e.i0[q] % br;
        x.cj[q] = e.j0[q] % bc;
    }
    return x;
}
__device__ inline bool col_erased_res(const ErasureRes &e, int64_t r, int64_t j, int64_t br) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= e.n) break;
        if (j < e.j0[q] || j >= e.j0[q] + e.w[q]) continue;
        if (e.h[q] >= br) return true;
        const int64_t off = r >= e.ri[q] ? r - e.ri[q] : r - e.ri[q] + br;
        if (off < e.h[q]) return true;
    }
    return false;
}
__device__ inline bool row_erased_res(const ErasureRes &e, int64_t i, int64_t c, int64_t bc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= e.n) break;
        if (i < e.i0[q] || i >= e.i0[q] + e.h[q]) continue;
        if (e.w[q] >= bc) return true;
        const int64_t off = c >= e.cj[q] ? c - e.cj[q] : c - e.cj[q] + bc;
        if (off < e.w[q]) return true;
    }
    return false;
}

// One pass over C_f for wide checksum blocks: thread t owns residue r and the
// V consecutive residues c0..c0+V-1 and walks the (Gr+1) x (Gc+1) grid of
// blocks (the last block row / column is the carried one), so it holds every
// member of the column relations (r, h*bc + c) and of the row relations
// (g*br + r, c): both directions from one read of C_f.  Sums run over the
// groups in increasing order with the carried term subtracted last, as in the
// two-pass kernels, so the residuals are the same numbers.  GC = Gc, 1..8.
constexpr int kBlockPassMaxG = 8;    // data block columns: up to 8 (the carried one makes 9)
// The thresholds of this pass with their row-, column- and problem-dependent
// factors loaded ahead of the sums (the same arithmetic as tau_row / tau_col).
struct VbFac {
    double sc, rowc, colc;          // tau_scale; per-residue factors of the row (c) and column (r) relations
};
__device__ inline double vb_row_fac(const VerifyArgs &a, int64_t i) {
    return a.mode == ABFT_TAU_DET ? a.na[i] : (a.mode == ABFT_TAU_STAT ? a.qr[i] : 0.0);
}
__device__ inline double vb_tau_row(const VerifyArgs &a, double sc, double fi, double fc, double tot) {
    if (a.mode == ABFT_TAU_DET) return sc * a.cr * fi * fc;
    if (a.mode == ABFT_TAU_STAT) {
        const double t = isfinite(tot) ? tot : 0.0;
        return sqrt(sc * sc * a.cr * (a.bc == 1 ? fi : fi * fc) + a.cst * t * t);
    }
    return 0.0;
}
__device__ inline double vb_tau_col(const VerifyArgs &a, double sc, double fr, double chr, double fj, double cwj,
                                    double tot) {
    if (a.mode == ABFT_TAU_DET) return sc * a.cc * fr * fj + chr * cwj;
    if (a.mode == ABFT_TAU_STAT) {
        const double t = isfinite(tot) ? tot : 0.0;
        return sqrt(sc * sc * a.cc * (a.br == 1 ? fj : fr * fj) + a.cst * t * t);
    }
    return 0.0;
}

template <typename T, int V, int GC>
__global__ __launch_bounds__(kThreads) void k_vblock(const T *C, VerifyArgs a, ErasureRes er) {
    const int64_t cv = a.bc / V, total = a.br * cv;
    const bool det = a.mode == ABFT_TAU_DET, stat = a.mode == ABFT_TAU_STAT;
    const double sc = (det || stat) ? tau_scale(a) : 0.0;
    double ratio_c = 0.0, ratio_r = 0.0;
    unsigned long long excl_c = 0, excl_r = 0;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        const int64_t r = t / cv, c0 = (t - r * cv) * V;
        // residue factors, loaded once: row relations (i, c0 + q), column relations (r, .)
        double fc[V];
#pragma unroll
        for (int q = 0; q < V; ++q) fc[q] = det ? a.nb_abs[c0 + q] : ((stat && a.bc > 1) ? a.nw[c0 + q] : 0.0);
        const double fr = det ? a.na_abs[r] : ((stat && a.br > 1) ? a.nv[r] : 0.0);
        const double chr = det ? a.chain_a[r] : 0.0;
        double cs[GC + 1][V];
#pragma unroll
        for (int h = 0; h <= GC; ++h)
#pragma unroll
            for (int q = 0; q < V; ++q) cs[h][q] = 0.0;
        // row relations (i, c0 + q): data columns summed, the carried column last
        auto rows_of = [&](int64_t i, double fi, const double (&v)[GC + 1][V]) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                double rs = 0.0;
#pragma unroll
                for (int h = 0; h < GC; ++h) rs += v[h][q];
                if (er.n && row_erased_res(er, i, c0 + q, a.bc)) excl_r++;
                else ratio_r = fmax(ratio_r, record(a.rep, false, i, c0 + q, rs - v[GC][q],
                                                    vb_tau_row(a, sc, fi, fc[q], v[GC][q])));
            }
        };
        auto add_col = [&](const double (&v)[GC + 1][V]) {
#pragma unroll
            for (int h = 0; h <= GC; ++h)
#pragma unroll
                for (int q = 0; q < V; ++q) cs[h][q] += v[h][q];
        };
        // two rows of blocks at a time: both rows' loads (and their row factors) in flight together
        int64_t g = 0;
        for (; g + 1 < a.Gr; g += 2) {
            const int64_t i0 = g * a.br + r, i1 = i0 + a.br;
            const double f0 = vb_row_fac(a, i0), f1 = vb_row_fac(a, i1);
            double v0[GC + 1][V], v1[GC + 1][V];
#pragma unroll
            for (int h = 0; h <= GC; ++h) {
                load_c<T, V>(C + i0 * a.ldc + h * a.bc + c0, v0[h]);
                load_c<T, V>(C + i1 * a.ldc + h * a.bc + c0, v1[h]);
            }
            rows_of(i0, f0, v0);
            add_col(v0);
            rows_of(i1, f1, v1);
            add_col(v1);
        }
        if (g < a.Gr) {
            const int64_t i0 = g * a.br + r;
            const double f0 = vb_row_fac(a, i0);
            double v0[GC + 1][V];
#pragma unroll
            for (int h = 0; h <= GC; ++h) load_c<T, V>(C + i0 * a.ldc + h * a.bc + c0, v0[h]);
            rows_of(i0, f0, v0);
            add_col(v0);
        }
        // the carried row: its row relations, then the column relations (r, j),
        // data rows summed, the carried row last
        const int64_t i = a.m + r;
        const double fi = vb_row_fac(a, i);
        double fj[GC + 1][V], cw[GC + 1][V], v[GC + 1][V];
#pragma unroll
        for (int h = 0; h <= GC; ++h)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = h * a.bc + c0 + q;
                fj[h][q] = det ? a.nb[j] : (stat ? a.qc[j] : 0.0);
                cw[h][q] = det ? a.chain_w[j] : 0.0;
            }
#pragma unroll
        for (int h = 0; h <= GC; ++h) load_c<T, V>(C + i * a.ldc + h * a.bc + c0, v[h]);
        rows_of(i, fi, v);
#pragma unroll
        for (int h = 0; h <= GC; ++h)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = h * a.bc + c0 + q;
                if (er.n && col_erased_res(er, r, j, a.br)) excl_c++;
                else ratio_c = fmax(ratio_c, record(a.rep, true, r, j, cs[h][q] - v[h][q],
                                                    vb_tau_col(a, sc, fr, chr, fj[h][q], cw[h][q], v[h][q])));
            }
    }
    fold_block(ratio_c, excl_c, &a.rep->max_ratio_c, &a.rep->n_excl_c);
    __syncthreads();   // fold_block's shared slots are reused
    fold_block(ratio_r, excl_r, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}
template <int GC>
static void launch_vblock(const double *C, const VerifyArgs &a, const ErasureRes &er, unsigned grid, hipStream_t s) {
    k_vblock<double, 2, GC><<<grid, kThreads, 0, s>>>(C, a, er);
}

// Re-read verification for b = 1 in one pass over C: tile partial sums of the
// data part, column sums of each kPartRows-row tile (pc[tile row][j]) and row
// sums of each 64V-column tile (pr[tile column][i]), the layout the product
// epilogue writes for the fused verification; k_vfused then finishes the
// relations.  A wave takes rows w, w + 4, ... of its tile, four at a time.
constexpr int64_t kPartRows = kVerifyPartRows;
template <typename T, int V>
__global__ __launch_bounds__(kThreads) void k_vpartials(const T *C, int64_t ldc, int64_t m, int64_t n, double *pc,
                                                        double *pr) {
    constexpr int NW = kThreads / kWave;
    constexpr int64_t TCW = (int64_t)kWave * V;
    __shared__ double sh[NW][TCW];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int64_t tiles_n = (n + TCW - 1) / TCW, tiles = ((m + kPartRows - 1) / kPartRows) * tiles_n;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t tm = tile / tiles_n, tn = tile - tm * tiles_n;
        const int64_t i0 = tm * kPartRows, i1 = min(m, i0 + kPartRows), j0 = tn * TCW + lane * V;
        double cs[V];
#pragma unroll
        for (int q = 0; q < V; ++q) cs[q] = 0.0;
        // rows of C are 16-byte aligned and ldc is a multiple of V: a vector that starts before n stays
        // inside its row; its elements at n and beyond are not summed
        auto add_row = [&](const double (&v)[V], double &rs) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const double x = j0 + q < n ? v[q] : 0.0;
                cs[q] += x;
                rs += x;
            }
        };
        int64_t i = i0 + w;
        for (; i + 3 * NW < i1; i += 4 * NW) {
            double v0[V], v1[V], v2[V], v3[V];
            if (j0 < n) {
                load_c<T, V>(C + i * ldc + j0, v0);
                load_c<T, V>(C + (i + NW) * ldc + j0, v1);
                load_c<T, V>(C + (i + 2 * NW) * ldc + j0, v2);
                load_c<T, V>(C + (i + 3 * NW) * ldc + j0, v3);
            } else {
#pragma unroll
                for (int q = 0; q < V; ++q) v0[q] = v1[q] = v2[q] = v3[q] = 0.0;
            }
            double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
            add_row(v0, r0);
            add_row(v1, r1);
            add_row(v2, r2);
            add_row(v3, r3);
            r0 = wave_sum(r0);
            r1 = wave_sum(r1);
            r2 = wave_sum(r2);
            r3 = wave_sum(r3);
            if (lane == 0) {
                pr[tn * m + i] = r0;
                pr[tn * m + i + NW] = r1;
                pr[tn * m + i + 2 * NW] = r2;
                pr[tn * m + i + 3 * NW] = r3;
            }
        }
        for (; i < i1; i += NW) {
            double v0[V];
            if (j0 < n) load_c<T, V>(C + i * ldc + j0, v0);
            else {
#pragma unroll
                for (int q = 0; q < V; ++q) v0[q] = 0.0;
            }
            double r0 = 0.0;
            add_row(v0, r0);
            r0 = wave_sum(r0);
            if (lane == 0) pr[tn * m + i] = r0;
        }
#pragma unroll
        for (int q = 0; q < V; ++q) sh[w][lane * V + q] = cs[q];
        __syncthreads();
        for (int64_t c = threadIdx.x; c < TCW; c += kThreads) {
            const int64_t j = tn * TCW + c;
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) t += sh[q][c];
            if (j < n) pc[tm * n + j] = t;
        }
        __syncthreads();
    }
}

// Fused verification (b = 1): the column relations of the data columns and
// the row relations of the data rows from the product epilogue's partial
// sums (pc: tiles_m x n, pr: tiles_n x m, summed over the tiles in a fixed
// order: four running sums over tiles q mod 4, then pairwise);
// the carried column and the carried row are summed from C_f directly.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vfused(const T *C, VerifyArgs a, const double *pc, const double *pr,
                                                     int64_t tiles_m, int64_t tiles_n) {
    if (a.tag && *a.tag != a.key) return;     // partials of another product: nothing is recorded
    double rc = 0.0, rr = 0.0;
    unsigned long long ec = 0, er = 0;
    const int64_t total = a.n + a.m;
    for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total; t += (int64_t)gridDim.x * kThreads) {
        // four independent running sums (tiles q mod 4) keep four loads in flight
        auto sum4 = [](const double *x, int64_t stride, int64_t cnt) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            int64_t q = 0;
            for (; q + 3 < cnt; q += 4) {
#pragma unroll
                for (int e = 0; e < 4; ++e) s4[e] += x[(q + e) * stride];
            }
            for (int e = 0; q < cnt; ++q, ++e) s4[e] += x[q * stride];
            return (s4[0] + s4[1]) + (s4[2] + s4[3]);
        };
        if (t < a.n) {
            finish_col<T>(a, C, 0, t, sum4(pc + t, a.n, tiles_m), rc, ec);
        } else {
            const int64_t i = t - a.n;
            finish_row<T>(a, C, i, 0, sum4(pr + i, a.m, tiles_n), rr, er);
        }
    }
    fold_block(rc, ec, &a.rep->max_ratio_c, &a.rep->n_excl_c);
    __syncthreads();   // fold_block's shared slots are reused by the second fold
    fold_block(rr, er, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

// Block 0: the carried column C_f[0:m, n] against the corner; block 1: the
// carried row C_f[m, 0:n] against the corner.  Fixed-order block reductions.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vfused_edges(const T *C, VerifyArgs a) {
    if (a.tag && *a.tag != a.key) return;
    __shared__ double sh[kThreads];
    const bool col = blockIdx.x == 0;
    const int64_t len = col ? a.m : a.n;
    // element t of the carried column (row); four running sums keep four loads in flight (the tail goes to the first)
    auto at = [&](int64_t t) { return col ? elem<T>::load(C + t * a.ldc + a.n) : elem<T>::load(C + a.m * a.ldc + t); };
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t t = threadIdx.x;
    for (; t + 3 * kThreads < len; t += 4 * kThreads) {
#pragma unroll
        for (int e = 0; e < 4; ++e) s4[e] += at(t + e * kThreads);
    }
    for (; t < len; t += kThreads) s4[0] += at(t);
    sh[threadIdx.x] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    double ratio = 0.0;
    unsigned long long excl = 0;
    if (threadIdx.x == 0) {
        if (col) finish_col<T>(a, C, 0, a.n, sh[0], ratio, excl);
        else finish_row<T>(a, C, a.m, 0, sh[0], ratio, excl);
    }
    if (col) fold_block(ratio, excl, &a.rep->max_ratio_c, &a.rep->n_excl_c);
    else fold_block(ratio, excl, &a.rep->max_ratio_r, &a.rep->n_excl_r);
}

template <typename T>
static int verify_typed(const abft_problem *p, const T *C, const Erasures &er, const char *ws, const VerifyScratch &sc,
                        hipStream_t s) {
    Geom g = geom_of(p);
    WsLayout L = ws_layout(p);
    TauCoef tc = tau_coef(p);
    VerifyArgs a{};
    a.m = g.m; a.n = g.n; a.br = g.br; a.bc = g.bc; a.S = g.S; a.Gr = g.Gr; a.Gc = g.Gc; a.M = g.M; a.N = g.N;
    a.ldc = p->ldc;
    a.mode = tc.mode; a.cc = tc.cc; a.cr = tc.cr; a.cst = tc.cst;
    a.na = (const double *)(ws + L.na); a.na_abs = (const double *)(ws + L.na_abs);
    a.nb = (const double *)(ws + L.nb); a.nb_abs = (const double *)(ws + L.nb_abs);
    a.chain_a = (const double *)(ws + L.chain_a); a.chain_w = (const double *)(ws + L.chain_w);
    a.qr = (const double *)(ws + L.qr); a.qc = (const double *)(ws + L.qc);
    a.nv = (const double *)(ws + L.nv); a.nw = (const double *)(ws + L.nw);
    a.scale_exp = p->dtype == ABFT_FP8_E4M3 ? (const int *)(ws + L.scale) : nullptr;
    a.rep = sc.rep;
    a.er = er;
    k_report_init<<<1, kThreads, 0, s>>>(a.rep);
    auto blocks = [](int64_t work) { return (unsigned)std::min<int64_t>((work + kThreads - 1) / kThreads, 4096); };
    // 16-byte loads when every row of C starts on a 16-byte boundary
    constexpr int VV = 16 / (int)sizeof(T);
    const bool vec = ((uintptr_t)C % 16 == 0) && (p->ldc % VV == 0);
    const int64_t V = vec ? VV : 1;
    // wide checksum blocks with few groups per row: one pass for both directions
    if (sizeof(T) == 8 && vec && g.bc % VV == 0 && g.bc >= 64 && g.Gc <= kBlockPassMaxG &&
        g.br * (g.bc / VV) >= 65536) {
        const double *Cd = (const double *)C;
        const ErasureRes ex = erasure_res(er, g.br, g.bc);
        const unsigned grid = blocks(g.br * (g.bc / 2));
        switch (g.Gc) {
        case 1: launch_vblock<1>(Cd, a, ex, grid, s); break;
        case 2: launch_vblock<2>(Cd, a, ex, grid, s); break;
        case 3: launch_vblock<3>(Cd, a, ex, grid, s); break;
        case 4: launch_vblock<4>(Cd, a, ex, grid, s); break;
        case 5: launch_vblock<5>(Cd, a, ex, grid, s); break;
        case 6: launch_vblock<6>(Cd, a, ex, grid, s); break;
        case 7: launch_vblock<7>(Cd, a, ex, grid, s); break;
        default: launch_vblock<8>(Cd, a, ex, grid, s); break;
        }
        ABFT_LAUNCHED();
        return ABFT_OK;
    }
    // b = 1: tile partials in one pass, then the relations from them
    if (g.br == 1 && g.bc == 1 && vec) {
        double *pc = sc.vpart_c, *pr = sc.vpart_r;
        const int64_t tiles_m = (g.m + kPartRows - 1) / kPartRows, tiles_n = (g.n + kWave * VV - 1) / (kWave * VV);
        k_vpartials<T, VV><<<(unsigned)std::min<int64_t>(tiles_m * tiles_n, 8192), kThreads, 0, s>>>(C, p->ldc, g.m,
                                                                                                   g.n, pc, pr);
        k_vfused<T><<<blocks(g.n + g.m), kThreads, 0, s>>>(C, a, pc, pr, tiles_m, tiles_n);
        k_vfused_edges<T><<<2, kThreads, 0, s>>>(C, a);
        ABFT_LAUNCHED();
        return ABFT_OK;
    }
    int64_t P = group_partitions(g.Gr, g.br, (g.N + V - 1) / V);
    if (P == 1) {
        if (vec) k_vcol_direct<T, VV><<<blocks(g.br * ((g.N + VV - 1) / VV)), kThreads, 0, s>>>(C, a);
        else k_vcol_direct<T, 1><<<blocks(g.br * g.N), kThreads, 0, s>>>(C, a);
    } else {
        int64_t chunk = (g.Gr + P - 1) / P;
        P = (g.Gr + chunk - 1) / chunk;
        double *part = sc.partial;
        if (vec) k_vcol_partial<T, VV><<<blocks(P * g.br * ((g.N + VV - 1) / VV)), kThreads, 0, s>>>(C, a, P, chunk, part);
        else k_vcol_partial<T, 1><<<blocks(P * g.br * g.N), kThreads, 0, s>>>(C, a, P, chunk, part);
        k_vcol_finish<T><<<blocks(g.br * g.N), kThreads, 0, s>>>(C, a, P, part);
    }
    if (g.bc == 1 && vec)
        k_vrow_block<T, VV><<<(unsigned)std::min<int64_t>(g.M, 8192), kThreads, 0, s>>>(C, a);
    else if (g.bc < 64 && (kThreads % g.bc) == 0)
        k_vrow_block<T, 1><<<(unsigned)std::min<int64_t>(g.M, 8192), kThreads, 0, s>>>(C, a);
    else
        k_vrow_strided<T><<<blocks(g.M * g.bc), kThreads, 0, s>>>(C, a);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

template <typename T>
static int verify_fused_typed(const abft_problem *p, const T *C, char *ws, int64_t tiles_m, int64_t tiles_n,
                              uint64_t key, hipStream_t s) {
    Geom g = geom_of(p);
    WsLayout L = ws_layout(p);
    TauCoef tc = tau_coef(p);
    VerifyArgs a{};
    a.m = g.m; a.n = g.n; a.br = g.br; a.bc = g.bc; a.S = g.S; a.Gr = g.Gr; a.Gc = g.Gc; a.M = g.M; a.N = g.N;
    a.ldc = p->ldc;
    a.mode = tc.mode; a.cc = tc.cc; a.cr = tc.cr; a.cst = tc.cst;
    a.na = (const double *)(ws + L.na); a.na_abs = (const double *)(ws + L.na_abs);
    a.nb = (const double *)(ws + L.nb); a.nb_abs = (const double *)(ws + L.nb_abs);
    a.chain_a = (const double *)(ws + L.chain_a); a.chain_w = (const double *)(ws + L.chain_w);
    a.qr = (const double *)(ws + L.qr); a.qc = (const double *)(ws + L.qc);
    a.nv = (const double *)(ws + L.nv); a.nw = (const double *)(ws + L.nw);
    a.scale_exp = p->dtype == ABFT_FP8_E4M3 ? (const int *)(ws + L.scale) : nullptr;
    a.rep = (abft_report *)(ws + L.report);
    a.er.n = 0;
    a.tag = (const uint64_t *)(ws + L.fused_tag);
    a.key = key;
    k_report_init_tag<<<1, kThreads, 0, s>>>(a.rep, a.tag, key);
    const unsigned blocks = (unsigned)std::min<int64_t>((g.n + g.m + kThreads - 1) / kThreads, 4096);
    k_vfused<T><<<blocks, kThreads, 0, s>>>(C, a, (const double *)(ws + L.fused_c), (const double *)(ws + L.fused_r),
                                            tiles_m, tiles_n);
    k_vfused_edges<T><<<2, kThreads, 0, s>>>(C, a);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int launch_verify_fused(const abft_problem *p, const void *C_f, char *ws, int64_t tiles_m, int64_t tiles_n,
                        uint64_t key, hipStream_t s) {
    if (p->dtype == ABFT_F64) return verify_fused_typed<double>(p, (const double *)C_f, ws, tiles_m, tiles_n, key, s);
    return verify_fused_typed<float>(p, (const float *)C_f, ws, tiles_m, tiles_n, key, s);
}

int launch_verify(const abft_problem *p, const void *C_f, const Erasures &er, char *ws, hipStream_t s) {
    const WsLayout L = ws_layout(p);
    VerifyScratch sc;
    sc.rep = (abft_report *)(ws + L.report);
    sc.vpart_c = (double *)(ws + L.vpart_c);
    sc.vpart_r = (double *)(ws + L.vpart_r);
    sc.partial = (double *)(ws + L.partial);
    return launch_verify_scratch(p, C_f, er, ws, sc, s);
}

// Bytes of scratch the verification of p on this C_f writes, by the path it
// takes (as verify_typed decides it), laid out from base (256-byte aligned
// parts; base may be null to size only).
size_t verify_scratch_layout(const abft_problem *p, const void *C_f, char *base, VerifyScratch *sc) {
    const Geom g = geom_of(p);
    const bool f64 = p->dtype == ABFT_F64;
    const int64_t VV = f64 ? 2 : 4;
    const bool vec = ((uintptr_t)C_f % 16 == 0) && (p->ldc % VV == 0);
    const int64_t V = vec ? VV : 1;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~(size_t)255; return o; };
    const size_t rep = take(sizeof(abft_report));
    size_t pc = 0, pr = 0, part = 0;
    bool use_pc = false, use_part = false;
    const bool block_pass = f64 && vec && g.bc % VV == 0 && g.bc >= 64 && g.Gc <= kBlockPassMaxG &&
                            g.br * (g.bc / VV) >= 65536;
    if (!block_pass) {
        if (g.br == 1 && g.bc == 1 && vec) {
            const int64_t tiles_m = (g.m + kPartRows - 1) / kPartRows, tiles_n = (g.n + kWave * VV - 1) / (kWave * VV);
            pc = take(sizeof(double) * tiles_m * g.n);
            pr = take(sizeof(double) * tiles_n * g.m);
            use_pc = true;
        } else {
            const int64_t P = group_partitions(g.Gr, g.br, (g.N + V - 1) / V);
            if (P > 1) {
                part = take(sizeof(double) * P * g.br * g.N);
                use_part = true;
            }
        }
    }
    if (sc) {
        sc->rep = (abft_report *)(base + rep);
        sc->vpart_c = use_pc ? (double *)(base + pc) : nullptr;
        sc->vpart_r = use_pc ? (double *)(base + pr) : nullptr;
        sc->partial = use_part ? (double *)(base + part) : nullptr;
    }
    return off;
}

int launch_verify_scratch(const abft_problem *p, const void *C_f, const Erasures &er, const char *ws,
                          const VerifyScratch &sc, hipStream_t s) {
    if (p->dtype == ABFT_F64) return verify_typed<double>(p, (const double *)C_f, er, ws, sc, s);
    return verify_typed<float>(p, (const float *)C_f, er, ws, sc, s);
}

}  // namespace abft
