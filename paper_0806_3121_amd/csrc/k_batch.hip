// Batched protected products: many independent bfloat16 products of uneven
// shapes.  Every step runs over flattened work spaces.  Each problem's range
// in a space is padded to a whole number of block iterations, so a block
// iteration belongs to one problem and finds it with one binary search on a
// block-uniform index (scalar loads).  Nothing here synchronises with the
// host or allocates, so the pass can be captured in a hipGraph.
//
// Per problem the arithmetic is that of the single-problem bfloat16 path
// (binary64 checksum sums rounded once to binary32, statistics of Sec. 3),
// except for the carried checksum blocks: the binary32 checksum rows are
// split into three bfloat16 rows hi + mid + lo that add up to them exactly,
// the product runs over the "virtual" operands [A; hi; mid; lo] and
// [Bt; hi; mid; lo] on the matrix cores, and the three (nine, for the
// corner) partial products are added in binary64 and rounded once.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "gemm_lowp_kernel.h"

namespace abft {

namespace {

constexpr int kT = 256;
constexpr int kW = 64;
constexpr int kRowsPerIter = 64;        // row statistics: rows per block iteration (16 per wave)
constexpr int kWLdsMax = 8192;          // row statistics: weights staged in LDS up to this k

struct BatchDesc {
    int64_t m, n, k, br, bc, lda, ldb, ldc, M, N, Gr, Gc;
    int64_t MV, NV;                   // virtual product rows m + 3 br, columns n + 3 bc
    int64_t PA, PB;                   // encode partitions of the group sums (A side, B side)
    const float *A32, *Bt32;
    uint16_t *A, *Bt;
    float *C;
    float *acs, *bcs;                 // binary32 checksum rows (br x k), (bc x k)
    uint16_t *asp, *bsp;              // the same split into bfloat16: (3 br x k), (3 bc x k), hi rows first
    double *grpA, *grpB;              // per-residue sums of squares (br x k), (bc x k)
    double *partA, *partB;            // encode partials [P][2][b][k] when P > 1
    float *S1, *S2;                   // product staging: rows m.. of the virtual C (3 br x ld1); columns n.. (m x 3 bc)
    int64_t ld1;                      // S1 row length: NV rounded up to 4 (16-byte rows)
    double *qr, *qc, *nv, *nw;        // threshold statistics (M, N, br, bc)
    double *rowpart;                  // strip partials of the data rows' statistics when ns > 1: A (ns x m), then B (ns x n)
    int64_t ns;                       // 128-column strips of a row: ceil(k / 128)
    double *vpart;                    // verification row partials [M][ceil(N / 1024)][bc]
    abft_report *rep;
    double cc, cr;                    // stat coefficients (lambda^2 (u^2/3)(T/2 + s))
    double cst;                       // lambda^2 (u^2/3)(1 + T/3): the stored total's rounding and accumulation
    int mode;                         // ABFT_TAU_STAT or ABFT_TAU_EXACT
    int orig;                         // index in the caller's order
    int tile;                         // the problem's own product tile shape (0 .. ABFT_BATCH_TILES-1)
    int cvec;                         // rows of C 16-byte aligned (C at 16 bytes, ldc a multiple of 4, below 2^27)
    int s1vec;                        // ld1 below 2^27 (the 16-byte stores of S1)
    // starts in the flattened work spaces: tiles of each uniform shape, then of the per-problem shapes
    int64_t s_tiles[2 * ABFT_BATCH_TILES][2];   // [map][plain]: maps of the uniform shapes, then the per-shape mixed ones
    int64_t s_quant, s_enc1, s_enc2, s_rows, s_comb, s_vcol, s_vrow, s_encB, s_rfin;
};

// Flattened work spaces (plan->n_work): s_enc1 is pass 1 of A, s_encB of B.
enum { W_QUANT = 0, W_ENC1, W_ENC2, W_ROWS, W_COMB, W_VCOL, W_VROW, W_UNALIGNED, W_ENCB, W_RFIN, W_COUNT };

// A pointer read from a descriptor, typed as global memory: offsets are added
// in the global address space, and the result is cast back to a generic
// pointer only where it is dereferenced (G<T> * -> T *), so the compiler emits
// global rather than flat memory instructions.
template <typename T> using G = T __attribute__((address_space(1)));
template <typename T>
__device__ inline G<T> *gp(T *p) {
    return (G<T> *)p;
}


// largest p with d[p].*F <= t (starts are non-decreasing; t block-uniform)
template <int64_t BatchDesc::*F>
__device__ inline int find_problem(const BatchDesc *__restrict__ d, int count, int64_t t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].*F <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A block's walk over its contiguous share of a flattened space, PER units per
// iteration: the problem is looked up again only when the walk crosses into
// the next problem's range.
template <int64_t BatchDesc::*F, int PER>
struct Walk {
    const BatchDesc *d;
    int count, p;
    int64_t end, first, last;
    __device__ Walk(const BatchDesc *d_, int count_, int64_t total) : d(d_), count(count_), p(0), end(-1) {
        const int64_t iters = (total + PER - 1) / PER, per = (iters + gridDim.x - 1) / gridDim.x;
        first = (int64_t)blockIdx.x * per * PER;
        last = min(total, first + per * PER);
    }
    __device__ const BatchDesc &at(int64_t t) {
        if (t >= end) {
            p = find_problem<F>(d, count, t);
            end = p + 1 < count ? d[p + 1].*F : INT64_MAX;
        }
        return d[p];
    }
};

typedef float v4f_ __attribute__((ext_vector_type(4)));
typedef uint32_t v4u_ __attribute__((ext_vector_type(4)));
typedef double v2d_ __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pack2(uint16_t a, uint16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

// One 16-byte load from global memory, widened to binary64.
template <typename T> struct gload;
template <> struct gload<uint16_t> {
    static constexpr int N = 8;
    __device__ static void load(const G<uint16_t> *p, double *o) {
        v4u_ v = *(const G<v4u_> *)p;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (double)bf16_to_f32((uint16_t)(v[q] & 0xFFFFu));
            o[2 * q + 1] = (double)bf16_to_f32((uint16_t)(v[q] >> 16));
        }
    }
};
template <> struct gload<float> {
    static constexpr int N = 4;
    __device__ static void load(const G<float> *p, double *o) {
        v4f_ v = *(const G<v4f_> *)p;
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
};
template <> struct gload<double> {
    static constexpr int N = 2;
    __device__ static void load(const G<double> *p, double *o) {
        v2d_ v = *(const G<v2d_> *)p;
        o[0] = v[0]; o[1] = v[1];
    }
};

// ------------------------------------------------------------------ quantize
// Unit = 8 consecutive elements of a row of A (first) or of Bt.
__global__ __launch_bounds__(kT) void kb_quantize(const BatchDesc *__restrict__ d, int count, int64_t total) {
    Walk<&BatchDesc::s_quant, kT> wk(d, count, total);
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT) {
        const BatchDesc &D = wk.at(b0);
        int64_t q = b0 - D.s_quant + threadIdx.x;
        const int64_t kv = D.k / 8, na = D.m * kv;
        if (q >= na + D.n * kv) continue;
        const bool isA = q < na;
        if (!isA) q -= na;
        const G<const float> *X0 = isA ? gp(D.A32) : gp(D.Bt32);
        if (!X0) continue;                             // this operand is already bfloat16
        const int64_t i = q / kv, c = (q - i * kv) * 8, ld = isA ? D.lda : D.ldb;
        const G<const float> *X = X0 + i * ld + c;
        v4f_ x0 = *(const G<v4f_> *)X, x1 = *(const G<v4f_> *)(X + 4);
        v4u_ o;
        o[0] = pack2(f32_to_bf16_rne(x0[0]), f32_to_bf16_rne(x0[1]));
        o[1] = pack2(f32_to_bf16_rne(x0[2]), f32_to_bf16_rne(x0[3]));
        o[2] = pack2(f32_to_bf16_rne(x1[0]), f32_to_bf16_rne(x1[1]));
        o[3] = pack2(f32_to_bf16_rne(x1[2]), f32_to_bf16_rne(x1[3]));
        *(G<v4u_> *)((isA ? gp(D.A) : gp(D.Bt)) + i * ld + c) = o;
    }
}

// ------------------------------------------------------------------ encode
// Final values of 8 consecutive checksum entries (r, l0..l0+7) of one side:
// the binary32 row, its exact bfloat16 split hi + mid + lo, and grp.
__device__ inline void enc_finish(G<float> *cs, G<uint16_t> *sp, G<double> *grp, int64_t b, int64_t k, int64_t r,
                                  int64_t l0, const double *s, const double *ss) {
    float c[8];
    uint16_t h[3][8];
    double g[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        c[e] = (float)s[e];
        g[e] = ss[e] + (double)c[e] * (double)c[e];
        uint16_t hi = f32_to_bf16_rne(c[e]);
        float r1 = c[e] - bf16_to_f32(hi);             // exact
        uint16_t mid = f32_to_bf16_rne(r1);
        float r2 = r1 - bf16_to_f32(mid);              // exact, at most 8 significant bits
        h[0][e] = hi;
        h[1][e] = mid;
        h[2][e] = f32_to_bf16_rne(r2);
    }
    G<float> *pc = cs + r * k + l0;
    *(G<v4f_> *)pc = v4f_{c[0], c[1], c[2], c[3]};
    *(G<v4f_> *)(pc + 4) = v4f_{c[4], c[5], c[6], c[7]};
    G<double> *pg = grp + r * k + l0;
#pragma unroll
    for (int e = 0; e < 8; e += 2) *(G<v2d_> *)(pg + e) = v2d_{g[e], g[e + 1]};
#pragma unroll
    for (int s3 = 0; s3 < 3; ++s3)
        *(G<v4u_> *)(sp + (s3 * b + r) * k + l0) =
            v4u_{pack2(h[s3][0], h[s3][1]), pack2(h[s3][2], h[s3][3]), pack2(h[s3][4], h[s3][5]),
                 pack2(h[s3][6], h[s3][7])};
}

// Element e of a 16-byte chunk of T, widened to binary64.
template <typename T> __device__ inline double chunk_elem(const v4u_ &w, int e);
template <> __device__ inline double chunk_elem<uint16_t>(const v4u_ &w, int e) {
    return (double)bf16_to_f32((uint16_t)((w[e / 2] >> (16 * (e % 2))) & 0xFFFFu));
}
template <> __device__ inline double chunk_elem<float>(const v4u_ &w, int e) { return (double)__uint_as_float(w[e]); }
template <> __device__ inline double chunk_elem<double>(const v4u_ &w, int e) {
    return __hiloint2double((int)w[2 * e + 1], (int)w[2 * e]);
}

// Row statistic of the data rows of a side (the thresholds' Q terms): 0 none
// here (B when br = 1: its rows are weighted by A's sums of squares, known only
// after A's pass; the row statistics pass takes them), 1 sum x^2 w with w the
// other side's per-column sums of squares (A when bc = 1), 2 ||x||_4^2.
__device__ inline int side_rowstat(const BatchDesc &D, int side) {
    return side ? (D.br == 1 ? 0 : 2) : (D.bc == 1 ? 1 : 2);
}

// Pass 1 of one side (SIDE 0: A, 1: B), unit = (partition p, residue r, strip,
// lane16): lane16 of a strip holds columns l0 = (16 strip + lane16) * 8 ..
// l0 + 7 (none past k).  Sums over the partition's groups g of X[g*b + r, l]
// and of its square; final values when the side has one partition, else
// partials.  The data rows' statistic is taken in the same read: each row's
// 16 lane partials (added over the lane's 8 columns in order) are added by a
// butterfly over the 16 lanes; with one strip that is the row's value, else
// the strip's partial, added in strip order by kb_rowsfin.  QUANT: the rows
// are read in binary32 (for the items that have them), rounded to bfloat16 and
// stored, and every sum is taken of the rounded values (quantize, pass 1 and
// the row statistics in one read of the binary32 operand).
template <bool QUANT, int SIDE>
__global__ __launch_bounds__(kT) void kb_encside(const BatchDesc *__restrict__ d, int count, int64_t total) {
    Walk<SIDE ? &BatchDesc::s_encB : &BatchDesc::s_enc1, kT> wk(d, count, total);
    const int lane16 = threadIdx.x % 16;
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT) {
        const BatchDesc &D = wk.at(b0);
        const int64_t q = b0 - (SIDE ? D.s_encB : D.s_enc1) + threadIdx.x;
        const int64_t b = SIDE ? D.bc : D.br, NG = SIDE ? D.Gc : D.Gr, P = SIDE ? D.PB : D.PA;
        const int64_t ld = SIDE ? D.ldb : D.lda, ns = D.ns, K = D.k;
        const int64_t grp = q / 16, strip = grp % ns, pr = grp / ns, r = pr % b, p = pr / b;
        if (p >= P) continue;                          // whole groups of 16 lanes
        const int64_t l0 = (strip * 16 + lane16) * 8;
        const bool has = l0 < K;
        const int rs = side_rowstat(D, SIDE);
        const int64_t ch = (NG + P - 1) / P, g0 = p * ch, g1 = min(NG, g0 + ch);
        double w[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = (rs == 1 && has) ? gp(D.grpB)[l0 + e] : 0.0;
        G<double> *rdst = rs == 0 ? nullptr
                          : ns == 1 ? (SIDE ? gp(D.qc) : gp(D.qr))
                                    : gp(D.rowpart) + (SIDE ? D.m * ns + strip * D.n : strip * D.m);
        G<uint16_t> *X = (SIDE ? gp(D.Bt) : gp(D.A)) + r * ld + l0;
        const G<const float> *X32 = QUANT ? (SIDE ? gp(D.Bt32) : gp(D.A32)) : nullptr;
        if (X32) X32 += r * ld + l0;
        double s[8], ss[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] = ss[e] = 0.0;
        // loads two rows ahead: row g + 2 is requested before row g is used
        // (quantize + pass 1 on the 512-problem batch: 1.86 ms one row at a time,
        // 1.89 one row ahead, 1.81 two rows ahead)
        v4u_ nx[2] = {}, ny[2] = {};
        auto fetch = [&](int64_t g, v4u_ *dst) {
            const int64_t o = g * b * ld;
            if (X32) {
                dst[0] = *(const G<v4u_> *)(X32 + o);
                dst[1] = *(const G<v4u_> *)(X32 + o + 4);
            } else {
                dst[0] = *(const G<v4u_> *)(X + o);
            }
        };
        if (has && g0 < g1) fetch(g0, nx);
        if (has && g0 + 1 < g1) fetch(g0 + 1, ny);
        for (int64_t g = g0; g < g1; ++g) {
            const v4u_ c0 = nx[0], c1 = nx[1];
            nx[0] = ny[0]; nx[1] = ny[1];
            if (has && g + 2 < g1) fetch(g + 2, ny);
            const int64_t o = g * b * ld;
            double x[8];
            if (!has) {
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = 0.0;
            } else if (X32) {
                uint16_t h[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    h[e] = f32_to_bf16_rne(__uint_as_float(c0[e]));
                    h[4 + e] = f32_to_bf16_rne(__uint_as_float(c1[e]));
                }
                *(G<v4u_> *)(X + o) = v4u_{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = (double)bf16_to_f32(h[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = chunk_elem<uint16_t>(c0, e);
            }
            double part = 0.0;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                s[e] += x[e];
                const double x2 = x[e] * x[e];
                ss[e] += x2;
                part += rs == 1 ? x2 * w[e] : x2 * x2;
            }
            if (rs) {
                // the 16 lanes of the strip (every lane of the group runs the same trip count)
                for (int off = 8; off > 0; off >>= 1) part += __shfl_xor(part, off, kW);
                if (lane16 == 0) rdst[g * b + r] = (ns == 1 && rs == 2) ? sqrt(part) : part;
            }
        }
        if (!has) continue;
        if (P == 1) {
            enc_finish(SIDE ? gp(D.bcs) : gp(D.acs), SIDE ? gp(D.bsp) : gp(D.asp), SIDE ? gp(D.grpB) : gp(D.grpA), b, K,
                       r, l0, s, ss);
        } else {
            G<double> *part = SIDE ? gp(D.partB) : gp(D.partA);
            G<double> *ps = part + ((2 * p) * b + r) * K + l0, *pq = part + ((2 * p + 1) * b + r) * K + l0;
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                *(G<v2d_> *)(ps + e) = v2d_{s[e], s[e + 1]};
                *(G<v2d_> *)(pq + e) = v2d_{ss[e], ss[e + 1]};
            }
        }
    }
}

// Pass 1 finish for the sides with several partitions: partials added in
// partition order.  Only the units of side `side` (0: A, 1: B).
__global__ __launch_bounds__(kT) void kb_encode2(const BatchDesc *__restrict__ d, int count, int64_t total, int side) {
    Walk<&BatchDesc::s_enc2, kT> wk(d, count, total);
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT) {
        const BatchDesc &D = wk.at(b0);
        int64_t q = b0 - D.s_enc2 + threadIdx.x;
        const int64_t kv = D.k / 8;
        const int64_t ua = D.PA > 1 ? D.br * kv : 0, ub = D.PB > 1 ? D.bc * kv : 0;
        if (q >= ua + ub) continue;
        const bool isA = q < ua;
        if (isA != (side == 0)) continue;
        if (!isA) q -= ua;
        const int64_t b = isA ? D.br : D.bc, P = isA ? D.PA : D.PB;
        const int64_t r = q / kv, l0 = (q - r * kv) * 8;
        const G<double> *part = isA ? gp(D.partA) : gp(D.partB);
        double s[8], ss[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] = ss[e] = 0.0;
        for (int64_t p = 0; p < P; ++p) {
            const G<double> *ps = part + ((2 * p) * b + r) * D.k + l0, *pq = part + ((2 * p + 1) * b + r) * D.k + l0;
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                v2d_ a = *(const G<v2d_> *)(ps + e), c = *(const G<v2d_> *)(pq + e);
                s[e] += a[0]; s[e + 1] += a[1];
                ss[e] += c[0]; ss[e + 1] += c[1];
            }
        }
        enc_finish(isA ? gp(D.acs) : gp(D.bcs), isA ? gp(D.asp) : gp(D.bsp), isA ? gp(D.grpA) : gp(D.grpB), b, D.k, r, l0, s, ss);
    }
}

// ------------------------------------------------------------------ row statistics
// The rows pass passes 1 do not take: segments per problem, each padded to
// kRowsPerIter rows: [acs rows br] [B rows n when br = 1, then bcs rows bc]
// [grpA rows br, grpB rows bc].  Data and checksum rows: sum x^2 w (the other
// side's b == 1, w = its grp) or ||x||_4^2; grp rows: ||.||_2.  Sixteen lanes
// per row, 16 rows per wave and block iteration.
__device__ inline int64_t pad_to(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// One row's statistic by a group of 16 lanes (lane16 = lane % 16).  U 16-byte
// loads per lane are in flight, kept as raw words until they are summed.
template <typename T, int MODE>   // MODE 0: sum x^4 -> sqrt; 1: sum x^2 w; 2: sum x^2 -> sqrt
__device__ inline double row_stat(const G<T> *row, int64_t k, const float *wsh, const G<double> *wg, int lane16) {
    constexpr int V = 16 / (int)sizeof(T), U = 8;
    double acc = 0.0;
    for (int64_t l0 = (int64_t)lane16 * V; l0 < k; l0 += U * 16 * V) {
        v4u_ raw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t l = l0 + (int64_t)u * 16 * V;
            if (l < k) raw[u] = *(const G<v4u_> *)(row + l);
        }
        // the same order of terms per lane as one load at a time
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t l = l0 + (int64_t)u * 16 * V;
            if (l < k) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const double x = chunk_elem<T>(raw[u], e);
                    double x2 = x * x;
                    if (MODE == 1) acc += x2 * (wsh ? (double)wsh[l + e] : wg[l + e]);
                    else if (MODE == 0) acc += x2 * x2;
                    else acc += x2;
                }
            }
        }
    }
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kW);
    return MODE == 1 ? acc : sqrt(acc);
}

// 64 rows per block iteration: 16 per wave, 4 at a time (16 lanes per row).
__global__ __launch_bounds__(kT) void kb_rowstats(const BatchDesc *__restrict__ d, int count, int64_t total) {
    __shared__ float wsh[kWLdsMax];
    const int lane = threadIdx.x % kW, wave = threadIdx.x / kW, lane16 = lane % 16;
    Walk<&BatchDesc::s_rows, kRowsPerIter> wk(d, count, total);
    const G<double> *staged = nullptr;                 // the weights wsh holds
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kRowsPerIter) {
        const BatchDesc &D = wk.at(b0);
        const int64_t q0 = b0 - D.s_rows;
        const int64_t nb = D.br == 1 ? D.n : 0;        // B data rows taken here
        const int64_t pa = pad_to(D.br, kRowsPerIter), pb = pad_to(nb + D.bc, kRowsPerIter);
        const int seg = q0 < pa ? 0 : (q0 < pa + pb ? 1 : 2);
        const int64_t r0 = seg == 0 ? q0 : (seg == 1 ? q0 - pa : q0 - pa - pb);
        const bool use_w = seg == 0 ? D.bc == 1 : (seg == 1 ? D.br == 1 : false);
        const G<double> *wg = seg == 0 ? gp(D.grpB) : gp(D.grpA);
        const bool wlds = use_w && D.k <= kWLdsMax;
        if (wlds && staged != wg) {
            __syncthreads();                           // every wave is done with the previous weights
            for (int64_t l = threadIdx.x; l < D.k; l += kT) wsh[l] = (float)wg[l];
            __syncthreads();
            staged = wg;
        }
        const float *ws = wlds ? wsh : nullptr;
#pragma unroll
        for (int e = 0; e < kRowsPerIter / 16; ++e) {
            const int64_t r = r0 + wave * (kRowsPerIter / 4) + e * 4 + lane / 16;
            double out = 0.0;
            G<double> *dst = nullptr;
            if (seg == 0) {
                if (r < D.br) {
                    const G<float> *row = gp(D.acs) + r * D.k;
                    out = use_w ? row_stat<float, 1>(row, D.k, ws, wg, lane16)
                                : row_stat<float, 0>(row, D.k, ws, wg, lane16);
                    dst = gp(D.qr) + D.m + r;
                }
            } else if (seg == 1) {
                if (r < nb) {
                    const G<uint16_t> *row = gp(D.Bt) + r * D.ldb;
                    out = use_w ? row_stat<uint16_t, 1>(row, D.k, ws, wg, lane16)
                                : row_stat<uint16_t, 0>(row, D.k, ws, wg, lane16);
                    dst = gp(D.qc) + r;
                } else if (r < nb + D.bc) {
                    const G<float> *row = gp(D.bcs) + (r - nb) * D.k;
                    out = use_w ? row_stat<float, 1>(row, D.k, ws, wg, lane16)
                                : row_stat<float, 0>(row, D.k, ws, wg, lane16);
                    dst = gp(D.qc) + D.n + (r - nb);
                }
            } else {
                if (r < D.br) {
                    out = row_stat<double, 2>(gp(D.grpA) + r * D.k, D.k, nullptr, nullptr, lane16);
                    dst = gp(D.nv) + r;
                } else if (r < D.br + D.bc) {
                    out = row_stat<double, 2>(gp(D.grpB) + (r - D.br) * D.k, D.k, nullptr, nullptr, lane16);
                    dst = gp(D.nw) + (r - D.br);
                }
            }
            if (dst && lane16 == 0) *dst = out;
        }
    }
}

// The data rows' statistics taken in strips (ns > 1): unit = a row of A (m),
// then of B (n, when pass 1 of B takes them); the strip partials added in
// strip order, then the square root for ||x||_4^2.
__global__ __launch_bounds__(kT) void kb_rowsfin(const BatchDesc *__restrict__ d, int count, int64_t total) {
    Walk<&BatchDesc::s_rfin, kT> wk(d, count, total);
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT) {
        const BatchDesc &D = wk.at(b0);
        const int64_t i = b0 - D.s_rfin + threadIdx.x;
        const int64_t nbr = side_rowstat(D, 1) ? D.n : 0;
        if (i >= D.m + nbr) continue;
        const int side = i < D.m ? 0 : 1;
        const int64_t row = side ? i - D.m : i, R = side ? D.n : D.m;
        const G<double> *pp = gp(D.rowpart) + (side ? D.m * D.ns : 0) + row;
        double acc = 0.0;
        for (int64_t t = 0; t < D.ns; ++t) acc += pp[t * R];
        const double v = side_rowstat(D, side) == 2 ? sqrt(acc) : acc;
        (side ? gp(D.qc) : gp(D.qr))[row] = v;
    }
}

// ------------------------------------------------------------------ product
// Direct-to-LDS tile (global_load_lds_dwordx4: lane L of a wave writes 16 bytes
// at base + 16 L), NS-stage ring of LDS slabs with NS - 1 slabs in flight.  A
// slab holds SLAB bytes of k per row: CPR = SLAB / 16 chunks.  Chunk kc of
// combined row rr (A rows first, then B rows) sits in slot
// kc ^ ((rr / RP) % CPR), RP = 256 / SLAB rows per 64-bank period, so the 16
// lanes of a quarter-wave reading chunk kc of 16 consecutive rows hit all 64
// banks once.  Chunks past K load a zero chunk.
template <int BM_, int BN_, int WM_, int WN_, int BPC_, int SLAB_, int NS_>
struct DCfg {
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, BPC = BPC_, SLAB = SLAB_, NS = NS_;
    static constexpr int NW = WM * WN, THREADS = 64 * NW;
    static constexpr int BK = SLAB / 2;                // bfloat16 per row and slab
    static constexpr int CPR = SLAB / 16, RP = 256 / SLAB, RPI = 1024 / SLAB;   // rows per load instruction
    static constexpr int KGS = SLAB / 64;              // 32-wide k groups per slab
    static constexpr int HDR = 256;
    static constexpr int STAGE = (BM + BN) * SLAB;
    static constexpr int LDS = HDR + NS * STAGE;
    static constexpr int LPW = (BM + BN) / RPI / NW;   // load instructions per wave and slab
    static constexpr int TMW = BM / WM / 16, TNW = BN / WN / 16;
    // s_waitcnt with vmcnt = the loads of NS - 2 later slabs (expcnt, lgkmcnt not waited)
    static constexpr int VM = LPW * (NS - 2);
    static constexpr int WAIT_AHEAD = (VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (15 << 8);
    static_assert(VM < 64, "vmcnt range");
    static_assert((BM + BN) % (RPI * NW) == 0 && BM % RPI == 0, "load split");
    static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "wave tile");
    static_assert(NS >= 2 && LDS <= 160 * 1024 / BPC, "LDS");
};
// The four tile shapes, all blocks of eight waves.  256 x 256 (waves of
// 64 x 128, 128 accumulators each) runs one block per CU.  The three smaller
// shapes run two blocks per CU (waves of 64 x 64 or 32 x 64, at most 128
// registers, at most 80 KB of LDS each), so that one block's tile start and
// end (its first slab's latency, the drain of its stores) overlap the other's
// k loop: measured on the 512-problem workload with one shape for every
// problem, 2.62 -> 2.42 ms (256 x 128), 2.70 -> 2.43 (128 x 256), 2.99 -> 2.40
// (128 x 128) against one block per CU.
typedef DCfg<256, 256, 4, 2, 1, 128, 2> Cfg0;    // 128 KB, one block per CU
typedef DCfg<256, 128, 4, 2, 2, 64, 3> Cfg1;     // 72 KB, two per CU
typedef DCfg<128, 256, 2, 4, 2, 64, 3> Cfg2;     // 72 KB
typedef DCfg<128, 128, 4, 2, 2, 128, 2> Cfg3;    // 64 KB, waves of 32 x 64
constexpr int kGemmThreads = 512;
static_assert(Cfg0::THREADS == kGemmThreads && Cfg1::THREADS == kGemmThreads && Cfg2::THREADS == kGemmThreads &&
              Cfg3::THREADS == kGemmThreads, "one block shape for every tile shape");

__device__ __align__(16) uint32_t kZeroChunk[4];      // never written: the source of chunks past K

// Tile queues: one per XCD (8), each a contiguous range [qb[x], qe[x]) of the
// flattened tiles, so the tiles an XCD runs together are neighbours and share
// operand rows in its L2.  A block takes tiles from its own XCD's queue
// (blockIdx.x % 8), then from the others in turn.  tmap (byte offset from the
// workspace) gives each tile's problem.  Map s (0 .. ABFT_BATCH_TILES-1): every
// problem with shape s; map kMix + s: the problems whose own shape
// (BatchDesc::tile) is s (the per-problem run is one launch per shape; every
// launch runs a kernel built for its one shape, which keeps each within its
// registers).
constexpr int kXcds = 8;
constexpr int kMix = ABFT_BATCH_TILES;
constexpr int kMaps = 2 * ABFT_BATCH_TILES;
// the tile shape of map c
__host__ __device__ inline int shape_of_map(int c) { return c < kMix ? c : c - kMix; }
// whether a problem with own shape `own` has tiles on map c
__host__ __device__ inline bool on_map(int c, int own) { return c < kMix || own == c - kMix; }
struct TileQueues {
    int64_t qb[kMaps][2][kXcds], qe[kMaps][2][kXcds];
    int64_t tmap[kMaps][2];
};
constexpr int kCtrWords = kXcds + 1;                   // queue counters, then the exit counter
constexpr size_t kCtlBytes = 4096;                     // counters (256 bytes) + TileQueues
static_assert(256 + sizeof(TileQueues) <= kCtlBytes, "control block");

__device__ inline int64_t next_tile(unsigned *ctr, const int64_t *qb, const int64_t *qe, int home, int &qi) {
    while (qi < kXcds) {
        const int x = (home + qi) % kXcds;
        const int64_t len = qe[x] - qb[x];
        if (len > 0) {
            const unsigned v = atomicAdd(ctr + x, 1u);
            if ((int64_t)v < len) return qb[x] + v;
        }
        ++qi;
    }
    return -1;
}

// A block-uniform value read from LDS, made visibly uniform (scalar registers)
// so that the descriptor loads it indexes are scalar loads.
__device__ inline int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lanes p and p ^ 1 (p ^ 2) of each quad exchange a value: DPP quad permutations.
__device__ inline float quad_xor1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ inline float quad_xor2(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
}
// 4 x 4 transpose inside a quad of lanes: lane p holds element (v, p) of the
// block in x[v] (a column of the matrix-core output), afterwards (p, c) in x[c]
// (a row).  Two butterfly steps, each exchanging the two elements whose index
// bit differs from the lane's.
__device__ inline void quad_transpose(v4f &x, int p) {
    const bool o1 = p & 1, o2 = p & 2;
    float s0 = o1 ? x[0] : x[1], s1 = o1 ? x[2] : x[3];
    float r0 = quad_xor1(s0), r1 = quad_xor1(s1);
    if (o1) { x[0] = r0; x[2] = r1; } else { x[1] = r0; x[3] = r1; }
    s0 = o2 ? x[0] : x[2];
    s1 = o2 ? x[1] : x[3];
    r0 = quad_xor2(s0);
    r1 = quad_xor2(s1);
    if (o2) { x[0] = r0; x[1] = r1; } else { x[2] = r0; x[3] = r1; }
}

// One tile `local` (in the problem's grouped tile order for shape CF) of
// problem D: the k loop through the LDS ring and the epilogue.  lds: the
// block's LDS (header first); fetch(): called by thread 0 during the last slab
// to take the next tile.
template <class CF, class Fetch>
__device__ __attribute__((always_inline)) inline void gemm_tile(const BatchDesc &D, int64_t local, int plain,
                                                                uint8_t *lds, Fetch fetch) {
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm = wave / CF::WN, wn = wave % CF::WN;
    const int lr = lane % 16, lq = lane / 16;
    const int64_t MV = plain ? D.m : D.MV, NV = plain ? D.n : D.NV, K = D.k;
    // grouped order: bands of GM tile rows, column by column within a band,
    // so the tiles running together share operand rows in L2
    const int64_t tm_count = (MV + CF::BM - 1) / CF::BM, tn_count = (NV + CF::BN - 1) / CF::BN;
    constexpr int GM = 1024 / CF::BM;
    const int64_t band = local / (GM * tn_count), in_band = local - band * (GM * tn_count);
    const int64_t gsz = min((int64_t)GM, tm_count - band * GM);
    const int64_t tm = band * GM + in_band % gsz, tn = in_band / gsz;
    const int64_t row0 = tm * CF::BM, col0 = tn * CF::BN;

    // The start of the row of A (of B) at row (column) offset rr of the tile: A or its checksum
    // rows (both addresses formed, then one selected; as a branch, the descriptor fields were
    // reloaded per row and the kernels spilled)
    const uint16_t *pA = D.A, *pAs = D.asp, *pB = D.Bt, *pBs = D.bsp;
    const int64_t dm = D.m, dn = D.n, lda = D.lda, ldb = D.ldb;
    auto row_a = [&](int rr) -> const uint16_t * {
        const int64_t gr = min(row0 + rr, MV - 1);
        const uint16_t *x = pA + gr * lda, *y = pAs + (gr - dm) * K;
        return gr < dm ? x : y;
    };
    auto row_b = [&](int rr) -> const uint16_t * {
        const int64_t gc = min(col0 + rr, NV - 1);
        const uint16_t *x = pB + gc * ldb, *y = pBs + (gc - dn) * K;
        return gc < dn ? x : y;
    };
    // the 16-byte chunk of combined row rr (A rows, then B rows) that lane ln fetches at k offset 0
    auto chunk_src = [&](int rr, int ln) -> const uint16_t * {
        const int kc = (ln % CF::CPR) ^ ((rr / CF::RP) % CF::CPR);
        return (rr < CF::BM ? row_a(rr) : row_b(rr - CF::BM)) + kc * 8;
    };
    // load instruction q of wave w fills the 1 KB of slab rows (w LPW + q) RPI ..: A rows, then B rows
    const uint16_t *src[CF::LPW];
#pragma unroll
    for (int q = 0; q < CF::LPW; ++q) src[q] = chunk_src((wave * CF::LPW + q) * CF::RPI + lane / CF::CPR, lane);
    const void *zero = (const void *)kZeroChunk;
    auto issue = [&](int stage, int64_t k0) {
        uint8_t *dst = lds + CF::HDR + stage * CF::STAGE + wave * CF::LPW * 1024;
        const bool full = k0 + CF::BK <= K;
#pragma unroll
        for (int q = 0; q < CF::LPW; ++q) {
            const int rr = (wave * CF::LPW + q) * CF::RPI + lane / CF::CPR;
            const int kc = (lane % CF::CPR) ^ ((rr / CF::RP) % CF::CPR);
            const void *g = (full || k0 + kc * 8 < K) ? (const void *)(src[q] + k0) : zero;
            __builtin_amdgcn_global_load_lds(g, (void *)(dst + q * 1024), 16, 0, 0);
        }
    };

    v4f acc[CF::TMW][CF::TNW];
#pragma unroll
    for (int a = 0; a < CF::TMW; ++a)
#pragma unroll
        for (int b = 0; b < CF::TNW; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int arow = wm * (CF::BM / CF::WM) + lr, brow = CF::BM + wn * (CF::BN / CF::WN) + lr;

    const int64_t nk = (K + CF::BK - 1) / CF::BK;
    // fragments of k group g of the slab in stage `stage`
    auto read = [&](int stage, int g, v4u (&fa)[CF::TMW], v4u (&fb)[CF::TNW]) {
        const uint8_t *S = lds + CF::HDR + stage * CF::STAGE;
        const int kc = 4 * g + lq;
#pragma unroll
        for (int a = 0; a < CF::TMW; ++a) {
            const int r = arow + 16 * a;
            fa[a] = *(const v4u *)(S + r * CF::SLAB + ((kc ^ ((r / CF::RP) % CF::CPR)) << 4));
        }
#pragma unroll
        for (int b = 0; b < CF::TNW; ++b) {
            const int r = brow + 16 * b;
            fb[b] = *(const v4u *)(S + r * CF::SLAB + ((kc ^ ((r / CF::RP) % CF::CPR)) << 4));
        }
    };
    auto mma = [&](const v4u (&fa)[CF::TMW], const v4u (&fb)[CF::TNW]) {
#pragma unroll
        for (int a = 0; a < CF::TMW; ++a)
#pragma unroll
            for (int b = 0; b < CF::TNW; ++b) Bf16Ops::mfma(fa[a], fb[b], acc[a][b]);
    };
    auto barrier = []() {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
#pragma unroll
    for (int s = 0; s < CF::NS - 1; ++s)
        if (s < nk) issue(s, (int64_t)s * CF::BK);
    for (int64_t kt = 0; kt < nk; ++kt) {
        // slab kt has landed once at most the loads of the NS - 2 later slabs are pending
        if (kt + CF::NS - 2 < nk) __builtin_amdgcn_s_waitcnt(CF::WAIT_AHEAD);
        else __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        // and every wave is done with slab kt - 1.  A bare barrier: the
        // fence of __syncthreads would wait for every slab in flight.
        barrier();
        if (kt + CF::NS - 1 < nk) issue((int)((kt + CF::NS - 1) % CF::NS), (kt + CF::NS - 1) * CF::BK);
        // the next tile, taken during the last slab (taken earlier, it would
        // sit reserved while idle blocks find the queues empty)
        if (kt == nk - 1 && tid == 0) fetch();
#pragma unroll
        for (int g = 0; g < CF::KGS; ++g) {
            v4u fa[CF::TMW], fb[CF::TNW];
            read((int)(kt % CF::NS), g, fa, fb);
            mma(fa, fb);
        }
    }

    // epilogue: data block -> C; rows >= m -> S1; columns >= n of data rows -> S2
    if (row0 + CF::BM <= D.m && col0 + CF::BN <= D.n && D.cvec) {
        // interior tile, aligned rows: each 4 x 4 block of a quad of lanes is transposed so that a
        // lane holds 4 consecutive columns of one row, stored with one 16-byte store (a quarter of
        // the store instructions of the element-wise form)
        const int p = lane & 3;
        G<float> *Ct = gp(D.C) + (row0 + wm * (CF::BM / CF::WM) + 4 * lq + p) * D.ldc + col0 +
                       wn * (CF::BN / CF::WN) + (lr & ~3);
#pragma unroll
        for (int a = 0; a < CF::TMW; ++a)
#pragma unroll
            for (int b = 0; b < CF::TNW; ++b) {
                v4f x = acc[a][b];
                quad_transpose(x, p);
                *(G<v4f> *)(Ct + 16 * a * D.ldc + 16 * b) = x;
            }
    } else if (row0 + CF::BM <= D.m && col0 + CF::BN <= D.n) {
        // interior tile: every element is a data element of C
        G<float> *Ct = gp(D.C) + (row0 + wm * (CF::BM / CF::WM) + 4 * lq) * D.ldc + col0 + wn * (CF::BN / CF::WN) + lr;
#pragma unroll
        for (int a = 0; a < CF::TMW; ++a)
#pragma unroll
            for (int b = 0; b < CF::TNW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) Ct[(16 * a + v) * D.ldc + 16 * b] = acc[a][b][v];
    } else {
        // edge tile: each 16 x 16 block of a wave (its bounds are wave-uniform) lying wholly in the
        // data block (C, aligned rows) or wholly in the checksum rows (S1, 16-byte rows) takes the
        // 16-byte form; only the blocks across a boundary, or in the columns >= n (S2), are stored
        // element by element (all blocks element-wise: 14.2 us per 256 x 256 edge tile, 3.7 for an
        // interior one)
        // (lane offsets in 32 bits: the 16-byte forms need ldc and ld1 below 2^27, which cvec and s1vec state)
        const int p = lane & 3;
        const int lc = (4 * lq + p) * (int)D.ldc + (lr & ~3), l1 = (4 * lq + p) * (int)D.ld1 + (lr & ~3);
#pragma unroll
        for (int a = 0; a < CF::TMW; ++a) {
#pragma unroll
            for (int b = 0; b < CF::TNW; ++b) {
                const int64_t r0 = row0 + wm * (CF::BM / CF::WM) + 16 * a, c0 = col0 + wn * (CF::BN / CF::WN) + 16 * b;
                if (r0 >= MV || c0 >= NV) continue;
                if (D.cvec && r0 + 16 <= D.m && c0 + 16 <= D.n) {
                    v4f x = acc[a][b];
                    quad_transpose(x, p);
                    *(G<v4f> *)(gp(D.C) + (r0 * D.ldc + c0) + lc) = x;
                } else if (D.s1vec && r0 >= D.m && r0 + 16 <= MV && c0 + 16 <= NV) {
                    v4f x = acc[a][b];
                    quad_transpose(x, p);
                    *(G<v4f> *)(gp(D.S1) + ((r0 - D.m) * D.ld1 + c0) + l1) = x;
                } else {
                    const int64_t gc = c0 + lr;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t gr = r0 + 4 * lq + v;
                        if (gr < MV && gc < NV) {
                            if (gr < D.m) {
                                if (gc < D.n) gp(D.C)[gr * D.ldc + gc] = acc[a][b][v];
                                else gp(D.S2)[gr * 3 * D.bc + (gc - D.n)] = acc[a][b][v];
                            } else {
                                gp(D.S1)[(gr - D.m) * D.ld1 + gc] = acc[a][b][v];
                            }
                        }
                    }
                }
            }
        }
    }
}

// The persistent product: resident blocks take tiles from the queues of map
// `mp` (all of shape CF) until they are empty; BPC blocks per CU.  ttime
// (null normally): the duration of every tile in ticks of the constant 100 MHz
// clock, for the tuner.
template <class CF, bool TIMED>
__global__ __launch_bounds__(kGemmThreads, CF::BPC == 1 ? 2 : 4) void kb_gemm(const BatchDesc *__restrict__ d, int mp,
                                                                              int plain, unsigned *ctr,
                                                                              const TileQueues *__restrict__ tq,
                                                                              uint64_t *ttime) {
    // One LDS object only: with a second one the compiler cannot tell the
    // fragment reads from the in-flight direct-to-LDS loads and waits for them.
    __shared__ __attribute__((aligned(16))) uint8_t lds[CF::LDS];
    int64_t &sh_next = *(int64_t *)lds;               // the header holds the next tile index
    const int tid = threadIdx.x;
    const int home = blockIdx.x % kXcds;
    const int64_t *qb = tq->qb[mp][plain], *qe = tq->qe[mp][plain];
    const int *tmap = (const int *)((const char *)d + tq->tmap[mp][plain]);
    int qi = 0;                                        // thread 0: queues tried so far
    if (tid == 0) sh_next = next_tile(ctr, qb, qe, home, qi);
    __syncthreads();
    int64_t t = uniform64(sh_next);
    while (t >= 0) {
        int64_t nx = -1;
        const BatchDesc &D = d[tmap[t]];
        const int64_t local = t - D.s_tiles[mp][plain];
        auto fetch = [&]() { nx = next_tile(ctr, qb, qe, home, qi); };
        uint64_t t0 = 0;
        if (TIMED) t0 = __builtin_amdgcn_s_memrealtime();
        gemm_tile<CF>(D, local, plain, lds, fetch);
        // every wave is done with the last slab's stage.  Bare barriers: the
        // tile's stores need not land before the next tile's loads (measured
        // 0.5 % faster than the fenced __syncthreads on the 512-problem batch).
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (tid == 0) {
            if (TIMED) ttime[t] = __builtin_amdgcn_s_memrealtime() - t0;
            sh_next = nx;
            __builtin_amdgcn_s_waitcnt(0xC07F);         // lgkmcnt(0): the header written before the barrier
        }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        t = uniform64(sh_next);
    }
    // the last block out resets the queue counters for the next launch
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(ctr + kXcds, 1u) == gridDim.x - 1) {
            for (int x = 0; x < kCtrWords; ++x) atomicExch(ctr + x, 0u);
        }
    }
}

// Carried checksums from the staged partial products.  Units per problem:
// C[m+q, j0..j0+3] (br x ceil(n/4): four columns each, 16-byte loads of the
// staged rows, whose length ld1 >= n + 3 is a multiple of 4), C[i, n+c]
// (m x bc), corner C[m+q, n+c] (br x bc).  Each entry: its three staged terms
// added in binary64 in order, rounded once.
__host__ __device__ inline int64_t comb_units(int64_t m, int64_t n, int64_t br, int64_t bc) {
    return br * ((n + 3) / 4) + m * bc + br * bc;
}
__global__ __launch_bounds__(kT) void kb_combine(const BatchDesc *__restrict__ d, int count, int64_t total) {
    Walk<&BatchDesc::s_comb, kT> wk(d, count, total);
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT) {
        const BatchDesc &D = wk.at(b0);
        int64_t u = b0 - D.s_comb + threadIdx.x;
        const int64_t br = D.br, bc = D.bc, n = D.n, m = D.m, NV = D.NV, n4 = (n + 3) / 4;
        if (u < br * n4) {
            const int64_t q = u / n4, j0 = (u - q * n4) * 4;
            double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s3 = 0; s3 < 3; ++s3) {
                const v4f_ x = *(const G<v4f_> *)(gp(D.S1) + (s3 * br + q) * D.ld1 + j0);
#pragma unroll
                for (int e = 0; e < 4; ++e) s[e] += (double)x[e];
            }
            G<float> *dst = gp(D.C) + (m + q) * D.ldc + j0;
            if (D.cvec && j0 + 4 <= n) {
                *(G<v4f_> *)dst = v4f_{(float)s[0], (float)s[1], (float)s[2], (float)s[3]};
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (j0 + e < n) dst[e] = (float)s[e];    // the corner columns are the third unit kind's
            }
            continue;
        }
        u -= br * n4;
        if (u < m * bc) {
            const int64_t i = u / bc, c = u - i * bc;
            double s = 0.0;
#pragma unroll
            for (int t3 = 0; t3 < 3; ++t3) s += (double)gp(D.S2)[i * 3 * bc + t3 * bc + c];
            gp(D.C)[i * D.ldc + n + c] = (float)s;
            continue;
        }
        u -= m * bc;
        if (u < br * bc) {
            const int64_t q = u / bc, c = u - q * bc;
            double s = 0.0;
#pragma unroll
            for (int s3 = 0; s3 < 3; ++s3)
#pragma unroll
                for (int t3 = 0; t3 < 3; ++t3) s += (double)gp(D.S1)[(s3 * br + q) * D.ld1 + n + t3 * bc + c];
            gp(D.C)[(m + q) * D.ldc + n + c] = (float)s;
        }
    }
}

// ------------------------------------------------------------------ verify
__global__ void kb_report_init(const BatchDesc *__restrict__ d, int count) {
    for (int p = blockIdx.x; p < count; p += gridDim.x) {
        uint64_t *w = (uint64_t *)d[p].rep;
        for (int q = threadIdx.x; q < (int)(sizeof(abft_report) / 8); q += blockDim.x) w[q] = 0;
    }
}

__device__ inline void bflag(G<abft_report> *rep, bool col, int64_t a, int64_t b, double dd, double tau) {
    if (!(fabs(dd) <= tau)) {
        unsigned long long *cnt = (unsigned long long *)(col ? &rep->n_flag_c : &rep->n_flag_r);
        unsigned long long q = atomicAdd(cnt, 1ull);
        if (q < ABFT_MAX_FLAGS) {
            G<abft_flag> *f = col ? &rep->flag_c[q] : &rep->flag_r[q];
            f->a = a; f->b = b; f->d = dd; f->tau = tau;
        }
        if (!isfinite(dd)) atomicAdd((unsigned long long *)&rep->n_nonfinite, 1ull);
    }
}

// Max ratio of a wave (all lanes on one problem) into the problem's report.
__device__ inline void bfold(G<abft_report> *rep, double ratio, bool col) {
    for (int off = kW / 2; off > 0; off >>= 1) ratio = fmax(ratio, __shfl_xor(ratio, off, kW));
    if (threadIdx.x % kW == 0 && ratio > 0) {
        unsigned long long bits;
        __builtin_memcpy(&bits, &ratio, 8);
        atomicMax((unsigned long long *)(col ? &rep->max_ratio_c : &rep->max_ratio_r), bits);
    }
}

__device__ inline double btau(const BatchDesc &D, bool col, int64_t a, int64_t b, double tot) {
    if (D.mode != ABFT_TAU_STAT) return 0.0;
    if (!isfinite(tot)) tot = 0.0;          // no rounding term: the residual is then non-finite and fails
    if (col) return sqrt(D.cc * (D.br == 1 ? gp(D.qc)[b] : gp(D.nv)[a] * gp(D.qc)[b]) + D.cst * tot * tot);
    return sqrt(D.cr * (D.bc == 1 ? gp(D.qr)[a] : gp(D.qr)[a] * gp(D.nw)[b]) + D.cst * tot * tot);
}

// Verification pass 1, one read of C: one wave per (residue r, strip of
// kVStrip columns).  The wave walks the rows i = g*br + r, g < Gr, then m + r;
// lane l keeps the column sums of columns l, l + 64, ... of the strip in
// registers, and each row's strip is folded once to its bc residues, into
// part[i][strip][c].  Column relation (r, j): the sum against C[m + r, j].
constexpr int kVCols = 16;                      // columns per lane and strip
constexpr int kVStrip = kVCols * kW;            // 1024
constexpr int kVStripV = 4 * kW;                // 256: the strip of the 16-byte form
constexpr int kVRows = 8;                       // rows loaded together by the 16-byte form
// Strips of a problem's verification (the 16-byte form when its rows are aligned).
__host__ __device__ inline int64_t vstrips(int64_t N, bool vec) {
    const int64_t w = vec ? kVStripV : kVStrip;
    return (N + w - 1) / w;
}

// The same pass where the rows of C are 16-byte aligned: strips of 256
// columns, lane l holds columns 4 l .. 4 l + 3 (one 16-byte non-temporal load
// per row), and kVRows rows are loaded before any is summed (8 KB of a wave in
// flight, few registers, so many waves).  Row partials: the lane's four
// columns have residues (4 l + q) mod bc, summed across the lanes that share
// them (bc is a power of two dividing 64).
__device__ __attribute__((always_inline)) inline void verify1_rows_vec(const BatchDesc &D, int64_t r, int64_t st,
                                                                       int64_t nst, int lane) {
    const int bc = (int)D.bc;
    const int64_t j0 = st * kVStripV + 4 * lane;       // the lane's first column
    const bool live = j0 < D.N;                        // a chunk that starts below N lies inside the row
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    auto load_row = [&](int64_t i, bool ok) {
        return (ok && live) ? __builtin_nontemporal_load((const G<v4f_> *)(gp(D.C) + i * D.ldc + j0))
                            : v4f_{0.f, 0.f, 0.f, 0.f};
    };
    auto sum_row = [&](int64_t i, bool carried, v4f_ x) {
        double y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = j0 + q < D.N ? (double)x[q] : 0.0;
            if (!carried) cs[q] += v;
            y[q] = j0 + q < D.n ? v : 0.0;
        }
        if (bc >= 4) {
            for (int off = kW / 2; off >= bc / 4; off >>= 1)
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] += __shfl_xor(y[q], off, kW);
            if (lane < bc / 4)
#pragma unroll
                for (int q = 0; q < 4; ++q) gp(D.vpart)[(i * nst + st) * bc + 4 * lane + q] = y[q];
        } else {
            double z0 = bc == 1 ? (y[0] + y[1]) + (y[2] + y[3]) : y[0] + y[2];
            double z1 = bc == 1 ? 0.0 : y[1] + y[3];
            for (int off = kW / 2; off >= 1; off >>= 1) {
                z0 += __shfl_xor(z0, off, kW);
                if (bc == 2) z1 += __shfl_xor(z1, off, kW);
            }
            if (lane == 0) {
                gp(D.vpart)[(i * nst + st) * bc] = z0;
                if (bc == 2) gp(D.vpart)[(i * nst + st) * bc + 1] = z1;
            }
        }
    };
    static_assert(kVRows == 8, "the reduce-scatter below takes 8 rows");
    for (int64_t g0 = 0; g0 < D.Gr; g0 += kVRows) {
        v4f_ x[kVRows];
#pragma unroll
        for (int q = 0; q < kVRows; ++q) x[q] = load_row((g0 + q) * D.br + r, g0 + q < D.Gr);
        if (bc == 1) {
            // bc = 1: each row's partial is its strip's sum; the 8 rows' sums across
            // the 64 lanes by a reduce-scatter (4 + 2 + 1 exchanges, then 3 within
            // groups of 8 lanes) instead of 8 full reductions
            double y[kVRows];
#pragma unroll
            for (int q = 0; q < kVRows; ++q) {
                double s = 0.0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double v = j0 + e < D.N ? (double)x[q][e] : 0.0;
                    cs[e] += v;
                    if (j0 + e < D.n) s += v;
                }
                y[q] = s;
            }
            const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
            double z[4], w[2];
#pragma unroll
            for (int h = 0; h < 4; ++h)
                z[h] = (b5 ? y[h + 4] : y[h]) + __shfl_xor(b5 ? y[h] : y[h + 4], 32, kW);
#pragma unroll
            for (int h = 0; h < 2; ++h)
                w[h] = (b4 ? z[h + 2] : z[h]) + __shfl_xor(b4 ? z[h] : z[h + 2], 16, kW);
            double v = (b3 ? w[1] : w[0]) + __shfl_xor(b3 ? w[0] : w[1], 8, kW);
            for (int off = 4; off >= 1; off >>= 1) v += __shfl_xor(v, off, kW);
            const int64_t g = g0 + 4 * b5 + 2 * b4 + (b3 ? 1 : 0);    // the row this lane now holds
            if ((lane & 7) == 0 && g < D.Gr) gp(D.vpart)[(g * D.br + r) * nst + st] = v;
        } else {
#pragma unroll
            for (int q = 0; q < kVRows; ++q)
                if (g0 + q < D.Gr) sum_row((g0 + q) * D.br + r, false, x[q]);
        }
    }
    const v4f_ x = load_row(D.m + r, true);
    sum_row(D.m + r, true, x);
    // column relations of the strip: the carried row's entries are the stored totals
    double ratio = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t j = j0 + q;
        if (j < D.N) {
            const double tot = (double)x[q];
            const double dd = cs[q] - tot;
            const double tau = btau(D, true, r, j, tot);
            bflag(gp(D.rep), true, r, j, dd, tau);
            if (isfinite(dd) && tau > 0) ratio = fmax(ratio, fabs(dd) / tau);
        }
    }
    bfold(gp(D.rep), ratio, true);
}

// VEC: this launch takes the problems whose rows of C are 16-byte aligned (the
// 16-byte form), else the others (two instantiations, so that each keeps its
// own register count and occupancy).
template <bool VEC>
__global__ __launch_bounds__(kT) void kb_verify1(const BatchDesc *__restrict__ d, int count, int64_t total) {
    const int lane = threadIdx.x % kW, wave = threadIdx.x / kW;
    Walk<&BatchDesc::s_vcol, kT / kW> wk(d, count, total);
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT / kW) {
        const BatchDesc &D = wk.at(b0);
        const int64_t u = b0 - D.s_vcol + wave;
        if ((D.cvec != 0) != VEC) continue;           // problem-uniform: the other launch's problem
        const int64_t nst = vstrips(D.N, D.cvec);
        if (u >= D.br * nst) continue;                // wave-uniform
        const int64_t r = u / nst, st = u - r * nst, j0 = st * kVStrip + lane;
        const int bc = (int)D.bc;
        if constexpr (VEC) {
            verify1_rows_vec(D, r, st, nst, lane);
            continue;
        }
        double cs[kVCols];
#pragma unroll
        for (int e = 0; e < kVCols; ++e) cs[e] = 0.0;
        auto do_row = [&](int64_t i, bool carried) {
            const G<float> *row = gp(D.C) + i * D.ldc;
            double x[kVCols], y = 0.0;
            float xf[kVCols];
#pragma unroll
            for (int e = 0; e < kVCols; ++e)           // clamped, unconditional loads: all in flight at once
                xf[e] = row[min(j0 + (int64_t)e * kW, D.N - 1)];
#pragma unroll
            for (int e = 0; e < kVCols; ++e) x[e] = j0 + (int64_t)e * kW < D.N ? (double)xf[e] : 0.0;
#pragma unroll
            for (int e = 0; e < kVCols; ++e) {
                const int64_t j = j0 + (int64_t)e * kW;
                if (!carried) cs[e] += x[e];
                if (j < D.n) y += x[e];
            }
            for (int off = kW / 2; off >= bc; off >>= 1) y += __shfl_xor(y, off, kW);
            if (lane < bc) gp(D.vpart)[(i * nst + st) * bc + lane] = y;
            return 0;
        };
        for (int64_t g = 0; g < D.Gr; ++g) do_row(g * D.br + r, false);
        do_row(D.m + r, true);
        // column relations of the strip
        const G<float> *crow = gp(D.C) + (D.m + r) * D.ldc;
        double ratio = 0.0;
#pragma unroll
        for (int e = 0; e < kVCols; ++e) {
            const int64_t j = j0 + (int64_t)e * kW;
            if (j < D.N) {
                const double tot = (double)crow[j];
                const double dd = cs[e] - tot;
                const double tau = btau(D, true, r, j, tot);
                bflag(gp(D.rep), true, r, j, dd, tau);
                if (isfinite(dd) && tau > 0) ratio = fmax(ratio, fabs(dd) / tau);
            }
        }
        bfold(gp(D.rep), ratio, true);
    }
}

// Verification pass 2: row relation (i, c) from the partials of pass 1, added
// in column order, against C[i, n + c].
__global__ __launch_bounds__(kT) void kb_verify2(const BatchDesc *__restrict__ d, int count, int64_t total) {
    Walk<&BatchDesc::s_vrow, kT> wk(d, count, total);
    for (int64_t b0 = wk.first; b0 < wk.last; b0 += kT) {
        const BatchDesc &D = wk.at(b0);
        const int64_t u = b0 - D.s_vrow + threadIdx.x;
        double ratio = 0.0;
        if (u < D.M * D.bc) {
            const int64_t i = u / D.bc, c = u - i * D.bc, nst = vstrips(D.N, D.cvec);
            double s = 0.0;
            for (int64_t w = 0; w < nst; ++w) s += gp(D.vpart)[(i * nst + w) * D.bc + c];
            const double tot = (double)gp(D.C)[i * D.ldc + D.n + c];
            const double dd = s - tot;
            const double tau = btau(D, false, i, c, tot);
            bflag(gp(D.rep), false, i, c, dd, tau);
            if (isfinite(dd) && tau > 0) ratio = fabs(dd) / tau;
        }
        bfold(gp(D.rep), ratio, false);
    }
}

// The thresholds of one problem (descriptor v), as the verification computes
// them: column relations (r, j) into tc (br x N), row relations (i, c) into tr
// (M x bc); the stored totals are read from C.
__global__ __launch_bounds__(kT) void kb_thresholds(const BatchDesc *__restrict__ d, int v, double *tc, double *tr) {
    const BatchDesc &D = d[v];
    int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t nc = D.br * D.N;
    if (u < nc) {
        const int64_t r = u / D.N, j = u - r * D.N;
        tc[u] = btau(D, true, r, j, (double)gp(D.C)[(D.m + r) * D.ldc + j]);
        return;
    }
    u -= nc;
    if (u < D.M * D.bc) {
        const int64_t i = u / D.bc, c = u - i * D.bc;
        tr[u] = btau(D, false, i, c, (double)gp(D.C)[i * D.ldc + D.n + c]);
    }
}

// ------------------------------------------------------------------ host side
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t pad_h(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

struct Parts {
    int64_t PA, PB;
    size_t acs, bcs, asp, bsp, grpA, grpB, partA, partB, S1, S2, qr, qc, nv, nw, vpart, rowpart;
    size_t total() const {
        return acs + bcs + asp + bsp + grpA + grpB + partA + partB + S1 + S2 + qr + qc + nv + nw + vpart + rowpart;
    }
};
int64_t strips_of(const abft_problem &q) { return (q.k + 127) / 128; }
Parts parts_of(const abft_problem &q) {
    Parts b;
    const int64_t Gr = q.m / q.br, Gc = q.n / q.bc;
    b.PA = std::min<int64_t>(Gr, (32 + q.br - 1) / q.br);
    b.PB = std::min<int64_t>(Gc, (32 + q.bc - 1) / q.bc);
    b.acs = align256(sizeof(float) * q.br * q.k);
    b.bcs = align256(sizeof(float) * q.bc * q.k);
    b.asp = align256(sizeof(uint16_t) * 3 * q.br * q.k);
    b.bsp = align256(sizeof(uint16_t) * 3 * q.bc * q.k);
    b.grpA = align256(sizeof(double) * q.br * q.k);
    b.grpB = align256(sizeof(double) * q.bc * q.k);
    b.partA = b.PA > 1 ? align256(sizeof(double) * 2 * b.PA * q.br * q.k) : 0;
    b.partB = b.PB > 1 ? align256(sizeof(double) * 2 * b.PB * q.bc * q.k) : 0;
    b.S1 = align256(sizeof(float) * 3 * q.br * ((q.n + 3 * q.bc + 3) / 4 * 4));
    b.S2 = align256(sizeof(float) * q.m * 3 * q.bc);
    b.qr = align256(sizeof(double) * (q.m + q.br));
    b.qc = align256(sizeof(double) * (q.n + q.bc));
    b.nv = align256(sizeof(double) * q.br);
    b.nw = align256(sizeof(double) * q.bc);
    b.vpart = align256(sizeof(double) * (q.m + q.br) * vstrips(q.n + q.bc, true) * q.bc);   // the larger count
    const int64_t ns = strips_of(q);
    b.rowpart = ns > 1 ? align256(sizeof(double) * (q.m + q.n) * ns) : 0;
    return b;
}

int check_batch_problem(const abft_problem &q) {
    if (q.dtype != ABFT_BF16) return ABFT_E_UNSUPPORTED;
    if (q.tau_mode != ABFT_TAU_STAT && q.tau_mode != ABFT_TAU_EXACT) return ABFT_E_UNSUPPORTED;
    if (q.m < 1 || q.n < 1 || q.k < 8 || q.br < 1 || q.bc < 1 || q.m % q.br || q.n % q.bc) return ABFT_E_ARG;
    if (q.k % 8 || q.lda < q.k || q.ldb < q.k || q.lda % 8 || q.ldb % 8) return ABFT_E_ARG;
    if (q.ldc < q.n + q.bc) return ABFT_E_ARG;
    if (q.bc > 64 || 64 % q.bc) return ABFT_E_UNSUPPORTED;   // row verification folds lanes to bc residues
    return ABFT_OK;
}

size_t header_bytes(int count) {
    return align256(sizeof(BatchDesc) * count) + kCtlBytes + align256(sizeof(abft_report) * count);
}

constexpr int kTileBM[ABFT_BATCH_TILES] = {Cfg0::BM, Cfg1::BM, Cfg2::BM, Cfg3::BM};
constexpr int kTileBN[ABFT_BATCH_TILES] = {Cfg0::BN, Cfg1::BN, Cfg2::BN, Cfg3::BN};

}  // namespace

// Tiles of one problem for tile shape c: [0] protected (virtual rows and
// columns), [1] data block only.
static int64_t tiles_of(const abft_problem &q, int c, int plain) {
    const int64_t R = plain ? q.m : q.m + 3 * q.br, Cn = plain ? q.n : q.n + 3 * q.bc;
    return ((R + kTileBM[c] - 1) / kTileBM[c]) * ((Cn + kTileBN[c] - 1) / kTileBN[c]);
}

// The model's tile for a problem (used until a tuned choice is given): the
// executed tile area over a per-shape efficiency, the smallest wins.  The
// efficiencies are the relative rates of the shapes on large products,
// measured on MI355X (256 x 256 = 1).
static int model_tile(const abft_problem &q) {
    static const double eff[ABFT_BATCH_TILES] = {1.0, 0.86, 0.86, 0.62};
    int best = 0;
    double cost = 0.0;
    for (int c = 0; c < ABFT_BATCH_TILES; ++c) {
        const double x = (double)tiles_of(q, c, 0) * kTileBM[c] * kTileBN[c] / eff[c];
        if (c == 0 || x < cost) { cost = x; best = c; }
    }
    return best;
}

static int64_t max_tiles(const abft_problem *probs, int count) {
    int64_t mx = 0;
    for (int c = 0; c < ABFT_BATCH_TILES; ++c) {
        int64_t n = 0;
        for (int p = 0; p < count; ++p) n += tiles_of(probs[p], c, 0);
        mx = std::max(mx, n);
    }
    return mx;
}

// per-problem tile shapes: the caller's where given (0 .. ABFT_BATCH_TILES-1), else the model's
static int tile_choice(const abft_problem *probs, const int32_t *tiles, int p) {
    return (tiles && tiles[p] >= 0 && tiles[p] < ABFT_BATCH_TILES) ? tiles[p] : model_tile(probs[p]);
}

// The tile map of the mixed shapes is sized for the largest shape count any
// choice can give (the map is rewritten when the choice changes); plus the
// tuner's per-tile durations.
static size_t tmap_bytes_any(const abft_problem *probs, int count) {
    size_t s = 0;
    for (int c = 0; c < ABFT_BATCH_TILES; ++c)
        for (int pl = 0; pl < 2; ++pl) {
            int64_t n = 0;
            for (int p = 0; p < count; ++p) n += tiles_of(probs[p], c, pl);
            s += align256(sizeof(int) * n);
        }
    for (int c = kMix; c < kMaps; ++c)                 // each mixed map sized for any choice
        for (int pl = 0; pl < 2; ++pl) {
            int64_t n = 0;
            for (int p = 0; p < count; ++p) n += tiles_of(probs[p], shape_of_map(c), pl);
            s += align256(sizeof(int) * n);
        }
    return s + align256(sizeof(uint64_t) * max_tiles(probs, count));
}

size_t batch_workspace_size(const abft_problem *probs, int count) {
    size_t s = header_bytes(count) + tmap_bytes_any(probs, count);
    for (int p = 0; p < count; ++p) s += parts_of(probs[p]).total();
    return s;
}

int batch_setup(const abft_problem *probs, const abft_batch_item *items, int count, const int32_t *tiles, void *bws,
                size_t bytes, abft_batch_plan *plan) {
    if (count < 1 || !probs || !items || !bws || !plan) return ABFT_E_ARG;
    if ((uintptr_t)bws & 255u) return ABFT_E_ARG;
    for (int p = 0; p < count; ++p) {
        int st = check_batch_problem(probs[p]);
        if (st) return st;
        if (!items[p].A_f || !items[p].B_f || !items[p].C_f) return ABFT_E_ARG;
        if (((uintptr_t)items[p].A_f | (uintptr_t)items[p].B_f) & 15u) return ABFT_E_ARG;
        if ((items[p].A32 && ((uintptr_t)items[p].A32 & 15u)) || (items[p].Bt32 && ((uintptr_t)items[p].Bt32 & 15u)))
            return ABFT_E_ARG;
        if (((uintptr_t)items[p].C_f & 3u)) return ABFT_E_ARG;
    }
    size_t need = batch_workspace_size(probs, count);
    if (bytes < need) return ABFT_E_WORKSPACE;
    // Problems in order of decreasing k; the flattened tiles are cut into 8
    // contiguous queues of equal work (tiles x k), one per XCD, so each XCD
    // runs a compact run of neighbouring tiles.
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].k > probs[b].k; });

    char *base = (char *)bws;
    const size_t off_ctr = align256(sizeof(BatchDesc) * count);
    abft_report *reps = (abft_report *)(base + off_ctr + kCtlBytes);
    TileQueues tq;
    for (int c = 0; c < kMaps; ++c)
        for (int pl = 0; pl < 2; ++pl)
            for (int x = 0; x < kXcds; ++x) tq.qb[c][pl][x] = tq.qe[c][pl][x] = 0;
    // per-tile problem maps (the uniform shapes, then the mixed one, sized for
    // any choice), the tuner's durations, then the per-problem arrays
    size_t off = header_bytes(count);
    std::vector<int> tmaps[kMaps][2];
    size_t tmap_off[kMaps][2];
    for (int c = 0; c < kMaps; ++c)
        for (int pl = 0; pl < 2; ++pl) {
            int64_t n = 0, cap = 0;
            for (int p = 0; p < count; ++p) {
                const int own = tile_choice(probs, tiles, p);
                if (on_map(c, own)) n += tiles_of(probs[p], shape_of_map(c), pl);
                cap += tiles_of(probs[p], shape_of_map(c), pl);   // any choice fits
            }
            if (cap >= (int64_t)INT32_MAX) return ABFT_E_ARG;
            tmaps[c][pl].reserve(n);
            tmap_off[c][pl] = off;
            tq.tmap[c][pl] = (int64_t)off;
            off += align256(sizeof(int) * cap);
        }
    const size_t ttime_off = off;
    off += align256(sizeof(uint64_t) * max_tiles(probs, count));
    std::vector<BatchDesc> h(count);
    int64_t ntl[kMaps][2] = {};
    int64_t w[W_COUNT] = {};
    static_assert(W_COUNT <= 12, "plan->n_work");
    for (int s = 0; s < count; ++s) {
        const int p = order[s];
        const abft_problem &q = probs[p];
        BatchDesc &D = h[s];
        D.m = q.m; D.n = q.n; D.k = q.k; D.br = q.br; D.bc = q.bc;
        D.lda = q.lda; D.ldb = q.ldb; D.ldc = q.ldc;
        D.cvec = ((uintptr_t)items[p].C_f % 16 == 0 && q.ldc % 4 == 0 && q.ldc < (1 << 27)) ? 1 : 0;
        D.M = q.m + q.br; D.N = q.n + q.bc; D.Gr = q.m / q.br; D.Gc = q.n / q.bc;
        D.MV = q.m + 3 * q.br; D.NV = q.n + 3 * q.bc; D.ld1 = (D.NV + 3) / 4 * 4;
        D.s1vec = D.ld1 < (1 << 27) ? 1 : 0;
        D.A32 = items[p].A32; D.Bt32 = items[p].Bt32;
        D.A = (uint16_t *)items[p].A_f; D.Bt = (uint16_t *)items[p].B_f; D.C = (float *)items[p].C_f;
        Parts b = parts_of(q);
        D.PA = b.PA; D.PB = b.PB;
        D.acs = (float *)(base + off); off += b.acs;
        D.bcs = (float *)(base + off); off += b.bcs;
        D.asp = (uint16_t *)(base + off); off += b.asp;
        D.bsp = (uint16_t *)(base + off); off += b.bsp;
        D.grpA = (double *)(base + off); off += b.grpA;
        D.grpB = (double *)(base + off); off += b.grpB;
        D.partA = (double *)(base + off); off += b.partA;
        D.partB = (double *)(base + off); off += b.partB;
        D.S1 = (float *)(base + off); off += b.S1;
        D.S2 = (float *)(base + off); off += b.S2;
        D.qr = (double *)(base + off); off += b.qr;
        D.qc = (double *)(base + off); off += b.qc;
        D.nv = (double *)(base + off); off += b.nv;
        D.nw = (double *)(base + off); off += b.nw;
        D.vpart = (double *)(base + off); off += b.vpart;
        D.rowpart = (double *)(base + off); off += b.rowpart;
        D.ns = strips_of(q);
        D.rep = reps + p;
        D.orig = p;
        D.tile = tile_choice(probs, tiles, p);
        TauCoef tc = tau_coef(&q);
        // the stored totals (carried rows and columns) are accumulated on the matrix cores in binary32,
        // k/4 steps of the hi, mid and lo parts: their running sums have the totals' own magnitude
        D.cc = tc.cc; D.cr = tc.cr; D.cst = tc.cst * (1.0 + ((double)q.k / 4.0) / 3.0); D.mode = q.tau_mode;
        for (int c = 0; c < kMaps; ++c) {
            for (int pl = 0; pl < 2; ++pl) {
                D.s_tiles[c][pl] = ntl[c][pl];
                const int64_t nt = on_map(c, D.tile) ? tiles_of(q, shape_of_map(c), pl) : 0;
                tmaps[c][pl].insert(tmaps[c][pl].end(), (size_t)nt, s);
                ntl[c][pl] += nt;
            }
        }
        const int64_t kv = q.k / 8;
        D.s_quant = w[W_QUANT]; w[W_QUANT] += pad_h((q.m + q.n) * kv, kT);
        const int64_t ns = strips_of(q), nbr = q.br == 1 ? 0 : q.n;   // B rows of pass 1 (else of the rows pass)
        D.s_enc1 = w[W_ENC1]; w[W_ENC1] += pad_h(b.PA * q.br * ns * 16, kT);
        D.s_encB = w[W_ENCB]; w[W_ENCB] += pad_h(b.PB * q.bc * ns * 16, kT);
        D.s_enc2 = w[W_ENC2]; w[W_ENC2] += pad_h(((b.PA > 1 ? q.br : 0) + (b.PB > 1 ? q.bc : 0)) * kv, kT);
        D.s_rows = w[W_ROWS];
        w[W_ROWS] += pad_h(q.br, kRowsPerIter) + pad_h((q.br == 1 ? q.n : 0) + q.bc, kRowsPerIter) +
                     pad_h(q.br + q.bc, kRowsPerIter);
        D.s_rfin = w[W_RFIN]; w[W_RFIN] += ns > 1 ? pad_h(q.m + nbr, kT) : 0;
        D.s_comb = w[W_COMB]; w[W_COMB] += pad_h(comb_units(q.m, q.n, q.br, q.bc), kT);
        D.s_vcol = w[W_VCOL]; w[W_VCOL] += pad_h(q.br * vstrips(q.n + q.bc, D.cvec), kT / kW);
        D.s_vrow = w[W_VROW]; w[W_VROW] += pad_h((q.m + q.br) * q.bc, kT);
        if (!D.cvec) ++w[W_UNALIGNED];
    }
    // queue cuts: equal shares of the total tile work (tile area x k)
    for (int c = 0; c < kMaps; ++c)
        for (int pl = 0; pl < 2; ++pl) {
            const std::vector<int> &tm = tmaps[c][pl];
            auto work = [&](int v) {
                const int sh = shape_of_map(c);
                return (double)kTileBM[sh] * kTileBN[sh] * (double)h[v].k;
            };
            double total = 0.0;
            for (int v : tm) total += work(v);
            double acc = 0.0;
            int64_t t = 0;
            for (int x = 0; x < kXcds; ++x) {
                tq.qb[c][pl][x] = t;
                const double goal = total * (x + 1) / kXcds;
                while (t < (int64_t)tm.size() && (x == kXcds - 1 || acc + 0.5 * work(tm[t]) <= goal))
                    acc += work(tm[t++]);
                tq.qe[c][pl][x] = t;
            }
        }
    ABFT_HIP(hipMemcpy(bws, h.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice));
    for (int c = 0; c < kMaps; ++c)
        for (int pl = 0; pl < 2; ++pl)
            if (!tmaps[c][pl].empty())
                ABFT_HIP(hipMemcpy(base + tmap_off[c][pl], tmaps[c][pl].data(), sizeof(int) * tmaps[c][pl].size(),
                                   hipMemcpyHostToDevice));
    std::vector<char> ctl(kCtlBytes, 0);                // zero counters, then the queue table
    std::memcpy(ctl.data() + 256, &tq, sizeof(tq));
    ABFT_HIP(hipMemcpy(base + off_ctr, ctl.data(), kCtlBytes, hipMemcpyHostToDevice));
    plan->bws = bws;
    plan->count = count;
    plan->dtype = ABFT_BF16;
    for (int c = 0; c < ABFT_BATCH_TILES; ++c)
        for (int pl = 0; pl < 2; ++pl) plan->n_tiles[c][pl] = ntl[c][pl];
    for (int c = 0; c < ABFT_BATCH_TILES; ++c) plan->n_shape[c] = 0;
    for (int v = 0; v < count; ++v) ++plan->n_shape[h[v].tile];
    for (int pl = 0; pl < 2; ++pl) {
        plan->n_tiles[ABFT_BATCH_MIXED][pl] = 0;
        for (int c = kMix; c < kMaps; ++c) plan->n_tiles[ABFT_BATCH_MIXED][pl] += ntl[c][pl];
    }
    plan->ttime_off = ttime_off;
    for (int e = 0; e < W_COUNT; ++e) plan->n_work[e] = w[e];
    plan->bytes = need;
    return ABFT_OK;
}

static const BatchDesc *descs(const abft_batch_plan *pl) { return (const BatchDesc *)pl->bws; }
static unsigned *counters(const abft_batch_plan *pl) {
    return (unsigned *)((char *)pl->bws + align256(sizeof(BatchDesc) * pl->count));
}
static unsigned blocks_for(int64_t work, int64_t per) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + per - 1) / per, 16384));
}

int batch_quantize(const abft_batch_plan *pl, hipStream_t s) {
    const int64_t n = pl->n_work[W_QUANT];
    kb_quantize<<<blocks_for(n, kT), kT, 0, s>>>(descs(pl), pl->count, n);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

// B first: A's row statistics are weighted by B's sums of squares when bc = 1.
int batch_encode(const abft_batch_plan *pl, bool quantize, hipStream_t s) {
    const int64_t na = pl->n_work[W_ENC1], nb = pl->n_work[W_ENCB], n2 = pl->n_work[W_ENC2];
    const int64_t nr = pl->n_work[W_ROWS], nf = pl->n_work[W_RFIN];
    if (quantize) kb_encside<true, 1><<<blocks_for(nb, kT), kT, 0, s>>>(descs(pl), pl->count, nb);
    else kb_encside<false, 1><<<blocks_for(nb, kT), kT, 0, s>>>(descs(pl), pl->count, nb);
    if (n2 > 0) kb_encode2<<<blocks_for(n2, kT), kT, 0, s>>>(descs(pl), pl->count, n2, 1);
    if (quantize) kb_encside<true, 0><<<blocks_for(na, kT), kT, 0, s>>>(descs(pl), pl->count, na);
    else kb_encside<false, 0><<<blocks_for(na, kT), kT, 0, s>>>(descs(pl), pl->count, na);
    if (n2 > 0) kb_encode2<<<blocks_for(n2, kT), kT, 0, s>>>(descs(pl), pl->count, n2, 0);
    kb_rowstats<<<blocks_for(nr, kRowsPerIter), kT, 0, s>>>(descs(pl), pl->count, nr);
    if (nf > 0) kb_rowsfin<<<blocks_for(nf, kT), kT, 0, s>>>(descs(pl), pl->count, nf);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

template <class CF>
static void launch_shape(const abft_batch_plan *pl, int mp, int plain, uint64_t *ttime, hipStream_t s) {
    // a whole number of blocks per XCD: CF::BPC per CU
    const TileQueues *tq = (const TileQueues *)((const char *)counters(pl) + 256);
    const unsigned grid = 256u * CF::BPC;
    if (ttime) kb_gemm<CF, true><<<grid, kGemmThreads, 0, s>>>(descs(pl), mp, plain, counters(pl), tq, ttime);
    else kb_gemm<CF, false><<<grid, kGemmThreads, 0, s>>>(descs(pl), mp, plain, counters(pl), tq, nullptr);
}
static void launch_gemm_map(const abft_batch_plan *pl, int mp, int plain, uint64_t *ttime, hipStream_t s) {
    switch (shape_of_map(mp)) {
    case 0: launch_shape<Cfg0>(pl, mp, plain, ttime, s); break;
    case 1: launch_shape<Cfg1>(pl, mp, plain, ttime, s); break;
    case 2: launch_shape<Cfg2>(pl, mp, plain, ttime, s); break;
    default: launch_shape<Cfg3>(pl, mp, plain, ttime, s); break;
    }
}

int batch_gemm(const abft_batch_plan *pl, int tile, uint32_t flags, hipStream_t s) {
    if (tile < 0 || tile > ABFT_BATCH_MIXED) return ABFT_E_ARG;
    const int plain = (flags & ABFT_PLAIN) ? 1 : 0;
    if (tile == ABFT_BATCH_MIXED) {                    // one launch per shape that has problems
        for (int c = kMix; c < kMaps; ++c)
            if (pl->n_shape[c - kMix]) launch_gemm_map(pl, c, plain, nullptr, s);
    } else {
        launch_gemm_map(pl, tile, plain, nullptr, s);
    }
    ABFT_LAUNCHED();
    if (!plain) {
        const int64_t n = pl->n_work[W_COMB];
        kb_combine<<<blocks_for(n, kT), kT, 0, s>>>(descs(pl), pl->count, n);
        ABFT_LAUNCHED();
    }
    return ABFT_OK;
}

int batch_verify(const abft_batch_plan *pl, hipStream_t s) {
    kb_report_init<<<(unsigned)std::min(pl->count, 1024), 64, 0, s>>>(descs(pl), pl->count);
    const int64_t nc = pl->n_work[W_VCOL], nr = pl->n_work[W_VROW], nu = pl->n_work[W_UNALIGNED];
    if (nu < pl->count) kb_verify1<true><<<blocks_for(nc, kT / kW), kT, 0, s>>>(descs(pl), pl->count, nc);
    if (nu > 0) kb_verify1<false><<<blocks_for(nc, kT / kW), kT, 0, s>>>(descs(pl), pl->count, nc);
    kb_verify2<<<blocks_for(nr, kT), kT, 0, s>>>(descs(pl), pl->count, nr);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int batch_reports(const abft_batch_plan *pl, abft_report *host, hipStream_t s) {
    const char *base = (const char *)pl->bws + align256(sizeof(BatchDesc) * pl->count) + kCtlBytes;
    ABFT_HIP(hipMemcpyAsync(host, base, sizeof(abft_report) * pl->count, hipMemcpyDeviceToHost, s));
    return ABFT_OK;
}

int batch_thresholds(const abft_batch_plan *pl, int problem, double *tc, double *tr, hipStream_t s) {
    std::vector<BatchDesc> h(pl->count);
    ABFT_HIP(hipMemcpy(h.data(), pl->bws, sizeof(BatchDesc) * pl->count, hipMemcpyDeviceToHost));
    for (int v = 0; v < pl->count; ++v)
        if (h[v].orig == problem) {
            const int64_t units = h[v].br * h[v].N + h[v].M * h[v].bc;
            kb_thresholds<<<blocks_for(units, kT), kT, 0, s>>>(descs(pl), v, tc, tr);
            ABFT_LAUNCHED();
            return ABFT_OK;
        }
    return ABFT_E_ARG;
}

// Tuner: each uniform tile shape runs once with the durations of its tiles
// recorded (after a warm-up launch); a problem's cost for a shape is the sum
// of its tiles' durations (CU time, in ticks of the 100 MHz clock).
int batch_tune(const abft_batch_plan *pl, double *costs, int32_t *best, hipStream_t s) {
    const int count = pl->count;
    std::vector<BatchDesc> h(count);
    ABFT_HIP(hipMemcpy(h.data(), pl->bws, sizeof(BatchDesc) * count, hipMemcpyDeviceToHost));
    uint64_t *ttime = (uint64_t *)((char *)pl->bws + pl->ttime_off);
    std::vector<uint64_t> tt;
    std::vector<double> cost((size_t)count * ABFT_BATCH_TILES, 0.0);
    for (int c = 0; c < ABFT_BATCH_TILES; ++c) {
        launch_gemm_map(pl, c, 0, nullptr, s);            // warm-up
        launch_gemm_map(pl, c, 0, ttime, s);
        ABFT_LAUNCHED();
        tt.resize((size_t)pl->n_tiles[c][0]);
        ABFT_HIP(hipMemcpyAsync(tt.data(), ttime, sizeof(uint64_t) * tt.size(), hipMemcpyDeviceToHost, s));
        ABFT_HIP(hipStreamSynchronize(s));
        for (int v = 0; v < count; ++v) {
            const int64_t t0 = h[v].s_tiles[c][0], t1 = v + 1 < count ? h[v + 1].s_tiles[c][0] : pl->n_tiles[c][0];
            double sum = 0.0;
            for (int64_t t = t0; t < t1; ++t) sum += (double)tt[(size_t)t];
            // CU time: the shapes that run two blocks per CU count half of each tile's duration
            cost[(size_t)h[v].orig * ABFT_BATCH_TILES + c] = c == 0 ? sum : 0.5 * sum;
        }
    }
    for (int p = 0; p < count; ++p) {
        const double *cp = &cost[(size_t)p * ABFT_BATCH_TILES];
        if (costs) std::copy(cp, cp + ABFT_BATCH_TILES, costs + (size_t)p * ABFT_BATCH_TILES);
        if (best) best[p] = (int32_t)(std::min_element(cp, cp + ABFT_BATCH_TILES) - cp);
    }
    return ABFT_OK;
}

// Launch-level choice: the whole protected product timed (device events,
// median of `reps` launches after one warm-up) with each uniform shape and
// with the per-problem shapes of the plan; returns the fastest.  The
// per-problem run is one launch per shape, each with its own tail, so the
// fastest tiles per problem need not give the fastest run.
// Candidates timed in sweeps (each once per sweep, in turn) after a warm-up
// sweep: the device clock still rises during the first launches of a run, and
// timing one candidate after another would favour the later ones.
int batch_choose(const abft_batch_plan *pl, int reps, double *ms, int32_t *choice, hipStream_t s) {
    constexpr int kCand = ABFT_BATCH_MIXED + 1;
    hipEvent_t e0, e1;
    ABFT_HIP(hipEventCreate(&e0));
    ABFT_HIP(hipEventCreate(&e1));
    std::vector<float> ts[kCand];
    int st = ABFT_OK;
    for (int r = 0; r <= reps && st == ABFT_OK; ++r) {
        for (int c = 0; c < kCand && st == ABFT_OK; ++c) {
            if (hipEventRecord(e0, s) != hipSuccess) { st = ABFT_E_HIP; break; }
            st = batch_gemm(pl, c, 0, s);
            if (st) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = ABFT_E_HIP; break; }
            float t = 0.f;
            if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) { st = ABFT_E_HIP; break; }
            if (r > 0) ts[c].push_back(t);             // sweep 0 warms up
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    double best = 0.0;
    int arg = 0;
    for (int c = 0; c < kCand; ++c) {
        std::sort(ts[c].begin(), ts[c].end());
        const double med = ts[c][ts[c].size() / 2];
        if (ms) ms[c] = med;
        if (c == 0 || med < best) { best = med; arg = c; }
    }
    if (choice) *choice = arg;
    return ABFT_OK;
}

// ------------------------------------------------------------------ tuning cache
// A text file, one line per bucket:
//   <dtype> <m bucket> <n bucket> <k bucket> <br> <bc> <arch> <problems> <cost of each shape>
// Buckets: m and n in steps of 128, k by powers of two.  The shape of a bucket
// is the one with the least summed cost over the problems measured in it.
struct CacheKey {
    int dtype;
    int64_t mb, nb, kb, br, bc;
    std::string arch;
    bool operator<(const CacheKey &o) const {
        return std::tie(dtype, mb, nb, kb, br, bc, arch) < std::tie(o.dtype, o.mb, o.nb, o.kb, o.br, o.bc, o.arch);
    }
};
struct CacheVal {
    int64_t problems = 0;
    double cost[ABFT_BATCH_TILES] = {};
};
static CacheKey cache_key(const abft_problem &q, const char *arch) {
    CacheKey k;
    k.dtype = q.dtype;
    k.mb = (q.m + 127) / 128;
    k.nb = (q.n + 127) / 128;
    int64_t kb = 0;
    while ((int64_t(1) << kb) < q.k) ++kb;
    k.kb = kb;
    k.br = q.br;
    k.bc = q.bc;
    k.arch = arch;
    return k;
}
static bool read_cache(const char *path, std::map<CacheKey, CacheVal> &out) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        CacheKey k;
        CacheVal v;
        char dt[16], arch[64];
        long long mb, nb, kb, br, bc, np;
        double c[4];
        if (std::sscanf(line, "%15s %lld %lld %lld %lld %lld %63s %lld %lf %lf %lf %lf", dt, &mb, &nb, &kb, &br, &bc,
                        arch, &np, &c[0], &c[1], &c[2], &c[3]) != 12)
            continue;
        if (std::strcmp(dt, "bf16") != 0) continue;
        k.dtype = ABFT_BF16; k.mb = mb; k.nb = nb; k.kb = kb; k.br = br; k.bc = bc; k.arch = arch;
        v.problems = np;
        for (int e = 0; e < ABFT_BATCH_TILES; ++e) v.cost[e] = c[e];
        out[k] = v;
    }
    std::fclose(f);
    return true;
}
static int best_of(const CacheVal &v) {
    return (int)(std::min_element(v.cost, v.cost + ABFT_BATCH_TILES) - v.cost);
}
static bool device_arch(std::string &arch) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return true;
}

}  // namespace abft

using namespace abft;

extern "C" {

size_t abft_batch_workspace_size(const abft_problem *probs, int count) {
    if (count < 1 || !probs) return 0;
    for (int p = 0; p < count; ++p)
        if (check_batch_problem(probs[p]) != ABFT_OK) return 0;
    return batch_workspace_size(probs, count);
}
int abft_batch_setup(const abft_problem *probs, const abft_batch_item *items, int count, void *bws, size_t bws_bytes,
                     abft_batch_plan *plan) {
    return batch_setup(probs, items, count, nullptr, bws, bws_bytes, plan);
}
int abft_batch_setup_tiles(const abft_problem *probs, const abft_batch_item *items, int count, const int32_t *tiles,
                           void *bws, size_t bws_bytes, abft_batch_plan *plan) {
    return batch_setup(probs, items, count, tiles, bws, bws_bytes, plan);
}
int abft_batch_quantize(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_quantize(plan, (hipStream_t)stream);
}
int abft_batch_encode(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_encode(plan, false, (hipStream_t)stream);
}
int abft_batch_quantize_encode(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_encode(plan, true, (hipStream_t)stream);
}
int abft_batch_gemm(const abft_batch_plan *plan, int tile, uint32_t flags, void *stream) {
    if (!plan || !plan->bws || (flags & ~ABFT_PLAIN)) return ABFT_E_ARG;
    return batch_gemm(plan, tile, flags, (hipStream_t)stream);
}
int abft_batch_tune(const abft_batch_plan *plan, double *costs, int32_t *tiles, void *stream) {
    if (!plan || !plan->bws || (!costs && !tiles)) return ABFT_E_ARG;
    return batch_tune(plan, costs, tiles, (hipStream_t)stream);
}
int abft_batch_choose(const abft_batch_plan *plan, int reps, double *ms, int32_t *choice, void *stream) {
    if (!plan || !plan->bws || reps < 1 || reps > 100 || (!ms && !choice)) return ABFT_E_ARG;
    return batch_choose(plan, reps, ms, choice, (hipStream_t)stream);
}
int abft_batch_cache_lookup(const char *path, const char *arch, const abft_problem *probs, int count, int32_t *tiles) {
    if (!path || !probs || !tiles || count < 1) return ABFT_E_ARG;
    std::string a = arch ? arch : "";
    if (!arch && !device_arch(a)) return ABFT_E_HIP;
    std::map<CacheKey, CacheVal> cache;
    read_cache(path, cache);
    int found = 0;
    for (int p = 0; p < count; ++p) {
        const auto it = cache.find(cache_key(probs[p], a.c_str()));
        tiles[p] = it == cache.end() ? -1 : best_of(it->second);
        found += it != cache.end();
    }
    return found;
}
int abft_batch_cache_store(const char *path, const char *arch, const abft_problem *probs, int count,
                           const double *costs) {
    if (!path || !probs || !costs || count < 1) return ABFT_E_ARG;
    std::string a = arch ? arch : "";
    if (!arch && !device_arch(a)) return ABFT_E_HIP;
    std::map<CacheKey, CacheVal> cache;
    read_cache(path, cache);
    std::map<CacheKey, CacheVal> fresh;
    for (int p = 0; p < count; ++p) {
        if (probs[p].dtype != ABFT_BF16) return ABFT_E_ARG;
        CacheVal &v = fresh[cache_key(probs[p], a.c_str())];
        v.problems += 1;
        for (int e = 0; e < ABFT_BATCH_TILES; ++e) v.cost[e] += costs[(size_t)p * ABFT_BATCH_TILES + e];
    }
    for (const auto &kv : fresh) cache[kv.first] = kv.second;      // a new measurement replaces the old one
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return ABFT_E_ARG;
    std::fprintf(f, "# batched product tile shapes: dtype m/128 n/128 log2(k) br bc arch problems "
                    "cost(256x256) cost(256x128) cost(128x256) cost(128x128) (ticks of 10 ns)\n");
    for (const auto &kv : cache) {
        const CacheKey &k = kv.first;
        const CacheVal &v = kv.second;
        std::fprintf(f, "bf16 %lld %lld %lld %lld %lld %s %lld %.0f %.0f %.0f %.0f\n", (long long)k.mb, (long long)k.nb,
                     (long long)k.kb, (long long)k.br, (long long)k.bc, k.arch.c_str(), (long long)v.problems, v.cost[0],
                     v.cost[1], v.cost[2], v.cost[3]);
    }
    std::fclose(f);
    return std::rename(tmp.c_str(), path) == 0 ? ABFT_OK : ABFT_E_ARG;
}
int abft_batch_verify(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_verify(plan, (hipStream_t)stream);
}
int abft_batch_reports(const abft_batch_plan *plan, abft_report *host_out, void *stream) {
    if (!plan || !plan->bws || !host_out) return ABFT_E_ARG;
    return batch_reports(plan, host_out, (hipStream_t)stream);
}
int abft_batch_thresholds(const abft_batch_plan *plan, int problem, double *tau_c, double *tau_r, void *stream) {
    if (!plan || !plan->bws || !tau_c || !tau_r || problem < 0 || problem >= plan->count) return ABFT_E_ARG;
    return batch_thresholds(plan, problem, tau_c, tau_r, (hipStream_t)stream);
}

}  // extern "C"
