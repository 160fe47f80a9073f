// Batched protected products (the batched workload: many independent
// bfloat16 products of uneven shapes).  Every step runs over flattened work
// spaces: each problem's descriptor holds the start of its range in each
// space, and a thread finds its problem by binary search.  The product is a
// persistent kernel striding over all problems' tiles.  Nothing here
// synchronises with the host or allocates, so the pass can be captured in a
// hipGraph.  The arithmetic of every step is the single-problem one
// (k_reduce.hip, gemm_lowp_kernel.h, sliver_kernel.h).
#include <algorithm>
#include <cmath>
#include <vector>

#include "gemm_lowp_kernel.h"

namespace abft {

namespace {

constexpr int kT = 256;
constexpr int kW = 64;

struct BatchDesc {
    int64_t m, n, k, br, bc, lda, ldb, ldc, M, N, Gr, Gc;
    const float *A32, *Bt32;
    uint16_t *A, *Bt;
    float *C;
    float *acs, *bcs;             // binary32 checksum rows (br x k), (bc x k)
    double *grpA, *grpB;          // per-residue sums of squares v (br x k), w (bc x k)
    double *qr, *qc, *nv, *nw;    // threshold statistics (M, N, br, bc)
    abft_report *rep;
    double cc, cr;                // stat coefficients (lambda^2 (u^2/3)(T/2 + s))
    int mode;                     // ABFT_TAU_STAT or ABFT_TAU_EXACT
    // starts in the flattened work spaces
    int64_t s_tiles[2], s_quant, s_enc, s_rows, s_many, s_vcol, s_vrow;
};

// largest p with d[p].*F <= t  (starts are non-decreasing)
template <int64_t BatchDesc::*F>
__device__ inline int find_problem(const BatchDesc *d, int count, int64_t t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].*F <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ inline int find_tile_problem(const BatchDesc *d, int count, int64_t t, int tile) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].s_tiles[tile] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline double bf(uint16_t x) { return (double)bf16_to_f32(x); }

// ------------------------------------------------------------------ quantize
__global__ __launch_bounds__(kT) void kb_quantize(const BatchDesc *d, int count, int64_t total) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef uint32_t v4u_ __attribute__((ext_vector_type(4)));
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        int p = find_problem<&BatchDesc::s_quant>(d, count, t);
        const BatchDesc &D = d[p];
        int64_t q = t - D.s_quant, kv = D.k / 8;
        bool isA = q < D.m * kv;
        if (!isA) q -= D.m * kv;
        int64_t i = q / kv, c = (q - i * kv) * 8;
        const float *X0 = isA ? D.A32 : D.Bt32;
        if (!X0) continue;                             // this operand is already bfloat16
        const float *X = X0 + i * (isA ? D.lda : D.ldb) + c;
        uint16_t *Q = isA ? D.A + i * D.lda + c : D.Bt + i * D.ldb + c;
        v4 x0 = *(const v4 *)X, x1 = *(const v4 *)(X + 4);
        v4u_ o;
        o[0] = f32_to_bf16_rne(x0[0]) | ((uint32_t)f32_to_bf16_rne(x0[1]) << 16);
        o[1] = f32_to_bf16_rne(x0[2]) | ((uint32_t)f32_to_bf16_rne(x0[3]) << 16);
        o[2] = f32_to_bf16_rne(x1[0]) | ((uint32_t)f32_to_bf16_rne(x1[1]) << 16);
        o[3] = f32_to_bf16_rne(x1[2]) | ((uint32_t)f32_to_bf16_rne(x1[3]) << 16);
        *(v4u_ *)Q = o;
    }
}

// ------------------------------------------------------------------ encode pass 1
// Per problem: br*k/8 A relations then bc*k/8 B relations; thread = 8 columns.
__global__ __launch_bounds__(kT) void kb_encode(const BatchDesc *d, int count, int64_t total) {
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kT) {
        int p = find_problem<&BatchDesc::s_enc>(d, count, t);
        const BatchDesc &D = d[p];
        int64_t q = t - D.s_enc, kv = D.k / 8;
        bool isA = q < D.br * kv;
        if (!isA) q -= D.br * kv;
        int64_t b = isA ? D.br : D.bc, G = isA ? D.Gr : D.Gc, ld = isA ? D.lda : D.ldb;
        int64_t r = q / kv, l0 = (q - r * kv) * 8;
        const uint16_t *X = (isA ? D.A : D.Bt) + r * ld + l0;
        double s[8], ss[8], v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] = ss[e] = 0.0;
        for (int64_t g = 0; g < G; ++g) {
            vec16<uint16_t>::load(X + g * b * ld, v);
#pragma unroll
            for (int e = 0; e < 8; ++e) { s[e] += v[e]; ss[e] += v[e] * v[e]; }
        }
        float *cs = (isA ? D.acs : D.bcs) + r * D.k + l0;
        double *grp = (isA ? D.grpA : D.grpB) + r * D.k + l0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float c = (float)s[e];
            cs[e] = c;
            grp[e] = ss[e] + (double)c * (double)c;
        }
    }
}

// ------------------------------------------------------------------ encode pass 2 (row statistics)
// Per problem, rows: [A m][Acs br][Bt n][Bcs bc][grpA br][grpB bc].  Data and
// checksum rows: sum x^2 w (other side's b == 1) or ||x||_4^2; grp rows: ||.||_2.
__global__ __launch_bounds__(kT) void kb_rowstats(const BatchDesc *d, int count, int64_t total) {
    __shared__ double sh[kT / kW];
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int p = find_problem<&BatchDesc::s_rows>(d, count, t);
        const BatchDesc &D = d[p];
        int64_t q = t - D.s_rows;
        int kind;                 // 0 bf16 row, 1 float row, 2 double row (L2)
        const void *row;
        const double *w = nullptr;
        double *out;
        bool use_w;
        if (q < D.m) { kind = 0; row = D.A + q * D.lda; use_w = D.bc == 1; w = D.grpB; out = D.qr + q; }
        else if ((q -= D.m) < D.br) { kind = 1; row = D.acs + q * D.k; use_w = D.bc == 1; w = D.grpB; out = D.qr + D.m + q; }
        else if ((q -= D.br) < D.n) { kind = 0; row = D.Bt + q * D.ldb; use_w = D.br == 1; w = D.grpA; out = D.qc + q; }
        else if ((q -= D.n) < D.bc) { kind = 1; row = D.bcs + q * D.k; use_w = D.br == 1; w = D.grpA; out = D.qc + D.n + q; }
        else if ((q -= D.bc) < D.br) { kind = 2; row = D.grpA + q * D.k; use_w = false; out = D.nv + q; }
        else { q -= D.br; kind = 2; row = D.grpB + q * D.k; use_w = false; out = D.nw + q; }
        double acc = 0.0;
        for (int64_t l = threadIdx.x; l < D.k; l += kT) {
            double x = kind == 0 ? bf(((const uint16_t *)row)[l])
                                 : (kind == 1 ? (double)((const float *)row)[l] : ((const double *)row)[l]);
            double x2 = x * x;
            acc += kind == 2 ? x2 : (use_w ? x2 * w[l] : x2 * x2);
        }
        for (int off = kW / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kW);
        if (threadIdx.x % kW == 0) sh[threadIdx.x / kW] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int e = 0; e < kT / kW; ++e) s += sh[e];
            *out = (kind != 2 && use_w) ? s : sqrt(s);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ product
template <class T>
__global__ __launch_bounds__(T::THREADS, T::MINB) void kb_gemm(const BatchDesc *d, int count, int64_t total, int tile) {
    __shared__ uint16_t lds[2 * T::BUF];
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int p = find_tile_problem(d, count, t, tile);
        const BatchDesc &D = d[p];
        int64_t q = t - D.s_tiles[tile];
        int64_t tn_count = (D.n + T::BN - 1) / T::BN;
        int64_t tm = q / tn_count, tn = q - tm * tn_count;
        lowp_tile<T>(D.A, D.lda, D.Bt, D.ldb, D.C, D.ldc, D.m, D.n, D.k, 1.0f, tm * T::BM, tn * T::BN, lds);
    }
}

// ------------------------------------------------------------------ carried blocks
// Per problem, "many" rows: [Bt n -> C[m+r, j]] [Bcs bc -> C[m+r, n+c]] [A m -> C[i, n+c]];
// the few rows are Acs (first two) or Bcs (last).  One wave per many row,
// binary64 accumulation, few rows in passes of 8.
__global__ __launch_bounds__(kT) void kb_sliver(const BatchDesc *d, int count, int64_t total) {
    const int lane = threadIdx.x % kW;
    const int64_t wave = ((int64_t)blockIdx.x * kT + threadIdx.x) / kW;
    const int64_t nwaves = (int64_t)gridDim.x * kT / kW;
    for (int64_t u = wave; u < total; u += nwaves) {
        int p = find_problem<&BatchDesc::s_many>(d, count, u);
        const BatchDesc &D = d[p];
        int64_t q = u - D.s_many;
        int seg;
        if (q < D.n) seg = 0;
        else if ((q -= D.n) < D.bc) seg = 1;
        else { q -= D.bc; seg = 2; }
        const uint16_t *xb = seg == 0 ? D.Bt + q * D.ldb : (seg == 2 ? D.A + q * D.lda : nullptr);
        const float *xf = seg == 1 ? D.bcs + q * D.k : nullptr;
        const float *Y = seg == 2 ? D.bcs : D.acs;
        int64_t R = seg == 2 ? D.bc : D.br;
        for (int64_t r0 = 0; r0 < R; r0 += 8) {
            double acc[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) acc[s] = 0.0;
            for (int64_t k0 = (int64_t)lane * 8; k0 < D.k; k0 += 64 * 8) {
                double xv[8], yv[8];
                if (xb) vec16<uint16_t>::load(xb + k0, xv);
                else { vec16<float>::load(xf + k0, xv); vec16<float>::load(xf + k0 + 4, xv + 4); }
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    if (r0 + s < R) {
                        vec16<float>::load(Y + (r0 + s) * D.k + k0, yv);
                        vec16<float>::load(Y + (r0 + s) * D.k + k0 + 4, yv + 4);
#pragma unroll
                        for (int e = 0; e < 8; ++e) acc[s] = fma(xv[e], yv[e], acc[s]);
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                double v = acc[s];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if (lane == 0 && r0 + s < R) {
                    int64_t rr = r0 + s;
                    float *o = seg == 0 ? D.C + (D.m + rr) * D.ldc + q
                                        : (seg == 1 ? D.C + (D.m + rr) * D.ldc + D.n + q : D.C + q * D.ldc + D.n + rr);
                    *o = (float)v;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ verify
__global__ void kb_report_init(const BatchDesc *d, int count) {
    for (int p = blockIdx.x; p < count; p += gridDim.x) {
        uint64_t *w = (uint64_t *)d[p].rep;
        for (int q = threadIdx.x; q < (int)(sizeof(abft_report) / 8); q += blockDim.x) w[q] = 0;
    }
}

__device__ inline void bflag(abft_report *rep, bool col, int64_t a, int64_t b, double dd, double tau) {
    if (!(fabs(dd) <= tau)) {
        unsigned long long *cnt = (unsigned long long *)(col ? &rep->n_flag_c : &rep->n_flag_r);
        unsigned long long q = atomicAdd(cnt, 1ull);
        if (q < ABFT_MAX_FLAGS) {
            abft_flag *f = col ? &rep->flag_c[q] : &rep->flag_r[q];
            f->a = a; f->b = b; f->d = dd; f->tau = tau;
        }
        if (!isfinite(dd)) atomicAdd((unsigned long long *)&rep->n_nonfinite, 1ull);
    }
}

// Fold the max ratio of a wave into its problem's report: one atomic per wave
// when every lane of the wave is on the same problem, else one per lane.
__device__ inline void bfold(int p, const BatchDesc *d, double ratio, bool col) {
    int p0 = __shfl(p, 0, kW);
    bool same = __all(p == p0);
    if (same) {
        for (int off = kW / 2; off > 0; off >>= 1) ratio = fmax(ratio, __shfl_xor(ratio, off, kW));
        if (threadIdx.x % kW != 0) return;
    }
    if (ratio > 0 && p >= 0) {
        unsigned long long bits;
        __builtin_memcpy(&bits, &ratio, 8);
        atomicMax((unsigned long long *)(col ? &d[p].rep->max_ratio_c : &d[p].rep->max_ratio_r), bits);
    }
}

__device__ inline double btau(const BatchDesc &D, bool col, int64_t a, int64_t b) {
    if (D.mode != ABFT_TAU_STAT) return 0.0;
    if (col) return sqrt(D.cc * (D.br == 1 ? D.qc[b] : D.nv[a] * D.qc[b]));
    return sqrt(D.cr * (D.bc == 1 ? D.qr[a] : D.qr[a] * D.nw[b]));
}

// Column relations: thread per (problem, r, j).
__global__ __launch_bounds__(kT) void kb_vcol(const BatchDesc *d, int count, int64_t total) {
    const int64_t nthreads = (int64_t)gridDim.x * kT;
    for (int64_t t0 = (int64_t)blockIdx.x * kT; t0 < total; t0 += nthreads) {
        int64_t t = t0 + threadIdx.x;
        int p = -1;
        double ratio = 0.0;
        if (t < total) {
            p = find_problem<&BatchDesc::s_vcol>(d, count, t);
            const BatchDesc &D = d[p];
            int64_t q = t - D.s_vcol, r = q / D.N, j = q - r * D.N;
            double s = 0.0;
            for (int64_t g = 0; g < D.Gr; ++g) s += (double)D.C[(g * D.br + r) * D.ldc + j];
            double dd = s - (double)D.C[(D.m + r) * D.ldc + j];
            double tau = btau(D, true, r, j);
            bflag(D.rep, true, r, j, dd, tau);
            if (isfinite(dd) && tau > 0) ratio = fabs(dd) / tau;
        }
        bfold(p, d, ratio, true);
    }
}

// Row relations: one block per (problem, row); bc divides 256.
__global__ __launch_bounds__(kT) void kb_vrow(const BatchDesc *d, int count, int64_t total) {
    __shared__ double sh[kT];
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int p = find_problem<&BatchDesc::s_vrow>(d, count, t);
        const BatchDesc &D = d[p];
        int64_t i = t - D.s_vrow;
        const float *row = D.C + i * D.ldc;
        double s = 0.0;
        for (int64_t j = threadIdx.x; j < D.n; j += kT) s += (double)row[j];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = kT / 2; w >= D.bc; w >>= 1) {
            if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        double ratio = 0.0;
        if (threadIdx.x < D.bc) {
            int64_t c = threadIdx.x;
            double dd = sh[c] - (double)row[D.n + c];
            double tau = btau(D, false, i, c);
            bflag(D.rep, false, i, c, dd, tau);
            if (isfinite(dd) && tau > 0) ratio = fabs(dd) / tau;
        }
        if (threadIdx.x < kW) bfold(p, d, ratio, false);
        __syncthreads();
    }
}

unsigned grid_of(int64_t work, int64_t per) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + per - 1) / per, 65536));
}

// Batch workspace layout: [descriptors][reports][per-problem arrays...]
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct PerProblemBytes {
    size_t acs, bcs, grpA, grpB, qr, qc, nv, nw;
    size_t total() const { return acs + bcs + grpA + grpB + qr + qc + nv + nw; }
};
PerProblemBytes per_problem_bytes(const abft_problem &q) {
    PerProblemBytes b;
    b.acs = align256(sizeof(float) * q.br * q.k);
    b.bcs = align256(sizeof(float) * q.bc * q.k);
    b.grpA = align256(sizeof(double) * q.br * q.k);
    b.grpB = align256(sizeof(double) * q.bc * q.k);
    b.qr = align256(sizeof(double) * (q.m + q.br));
    b.qc = align256(sizeof(double) * (q.n + q.bc));
    b.nv = align256(sizeof(double) * q.br);
    b.nw = align256(sizeof(double) * q.bc);
    return b;
}

int check_batch_problem(const abft_problem &q) {
    if (q.dtype != ABFT_BF16) return ABFT_E_UNSUPPORTED;
    if (q.tau_mode != ABFT_TAU_STAT && q.tau_mode != ABFT_TAU_EXACT) return ABFT_E_UNSUPPORTED;
    if (q.m < 1 || q.n < 1 || q.k < 8 || q.br < 1 || q.bc < 1 || q.m % q.br || q.n % q.bc) return ABFT_E_ARG;
    if (q.k % 8 || q.lda < q.k || q.ldb < q.k || q.lda % 8 || q.ldb % 8) return ABFT_E_ARG;
    if (q.ldc < q.n + q.bc) return ABFT_E_ARG;
    if (256 % q.bc) return ABFT_E_UNSUPPORTED;     // row verification: one block per row
    return ABFT_OK;
}

}  // namespace

size_t batch_workspace_size(const abft_problem *probs, int count) {
    size_t s = align256(sizeof(BatchDesc) * count) + align256(sizeof(abft_report) * count);
    for (int p = 0; p < count; ++p) s += per_problem_bytes(probs[p]).total();
    return s;
}

int batch_setup(const abft_problem *probs, const abft_batch_item *items, int count, void *bws, size_t bytes,
                abft_batch_plan *plan) {
    if (count < 1 || !probs || !items || !bws || !plan) return ABFT_E_ARG;
    for (int p = 0; p < count; ++p) {
        int st = check_batch_problem(probs[p]);
        if (st) return st;
        if (!items[p].A_f || !items[p].B_f || !items[p].C_f) return ABFT_E_ARG;
        if (((uintptr_t)items[p].A_f | (uintptr_t)items[p].B_f) & 15u) return ABFT_E_ARG;
        if ((items[p].A32 && ((uintptr_t)items[p].A32 & 15u)) || (items[p].Bt32 && ((uintptr_t)items[p].Bt32 & 15u)))
            return ABFT_E_ARG;
    }
    size_t need = batch_workspace_size(probs, count);
    if (bytes < need) return ABFT_E_WORKSPACE;
    char *base = (char *)bws;
    size_t off = align256(sizeof(BatchDesc) * count);
    abft_report *reps = (abft_report *)(base + off);
    off += align256(sizeof(abft_report) * count);
    std::vector<BatchDesc> h(count);
    int64_t tiles0 = 0, tiles1 = 0, quant = 0, enc = 0, rows = 0, many = 0, vcol = 0, vrow = 0;
    for (int p = 0; p < count; ++p) {
        const abft_problem &q = probs[p];
        BatchDesc &D = h[p];
        D.m = q.m; D.n = q.n; D.k = q.k; D.br = q.br; D.bc = q.bc;
        D.lda = q.lda; D.ldb = q.ldb; D.ldc = q.ldc;
        D.M = q.m + q.br; D.N = q.n + q.bc; D.Gr = q.m / q.br; D.Gc = q.n / q.bc;
        D.A32 = items[p].A32; D.Bt32 = items[p].Bt32;
        D.A = (uint16_t *)items[p].A_f; D.Bt = (uint16_t *)items[p].B_f; D.C = (float *)items[p].C_f;
        PerProblemBytes b = per_problem_bytes(q);
        D.acs = (float *)(base + off); off += b.acs;
        D.bcs = (float *)(base + off); off += b.bcs;
        D.grpA = (double *)(base + off); off += b.grpA;
        D.grpB = (double *)(base + off); off += b.grpB;
        D.qr = (double *)(base + off); off += b.qr;
        D.qc = (double *)(base + off); off += b.qc;
        D.nv = (double *)(base + off); off += b.nv;
        D.nw = (double *)(base + off); off += b.nw;
        D.rep = reps + p;
        TauCoef tc = tau_coef(&q);
        D.cc = tc.cc; D.cr = tc.cr; D.mode = q.tau_mode;
        D.s_tiles[0] = tiles0; tiles0 += ((q.m + 127) / 128) * ((q.n + 127) / 128);
        D.s_tiles[1] = tiles1; tiles1 += ((q.m + 63) / 64) * ((q.n + 63) / 64);
        D.s_quant = quant; quant += (q.m + q.n) * (q.k / 8);
        D.s_enc = enc; enc += (q.br + q.bc) * (q.k / 8);
        D.s_rows = rows; rows += (q.m + q.br) + (q.n + q.bc) + q.br + q.bc;
        D.s_many = many; many += q.n + q.bc + q.m;
        D.s_vcol = vcol; vcol += q.br * (q.n + q.bc);
        D.s_vrow = vrow; vrow += q.m + q.br;
    }
    ABFT_HIP(hipMemcpy(bws, h.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice));
    plan->bws = bws;
    plan->count = count;
    plan->dtype = probs[0].dtype;
    plan->n_tiles[0] = tiles0;
    plan->n_tiles[1] = tiles1;
    plan->n_quant = quant;
    plan->n_enc = enc;
    plan->n_rows = rows;
    plan->n_many = many;
    plan->n_vcol = vcol;
    plan->n_vrow = vrow;
    plan->bytes = need;
    return ABFT_OK;
}

static const BatchDesc *descs(const abft_batch_plan *pl) { return (const BatchDesc *)pl->bws; }

int batch_quantize(const abft_batch_plan *pl, hipStream_t s) {
    kb_quantize<<<grid_of(pl->n_quant, kT), kT, 0, s>>>(descs(pl), pl->count, pl->n_quant);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int batch_encode(const abft_batch_plan *pl, hipStream_t s) {
    kb_encode<<<grid_of(pl->n_enc, kT), kT, 0, s>>>(descs(pl), pl->count, pl->n_enc);
    kb_rowstats<<<(unsigned)std::min<int64_t>(pl->n_rows, 65536), kT, 0, s>>>(descs(pl), pl->count, pl->n_rows);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

using BatchTile0 = LowpTile<Bf16Ops, 128, 128, 64, 2, 2, 8, 2>;
using BatchTile1 = LowpTile<Bf16Ops, 64, 64, 64, 2, 2, 8, 4>;

int batch_gemm(const abft_batch_plan *pl, int tile, uint32_t flags, hipStream_t s) {
    if (tile != 0 && tile != 1) return ABFT_E_ARG;
    const int64_t tiles = pl->n_tiles[tile];
    if (tile == 0)
        kb_gemm<BatchTile0><<<(unsigned)std::min<int64_t>(tiles, 256 * 2), BatchTile0::THREADS, 0, s>>>(
            descs(pl), pl->count, tiles, 0);
    else
        kb_gemm<BatchTile1><<<(unsigned)std::min<int64_t>(tiles, 256 * 4), BatchTile1::THREADS, 0, s>>>(
            descs(pl), pl->count, tiles, 1);
    ABFT_LAUNCHED();
    if (!(flags & ABFT_PLAIN)) {
        kb_sliver<<<grid_of(pl->n_many, kT / kW), kT, 0, s>>>(descs(pl), pl->count, pl->n_many);
        ABFT_LAUNCHED();
    }
    return ABFT_OK;
}

int batch_verify(const abft_batch_plan *pl, hipStream_t s) {
    kb_report_init<<<(unsigned)std::min(pl->count, 1024), 64, 0, s>>>(descs(pl), pl->count);
    kb_vcol<<<grid_of(pl->n_vcol, kT), kT, 0, s>>>(descs(pl), pl->count, pl->n_vcol);
    kb_vrow<<<(unsigned)std::min<int64_t>(pl->n_vrow, 65536), kT, 0, s>>>(descs(pl), pl->count, pl->n_vrow);
    ABFT_LAUNCHED();
    return ABFT_OK;
}

int batch_reports(const abft_batch_plan *pl, abft_report *host, hipStream_t s) {
    const char *base = (const char *)pl->bws + align256(sizeof(BatchDesc) * pl->count);
    ABFT_HIP(hipMemcpyAsync(host, base, sizeof(abft_report) * pl->count, hipMemcpyDeviceToHost, s));
    return ABFT_OK;
}

int batch_tune(const abft_batch_plan *pl, int *best, hipStream_t s) {
    float t[2];
    hipEvent_t e0, e1;
    ABFT_HIP(hipEventCreate(&e0));
    ABFT_HIP(hipEventCreate(&e1));
    for (int tile = 0; tile < 2; ++tile) {
        int st = batch_gemm(pl, tile, ABFT_PLAIN, s);          // warm-up
        if (st) return st;
        ABFT_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r)
            if ((st = batch_gemm(pl, tile, ABFT_PLAIN, s))) return st;
        ABFT_HIP(hipEventRecord(e1, s));
        ABFT_HIP(hipEventSynchronize(e1));
        ABFT_HIP(hipEventElapsedTime(&t[tile], e0, e1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best = t[1] < t[0] ? 1 : 0;
    return ABFT_OK;
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
    return batch_setup(probs, items, count, bws, bws_bytes, plan);
}
int abft_batch_quantize(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_quantize(plan, (hipStream_t)stream);
}
int abft_batch_encode(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_encode(plan, (hipStream_t)stream);
}
int abft_batch_gemm(const abft_batch_plan *plan, int tile, uint32_t flags, void *stream) {
    if (!plan || !plan->bws || (flags & ~ABFT_PLAIN)) return ABFT_E_ARG;
    return batch_gemm(plan, tile, flags, (hipStream_t)stream);
}
int abft_batch_tune(const abft_batch_plan *plan, int *best_tile, void *stream) {
    if (!plan || !plan->bws || !best_tile) return ABFT_E_ARG;
    return batch_tune(plan, best_tile, (hipStream_t)stream);
}
int abft_batch_verify(const abft_batch_plan *plan, void *stream) {
    if (!plan || !plan->bws) return ABFT_E_ARG;
    return batch_verify(plan, (hipStream_t)stream);
}
int abft_batch_reports(const abft_batch_plan *plan, abft_report *host_out, void *stream) {
    if (!plan || !plan->bws || !host_out) return ABFT_E_ARG;
    return batch_reports(plan, host_out, (hipStream_t)stream);
}

}  // extern "C"
