// Low-precision product, direct-to-LDS variant: 256 x 256 block, 2*WM waves
// (WM = 4: eight waves of 64 x 128, two per SIMD; WM = 2: four waves of
// 128 x 128).  Operand slabs of 128 bytes of k per row go global -> LDS
// directly (global_load_lds_dwordx4: lane L of a wave writes 16 bytes at
// base + 16 L; measured on gfx950), double-buffered, with no register staging
// and no LDS write instructions.  Each slab is two k groups of 64 bytes, the
// same chunks for A and B: bfloat16 (16 x 16 x 32 instruction) takes chunk
// 4 g + lane / 16 of group g per lane, FP8 (32 x 32 x 64 instruction) chunks
// 4 g + 2 (lane / 32) and the next.  Both run a software pipeline over the
// groups with the slab's barrier between them (see the main loops).
//
// LDS layout per slab and operand: row r occupies 128 bytes = 8 chunks of 16
// bytes; chunk kc of row r is stored at slot kc ^ ((r >> 1) & 7).  The 16 lanes
// of a quarter-wave read chunk kc of 16 consecutive rows: (r & 1, slot) then
// covers all 16 four-bank groups, so fragment reads are conflict-free.  The
// swizzle is applied on the global side: lane L of a load instruction fetches
// the chunk that belongs in slot L % 8 of row L / 8.
//
// Rows beyond M (columns beyond N) load a clamped valid row; they only feed
// results that are not stored.  K must be a multiple of the slab (128 bytes);
// other K use the padded-LDS kernel of gemm_lowp_kernel.h.
#pragma once

#include "gemm_lowp_kernel.h"
#include "gemm_mfma2_kernel.h"

namespace abft {

template <class Ops, int WM = 2, bool FUSED = false, int GROUP_M = 8>
__global__ __launch_bounds__(128 * WM, 1) void k_gemm_lowp2(const typename Ops::E *__restrict__ A, int64_t lda,
                                                       const typename Ops::E *__restrict__ Bt, int64_t ldb,
                                                       float *__restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                                       int64_t K, const int *__restrict__ scale_exp, EpiArgs epi) {
    typedef typename Ops::E E;
    constexpr int BM = 256, BN = 256;
    constexpr int SLAB = 128;                          // bytes of k per row and slab
    constexpr int BK = SLAB / (int)sizeof(E);          // elements of k per slab
    constexpr int VEC = 16 / (int)sizeof(E);           // elements per 16-byte chunk
    constexpr int STAGE = (BM + BN) * SLAB;            // 64 KB per slab of both operands
    constexpr int HDR = 256;                           // keeps every LDS base address non-zero
    __shared__ __attribute__((aligned(16))) uint8_t lds[HDR + 2 * STAGE];

    const int64_t tiles_m = (M + BM - 1) / BM, tiles_n = (N + BN - 1) / BN;
    int64_t tm, tn;
    tile_of<GROUP_M>(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = tm * BM, col0 = tn * BN;

    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wm = wave / 2, wn = wave % 2;
    constexpr int NW = 2 * WM;                         // waves per block
    constexpr int LPW = 32 / NW;                       // load instructions per wave and operand
    constexpr int TMW = 16 / WM;                       // 16-row MFMA tiles per wave along M (wave tile 256/WM x 128)

    // global sources of this lane's A and B chunks per slab
    const E *srcA[LPW], *srcB[LPW];
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
        int c = (wave * LPW + q) * 64 + lane;          // chunk index within the operand's slab
        int r = c / 8, slot = c % 8;
        int kc = slot ^ ((r >> 1) & 7);
        int64_t ga = row0 + r < M ? row0 + r : M - 1;
        int64_t gb = col0 + r < N ? col0 + r : N - 1;
        srcA[q] = A + ga * lda + kc * VEC;
        srcB[q] = Bt + gb * ldb + kc * VEC;
    }
    auto issue = [&](int buf, int64_t k0) {
        uint8_t *base = lds + HDR + buf * STAGE + wave * LPW * 1024;
#pragma unroll
        for (int q = 0; q < LPW; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(srcA[q] + k0), (void *)(base + q * 1024), 16, 0, 0);
#pragma unroll
        for (int q = 0; q < LPW; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(srcB[q] + k0), (void *)(base + BM * SLAB + q * 1024), 16,
                                             0, 0);
    };

    v4f acc[TMW][8];
#pragma unroll
    for (int a = 0; a < TMW; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    // fragment addresses: row r = wave-tile base + 16 a + lane % 16, chunk kc = 4 g + lane / 16
    const int lr = lane % 16, lq = lane / 16;
    const int arow = wm * (BM / WM) + lr, brow = wn * 128 + lr;

    const int64_t nk = K / BK;
    if constexpr (Ops::MT == 32) {
        // FP8 through the 32 x 32 x 64 instruction: the pipeline of the
        // bfloat16 branch below with two 64-deep groups per slab.  A fragment
        // is 32 bytes of k (chunks 4 g + 2 (lane / 32) and the next) of row
        // lane % 32 of a 32-row tile; the wave tile is TA x TB such tiles.
        // After the k loop the accumulators are moved into the 16 x 16 layout
        // of the other branches through LDS, so the epilogue is shared.
        typedef typename Ops::v8i v8i;
        constexpr int TA = (BM / WM) / 32, TB = 128 / 32;
        static_assert(TA * TB * 16 == TMW * 8 * 4, "same accumulator count as the 16 x 16 layout");
        constexpr int NRD = (TA + TB) * 2;             // 16-byte LDS reads per group
        static_assert(NRD % 4 == 0 && NRD / 2 <= TA * TB && LPW + 4 <= TA * TB, "one MFMA per scheduling group");
        v16f acc32[TA][TB];
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc32[a][b][v] = 0.f;
        const int lr = lane % 32, lh = lane / 32;
        const int ar = wm * (BM / WM) + lr, br = wn * 128 + lr;
        v8i fa0[TA], fb0[TB], fa1[TA], fb1[TB];
        auto frag = [&](const uint8_t *S, int r, int g) {
            const int k0 = 4 * g + 2 * lh, sw = (r >> 1) & 7;
            typedef int v4i __attribute__((ext_vector_type(4)));
            const v4i lo = *(const v4i *)(S + r * SLAB + ((k0 ^ sw) << 4));
            const v4i hi = *(const v4i *)(S + r * SLAB + (((k0 + 1) ^ sw) << 4));
            return (v8i)__builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        };
        auto read = [&](int buf, int g, v8i (&fa)[TA], v8i (&fb)[TB]) {
            const uint8_t *As = lds + HDR + buf * STAGE, *Bs = As + BM * SLAB;
#pragma unroll
            for (int a = 0; a < TA; ++a) fa[a] = frag(As, ar + 32 * a, g);
#pragma unroll
            for (int b = 0; b < TB; ++b) fb[b] = frag(Bs, br + 32 * b, g);
        };
        auto mma = [&](const v8i (&fa)[TA], const v8i (&fb)[TB]) {
#pragma unroll
            for (int a = 0; a < TA; ++a)
#pragma unroll
                for (int b = 0; b < TB; ++b) Ops::mfma(fa[a], fb[b], acc32[a][b]);
        };
        // scheduling groups: two reads per MFMA; then the slab loads two per
        // MFMA and the reads three per MFMA
        auto spread_reads = [&]() {
#pragma unroll
            for (int i = 0; i < NRD / 2; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
        };
        auto spread_loads_reads = [&]() {
#pragma unroll
            for (int i = 0; i < LPW; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, NRD / 4, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
        };
        issue(0, 0);
        if (nk > 1) {
            issue(1, BK);
            wait_vm<2 * LPW>();
        } else {
            wait_vm<0>();
        }
        bare_barrier();
        read(0, 0, fa0, fb0);
        int64_t kt = 0;
        for (; kt + 2 < nk; ++kt) {                // steady state, as in the bfloat16 branch
            const int x = (int)(kt & 1);
            read(x, 1, fa1, fb1);
            mma(fa0, fb0);
            spread_reads();
            __builtin_amdgcn_s_waitcnt(0x0070);    // vmcnt(0) lgkmcnt(0)
            bare_barrier();
            issue(x, (kt + 2) * BK);
            read(x ^ 1, 0, fa0, fb0);
            mma(fa1, fb1);
            spread_loads_reads();
        }
        if (kt + 2 == nk) {                        // two slabs left: no more loads
            const int x = (int)(kt & 1);
            read(x, 1, fa1, fb1);
            mma(fa0, fb0);
            __builtin_amdgcn_s_waitcnt(0x0070);
            bare_barrier();
            read(x ^ 1, 0, fa0, fb0);
            mma(fa1, fb1);
            ++kt;
        }
        {                                          // the last slab (landed before the last barrier)
            const int x = (int)(kt & 1);
            read(x, 1, fa1, fb1);
            mma(fa0, fb0);
            mma(fa1, fb1);
        }
        __syncthreads();                           // LDS is reused below and by the epilogue
        // 32 x 32 -> 16 x 16 layout, one 32 x 32 tile at a time through a
        // wave-private column-major 32 x 36 float block placed after the
        // epilogue's partial-sum area: lane l writes its column l % 32, rows
        // 8 j + 4 (l / 32) + 0..3, then reads column 16 sb + l % 16, rows
        // 16 sa + 4 (l / 16) + 0..3 of quarter (sa, sb).
        constexpr int TLD = 36;
        static_assert(16384 + 2 * WM * 32 * TLD * 4 <= 2 * STAGE, "conversion block inside LDS");
        static_assert((WM * BN + 2 * BM) * 8 <= 16384, "clear of the epilogue's partial sums");
        float *T = (float *)(lds + HDR + 16384) + wave * (32 * TLD);
        auto lds_order = [] {
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0xC07F);    // lgkmcnt(0)
            asm volatile("" ::: "memory");
        };
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    *(v4f *)(T + lr * TLD + 8 * j + 4 * lh) =
                        v4f{acc32[a][b][4 * j], acc32[a][b][4 * j + 1], acc32[a][b][4 * j + 2], acc32[a][b][4 * j + 3]};
                lds_order();
#pragma unroll
                for (int sa = 0; sa < 2; ++sa)
#pragma unroll
                    for (int sb = 0; sb < 2; ++sb)
                        acc[2 * a + sa][2 * b + sb] = *(const v4f *)(T + (16 * sb + lane % 16) * TLD + 16 * sa + 4 * (lane / 16));
                lds_order();
            }
    } else {
        static_assert(Ops::CPM == 1 && Ops::MT == 16, "16 x 16 instructions: one 16-byte chunk per lane");
        // Two 32-deep k groups per slab (bfloat16).  The fragments of each group
        // are read from LDS while the previous group's MFMAs run; the one barrier
        // per slab sits between the slab's two groups (slab kt + 1 has landed and
        // every wave holds its fragments of slab kt, so its buffer takes slab
        // kt + 2); and the scheduler is asked to spread the fragment reads and
        // the slab loads evenly over the MFMAs.  Same products in the same order
        // as one group after the other.
        constexpr int NMF = TMW * 8, NRD = TMW + 8;
        v4u fa0[TMW], fb0[8], fa1[TMW], fb1[8];
        auto read = [&](int buf, int g, v4u (&fa)[TMW], v4u (&fb)[8]) {
            const uint8_t *As = lds + HDR + buf * STAGE, *Bs = As + BM * SLAB;
            const int kc = 4 * g + lq;
#pragma unroll
            for (int a = 0; a < TMW; ++a) {
                const int r = arow + 16 * a;
                fa[a] = *(const v4u *)(As + r * SLAB + ((kc ^ ((r >> 1) & 7)) << 4));
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int r = brow + 16 * b;
                fb[b] = *(const v4u *)(Bs + r * SLAB + ((kc ^ ((r >> 1) & 7)) << 4));
            }
        };
        auto mma = [&](const v4u (&fa)[TMW], const v4u (&fb)[8]) {
#pragma unroll
            for (int a = 0; a < TMW; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) Ops::mfma(fa[a], fb[b], acc[a][b]);
        };
        // scheduling groups (masks: 0x008 MFMA, 0x020 global load, 0x100 LDS read)
        auto spread_reads = [&]() {
#pragma unroll
            for (int i = 0; i < NRD; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMF / NRD, 0);
            }
        };
        auto spread_loads_reads = [&]() {
#pragma unroll
            for (int i = 0; i < 2 * LPW; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMF / (4 * LPW), 0);
            }
#pragma unroll
            for (int i = 0; i < NRD; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMF / (2 * NRD), 0);
            }
        };
        issue(0, 0);
        if (nk > 1) {
            issue(1, BK);
            wait_vm<2 * LPW>();
        } else {
            wait_vm<0>();
        }
        bare_barrier();
        read(0, 0, fa0, fb0);
        int64_t kt = 0;
        for (; kt + 2 < nk; ++kt) {                // steady state: no branches inside
            const int x = (int)(kt & 1);
            read(x, 1, fa1, fb1);
            mma(fa0, fb0);
            spread_reads();
            __builtin_amdgcn_s_waitcnt(0x0070);    // vmcnt(0) lgkmcnt(0)
            bare_barrier();
            issue(x, (kt + 2) * BK);
            read(x ^ 1, 0, fa0, fb0);
            mma(fa1, fb1);
            spread_loads_reads();
        }
        for (; kt < nk; ++kt) {                    // the last one or two slabs
            const int x = (int)(kt & 1);
            read(x, 1, fa1, fb1);
            mma(fa0, fb0);
            __builtin_amdgcn_s_waitcnt(0x0070);
            bare_barrier();
            if (kt + 1 < nk) read(x ^ 1, 0, fa0, fb0);
            mma(fa1, fb1);
        }
        __syncthreads();                           // LDS is reused by the epilogue
    }

    // FP8: the result is scaled back by 2^-(eA + eB) with ldexp (exact unless it leaves binary32's range;
    // the factor itself may not be a binary32 number)
    const int sh = scale_exp ? -(scale_exp[0] + scale_exp[1]) : 0;
    // epilogue extras (uniform branches): the accumulator flip hook, then the
    // store with the fused partial sums
    auto rowof = [](int l, int v) { return 4 * (l / 16) + v; };
    if (epi.fbit >= 0 && epi.fi >= row0 && epi.fi < row0 + BM && epi.fj >= col0 && epi.fj < col0 + BN)
        epi_flip(acc, epi, row0 + wm * (BM / WM), col0 + wn * 128, lane, rowof);
    if constexpr (FUSED) {
        epi_store_fused<TMW, 8, WM, 2, BM, BN>(acc, epi, (double *)(lds + HDR), row0, col0, tm, tn, M, N, wm, wn, lane,
                                               sh, C, ldc, false, rowof);
        return;
    }
    const int ccol = lane % 16;
#pragma unroll
    for (int a = 0; a < TMW; ++a) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            int64_t gc = col0 + wn * 128 + b * 16 + ccol;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t gr = row0 + wm * (BM / WM) + a * 16 + 4 * (lane / 16) + v;
                if (gr < M && gc < N) C[gr * ldc + gc] = __builtin_ldexpf(acc[a][b][v], sh);
            }
        }
    }
}

template <class Ops, int WM = 2>
inline int launch_gemm_lowp2(const typename Ops::E *A, int64_t lda, const typename Ops::E *Bt, int64_t ldb, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, const int *scale_exp, hipStream_t s,
                             EpiArgs *epi = nullptr) {
    int64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
    if (tiles > INT32_MAX) return ABFT_E_ARG;
    EpiArgs e = epi ? *epi : epi_none();
    if (epi) {
        epi->tiles_m = (M + 255) / 256;
        epi->tiles_n = (N + 255) / 256;
    }
    if (e.pc)
        k_gemm_lowp2<Ops, WM, true><<<(unsigned)tiles, 128 * WM, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, scale_exp, e);
    else
        k_gemm_lowp2<Ops, WM, false><<<(unsigned)tiles, 128 * WM, 0, s>>>(A, lda, Bt, ldb, C, ldc, M, N, K, scale_exp, e);
    return ABFT_OK;
}

}  // namespace abft
