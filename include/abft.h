/*
 * abft.h -- C ABI of libabft: checksum-encoded matrix multiplication with
 * error detection, location, correction and erased-block rebuild, on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Bosilca, Delmas, Dongarra, Langou, "Algorithmic Based Fault
 * Tolerance Applied to High Performance Computing" (2008), Sec. 2.1 (the
 * single-checksum recovery y = a_1 x_1 + ... + a_p x_p, here with unit
 * weights) and Sec. 2.2, Eq. ABFT-GEMM:
 *
 *     [ A       ]                 [ AB         AB C_R       ]
 *     [ C_C^T A ] [ B   B C_R ] = [ C_C^T AB   C_C^T AB C_R ] = (AB)_F
 *
 * whose result is "consistent": it keeps the checksum relations of its
 * operands, which lets errors in it be detected, located and corrected, and
 * lost parts be rebuilt.  C_C (m x br) stacks m/br identity blocks and C_R
 * (n x bc) stacks n/bc identity blocks, so C_C^T A sums the row blocks of A
 * and B C_R sums the column blocks of B.  br = bc = 1 is the classic
 * all-ones checksum; br = bc = nloc is the paper's per-process block scheme
 * (Sec. 3.2, the (n+nloc)-by-n-by-(n+nloc) product).
 *
 * Relations checked in C_f (the encoded product, M = m + br rows, N = n + bc
 * columns):
 *   column relation (r, j), r < br, j < N:  sum_{g<m/br} C_f[g*br + r, j] = C_f[m + r, j]
 *   row relation    (i, c), i < M, c < bc:  sum_{h<n/bc} C_f[i, h*bc + c] = C_f[i, n + c]
 * (the right-hand sides are the carried checksums).
 *
 * Conventions
 *  - Every pointer named *_f, ws or dst is DEVICE memory owned by the caller;
 *    the library never allocates or frees.  Host pointers are marked "host".
 *  - stream is a hipStream_t (passed as void*); every call that launches work
 *    is asynchronous on it and returns as soon as the work is queued.
 *  - Return values: 0 = ABFT_OK, > 0 informative, < 0 error.  Errors in the
 *    arguments are reported before anything is launched; no C++ exception or
 *    abort crosses this boundary.  After ABFT_E_HIP, abft_last_hip_error()
 *    gives the hipError_t.
 *  - Every call that takes a workspace ws also takes its size in bytes,
 *    ws_bytes; a missing workspace, or one smaller than the problem's
 *    workspace size, is refused with ABFT_E_WORKSPACE before any launch.
 *  - The library keeps no state besides the last HIP error (thread-local):
 *    whatever one call leaves for a later one (threshold statistics, the
 *    fused partial sums and their owner) lives in the caller's workspace.
 *    Calls on distinct buffers are independent and reentrant.
 */
#ifndef ABFT_H
#define ABFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element type of A_f and B_f.  C_f is binary64 for ABFT_F64 and binary32
 * (FP32 accumulation) for every other input type. */
typedef enum {
    ABFT_F64 = 0,
    ABFT_F32 = 1,
    ABFT_BF16 = 2,
    ABFT_FP8_E4M3 = 3
} abft_dtype;

typedef enum {
    ABFT_OK = 0,
    ABFT_FAULT_DETECTED = 1,     /* abft_verify: at least one relation failed */
    ABFT_E_ARG = -1,             /* invalid sizes, leading dimensions, alignment or pointers */
    ABFT_E_HIP = -2,             /* a HIP runtime call failed (see abft_last_hip_error) */
    ABFT_E_UNCORRECTABLE = -3,   /* abft_correct: the flags do not name one element */
    ABFT_E_UNRECOVERABLE = -4,   /* abft_recover_block: more unknowns than relations */
    ABFT_E_WORKSPACE = -5,       /* workspace missing or smaller than the problem's workspace size */
    ABFT_E_UNSUPPORTED = -6,     /* combination not implemented (e.g. dtype, tau mode) */
    ABFT_E_STALE = -7            /* abft_verify_fused (reported in abft_report.status): the partial
                                    sums in ws are not those of the last fused product of this
                                    problem into this C_f */
} abft_status;

/* Detection threshold tau per relation (a relation fails when !(|D| <= tau),
 * so NaN residuals always fail).  The paper fixes no threshold: it only
 * notes that checksum rounding is of the order of the method's own
 * (Sec. 2.1).
 *  ABFT_TAU_DET   rigorous rounding bound, (2 gamma_k + 2 gamma_{G+1} + u_st) S
 *                 with S bounded by Cauchy-Schwarz from per-row/column norms
 *                 (binary64 paths);
 *  ABFT_TAU_STAT  lambda times the standard deviation of the rounding error:
 *                 sigma^2 = (u^2/3)(T/2 + s) Q, u = 2^-24, Q the sum of the
 *                 squared products of the relation (exact for b = 1, a
 *                 Cauchy-Schwarz bound otherwise), T = k for F32 and k/4 for
 *                 BF16 / FP8 (accumulation steps), s = 2, plus 2^18 for FP8
 *                 (the FP8 matrix core's product-sum window, a per-product
 *                 error of 2^-15); for binary32 accumulation, where the
 *                 rigorous bound is far too loose;
 *  ABFT_TAU_EXACT tau = 0, for integer-valued inputs whose sums are exact. */
typedef enum { ABFT_TAU_DET = 0, ABFT_TAU_STAT = 1, ABFT_TAU_EXACT = 2 } abft_tau_mode;

/* abft_gemm flags */
#define ABFT_PLAIN 1u   /* multiply only the data part (C = A B, m x n): the
                           unprotected baseline the overhead is measured against */
#define ABFT_ACCUMULATE 2u /* abft_gemm_panel only: add the panel product to C_f
                              instead of overwriting it */
#define ABFT_FUSED 4u      /* abft_gemm, br = bc = 1 only: the product kernel's
                              epilogue also writes binary64 partial sums of each
                              tile's columns and rows into ws (the fused checksum
                              accumulation) for abft_verify_fused */

/*
 * Problem descriptor.  Layouts (elements of the dtype, not bytes):
 *   A_f  row-major (m + br) x k, row i at A_f + i*lda, lda >= k.
 *        Rows [0, m) are the caller's A; abft_encode writes rows [m, m+br).
 *   B_f  column-major k x (n + bc), column j at B_f + j*ldb, ldb >= k
 *        (equivalently, B_f^T is row-major).  Columns [0, n) are the caller's
 *        B; abft_encode writes columns [n, n+bc).
 *   C_f  row-major (m + br) x (n + bc), ldc >= n + bc.
 * For ABFT_BF16 (and ABFT_FP8_E4M3) A_f holds only the m data rows and B_f
 * only the n data columns: their checksums are binary32 values that the
 * element type cannot hold, so abft_encode keeps them in the workspace.
 * Requirements: m % br == 0, n % bc == 0, k >= 1, and rows of A_f / columns
 * of B_f start on 16-byte boundaries (lda*size and ldb*size multiples of 16,
 * base pointers 16-byte aligned); k is a multiple of 16/size (ABFT_E_ARG
 * otherwise: for another k, pad A_f with zero columns and B_f with zero rows
 * up to the next multiple, which leaves the product and its checksums
 * unchanged and the thresholds larger only through the larger k).  C_f only
 * needs its natural alignment (any ldc >= its minimum, e.g. n+1).
 */
typedef struct {
    int32_t dtype;     /* abft_dtype */
    int32_t tau_mode;  /* abft_tau_mode */
    int64_t m, n, k;   /* data sizes: A is m x k, B is k x n */
    int64_t br, bc;    /* checksum block height (divides m) and width (divides n) */
    int64_t lda, ldb, ldc;
    double lambda;     /* ABFT_TAU_STAT multiplier (0 selects 10) */
    double kappa;      /* ABFT_TAU_DET safety factor >= 1 (0 selects 1 + 2^-20) */
} abft_problem;

/* A rectangle of C_f: rows [i0, i0+h), columns [j0, j0+w). */
typedef struct {
    int64_t i0, j0, h, w;
} abft_rect;

#define ABFT_MAX_FLAGS 64

/* One failed relation: column relation (a = r, b = j) or row relation
 * (a = i, b = c), its residual d and threshold tau. */
typedef struct {
    int64_t a, b;
    double d, tau;
} abft_flag;

/* Result of abft_verify.  The flag lists hold up to ABFT_MAX_FLAGS failed
 * relations of each direction in the order the device recorded them (the
 * counts are exact; when more fail, which ones are kept is unspecified).
 * abft_classify sorts what it is given, and a report with more than one
 * failed relation in a direction is MULTI whichever flags were kept. */
typedef struct {
    int64_t n_flag_c, n_flag_r;       /* failed column / row relations */
    int64_t n_excl_c, n_excl_r;       /* relations skipped: they hold a known erased element */
    int64_t n_nonfinite;              /* failed relations with a NaN/Inf residual */
    int64_t status;                   /* ABFT_OK; ABFT_E_STALE from abft_verify_fused, the rest then empty */
    double max_ratio_c, max_ratio_r;  /* max |D|/tau over finite, checked relations */
    abft_flag flag_c[ABFT_MAX_FLAGS];
    abft_flag flag_r[ABFT_MAX_FLAGS];
} abft_report;

typedef enum { ABFT_CLS_CLEAN = 0, ABFT_CLS_DATA = 1, ABFT_CLS_CHECKSUM = 2, ABFT_CLS_MULTI = 3 } abft_class;
typedef enum { ABFT_DIR_COL = 0, ABFT_DIR_ROW = 1 } abft_direction;

/* Result of abft_classify: the class, the element (i, j) of C_f and the
 * direction of the relation it is rebuilt from. */
typedef struct {
    int32_t cls;   /* abft_class */
    int32_t dir;   /* abft_direction */
    int64_t i, j;
} abft_location;

/* Bytes of device workspace the calls below need for problem p (threshold
 * statistics, verification partials, the fused partial sums and their owner
 * tag, and the device report); 0 for an invalid problem. */
size_t abft_workspace_size(const abft_problem *p);

/*
 * Quantize a binary32 operand into the problem's element type (a step of the
 * low-precision workloads, not of the paper's method).  which == 0: X is A
 * (m x k, row-major, ldx) and dst receives the data rows of A_f (lda);
 * which == 1: X is B^T (n x k, row-major, ldx) and dst receives the data
 * columns of the column-major B_f (ldb).  ABFT_BF16: round to nearest even.
 * X and dst 16-byte aligned, ldx*4 a multiple of 16.  Asynchronous.
 */
int abft_quantize(const abft_problem *p, int which, const float *X, int64_t ldx, void *dst, void *ws, size_t ws_bytes,
                  void *stream);

/*
 * Quantize both binary32 operands and encode them: the same A_f, B_f and
 * workspace contents, bit for bit, as abft_quantize(p, 0, A32, lda32, A_f,
 * ws), abft_quantize(p, 1, B32, ldb32, B_f, ws) and abft_encode(p, A_f, B_f,
 * ws).  bfloat16: one pass per operand, each binary32 operand read once and
 * its quantized values encoded as they are stored; FP8: the same three calls
 * in sequence (measured faster than one pass).  A32: A (m x k, row-major,
 * lda32); B32: B^T (n x k, row-major, ldb32).  ABFT_BF16 and ABFT_FP8_E4M3 only (ABFT_E_UNSUPPORTED otherwise);
 * A32 and B32 16-byte aligned with lda32, ldb32 >= k and multiples of 4;
 * A_f, B_f and ws as for abft_quantize and abft_encode.  Asynchronous.
 */
int abft_quantize_encode(const abft_problem *p, const float *A32, int64_t lda32, const float *B32, int64_t ldb32,
                         void *A_f, void *B_f, void *ws, size_t ws_bytes, void *stream);

/*
 * Encode (Eq. ABFT-GEMM, the checkpointed operands A_F and B_F): writes
 * C_C^T A into rows [m, m+br) of A_f and B C_R into columns [n, n+bc) of
 * B_f (F64, F32; for BF16 / FP8 into ws, in binary32), summing in binary64
 * and rounding once, and writes the
 * per-row / per-column statistics the thresholds are built from into ws.
 * HBM-bound: A and B are read once each when k / (16 / element size) is a
 * multiple of 64 (the row statistics are taken in the same pass); otherwise,
 * and for the statistical thresholds' weighted row sums of A (whose weights
 * exist only after B's encode), a second pass reads the operand again.
 */
int abft_encode(const abft_problem *p, void *A_f, void *B_f, void *ws, size_t ws_bytes, void *stream);

/*
 * Chained products (stacked fault-tolerant routines; Sec. 3.2 notes that the
 * initial checksum is not paid again when calls are chained): the result C_f
 * of a previous product is the A_f of the next one, D_f = C_f[:, 0:n_prev)
 * B_f, without recomputing its checksum rows: the carried rows of C_f are
 * already A's checksum rows.  This call encodes B_f (checksum columns as
 * abft_encode) and fills ws for the new problem p: the threshold statistics
 * of A_f taken over the rows that enter the product (the carried rows as they
 * are), and the inherited threshold term.  The previous column relations hold
 * only up to their residual, at most tau_prev(r, l); through the product it
 * adds at most sum_l tau_prev(r, l) |B_f[l, j]| to relation (r, j), which the
 * det threshold of p then includes.  Requirements: both problems ABFT_F64, or
 * both ABFT_F32, with the same tau mode (ABFT_TAU_DET or ABFT_TAU_EXACT); p->m = prev->m,
 * p->br = prev->br, p->k = prev->n, p->lda = prev->ldc (A_f is the previous
 * C_f, unchanged); ws_prev is the previous product's workspace after its
 * abft_encode (read during this call only).
 */
int abft_encode_chained(const abft_problem *p, const void *A_f, void *B_f, void *ws, size_t ws_bytes,
                        const abft_problem *prev, const void *ws_prev, size_t ws_prev_bytes, void *stream);

/*
 * Protected product (Eq. ABFT-GEMM): C_f = A_f B_f over all (m+br) x (n+bc)
 * entries.  The data part and checksum blocks wider than 8 run on the matrix
 * cores with binary64 (F64) or binary32 (other dtypes) accumulation;
 * checksum blocks of width <= 8, and every checksum block of a bfloat16 / FP8
 * problem (whose binary32 checksum rows live in ws), are computed by a
 * streaming kernel with binary64 accumulation.  With flags & ABFT_PLAIN only
 * C = A B (m x n) is computed, on the matrix cores, and ws may be NULL.
 * A_f and B_f must have been encoded (unless ABFT_PLAIN); ws is the one
 * abft_encode filled (required for BF16 / FP8 and for ABFT_FUSED; optional
 * otherwise).  When ws is given, the product records in it whether its fused
 * partial sums are valid and for which problem and C_f (a product without
 * ABFT_FUSED on this ws invalidates them).
 */
int abft_gemm(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, void *ws, size_t ws_bytes,
              uint32_t flags, void *stream);

/*
 * Test hook (a fault inside the computation): abft_gemm with one bit of one
 * accumulator flipped.  The product kernel flips bit `fault->bit` of the
 * accumulator of element (fault->i, fault->j) of C (i < m, j < n) after its
 * k loop, before the epilogue stores C and forms the fused partial sums, so
 * the flipped value reaches both.  bit < 64 for ABFT_F64 (binary64
 * accumulator), < 32 otherwise.  fault is a host pointer (NULL: abft_gemm).
 * Other arguments as abft_gemm.
 */
typedef struct {
    int64_t i, j;
    int32_t bit;
} abft_fault;
int abft_gemm_fault(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, void *ws, size_t ws_bytes,
                    uint32_t flags, const abft_fault *fault, void *stream);

/*
 * Diagnostic: writes to buf (len bytes, NUL-terminated) the kernels and the
 * block tile abft_gemm would launch for p and flags, e.g.
 * "k_gemm_mfma2 f64 96x96 on 9216x9216 k=8192" or
 * "k_gemm_mfma2 f64 128x128 on 8192x8192 k=8192 + k_sliver carried rows + k_sliver carried columns".
 * No device work, no allocation.  Returns ABFT_OK; ABFT_E_ARG for an invalid
 * problem, unknown flags, a NULL buf or a len too short for the text (buf
 * then holds a truncated string).
 */
int abft_describe_gemm(const abft_problem *p, uint32_t flags, char *buf, size_t len);

/*
 * Panel update (outer-product form of the product, Sec. 2.2 and the rank-nb
 * updates of Sec. 3.2): C_f = A_f[:, k0:k1) B_f[k0:k1, :), or with
 * flags & ABFT_ACCUMULATE, C_f += A_f[:, k0:k1) B_f[k0:k1, :), over the same
 * (m+br) x (n+bc) entries (m x n with ABFT_PLAIN) and on the same kernels as
 * abft_gemm.  Every checksum relation is linear in the inner index, so after
 * any sequence of panels covering [0, k1) C_f is the encoded product of
 * A[:, 0:k1) and B[0:k1, :) and stays consistent: abft_verify may run and a
 * lost block may be rebuilt (abft_recover) between panels, and the loop then
 * goes on.  The thresholds are those of the whole product (an upper bound for
 * every partial sum: partial row norms and step counts are no larger).
 * Accumulation adds one rounding per panel to each entry.
 * dtype ABFT_F64 or ABFT_F32 (ABFT_E_UNSUPPORTED otherwise); A_f and B_f must
 * have been encoded; 0 <= k0 < k1 <= k with k0 and k1 multiples of 16/size
 * (panels start and end on 16-byte boundaries).  No workspace.  flags:
 * ABFT_PLAIN, ABFT_ACCUMULATE.
 */
int abft_gemm_panel(const abft_problem *p, const void *A_f, const void *B_f, void *C_f, int64_t k0, int64_t k1,
                    uint32_t flags, void *stream);

/*
 * Verify (consistency, Sec. 2.2): recomputes every column and row relation of
 * C_f from C_f in binary64, compares each residual with its threshold and
 * records the failures.  Relations that hold an element of a known erased
 * rectangle (host array `known`, n_known <= 4) are skipped.  The report is
 * built in ws; if host_out is not NULL it is also copied there (asynchronous
 * on stream: pass pinned memory and synchronise the stream before reading).
 * Returns ABFT_OK once queued; the outcome is in the report.
 */
int abft_verify(const abft_problem *p, const void *C_f, const abft_rect *known, int n_known,
                void *ws, size_t ws_bytes, abft_report *host_out, void *stream);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): abft_verify with
 * its scratch -- the device report, the tile partial sums and the reduction
 * partials -- in a static device array of the library, ABFT_NOALLOC_SCRATCH_BYTES
 * per GPU (held until the process ends), instead of ws.  ws is read only: the
 * threshold statistics abft_encode wrote (ws_bytes as for abft_verify).  The
 * report is copied to host_out (required; pinned host memory, valid after a
 * stream synchronisation).  Same checks, thresholds, flags and report as
 * abft_verify.  Allocates nothing.  ABFT_E_WORKSPACE if the problem's scratch
 * exceeds the array (e.g. b = 1 products beyond about 16384 x 16384).  Every
 * call on one GPU uses that GPU's one array, so calls that overlap on one GPU
 * (other streams, other threads) race; the stream must belong to the current
 * device.
 */
#define ABFT_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int abft_verify_noalloc(const abft_problem *p, const void *C_f, const abft_rect *known, int n_known,
                        const void *ws, size_t ws_bytes, abft_report *host_out, void *stream);

/*
 * Fused verification (Sec. 2.2 consistency, br = bc = 1): the column
 * relations of the data columns and the row relations of the data rows are
 * formed from the partial sums the last abft_gemm with ABFT_FUSED on this ws
 * wrote in its epilogue (summed over the tiles in binary64), instead of
 * re-reading C; the carried row and column are summed from C_f.  The partials
 * describe C as the product kernel produced it: an error made inside the
 * computation (see abft_gemm_fault) reaches both C and the partials
 * and is seen here, while a change of C_f in memory after the product is seen
 * only by abft_verify.  Same report, thresholds and flags as abft_verify (no
 * known erasures).  The device checks that the last product recorded in ws
 * was a fused product of this problem (dtype, sizes, ldc, tile grid) into
 * this C_f; otherwise the report carries status ABFT_E_STALE and no flags.
 */
int abft_verify_fused(const abft_problem *p, const void *C_f, void *ws, size_t ws_bytes, abft_report *host_out,
                      void *stream);

/*
 * Classify a report (host only, no device work; single-error model):
 *  no failed relation                                   -> CLEAN
 *  one failed column relation (r, j) and one failed row relation (i, c) with
 *  i mod br = r, j mod bc = c and consistent residuals  -> DATA (i < m, j < n)
 *                                                          or CHECKSUM (a carried entry)
 *  with known erasures, a lone failed relation whose partner relation is
 *  skipped and names exactly one element                -> DATA / CHECKSUM
 *  anything else                                        -> MULTI
 * The rebuild direction is the column relation unless that relation holds an
 * erased element.  report and out are host pointers.
 */
int abft_classify(const abft_problem *p, const abft_report *report, const abft_rect *known, int n_known,
                  abft_location *out);

/*
 * Correct one located element (Sec. 2.1 recovery with unit weights): the
 * element is rebuilt from the other members of its relation in binary64,
 * without reading its (possibly non-finite) value, and rounded once to C's
 * type.  loc is a host pointer from abft_classify.  CLEAN: nothing is queued,
 * returns ABFT_OK.  MULTI: returns ABFT_E_UNCORRECTABLE, C_f untouched.
 */
int abft_correct(const abft_problem *p, void *C_f, const abft_location *loc, void *stream);

/*
 * Rebuild an erased rectangle of C_f (the one-GPU image of the lost process,
 * Sec. 3.3's checksum step): each element is solved from its column relation
 * (use_rows == 0; needs e.h <= br) or its row relation (use_rows != 0; needs
 * e.w <= bc), which then hold exactly one unknown each.  Otherwise returns
 * ABFT_E_UNRECOVERABLE and queues nothing.  HBM-bound.
 */
int abft_recover_block(const abft_problem *p, void *C_f, abft_rect e, int use_rows, void *stream);

/* Test-only fault injectors.  abft_inject_flip XORs bit `bit` of element
 * (i, j) of C_f (bit < 64 for binary64 C, < 32 for binary32 C).
 * abft_inject_erase overwrites a rectangle with zeros (nan_fill == 0) or NaN. */
int abft_inject_flip(const abft_problem *p, void *C_f, int64_t i, int64_t j, int bit, void *stream);
int abft_inject_erase(const abft_problem *p, void *C_f, abft_rect e, int nan_fill, void *stream);

/* Synthetic inputs: splitmix64 counter stream (seed, stream_id); logical
 * element (r, c) of a rows x cols matrix uses counter r*cols + c and maps to
 * uniform [-1, 1) (binary64: 2*((x>>11)*2^-53)-1; binary32: 2*((x>>40)*2^-24)-1).
 * It is stored at dst[r*ld + c] (transpose == 0) or dst[c*ld + r]
 * (transpose != 0).  dtype ABFT_F64 or ABFT_F32. */
int abft_fill_uniform(int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed,
                      int32_t stream_id, void *dst, void *stream);

/* Heavy-tailed binary32 inputs (the second input set of the binary32
 * workload): N(0,1) by Box-Muller in binary64 from the splitmix64 streams 0
 * (u1 in (0, 1]) and 1 (u2 in [0, 1)) of seed at the logical element's
 * row-major counter, rounded to binary32, and multiplied by fl32(scale) with
 * probability frac (stream 6).  Layout as abft_fill_uniform.  The device's
 * log and cos may round differently from a host library's, so a value can
 * differ from a host generator's by one binary32 rounding: for runs whose
 * expected outcome needs no reference (clean products). */
int abft_fill_normal(int64_t rows, int64_t cols, int64_t ld, int transpose, uint64_t seed, double frac, float scale,
                     float *dst, void *stream);

/*
 * Peak probes (measurement aids, not part of the protected product): what the
 * matrix cores and HBM deliver on this device, so that kernel rates can be
 * read against measured peaks as well as datasheet ones.
 * abft_probe_mfma launches a register-only loop of `iters` rounds of 8 (binary64: 16)
 * independent matrix-core instructions per wave (dtype ABFT_F64:
 * v_mfma_f64_16x16x4, ABFT_F32: v_mfma_f32_16x16x4, ABFT_BF16:
 * v_mfma_f32_16x16x32_bf16) on 512 blocks of 4 waves, writes one value per
 * block to sink (device, sink_len >= 512 doubles) and stores the flops it
 * executes in *flops (host).  abft_probe_stream launches a read-only pass over
 * buf (device, 16-byte aligned, bytes >= 16, at most 2^31 - 1 blocks of 16 KB):
 * one block per 16 KB chunk, 16-byte non-temporal loads; sink (device,
 * sink_len >= 1) is written only if the fold of the loaded words hits a fixed
 * constant.  Both are asynchronous on stream; time them with events.
 */
int abft_probe_mfma(int32_t dtype, int64_t iters, double *sink, int64_t sink_len, double *flops, void *stream);
int abft_probe_stream(const void *buf, size_t bytes, double *sink, int64_t sink_len, void *stream);

/*
 * Batched problems: many independent protected products of uneven shapes in
 * one pass (bfloat16 inputs, binary32 C, statistical or exact thresholds).
 * Every step is one or two launches over all problems (flattened
 * per-problem descriptors; a persistent product kernel that takes tiles of
 * all problems, largest k first, from a device counter), takes no host
 * synchronisation and allocates nothing, so the pass quantize -> encode ->
 * gemm -> verify can be captured in a hipGraph and replayed.  The binary32
 * checksum rows are also stored as three bfloat16 rows whose sum is exact
 * (hi + mid + lo), so the carried checksum blocks are products on the matrix
 * cores like the data block; their three partial products are summed in
 * binary64 and rounded once.  Classification, correction and block rebuild
 * use the single-problem calls above (abft_classify, abft_correct,
 * abft_recover_block) with each problem's descriptor.  The calls on one plan
 * must be ordered on one stream: they share the workspace and its counters.
 */
typedef struct {
    const float *A32;   /* binary32 A (m x k, row-major, leading dimension lda) for abft_batch_quantize, or NULL */
    const float *Bt32;  /* binary32 B^T (n x k, row-major, leading dimension ldb), or NULL */
    void *A_f;          /* bfloat16 A (m x k, lda) */
    void *B_f;          /* bfloat16 B, column-major (n columns of length k, ldb) */
    void *C_f;          /* binary32 C_f, (m+br) x (n+bc), ldc */
} abft_batch_item;

/* Product tile shapes of the batched kernel: 0 = 256 x 256 (blocks of eight
 * waves, one per CU), 1 = 256 x 128, 2 = 128 x 256, 3 = 128 x 128 (blocks of
 * eight waves, two per CU).  ABFT_BATCH_MIXED: every problem with its own
 * shape (chosen at setup), in two persistent launches (shape 0, the others). */
#define ABFT_BATCH_TILES 4
#define ABFT_BATCH_MIXED ABFT_BATCH_TILES

/* Host-side plan filled by abft_batch_setup (caller-owned, plain data). */
typedef struct {
    void *bws;                                 /* the device batch workspace */
    int32_t count;
    int32_t dtype;
    int64_t n_tiles[ABFT_BATCH_TILES + 1][2];  /* product tiles per shape and for the per-problem shapes:
                                                  [.][0] protected, [.][1] ABFT_PLAIN */
    int64_t n_work[12];                        /* flattened work sizes of the other steps; [7]: problems
                                                  whose C_f rows are not 16-byte aligned */
    size_t bytes;
    size_t ttime_off;                          /* the tuner's per-tile durations in bws */
    int32_t n_shape[ABFT_BATCH_TILES];         /* problems per own tile shape (ABFT_BATCH_MIXED) */
} abft_batch_plan;

/* Device bytes of the batch workspace for these problems (0 if invalid). */
size_t abft_batch_workspace_size(const abft_problem *probs, int count);

/* Validate every problem (dtype ABFT_BF16; tau mode STAT or EXACT; k, lda,
 * ldb multiples of 8; ldc >= n + bc; br divides m; bc divides n and 64) and
 * write the descriptors and counters into bws (synchronous copy, not
 * capturable).  probs, items and plan are host arrays; A_f and B_f 16-byte
 * aligned, A32 and Bt32 16-byte aligned when set.  ABFT_E_ARG / ABFT_E_UNSUPPORTED
 * on a bad problem, ABFT_E_WORKSPACE if bws_bytes is too small. */
int abft_batch_setup(const abft_problem *probs, const abft_batch_item *items, int count, void *bws, size_t bws_bytes,
                     abft_batch_plan *plan);
/* abft_batch_setup with each problem's product tile shape for
 * ABFT_BATCH_MIXED: tiles (host, count entries in the caller's order) holds a
 * shape 0 .. ABFT_BATCH_TILES-1, or a negative value for the library's model
 * (the executed tile area over a per-shape efficiency).  abft_batch_setup is
 * this call with the model for every problem. */
int abft_batch_setup_tiles(const abft_problem *probs, const abft_batch_item *items, int count, const int32_t *tiles,
                           void *bws, size_t bws_bytes, abft_batch_plan *plan);

/* The batched steps (asynchronous, capturable), each the single-problem
 * step of the same name applied to every problem of the plan:
 *   abft_batch_quantize: A32 -> A_f and Bt32 -> B_f (round to nearest even)
 *     for the items whose binary32 pointers are set;
 *   abft_batch_encode: checksum rows C_C^T A and (B C_R)^T (Eq. ABFT-GEMM),
 *     kept in binary32 and as three bfloat16 rows in bws, and the statistics
 *     of the thresholds (Sec. 3);
 *   abft_batch_gemm: C_f = A_f B_f; flags 0 or ABFT_PLAIN (data block only);
 *     tile: one of the ABFT_BATCH_TILES shapes for every problem, or
 *     ABFT_BATCH_MIXED (each problem's own);
 *   abft_batch_verify: every column and row relation of every C_f (Sec. 2),
 *     into the problem's report in bws (no erased-element exclusion).
 * All return ABFT_E_ARG on a NULL plan or a bad tile. */
int abft_batch_quantize(const abft_batch_plan *plan, void *stream);
int abft_batch_encode(const abft_batch_plan *plan, void *stream);
/* abft_batch_quantize then abft_batch_encode in one read of the binary32
 * operands (same results, bit for bit); items without A32 / Bt32 are encoded
 * from their bfloat16 operands as they are. */
int abft_batch_quantize_encode(const abft_batch_plan *plan, void *stream);
int abft_batch_gemm(const abft_batch_plan *plan, int tile, uint32_t flags, void *stream);
/* Tuner (synchronous; overwrites every C_f): runs the product once with each
 * tile shape for every problem, recording each tile's duration on the device
 * (100 MHz clock), and gives per problem (caller's order) the CU time of its
 * tiles for each shape in costs (host, count x ABFT_BATCH_TILES, or NULL: the
 * summed durations, halved for the shapes that run two blocks per CU, 1 .. 3)
 * and the shape with the least in tiles (host, count, or NULL).  With
 * ABFT_BATCH_MIXED the problems of shape 0 run in one launch (one block per
 * CU) and the others in a second (two blocks per CU). */
int abft_batch_tune(const abft_batch_plan *plan, double *costs, int32_t *tiles, void *stream);
/* Launch-level choice (synchronous; overwrites every C_f): the protected
 * product timed with device events, median of reps launches (1 .. 100) after a
 * warm-up, with each uniform shape (0 .. ABFT_BATCH_TILES-1) and with the
 * plan's per-problem shapes (ABFT_BATCH_MIXED), the candidates taken in turn
 * within each sweep of launches (a warm-up sweep first); ms (host, ABFT_BATCH_TILES + 1
 * doubles, or NULL) receives the times, *choice (host, or NULL) the fastest,
 * the value to pass as `tile` to abft_batch_gemm.  The per-problem run is one
 * launch per shape, so its tiles' lower summed cost need not make it faster. */
int abft_batch_choose(const abft_batch_plan *plan, int reps, double *ms, int32_t *choice, void *stream);
/* Persisted tuning results: a text file keyed by (dtype, m / 128, n / 128,
 * log2 k rounded up, br, bc, arch) with the summed cost of each shape over the
 * problems measured in that bucket.  abft_batch_cache_store merges the costs
 * of these problems (from abft_batch_tune) into the file at path (a bucket
 * measured again is replaced); abft_batch_cache_lookup fills tiles (host,
 * count) with each problem's bucket's best shape, or -1 where the file has no
 * entry, and returns how many were found.  arch: the device architecture name
 * (e.g. "gfx950"), or NULL for the current device's.  Host only. */
int abft_batch_cache_lookup(const char *path, const char *arch, const abft_problem *probs, int count, int32_t *tiles);
int abft_batch_cache_store(const char *path, const char *arch, const abft_problem *probs, int count,
                           const double *costs);
int abft_batch_verify(const abft_batch_plan *plan, void *stream);
/* Copy the count reports (verify results, in the caller's problem order) to
 * host_out (pinned; valid after a stream synchronisation). */
int abft_batch_reports(const abft_batch_plan *plan, abft_report *host_out, void *stream);
/* Diagnostic (for tests): the thresholds the verification uses for problem
 * `problem` (caller's order), from the threshold statistics of the last encode
 * and the stored totals now in its C_f: tau_c (device, br x (n + bc),
 * row-major) for the column relations (r, j), tau_r (device, (m + br) x bc)
 * for the row relations (i, c); 0 under ABFT_TAU_EXACT.  Reads the
 * descriptors back (synchronous copy), then launches on the stream. */
int abft_batch_thresholds(const abft_batch_plan *plan, int problem, double *tau_c, double *tau_r, void *stream);

/*
 * Weighted f-checksums (Sec. 2.1).  Sec. 2.1 protects p values x_g with f
 * weighted checksums y_r = sum_g w_rg x_g and rebuilds any f lost values when
 * every f x f submatrix of the f x p weight matrix is nonsingular.  Applied to
 * the block product (Sec. 2.2, Eq. ABFT-GEMM with weighted checksum matrices):
 * the values are the Gr = m/br row blocks A_g of A and the Gc = n/bc column
 * blocks B_h of B,
 *   A_f = [A; Y_0 .. Y_{fr-1}],  Y_r = sum_g wr[r][g] A_g   (m + fr*br rows)
 *   B_f = [B, Z_0 .. Z_{fc-1}],  Z_c = sum_h wc[c][h] B_h   (n + fc*bc columns)
 * and C_f = A_f B_f satisfies, for every column j < N = n + fc*bc and every
 * row x < M = m + fr*br (corner included):
 *   column relation (r, i, j): sum_g wr[r][g] C_f[g*br + i, j] = C_f[m + r*br + i, j]
 *   row relation (x, c, jj):   sum_h wc[c][h] C_f[x, h*bc + jj] = C_f[x, n + c*bc + jj]
 * The fr relations of one (i, j) form a column group, the fc relations of one
 * (x, jj) a row group.  Binary64 or binary32 operands and C_f (every sum in
 * binary64, a stored result rounded once to the element type); layouts as for
 * abft_problem with these sizes (A_f row-major, B_f column-major, C_f
 * row-major, ldc >= N); k, lda and ldb multiples of 16 bytes' elements.
 */
#define ABFT_WMAX 4

typedef struct {
    abft_problem p;    /* dtype ABFT_F64 or ABFT_F32, tau_mode ABFT_TAU_DET or ABFT_TAU_EXACT;
                          br, bc are the block height and width */
    int32_t fr, fc;    /* checksum block rows / columns, 1 .. ABFT_WMAX */
    const double *wr;  /* host, fr x (m/br) row-major: wr[r*(m/br) + g] (finite) */
    const double *wc;  /* host, fc x (n/bc) row-major */
} abft_wproblem;

/* One failed group: (a, b) = (i, j) for a column group, (x, jj) for a row
 * group; the residual and threshold of each of its f relations. */
typedef struct {
    int64_t a, b;
    double d[ABFT_WMAX];
    double tau[ABFT_WMAX];
} abft_wgroup;

/* Result of abft_wverify.  A group fails when one of its relations has
 * !(|D| <= tau) (NaN fails); the lists hold the first ABFT_MAX_FLAGS failed
 * groups of each direction in no particular order (counts are exact). */
typedef struct {
    int64_t n_fail_c, n_fail_r;       /* failed column / row groups */
    int64_t n_excl_c, n_excl_r;       /* groups skipped: they hold a known erased element */
    double max_ratio_c, max_ratio_r;  /* max |D|/tau over finite relations with tau > 0 */
    abft_wgroup col[ABFT_MAX_FLAGS];
    abft_wgroup row[ABFT_MAX_FLAGS];
} abft_wreport;

/* Workspace bytes for p (weights, norms, partial sums, report); 0 if p is invalid. */
size_t abft_wworkspace_size(const abft_wproblem *p);
/* Copy the weights into ws (a blocking copy; once per problem and weight set). */
int abft_wsetup(const abft_wproblem *p, void *ws, size_t ws_bytes);
/* Checksum rows Y_r of A_f and columns Z_c of B_f (binary64 weighted sums over
 * the blocks in increasing order, one rounding per step; binary32 problems
 * store them rounded once to binary32), then the threshold statistics:
 * ||A_f[x, :]||_2, ||B_f[:, j]||_2 and S_r[i] = sum_g |wr[r][g]|
 * ||A_f[g*br + i, :]||_2 (and its column analogue).  ABFT_TAU_DET: tau of
 * column relation (r, i, j) = kappa (2 gamma_k(u_acc) + u_st +
 * 3 gamma_{Gr+1}) S_r[i] ||B_f[:, j]||_2, a rigorous bound on the rounding of
 * the product (accumulated with unit roundoff u_acc: 2^-53, binary32 2^-24),
 * the stored checksum rows (u_st: 0, binary32 2^-24) and the binary64
 * relation sum; rows alike with Gc. */
int abft_wencode(const abft_wproblem *p, void *A_f, void *B_f, void *ws, size_t ws_bytes, void *stream);
/* C_f = A_f B_f, all M x N entries: on the matrix cores (accumulated in the
 * element type), or for N <= 8 (the matrix-vector product: n = 1, bc = 1,
 * fc = 1) by a streaming kernel that reads A_f once (binary64 accumulation).  A protected matrix-vector product y = A x is
 * the problem with n = 1: B_f = [x, wc x], C_f = [y_f, wc y_f] with y_f the
 * encoded result; every weighted relation, location and recovery applies. */
int abft_wgemm(const abft_wproblem *p, const void *A_f, const void *B_f, void *C_f, void *stream);
/* Every column and row group of C_f (binary64 sums); groups holding an
 * element of a known erased rectangle (n_known <= 4) are skipped.  The report
 * is built in ws and, if host_out is not NULL, copied there asynchronously. */
int abft_wverify(const abft_wproblem *p, const void *C_f, const abft_rect *known, int n_known, void *ws,
                 size_t ws_bytes, abft_wreport *host_out, void *stream);
/* Locate (host only, one error per group).  When fr >= 2 each failed column
 * group is located on its own, so errors in distinct groups are found
 * together: a data member g with error e gives residuals wr[.][g] e (every
 * relation of the group fails and the residual vector fits that column of
 * the weights, for exactly one g), a checksum entry r gives one failed
 * relation; else when fc >= 2 the row groups alike; with fr = fc = 1 one
 * failed column group and one failed row group meet in one element.  Groups
 * that fit no member or several, or hold a non-finite residual, give MULTI.
 * Writes min(count, max_out) locations to out and the count to *n_out; returns
 * ABFT_E_UNCORRECTABLE if any location is MULTI. */
int abft_wlocate(const abft_wproblem *p, const abft_wreport *report, abft_location *out, int max_out, int *n_out);
/* Rebuild located elements in place from their groups (never reading them):
 * a data member from the lowest-numbered checksum relation of its group, a
 * checksum entry as its weighted sum.  MULTI locations are refused. */
int abft_wcorrect(const abft_wproblem *p, void *C_f, const abft_location *locs, int n, void *ws, size_t ws_bytes,
                  void *stream);
/* Sec. 2.1 recovery of lost blocks.  dir ABFT_DIR_COL: blocks[] are block-row
 * indices (g < Gr data block rows, Gr + r checksum block row r) lost over the
 * columns [lo, lo + len); every column group solves for the lost data members
 * with the lowest-numbered intact checksum relations (an s x s system, s <= fr,
 * inverted on the host in binary64 with partial pivoting), then recomputes the
 * lost checksum entries.  ABFT_DIR_ROW: block columns over the rows
 * [lo, lo + len).  ABFT_E_UNRECOVERABLE when more data blocks are lost than
 * checksum blocks survive or the system's 1-norm condition number exceeds 1e12. */
int abft_wrecover(const abft_wproblem *p, void *C_f, int dir, const int32_t *blocks, int n_blocks, int64_t lo,
                  int64_t len, void *ws, size_t ws_bytes, void *stream);

/*
 * 2-D block-cyclic distribution (Sec. 4.1: matrices spread over a process grid
 * in the 2-D block-cyclic format, checksums by rows, by columns or both) on
 * one GPU.  Over a P x Q grid with blocks of nb, global block (I, J) belongs to
 * process (I mod P, J mod Q) as its local block (I div P, J div Q).
 * abft_block_cyclic_stack copies a rows x cols matrix into the stacked
 * local-array layout: process (p, q)'s local array at rows [p rows/P,
 * (p+1) rows/P) and columns [q cols/Q, (q+1) cols/Q); unstack is the inverse.
 * A dimension over one process (P = 1 or Q = 1) is left as it is.  With A's
 * rows stacked over P and B's columns over Q (B_f^T's rows: stack it with
 * P = Q_grid, Q = 1), the product in the stacked layout is C stacked, and the
 * block checksum with br = m/P, bc = n/Q is the grid's checksum process row
 * and column (the sum of the local arrays over the process rows / columns):
 * losing process (p, q) is losing block (p, q) of C_f, rebuilt by
 * abft_recover_block.  elem_size 1, 2, 4 or 8 bytes; rows % (nb P) == 0 when
 * P > 1, cols % (nb Q) == 0 when Q > 1; source and destination distinct.
 */
int abft_block_cyclic_stack(const void *G, int64_t ldg, int64_t rows, int64_t cols, int32_t elem_size, int64_t nb,
                            int32_t P, int32_t Q, void *S, int64_t lds, void *stream);
int abft_block_cyclic_unstack(const void *S, int64_t lds, int64_t rows, int64_t cols, int32_t elem_size, int64_t nb,
                              int32_t P, int32_t Q, void *G, int64_t ldg, void *stream);

/* Last hipError_t seen by this thread (0 if none), and a status message. */
int abft_last_hip_error(void);
const char *abft_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* ABFT_H */
