/*
 * abft_oracle.c -- plain, slow, FP64 CPU oracle for checksum-encoded matrix
 * multiplication (Bosilca, Delmas, Dongarra, Langou, "Algorithmic Based Fault
 * Tolerance Applied to High Performance Computing", 2008).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library never
 * links it, and this file shares no header, helper, table or constant with it.
 *
 * Everything is binary64, in a fixed ascending loop order; build with
 * -O2 -ffp-contract=off and without fast-math so that every + and * is one
 * IEEE operation.  All matrices are row-major host arrays.
 *
 * Notation (Sec. 2.2, Eq. ABFT-GEMM).  A is m x k, B is k x n.  The column
 * checksum matrix C_C (m x br) stacks G_r = m/br identity blocks, so
 * C_C^T A sums the row blocks of A; the row checksum matrix C_R (n x bc)
 * stacks G_c = n/bc identity blocks, so B C_R sums the column blocks of B.
 * br = bc = 1 gives the all-ones vector of the classic scheme.
 *   A_f = [A ; C_C^T A]                    ((m+br) x k)
 *   B_f = [B , B C_R]                      (k x (n+bc))
 *   C_f = A_f B_f = [[AB, AB C_R], [C_C^T AB, C_C^T AB C_R]]
 * C_f is "consistent" (Sec. 2.2): every column relation
 *   sum_{g<G_r} C_f[g*br + r, j] = C_f[m + r, j]        (r < br, j < n+bc)
 * and every row relation
 *   sum_{h<G_c} C_f[i, h*bc + c] = C_f[i, n + c]        (i < m+br, c < bc)
 * holds up to rounding.  A relation that fails flags an error; one failed
 * column relation and one failed row relation that meet in one element locate
 * it; the element is rebuilt from the other members of its relation, which is
 * the single-checksum recovery of Sec. 2.1 with unit weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXFLAG 64

/* ------------------------------------------------------------------------ */
/* Encoding (Eq. ABFT-GEMM: C_C^T A and B C_R)                               */
/* ------------------------------------------------------------------------ */

/* Rows m..m+br-1 of A_f receive C_C^T A: A_f[m+r, l] = sum_g A[g*br + r, l],
 * summed over ascending g.  store_f32 != 0 rounds each sum once to binary32
 * (the low-precision paths keep their checksums in binary32). */
void orc_encode_rows(int64_t m, int64_t k, int64_t br, double *A, int64_t lda, int store_f32)
{
    int64_t G = m / br;
    for (int64_t r = 0; r < br; ++r) {
        double *dst = A + (m + r) * lda;
        for (int64_t l = 0; l < k; ++l) dst[l] = 0.0;
        for (int64_t g = 0; g < G; ++g) {
            const double *src = A + (g * br + r) * lda;
            for (int64_t l = 0; l < k; ++l) dst[l] += src[l];
        }
        if (store_f32)
            for (int64_t l = 0; l < k; ++l) dst[l] = (double)(float)dst[l];
    }
}

/* Columns n..n+bc-1 of B_f (k x (n+bc), row-major) receive B C_R:
 * B_f[l, n+c] = sum_h B[l, h*bc + c], ascending h. */
void orc_encode_cols(int64_t k, int64_t n, int64_t bc, double *B, int64_t ldb, int store_f32)
{
    int64_t G = n / bc;
    for (int64_t l = 0; l < k; ++l) {
        double *row = B + l * ldb;
        for (int64_t c = 0; c < bc; ++c) {
            double s = 0.0;
            for (int64_t h = 0; h < G; ++h) s += row[h * bc + c];
            row[n + c] = store_f32 ? (double)(float)s : s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Product                                                                   */
/* ------------------------------------------------------------------------ */

/* C = A B (M x K times K x N), i-l-j order: each C[i,j] is the ascending-l
 * sum of A[i,l]*B[l,j], one rounding per multiply and per add.  Rows are
 * independent, so they are shared among threads without changing any sum. */
void orc_gemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
              const double *B, int64_t ldb, double *C, int64_t ldc)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < M; ++i) {
        double *crow = C + i * ldc;
        for (int64_t j = 0; j < N; ++j) crow[j] = 0.0;
        for (int64_t l = 0; l < K; ++l) {
            double a = A[i * lda + l];
            const double *brow = B + l * ldb;
            for (int64_t j = 0; j < N; ++j) crow[j] += a * brow[j];
        }
    }
}

/* One element of a product, same ascending order as orc_gemm. */
double orc_dot(int64_t K, const double *a, int64_t inca, const double *b, int64_t incb)
{
    double s = 0.0;
    for (int64_t l = 0; l < K; ++l) s += a[l * inca] * b[l * incb];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Statistics the thresholds are built from                                  */
/* ------------------------------------------------------------------------ */

/* out[i] = ||A[i,:]||_2 for i < M */
void orc_row_norms(int64_t M, int64_t K, const double *A, int64_t lda, double *out)
{
    for (int64_t i = 0; i < M; ++i) {
        double s = 0.0;
        for (int64_t l = 0; l < K; ++l) s += A[i * lda + l] * A[i * lda + l];
        out[i] = sqrt(s);
    }
}

/* out[r] = || sum_g |A[g*br + r, :]| ||_2  (the row r of C_C^T |A|) */
void orc_group_abs_row_norms(int64_t m, int64_t k, int64_t br, const double *A, int64_t lda, double *out)
{
    int64_t G = m / br;
    double *t = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int64_t r = 0; r < br; ++r) {
        for (int64_t l = 0; l < k; ++l) t[l] = 0.0;
        for (int64_t g = 0; g < G; ++g)
            for (int64_t l = 0; l < k; ++l) t[l] += fabs(A[(g * br + r) * lda + l]);
        double s = 0.0;
        for (int64_t l = 0; l < k; ++l) s += t[l] * t[l];
        out[r] = sqrt(s);
    }
    free(t);
}

/* out[j] = ||B[:,j]||_2 for j < N (B is K x N row-major) */
void orc_col_norms(int64_t K, int64_t N, const double *B, int64_t ldb, double *out)
{
    for (int64_t j = 0; j < N; ++j) {
        double s = 0.0;
        for (int64_t l = 0; l < K; ++l) s += B[l * ldb + j] * B[l * ldb + j];
        out[j] = sqrt(s);
    }
}

/* out[c] = || sum_h |B[:, h*bc + c]| ||_2  (the column c of |B| C_R) */
void orc_group_abs_col_norms(int64_t k, int64_t n, int64_t bc, const double *B, int64_t ldb, double *out)
{
    int64_t G = n / bc;
    for (int64_t c = 0; c < bc; ++c) {
        double s = 0.0;
        for (int64_t l = 0; l < k; ++l) {
            double t = 0.0;
            for (int64_t h = 0; h < G; ++h) t += fabs(B[l * ldb + h * bc + c]);
            s += t * t;
        }
        out[c] = sqrt(s);
    }
}

/* Higham's gamma_n = n u / (1 - n u). */
double orc_gamma(double n, double u) { return n * u / (1.0 - n * u); }

/*
 * Rigorous ("det") thresholds.  For a column relation (r, j) every member is a
 * k-term dot product, each with error at most gamma_k * sum_l |a_l||b_l|; the
 * stored checksum row carries the error of its own (G_r-1)-term sum; the
 * G_r-term check sum adds gamma_{G_r}.  Collecting terms, with
 * S = sum_l (C_C^T|A|)[r,l] |B_f[l,j]| <= ||(C_C^T|A|)[r,:]||_2 ||B_f[:,j]||_2
 * (Cauchy-Schwarz), gives |D| <= (2 gamma_k + 2 gamma_{G_r+1} + u_st) S.
 * kappa (>= 1) absorbs the rounding of the norms themselves.
 * tau_c is br x (n+bc), tau_r is (m+br) x bc.
 */
void orc_tau_det(int64_t m, int64_t n, int64_t k, int64_t br, int64_t bc,
                 const double *na, const double *na_abs, const double *nb, const double *nb_abs,
                 double u_acc, double u_st, double kappa, double *tau_c, double *tau_r)
{
    const double u64 = ldexp(1.0, -53);
    double cc = kappa * (2.0 * orc_gamma((double)k, u_acc) + 2.0 * orc_gamma((double)(m / br + 1), u64) + u_st);
    double cr = kappa * (2.0 * orc_gamma((double)k, u_acc) + 2.0 * orc_gamma((double)(n / bc + 1), u64) + u_st);
    for (int64_t r = 0; r < br; ++r)
        for (int64_t j = 0; j < n + bc; ++j) tau_c[r * (n + bc) + j] = cc * na_abs[r] * nb[j];
    for (int64_t i = 0; i < m + br; ++i)
        for (int64_t c = 0; c < bc; ++c) tau_r[i * bc + c] = cr * na[i] * nb_abs[c];
}

/*
 * Statistical ("stat") thresholds for binary32 accumulation, where the
 * rigorous bound is orders of magnitude above the actual residual.  Model:
 * each of the T accumulation steps of a dot product rounds once with an error
 * uniform in [-u, u] relative to the running sum, so a k-term dot of
 * independent zero-mean terms has variance (u^2/3)(T/2) sum_l a_l^2 b_l^2.
 * The members of a relation round independently, so
 *   sigma^2 = (u^2/3) (T/2 + s) Q,
 *   Q_c[r,j] = sum_l v[r,l] B_f[l,j]^2,   v = C_C^T (A o A) + (C_C^T A) o (C_C^T A),
 * and likewise Q_r[i,c] = sum_l A_f[i,l]^2 w[l,c].  s covers the one
 * rounding of a binary32-stored checksum.  tau = lambda * sigma.
 * For br == 1 (bc == 1) Q is computed exactly; otherwise it is replaced by
 * the Cauchy-Schwarz bound ||v[r,:]||_2 ||B_f[:,j]||_4^2.
 * The stored total of each relation, the carried entry t = C_f[m+r, j]
 * (C_f[i, n+c] for a row relation), is rounded once to binary32, an error of
 * variance (u^2/3) t^2 taken with the entry's own magnitude: when C_f is
 * given (NULL: no such term), sigma^2 += (u^2/3) t^2.  For data of one sign
 * t is far above the root-sum-square of its products.  A non-finite t (a
 * fault in the stored total) adds no term, so that the relation's residual,
 * non-finite too, fails against a finite threshold.
 * Where the stored totals are themselves accumulated in steps of the same
 * precision (T_c steps, e.g. a carried checksum row computed on the matrix
 * cores; T_c = 0 when they are summed in binary64), their running sums carry
 * the total's own magnitude: for terms of one sign the partial sums grow
 * linearly, sum_l s_l^2 = t^2 T_c / 3, which adds (u^2/3)(T_c/3) t^2:
 * sigma^2 += (u^2/3) (1 + T_c/3) t^2 in all.
 * A_f is (m+br) x k and B_f is k x (n+bc), both row-major and encoded; C_f is
 * (m+br) x (n+bc) with leading dimension ldc.
 */
void orc_tau_stat(int64_t m, int64_t n, int64_t k, int64_t br, int64_t bc,
                  const double *Af, int64_t lda, const double *Bf, int64_t ldb,
                  double u_acc, double T, double s_store, double lambda,
                  const double *Cf, int64_t ldc, double T_c, double *tau_c, double *tau_r)
{
    int64_t Gr = m / br, Gc = n / bc, N = n + bc, M = m + br;
    double coef = u_acc * u_acc / 3.0 * (T / 2.0 + s_store);
    double cst = u_acc * u_acc / 3.0 * (1.0 + T_c / 3.0);
    double *v = (double *)calloc((size_t)(br * k), sizeof(double));
    double *w = (double *)calloc((size_t)(k * bc), sizeof(double));
    for (int64_t r = 0; r < br; ++r) {
        for (int64_t g = 0; g <= Gr; ++g) {           /* g == Gr is the checksum row */
            const double *a = Af + (g * br + r) * lda;
            for (int64_t l = 0; l < k; ++l) v[r * k + l] += a[l] * a[l];
        }
    }
    for (int64_t l = 0; l < k; ++l)
        for (int64_t c = 0; c < bc; ++c)
            for (int64_t h = 0; h <= Gc; ++h) {         /* h == Gc is the checksum column */
                double b = Bf[l * ldb + h * bc + c];
                w[l * bc + c] += b * b;
            }
    if (br == 1) {
        for (int64_t j = 0; j < N; ++j) {
            double q = 0.0;
            for (int64_t l = 0; l < k; ++l) q += v[l] * (Bf[l * ldb + j] * Bf[l * ldb + j]);
            double t = Cf && isfinite(Cf[m * ldc + j]) ? Cf[m * ldc + j] : 0.0;
            tau_c[j] = lambda * sqrt(coef * q + cst * t * t);
        }
    } else {
        double *nv = (double *)malloc(sizeof(double) * (size_t)br);
        for (int64_t r = 0; r < br; ++r) {
            double s = 0.0;
            for (int64_t l = 0; l < k; ++l) s += v[r * k + l] * v[r * k + l];
            nv[r] = sqrt(s);
        }
        for (int64_t j = 0; j < N; ++j) {
            double s4 = 0.0;
            for (int64_t l = 0; l < k; ++l) { double b2 = Bf[l * ldb + j] * Bf[l * ldb + j]; s4 += b2 * b2; }
            double n4sq = sqrt(s4);
            for (int64_t r = 0; r < br; ++r) {
                double t = Cf && isfinite(Cf[(m + r) * ldc + j]) ? Cf[(m + r) * ldc + j] : 0.0;
                tau_c[r * N + j] = lambda * sqrt(coef * nv[r] * n4sq + cst * t * t);
            }
        }
        free(nv);
    }
    if (bc == 1) {
        for (int64_t i = 0; i < M; ++i) {
            double q = 0.0;
            for (int64_t l = 0; l < k; ++l) q += (Af[i * lda + l] * Af[i * lda + l]) * w[l];
            double t = Cf && isfinite(Cf[i * ldc + n]) ? Cf[i * ldc + n] : 0.0;
            tau_r[i] = lambda * sqrt(coef * q + cst * t * t);
        }
    } else {
        double *nw = (double *)malloc(sizeof(double) * (size_t)bc);
        for (int64_t c = 0; c < bc; ++c) {
            double s = 0.0;
            for (int64_t l = 0; l < k; ++l) s += w[l * bc + c] * w[l * bc + c];
            nw[c] = sqrt(s);
        }
        for (int64_t i = 0; i < M; ++i) {
            double s4 = 0.0;
            for (int64_t l = 0; l < k; ++l) { double a2 = Af[i * lda + l] * Af[i * lda + l]; s4 += a2 * a2; }
            double n4sq = sqrt(s4);
            for (int64_t c = 0; c < bc; ++c) {
                double t = Cf && isfinite(Cf[i * ldc + n + c]) ? Cf[i * ldc + n + c] : 0.0;
                tau_r[i * bc + c] = lambda * sqrt(coef * n4sq * nw[c] + cst * t * t);
            }
        }
        free(nw);
    }
    free(v);
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Verification: relation residuals, flags                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n_flag_c, n_flag_r;   /* failed column / row relations (not excluded) */
    int64_t n_excl_c, n_excl_r;   /* relations skipped because they hold an erased element */
    int64_t n_nonfinite;          /* failed relations whose residual is not finite */
    double max_ratio_c, max_ratio_r;  /* max |D|/tau over finite, non-excluded relations */
    int64_t fc_r[ORC_MAXFLAG], fc_j[ORC_MAXFLAG];
    double fc_d[ORC_MAXFLAG], fc_t[ORC_MAXFLAG];
    int64_t fr_i[ORC_MAXFLAG], fr_c[ORC_MAXFLAG];
    double fr_d[ORC_MAXFLAG], fr_t[ORC_MAXFLAG];
} orc_report;

int64_t orc_report_size(void) { return (int64_t)sizeof(orc_report); }

/* Erasures are rectangles {i0, j0, h, w} of C_f, 4 int64 each. */
static int col_rel_has_erased(int64_t r, int64_t j, int64_t br, const int64_t *er, int ner)
{
    for (int e = 0; e < ner; ++e) {
        int64_t i0 = er[4 * e], j0 = er[4 * e + 1], h = er[4 * e + 2], w = er[4 * e + 3];
        if (j < j0 || j >= j0 + w) continue;
        for (int64_t i = i0; i < i0 + h; ++i)
            if (i % br == r) return 1;
    }
    return 0;
}

static int row_rel_has_erased(int64_t i, int64_t c, int64_t bc, const int64_t *er, int ner)
{
    for (int e = 0; e < ner; ++e) {
        int64_t i0 = er[4 * e], j0 = er[4 * e + 1], h = er[4 * e + 2], w = er[4 * e + 3];
        if (i < i0 || i >= i0 + h) continue;
        for (int64_t j = j0; j < j0 + w; ++j)
            if (j % bc == c) return 1;
    }
    return 0;
}

/*
 * Dc[r*(n+bc) + j] = sum_{g<G_r} C[g*br + r, j] - C[m + r, j]
 * Dr[i*bc + c]     = sum_{h<G_c} C[i, h*bc + c] - C[i, n + c]
 * A relation is flagged when !(|D| <= tau), so a NaN residual is flagged.
 * Flagged entries are listed in ascending index order (first 64).
 */
void orc_verify(int64_t m, int64_t n, int64_t br, int64_t bc, const double *C, int64_t ldc,
                const double *tau_c, const double *tau_r, const int64_t *erasures, int n_erasures,
                double *Dc, double *Dr, orc_report *rep)
{
    int64_t Gr = m / br, Gc = n / bc, N = n + bc, M = m + br;
    memset(rep, 0, sizeof(*rep));
    for (int64_t r = 0; r < br; ++r) {
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            for (int64_t g = 0; g < Gr; ++g) s += C[(g * br + r) * ldc + j];
            double d = s - C[(m + r) * ldc + j];
            double t = tau_c[r * N + j];
            Dc[r * N + j] = d;
            if (col_rel_has_erased(r, j, br, erasures, n_erasures)) { rep->n_excl_c++; continue; }
            if (isfinite(d) && t > 0 && fabs(d) / t > rep->max_ratio_c) rep->max_ratio_c = fabs(d) / t;
            if (!(fabs(d) <= t)) {
                if (!isfinite(d)) rep->n_nonfinite++;
                if (rep->n_flag_c < ORC_MAXFLAG) {
                    int64_t q = rep->n_flag_c;
                    rep->fc_r[q] = r; rep->fc_j[q] = j; rep->fc_d[q] = d; rep->fc_t[q] = t;
                }
                rep->n_flag_c++;
            }
        }
    }
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t c = 0; c < bc; ++c) {
            double s = 0.0;
            for (int64_t h = 0; h < Gc; ++h) s += C[i * ldc + h * bc + c];
            double d = s - C[i * ldc + n + c];
            double t = tau_r[i * bc + c];
            Dr[i * bc + c] = d;
            if (row_rel_has_erased(i, c, bc, erasures, n_erasures)) { rep->n_excl_r++; continue; }
            if (isfinite(d) && t > 0 && fabs(d) / t > rep->max_ratio_r) rep->max_ratio_r = fabs(d) / t;
            if (!(fabs(d) <= t)) {
                if (!isfinite(d)) rep->n_nonfinite++;
                if (rep->n_flag_r < ORC_MAXFLAG) {
                    int64_t q = rep->n_flag_r;
                    rep->fr_i[q] = i; rep->fr_c[q] = c; rep->fr_d[q] = d; rep->fr_t[q] = t;
                }
                rep->n_flag_r++;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Location (single-error model) and correction                             */
/* ------------------------------------------------------------------------ */

enum { ORC_CLEAN = 0, ORC_DATA = 1, ORC_CHECKSUM = 2, ORC_MULTI = 3 };
enum { ORC_DIR_COL = 0, ORC_DIR_ROW = 1 };

/*
 * One bad element (i, j) of C_f fails exactly one column relation
 * (i mod br, j) and one row relation (i, j mod bc).  Its residuals are
 * +delta where it is a summand and -delta where it is the stored total, so
 * sc*Dc and sr*Dr (sc = +1 for i < m, else -1; sr = +1 for j < n, else -1)
 * agree to within tau_c + tau_r plus the rounding of the two residual sums,
 * which both hold the bad value (gamma_{G+2} |delta| each), when both are
 * finite.
 * With known erasures, the relation through the erased rectangle is not
 * checked; a lone flag on one side then names the element when exactly one
 * candidate lies on an excluded relation of the other side.
 * Output: cls, (i, j) and the direction of the relation to rebuild it from.
 */
int orc_classify(int64_t m, int64_t n, int64_t br, int64_t bc, const orc_report *rep,
                 const int64_t *erasures, int n_erasures, int64_t *oi, int64_t *oj, int *odir)
{
    int64_t N = n + bc, M = m + br;
    *oi = -1; *oj = -1; *odir = ORC_DIR_COL;
    if (rep->n_flag_c == 0 && rep->n_flag_r == 0) return ORC_CLEAN;
    if (rep->n_flag_c == 1 && rep->n_flag_r == 1) {
        int64_t r = rep->fc_r[0], j = rep->fc_j[0], i = rep->fr_i[0], c = rep->fr_c[0];
        if (i % br != r || j % bc != c) return ORC_MULTI;
        double dc = rep->fc_d[0], dr = rep->fr_d[0];
        if (isfinite(dc) && isfinite(dr)) {
            /* each residual also carries the rounding of its own sum, which
             * holds the bad value: up to gamma_{G+2} |delta| (large when an
             * exponent bit flipped) */
            const double u64 = ldexp(1.0, -53);
            double big = fmax(fabs(dc), fabs(dr));
            double tol = rep->fc_t[0] + rep->fr_t[0] +
                         (orc_gamma((double)(m / br + 2), u64) + orc_gamma((double)(n / bc + 2), u64)) * big;
            double sc = (i < m) ? 1.0 : -1.0, sr = (j < n) ? 1.0 : -1.0;
            if (!(fabs(sc * dc - sr * dr) <= tol)) return ORC_MULTI;
        }
        *oi = i; *oj = j; *odir = ORC_DIR_COL;
        return (i < m && j < n) ? ORC_DATA : ORC_CHECKSUM;
    }
    if (n_erasures > 0 && rep->n_flag_c == 0 && rep->n_flag_r == 1) {
        int64_t i = rep->fr_i[0], c = rep->fr_c[0], found = -1, cnt = 0;
        for (int64_t j = c; j < N; j += bc)
            if (col_rel_has_erased(i % br, j, br, erasures, n_erasures)) { found = j; cnt++; }
        if (cnt != 1) return ORC_MULTI;
        *oi = i; *oj = found; *odir = ORC_DIR_ROW;
        return (i < m && found < n) ? ORC_DATA : ORC_CHECKSUM;
    }
    if (n_erasures > 0 && rep->n_flag_c == 1 && rep->n_flag_r == 0) {
        int64_t r = rep->fc_r[0], j = rep->fc_j[0], found = -1, cnt = 0;
        for (int64_t i = r; i < M; i += br)
            if (row_rel_has_erased(i, j % bc, bc, erasures, n_erasures)) { found = i; cnt++; }
        if (cnt != 1) return ORC_MULTI;
        *oi = found; *oj = j; *odir = ORC_DIR_COL;
        return (found < m && j < n) ? ORC_DATA : ORC_CHECKSUM;
    }
    return ORC_MULTI;
}

/*
 * Value of C_f[i, j] rebuilt from the other members of its relation
 * (Sec. 2.1 with unit weights: x_i = y - sum_{k != i} x_k).  The element
 * itself is never read.  Column direction: relation (i mod br, j); row
 * direction: relation (i, j mod bc).
 */
double orc_rebuild_value(int64_t m, int64_t n, int64_t br, int64_t bc, const double *C, int64_t ldc,
                         int64_t i, int64_t j, int dir)
{
    double s = 0.0;
    if (dir == ORC_DIR_COL) {
        int64_t r = i % br, Gr = m / br;
        for (int64_t g = 0; g < Gr; ++g) {
            int64_t ii = g * br + r;
            if (ii != i) s += C[ii * ldc + j];
        }
        return (i < m) ? C[(m + r) * ldc + j] - s : s;
    } else {
        int64_t c = j % bc, Gc = n / bc;
        for (int64_t h = 0; h < Gc; ++h) {
            int64_t jj = h * bc + c;
            if (jj != j) s += C[i * ldc + jj];
        }
        return (j < n) ? C[i * ldc + n + c] - s : s;
    }
}

/* Rebuild every element of an erased rectangle {i0, j0, h, w}.
 * Column direction needs h <= br (one unknown per column relation); row
 * direction needs w <= bc.  Returns 0, or -4 (unrecoverable) without writing.
 * round_f32 != 0 rounds each rebuilt value to binary32 (binary32 C). */
int orc_recover(int64_t m, int64_t n, int64_t br, int64_t bc, double *C, int64_t ldc,
                int64_t i0, int64_t j0, int64_t h, int64_t w, int use_rows, int round_f32)
{
    int64_t M = m + br, N = n + bc;
    if (i0 < 0 || j0 < 0 || h <= 0 || w <= 0 || i0 + h > M || j0 + w > N) return -1;
    if (!use_rows && h > br) return -4;
    if (use_rows && w > bc) return -4;
    /* Each rebuilt value only reads elements outside the rectangle, so the
     * order of the writes does not matter; stage them to keep it obvious. */
    double *out = (double *)malloc(sizeof(double) * (size_t)(h * w));
    for (int64_t a = 0; a < h; ++a)
        for (int64_t b = 0; b < w; ++b) {
            double v = orc_rebuild_value(m, n, br, bc, C, ldc, i0 + a, j0 + b, use_rows ? ORC_DIR_ROW : ORC_DIR_COL);
            out[a * w + b] = round_f32 ? (double)(float)v : v;
        }
    for (int64_t a = 0; a < h; ++a)
        for (int64_t b = 0; b < w; ++b) C[(i0 + a) * ldc + j0 + b] = out[a * w + b];
    free(out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Residual check (Sec. 4.3, stress test)                                    */
/* ------------------------------------------------------------------------ */

/* rho = ||C x - A (B x)||_inf / (k u ||C||_inf ||x||_inf), over the data part
 * C (m x n) = A (m x k) B (k x n).  u is the unit roundoff of the product. */
double orc_residual(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                    const double *C, int64_t ldc, const double *x, double u)
{
    double *bx = (double *)malloc(sizeof(double) * (size_t)k);
    for (int64_t l = 0; l < k; ++l) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += B[l * ldb + j] * x[j];
        bx[l] = s;
    }
    double rmax = 0.0, cnorm = 0.0, xnorm = 0.0;
    for (int64_t j = 0; j < n; ++j) xnorm = fmax(xnorm, fabs(x[j]));
    for (int64_t i = 0; i < m; ++i) {
        double cx = 0.0, abx = 0.0, rs = 0.0;
        for (int64_t j = 0; j < n; ++j) { cx += C[i * ldc + j] * x[j]; rs += fabs(C[i * ldc + j]); }
        for (int64_t l = 0; l < k; ++l) abx += A[i * lda + l] * bx[l];
        rmax = fmax(rmax, fabs(cx - abx));
        cnorm = fmax(cnorm, rs);
    }
    free(bx);
    return rmax / ((double)k * u * cnorm * xnorm);
}

/* ------------------------------------------------------------------------ */
/* Quantizers (round to nearest, ties to even)                               */
/* ------------------------------------------------------------------------ */

/* binary32 -> bfloat16 bits (1 sign, 8 exponent, 7 fraction).  The result is
 * the bfloat16 nearest to x, ties to even mantissa; NaN stays NaN. */
void orc_to_bf16(int64_t count, const float *x, uint16_t *out)
{
    for (int64_t q = 0; q < count; ++q) {
        float v = x[q];
        uint32_t u;
        memcpy(&u, &v, 4);
        if (isnan(v)) { out[q] = (uint16_t)((u >> 16) | 0x40); continue; }
        uint32_t hi = u >> 16, lo = u & 0xFFFFu;
        if (lo > 0x8000u || (lo == 0x8000u && (hi & 1u))) hi += 1;   /* carries into the exponent as needed */
        out[q] = (uint16_t)hi;
    }
}

/* Value of an OCP FP8 E4M3 ("e4m3fn") code: bias 7, 3 fraction bits,
 * no infinities, S.1111.111 is NaN, largest finite 448. */
double orc_e4m3_value(uint8_t code)
{
    int s = code >> 7, e = (code >> 3) & 15, f = code & 7;
    double v;
    if (e == 15 && f == 7) return NAN;
    if (e == 0) v = ldexp((double)f, -9);            /* subnormal: f/8 * 2^-6 */
    else v = ldexp(1.0 + f / 8.0, e - 7);
    return s ? -v : v;
}

/* binary32 -> E4M3 code, nearest value, ties to even fraction; inputs
 * beyond 448 (the infinities too: the format has none) saturate to +-448;
 * NaN -> 0x7F. */
void orc_to_e4m3(int64_t count, const float *x, uint8_t *out)
{
    for (int64_t q = 0; q < count; ++q) {
        double v = (double)x[q];
        if (isnan(v)) { out[q] = 0x7F; continue; }
        uint8_t sign = signbit(v) ? 0x80 : 0;
        if (isinf(v)) { out[q] = (uint8_t)(sign | 0x7E); continue; }
        double a = fabs(v);
        /* spacing of the E4M3 grid around a: 2^-9 below 2^-6, else 2^(floor(log2 a) - 3) */
        int ex;
        double spacing;
        if (a < ldexp(1.0, -6)) spacing = ldexp(1.0, -9);
        else { frexp(a, &ex); spacing = ldexp(1.0, (ex - 1) - 3); }
        double t = a / spacing;                   /* exact: power-of-two scaling */
        double fl = floor(t), rem = t - fl;
        double qv = fl;
        if (rem > 0.5 || (rem == 0.5 && fmod(fl, 2.0) == 1.0)) qv = fl + 1.0;
        double y = qv * spacing;
        if (y > 448.0) y = 448.0;
        /* encode y (a grid value, possibly one binade up after rounding) */
        uint8_t code;
        if (y == 0.0) code = 0;
        else if (y < ldexp(1.0, -6)) code = (uint8_t)(y / ldexp(1.0, -9));
        else {
            int e2;
            double fr = frexp(y, &e2);            /* y = fr * 2^e2, fr in [0.5,1) */
            int E = e2 - 1 + 7;
            int F = (int)((fr * 2.0 - 1.0) * 8.0);
            code = (uint8_t)((E << 3) | F);
        }
        out[q] = (uint8_t)(sign | code);
    }
}

/* Per-tensor power-of-two scale exponent: the largest e with amax * 2^e <= 448
 * (amax = max |x| over the finite entries: NaN and infinities cannot set a
 * scale); 0 when amax is 0.  Scaling by 2^e is exact. */
int orc_e4m3_scale_exp(int64_t count, const float *x)
{
    double amax = 0.0;
    for (int64_t q = 0; q < count; ++q)
        if (isfinite(x[q])) amax = fmax(amax, fabs((double)x[q]));
    if (amax == 0.0) return 0;
    int e = 0;
    while (ldexp(amax, e + 1) <= 448.0) ++e;
    while (ldexp(amax, e) > 448.0) --e;
    return e;
}

/* Threads the OpenMP loops of this library run on (1 without OpenMP), and a
 * way to change it (the single-core timing of the CPU baseline). */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int orc_num_threads(void) { return 1; }
void orc_set_num_threads(int n) { (void)n; }
#endif
