/*
 * Plain CPU FP64 oracle for Cholesky factorization, solution and inversion of a
 * symmetric positive definite matrix held in Rectangular Full Packed Format
 * (Gustavson, Wasniewski, Dongarra, Langou, "Rectangular Full Packed Format for
 * Cholesky's Algorithm: Factorization, Solution and Inversion").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library and never calls it.
 *
 * Everything here is deliberately slow and written to be checked by eye:
 *   - the element map of the eight RFP layouts is read off Figures 4, 5 and 6;
 *   - the factor is the textbook definition of the Cholesky factor
 *     (l_jj = sqrt(a_jj - sum l_jk^2), l_ij = (a_ij - sum l_ik l_jk) / l_jj),
 *     the unique lower-triangular L with positive diagonal and L L^T = A
 *     (Section 3, equations (alu)/(lluu));
 *   - a second factor path takes the paper's four steps (Figure 3, Section 3:
 *     POTRF on T1, TRSM on S, SYRK on T2, POTRF on T2) with naive loops over
 *     the three blocks of the rectangle, for the layout table of Figures 4-6;
 *   - the solve is forward then back substitution, L Y = B and L^T X = Y
 *     (Section 4, equations (sol:l)/(sol:u));
 *   - the inverse is W = L^{-1} by forward substitution on the identity and
 *     A^{-1} = W^T W (Section 5, equation (alum1)).
 *
 * Indices are 0-based and int64.  Characters are case-insensitive.
 * All floating point is IEEE binary64; metrics accumulate in long double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;

static int up(char c) { return (c >= 'a' && c <= 'z') ? c - 'a' + 'A' : c; }

/* ------------------------------------------------------------------------ */
/* Index layer                                                               */
/* ------------------------------------------------------------------------ */

/* Full format (Figure 1): element (i,j) of a column-major array, lda >= n. */
i64 orc_full_pos(i64 lda, i64 i, i64 j) { return i + j * lda; }

/* Packed format (Figure 2): columns of the stored triangle one after another.
 * Lower: column j holds rows j..n-1, so it starts after sum_{c<j} (n-c) entries.
 * Upper: column j holds rows 0..j, so it starts after sum_{c<j} (c+1) entries. */
i64 orc_packed_pos(char uplo, i64 n, i64 i, i64 j)
{
    if (up(uplo) == 'L') {
        if (i < j) { i64 t = i; i = j; j = t; }
        return (i - j) + j * n - (j * (j - 1)) / 2;
    } else {
        if (i > j) { i64 t = i; i = j; j = t; }
        return i + (j * (j + 1)) / 2;
    }
}

/* RFP (Figures 4, 5, 6).  (i,j) is any element of the symmetric matrix; the
 * stored copy is (max,min) for UPLO='L' and (min,max) for UPLO='U'.
 * The TRANSR='N' rectangle AR has LDAR = n (n odd) or n+1 (n even) rows and
 * C = ceil(n/2) columns.  Reading the figures:
 *   L, n odd  (Fig 4, Fig 6.1): column j < n1 of A sits in column j of AR,
 *             same rows; the lower triangle of A22 is transposed into the
 *             strict upper part of the top n1 x n1 square, shifted one column
 *             right: a(i,j) with j >= n1 -> AR(j-n1, i-n1+1).
 *   L, n even (Fig 5.2, Fig 6.2): column j < k of A sits one row down in
 *             column j of AR; A22's lower triangle is transposed into the top
 *             k x k square: a(i,j), j >= k -> AR(j-k, i-k).
 *   U, n odd  (Fig 5.3, Fig 6.1): columns j >= n2 of A sit in columns j-n2
 *             of AR; A11's upper triangle is transposed below row n1-1:
 *             a(i,j), j < n2 -> AR(n1+j, i).
 *   U, n even (Fig 5.4, Fig 6.2): columns j >= k sit in columns j-k; A11's
 *             upper triangle goes below row k: a(i,j), j < k -> AR(k+1+j, i).
 * TRANSR='T' stores AR^T: a C x LDAR array with leading dimension C, so the
 * element at AR(r,c) moves to offset c + r*C (Fig 6, "transpose, lda=n1"). */
i64 orc_rfp_pos(char transr, char uplo, i64 n, i64 i, i64 j)
{
    int lower = up(uplo) == 'L';
    int odd = (n % 2) == 1;
    i64 ldar = odd ? n : n + 1;
    i64 ncol = odd ? (n + 1) / 2 : n / 2;
    i64 r, c;
    if (lower) {
        if (i < j) { i64 t = i; i = j; j = t; }
        if (odd) {
            i64 n1 = (n + 1) / 2;
            if (j < n1) { r = i; c = j; } else { r = j - n1; c = i - n1 + 1; }
        } else {
            i64 k = n / 2;
            if (j < k) { r = i + 1; c = j; } else { r = j - k; c = i - k; }
        }
    } else {
        if (i > j) { i64 t = i; i = j; j = t; }
        if (odd) {
            i64 n1 = (n + 1) / 2, n2 = n / 2;
            if (j >= n2) { r = i; c = j - n2; } else { r = n1 + j; c = i; }
        } else {
            i64 k = n / 2;
            if (j >= k) { r = i; c = j - k; } else { r = k + 1 + j; c = i; }
        }
    }
    if (up(transr) == 'N') return r + c * ldar;
    return c + r * ncol;
}

/* TRTTF: full (column-major, lda) -> RFP.  Only the UPLO triangle is read. */
void orc_trttf(char transr, char uplo, i64 n, const double *a, i64 lda, double *arf)
{
    int lower = up(uplo) == 'L';
    for (i64 j = 0; j < n; j++)
        for (i64 i = lower ? j : 0; i < (lower ? n : j + 1); i++)
            arf[orc_rfp_pos(transr, uplo, n, i, j)] = a[orc_full_pos(lda, i, j)];
}

/* TFTTR: RFP -> full.  Only the UPLO triangle of a is written. */
void orc_tfttr(char transr, char uplo, i64 n, const double *arf, double *a, i64 lda)
{
    int lower = up(uplo) == 'L';
    for (i64 j = 0; j < n; j++)
        for (i64 i = lower ? j : 0; i < (lower ? n : j + 1); i++)
            a[orc_full_pos(lda, i, j)] = arf[orc_rfp_pos(transr, uplo, n, i, j)];
}

/* TPTTF / TFTTP: packed <-> RFP. */
void orc_tpttf(char transr, char uplo, i64 n, const double *ap, double *arf)
{
    int lower = up(uplo) == 'L';
    for (i64 j = 0; j < n; j++)
        for (i64 i = lower ? j : 0; i < (lower ? n : j + 1); i++)
            arf[orc_rfp_pos(transr, uplo, n, i, j)] = ap[orc_packed_pos(uplo, n, i, j)];
}

void orc_tfttp(char transr, char uplo, i64 n, const double *arf, double *ap)
{
    int lower = up(uplo) == 'L';
    for (i64 j = 0; j < n; j++)
        for (i64 i = lower ? j : 0; i < (lower ? n : j + 1); i++)
            ap[orc_packed_pos(uplo, n, i, j)] = arf[orc_rfp_pos(transr, uplo, n, i, j)];
}

/* Unpack the symmetric matrix (or the factor) into a dense row-major lower
 * triangle F[i*n+j], i >= j.  For UPLO='U' the stored upper element (j,i)
 * is the lower element (i,j): A is symmetric and U = L^T. */
static void unpack_lower(char transr, char uplo, i64 n, const double *arf, double *F)
{
    memset(F, 0, sizeof(double) * (size_t)(n * n));
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++)
            F[i * n + j] = arf[orc_rfp_pos(transr, uplo, n, i, j)];
}

static void pack_lower(char transr, char uplo, i64 n, const double *F, double *arf)
{
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++)
            arf[orc_rfp_pos(transr, uplo, n, i, j)] = F[i * n + j];
}

/* ------------------------------------------------------------------------ */
/* Factorization by definition (Section 3)                                   */
/* ------------------------------------------------------------------------ */

/* Cholesky factor of the dense lower triangle F (row-major), in place.
 * Returns 0, or j+1 when the leading minor of order j+1 is not positive
 * definite (the diagonal quantity is <= 0 or NaN); F is then left partly
 * overwritten.  Column j is finished before column j+1 starts; each l_ij is
 * the plain formula.  Rows of one column are independent, so the row loop
 * may run on several threads without changing any result. */
static int chol_def(i64 n, double *F)
{
    for (i64 j = 0; j < n; j++) {
        double s = F[j * n + j];
        for (i64 k = 0; k < j; k++) s -= F[j * n + k] * F[j * n + k];
        if (!(s > 0.0)) return (int)(j + 1);
        double ljj = sqrt(s);
        F[j * n + j] = ljj;
        const double *rj = F + j * n;
#pragma omp parallel for schedule(static)
        for (i64 i = j + 1; i < n; i++) {
            double *ri = F + i * n;
            double t = ri[j];
            for (i64 k = 0; k < j; k++) t -= ri[k] * rj[k];
            ri[j] = t / ljj;
        }
    }
    return 0;
}

/* PFTRF: A = L L^T (UPLO='L') or A = U^T U (UPLO='U'), overwriting arf with
 * the factor in the same layout.  On failure arf is left untouched and the
 * global order of the first non-positive-definite leading minor is returned. */
int orc_pftrf(char transr, char uplo, i64 n, double *arf)
{
    if (n <= 0) return 0;
    double *F = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!F) return -100;
    unpack_lower(transr, uplo, n, arf, F);
    int info = chol_def(n, F);
    if (info == 0) pack_lower(transr, uplo, n, F, arf);
    free(F);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Factorization by the paper's four steps (Figure 3, Section 3)             */
/* ------------------------------------------------------------------------ */

/* One of the three blocks T1, S, T2 of the rectangle, addressed as the
 * corresponding block of the lower factor: L11 (m1 x m1), L21 (m2 x m1),
 * L22 (m2 x m2).  Element (i,j) of the block is arf[off + i*rs + j*cs].
 * Offsets and orientations follow Figures 4-6:
 *   (N,L): T1 = L11 stored 'L' at the top-left; S = A21 below it;
 *          T2 = A22 stored 'U' (i.e. L22^T) in the upper part, one column
 *          right (odd) or one row up (even).
 *   (N,U): S = A12 on top; T1 = A11 stored 'L' below (A11^T); T2 = A22 'U'.
 *   (T,*): the same rectangle transposed, so row and column strides swap. */
typedef struct { i64 off, rs, cs; } blk;

static void srpa_blocks(char transr, char uplo, i64 n, i64 *m1, i64 *m2, blk *t1, blk *s, blk *t2)
{
    int lower = up(uplo) == 'L', odd = n % 2, tr = up(transr) == 'T';
    i64 ldar = odd ? n : n + 1;
    i64 ncol = odd ? (n + 1) / 2 : n / 2;
    /* Position (r,c) of each block's (0,0) element in AR, and whether the
     * block's (i,j) runs down rows (i -> r) or along columns (i -> c). */
    i64 r1, c1, rs2, cs2, r3, c3;
    int t1_rowwise, s_rowwise, t2_rowwise; /* 1: block row index i moves down AR rows */
    if (lower) {
        *m1 = odd ? (n + 1) / 2 : n / 2;
        *m2 = n - *m1;
        /* T1: a(i,j), i,j < m1 at AR(i + (odd?0:1), j) */
        r1 = odd ? 0 : 1; c1 = 0; t1_rowwise = 1;
        /* S: a(m1+i, j) at AR(m1 + i + (odd?0:1), j) */
        rs2 = *m1 + (odd ? 0 : 1); cs2 = 0; s_rowwise = 1;
        /* T2: a(m1+i, m1+j) at AR(j, i + (odd?1:0)) : transposed */
        r3 = 0; c3 = odd ? 1 : 0; t2_rowwise = 0;
    } else {
        *m1 = n / 2;             /* odd: A11 has order floor(n/2) (Fig 5.3) */
        *m2 = n - *m1;
        /* Upper storage holds U = L^T.  L11(i,j) = U11(j,i) = a(j,i), j<=i<m1,
         * stored at AR(r, c) = (ncolA + i, j) with ncolA = n1 (odd) or k+1. */
        i64 base = odd ? (n + 1) / 2 : n / 2 + 1;
        r1 = base; c1 = 0; t1_rowwise = 1;
        /* L21(i,j) = U12(j, i) = a(j, m1+i): column m1+i of A -> AR column i,
         * row j. */
        rs2 = 0; cs2 = 0; s_rowwise = 0;
        /* L22(i,j) = U22(j,i) = a(m1+j, m1+i): AR(m1 + j, i) */
        r3 = *m1; c3 = 0; t2_rowwise = 0;
    }
    /* convert to offsets/strides in the TRANSR='N' array, then transpose */
    i64 rstride = tr ? ncol : 1, cstride = tr ? 1 : ldar;
    t1->off = r1 * rstride + c1 * cstride;
    t1->rs = t1_rowwise ? rstride : cstride;
    t1->cs = t1_rowwise ? cstride : rstride;
    s->off = rs2 * rstride + cs2 * cstride;
    s->rs = s_rowwise ? rstride : cstride;
    s->cs = s_rowwise ? cstride : rstride;
    t2->off = r3 * rstride + c3 * cstride;
    t2->rs = t2_rowwise ? rstride : cstride;
    t2->cs = t2_rowwise ? cstride : rstride;
}

#define AT(b, i, j) arf[(b).off + (i) * (b).rs + (j) * (b).cs]

/* Unblocked Cholesky on the lower triangle of a block (step 1 / step 4). */
static int potrf_blk(double *arf, blk b, i64 m)
{
    for (i64 j = 0; j < m; j++) {
        double s = AT(b, j, j);
        for (i64 k = 0; k < j; k++) s -= AT(b, j, k) * AT(b, j, k);
        if (!(s > 0.0)) return (int)(j + 1);
        double ljj = sqrt(s);
        AT(b, j, j) = ljj;
        for (i64 i = j + 1; i < m; i++) {
            double t = AT(b, i, j);
            for (i64 k = 0; k < j; k++) t -= AT(b, i, k) * AT(b, j, k);
            AT(b, i, j) = t / ljj;
        }
    }
    return 0;
}

/* The paper's four steps.  Returns INFO in the global order of A. */
int orc_pftrf_srpa(char transr, char uplo, i64 n, double *arf)
{
    if (n <= 0) return 0;
    i64 m1, m2;
    blk t1, s, t2;
    srpa_blocks(transr, uplo, n, &m1, &m2, &t1, &s, &t2);
    /* step 1: L11 L11^T = A11 */
    int info = potrf_blk(arf, t1, m1);
    if (info) return info;
    /* step 2: L21 L11^T = A21, i.e. L21 = A21 L11^{-T}, row by row */
    for (i64 i = 0; i < m2; i++)
        for (i64 j = 0; j < m1; j++) {
            double t = AT(s, i, j);
            for (i64 k = 0; k < j; k++) t -= AT(s, i, k) * AT(t1, j, k);
            AT(s, i, j) = t / AT(t1, j, j);
        }
    /* step 3: A22 <- A22 - L21 L21^T on the stored triangle */
    for (i64 i = 0; i < m2; i++)
        for (i64 j = 0; j <= i; j++) {
            double t = 0.0;
            for (i64 k = 0; k < m1; k++) t += AT(s, i, k) * AT(s, j, k);
            AT(t2, i, j) -= t;
        }
    /* step 4: L22 L22^T = updated A22 */
    info = potrf_blk(arf, t2, m2);
    return info ? (int)(m1 + info) : 0;
}

/* Exported so tests can check the block table against the element map. */
void orc_srpa_blocks(char transr, char uplo, i64 n, i64 *out /* m1,m2, t1(off,rs,cs), s(...), t2(...) */)
{
    i64 m1, m2;
    blk t1, s, t2;
    srpa_blocks(transr, uplo, n, &m1, &m2, &t1, &s, &t2);
    out[0] = m1; out[1] = m2;
    out[2] = t1.off; out[3] = t1.rs; out[4] = t1.cs;
    out[5] = s.off; out[6] = s.rs; out[7] = s.cs;
    out[8] = t2.off; out[9] = t2.rs; out[10] = t2.cs;
}

/* ------------------------------------------------------------------------ */
/* Solution (Section 4)                                                      */
/* ------------------------------------------------------------------------ */

/* PFTRS: given the PFTRF factor in arf, solve A X = B; X overwrites B
 * (column-major, ldb >= n).  L Y = B by forward substitution, then
 * L^T X = Y by back substitution, one right-hand side at a time. */
void orc_pftrs(char transr, char uplo, i64 n, i64 nrhs, const double *arf, double *b, i64 ldb)
{
    if (n <= 0 || nrhs <= 0) return;
    double *F = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!F) return;
    unpack_lower(transr, uplo, n, arf, F);
#pragma omp parallel for schedule(static)
    for (i64 c = 0; c < nrhs; c++) {
        double *x = b + c * ldb;
        for (i64 i = 0; i < n; i++) {          /* L y = b */
            double t = x[i];
            for (i64 k = 0; k < i; k++) t -= F[i * n + k] * x[k];
            x[i] = t / F[i * n + i];
        }
        for (i64 i = n - 1; i >= 0; i--) {     /* L^T x = y */
            double t = x[i];
            for (i64 k = i + 1; k < n; k++) t -= F[k * n + i] * x[k];
            x[i] = t / F[i * n + i];
        }
    }
    free(F);
}

/* ------------------------------------------------------------------------ */
/* Inversion (Section 5)                                                     */
/* ------------------------------------------------------------------------ */

/* PFTRI: given the PFTRF factor, overwrite arf with the same triangle of
 * A^{-1} in the same layout.  W = L^{-1} column by column (L w_j = e_j),
 * then A^{-1} = W^T W, i.e. (A^{-1})_ij = sum_{k >= i} W_ki W_kj for i >= j.
 * Returns i+1 if the factor's diagonal entry i is exactly zero. */
int orc_pftri(char transr, char uplo, i64 n, double *arf)
{
    if (n <= 0) return 0;
    double *F = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *W = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!F || !W) { free(F); free(W); return -100; }
    unpack_lower(transr, uplo, n, arf, F);
    for (i64 i = 0; i < n; i++)
        if (F[i * n + i] == 0.0) { free(F); free(W); return (int)(i + 1); }
    memset(W, 0, sizeof(double) * (size_t)(n * n));
#pragma omp parallel for schedule(dynamic, 8)
    for (i64 j = 0; j < n; j++) {               /* column j of W */
        for (i64 i = j; i < n; i++) {
            double t = (i == j) ? 1.0 : 0.0;
            for (i64 k = j; k < i; k++) t -= F[i * n + k] * W[k * n + j];
            W[i * n + j] = t / F[i * n + i];
        }
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) {
            double t = 0.0;
            for (i64 k = i; k < n; k++) t += W[k * n + i] * W[k * n + j];
            F[i * n + j] = t;
        }
    pack_lower(transr, uplo, n, F, arf);
    free(F);
    free(W);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Metrics (long double accumulation)                                        */
/* ------------------------------------------------------------------------ */

static double sym_at(char transr, char uplo, i64 n, const double *arf, i64 i, i64 j)
{
    return arf[orc_rfp_pos(transr, uplo, n, i, j)];
}

/* ||A||_inf of the symmetric matrix held in RFP (max absolute row sum). */
double orc_norm_inf(char transr, char uplo, i64 n, const double *arf)
{
    long double best = 0.0L;
    for (i64 i = 0; i < n; i++) {
        long double s = 0.0L;
        for (i64 j = 0; j < n; j++) s += fabsl((long double)sym_at(transr, uplo, n, arf, i, j));
        if (s > best) best = s;
    }
    return (double)best;
}

/* max |a_ij| and the Frobenius norm of the symmetric matrix held in RFP
 * (the LANSF norms of the paper's routine table), by visiting every (i, j). */
double orc_norm_max(char transr, char uplo, i64 n, const double *arf)
{
    double best = 0.0;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            double v = fabs(sym_at(transr, uplo, n, arf, i, j));
            if (v > best) best = v;
        }
    return best;
}

double orc_norm_fro(char transr, char uplo, i64 n, const double *arf)
{
    long double s = 0.0L;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            long double v = (long double)sym_at(transr, uplo, n, arf, i, j);
            s += v * v;
        }
    return (double)sqrtl(s);
}

/* Y = alpha A X + beta Y for the symmetric A held in RFP (X, Y n x nrhs
 * column-major), by the definition of the product over the full symmetric
 * matrix, each sum in long double; beta = 0 does not read Y. */
void orc_sfmv(char transr, char uplo, i64 n, i64 nrhs, double alpha, const double *arf, const double *x, i64 ldx,
              double beta, double *y, i64 ldy)
{
    for (i64 c = 0; c < nrhs; c++)
        for (i64 i = 0; i < n; i++) {
            long double s = 0.0L;
            for (i64 j = 0; j < n; j++) s += (long double)sym_at(transr, uplo, n, arf, i, j) * x[j + c * ldx];
            double v = (double)((long double)alpha * s);
            if (beta != 0.0) v += beta * y[i + c * ldy];
            y[i + c * ldy] = v;
        }
}

/* Scaled cast of the mixed-precision solve (not part of the paper; the
 * scaling D^{-1/2} A D^{-1/2} with D = diag(A) is the classical symmetric
 * equilibration, the diagonal shift that of Higham and Pranesh's
 * low-precision Cholesky, SIAM J. Sci. Comput. 43 (2021)): s_i = 1 / sqrt(a_ii)
 * when scale is set (NaN for a non-positive a_ii), else 1; then every stored
 * entry becomes (float)(((a_ij * s_i) * s_j) * mu) with i > j, and a diagonal
 * one (float)((((a_ii * s_i) * s_i) + shift) * mu), each operation rounded in
 * binary64 in that order. */
void orc_pfcast_s(char transr, char uplo, i64 n, const double *arf, int scale, double mu, double shift, double *s,
                  float *out)
{
    for (i64 i = 0; i < n; i++) {
        double d = sym_at(transr, uplo, n, arf, i, i);
        s[i] = scale ? (d > 0.0 ? 1.0 / sqrt(d) : NAN) : 1.0;
    }
    for (i64 j = 0; j < n; j++)
        for (i64 i = j; i < n; i++) {
            i64 p = orc_rfp_pos(transr, uplo, n, i, j);
            double v = arf[p] * s[i];
            v = v * s[j];
            if (i == j) v = v + shift;
            v = v * mu;
            out[p] = (float)v;
        }
}

/* ------------------------------------------------------------------------ */
/* The rest of the routine table: TFTRI, TFSM, SFRK                          */
/* ------------------------------------------------------------------------ */

/* Dense triangular matrix T (row-major n x n, zero outside its triangle) of a
 * triangular matrix held in RFP: UPLO='L' lower, 'U' upper; DIAG='U' puts ones
 * on the diagonal (the stored diagonal is not read). */
static void unpack_tri(char transr, char uplo, char diag, i64 n, const double *arf, double *T)
{
    int lower = up(uplo) == 'L';
    memset(T, 0, sizeof(double) * (size_t)(n * n));
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            if (lower ? j > i : j < i) continue;
            T[i * n + j] = (i == j && up(diag) == 'U') ? 1.0 : arf[orc_rfp_pos(transr, uplo, n, i, j)];
        }
}

/* TFTRI (the routine table, "Triangular inversion"): the inverse of the
 * triangular matrix T held in RFP overwrites it, same layout.  By definition
 * T X = I, column by column: forward substitution for a lower T, back
 * substitution for an upper T.  Returns 0, or i+1 when T(i,i) is exactly zero
 * (DIAG='N'); the array is then untouched.  DIAG='U' leaves the stored
 * diagonal as it was. */
int orc_tftri(char transr, char uplo, char diag, i64 n, double *arf)
{
    if (n <= 0) return 0;
    int lower = up(uplo) == 'L', unit = up(diag) == 'U';
    double *T = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *X = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!T || !X) { free(T); free(X); return -100; }
    unpack_tri(transr, uplo, diag, n, arf, T);
    for (i64 i = 0; i < n; i++)
        if (T[i * n + i] == 0.0) { free(T); free(X); return (int)(i + 1); }
    memset(X, 0, sizeof(double) * (size_t)(n * n));
    for (i64 c = 0; c < n; c++) {
        if (lower) {
            for (i64 i = 0; i < n; i++) {
                double t = (i == c) ? 1.0 : 0.0;
                for (i64 k = 0; k < i; k++) t -= T[i * n + k] * X[k * n + c];
                X[i * n + c] = t / T[i * n + i];
            }
        } else {
            for (i64 i = n - 1; i >= 0; i--) {
                double t = (i == c) ? 1.0 : 0.0;
                for (i64 k = i + 1; k < n; k++) t -= T[i * n + k] * X[k * n + c];
                X[i * n + c] = t / T[i * n + i];
            }
        }
    }
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            if (lower ? j > i : j < i) continue;
            if (i == j && unit) continue;
            arf[orc_rfp_pos(transr, uplo, n, i, j)] = X[i * n + j];
        }
    free(T);
    free(X);
    return 0;
}

/* TFSM (the routine table, "Triangular solve"): B (m x n, column-major, ldb)
 * becomes X with
 *   SIDE='L': op(A) X = alpha B,   A of order m;
 *   SIDE='R': X op(A) = alpha B,   A of order n;
 * op(A) = A (TRANS='N') or A^T (TRANS='T'); A triangular in RFP (UPLO, DIAG).
 * alpha = 0 sets B to zero without reading A.  Plain substitution on the
 * dense op(A), one right-hand side (a column for SIDE='L', a row for
 * SIDE='R') at a time. */
void orc_tfsm(char transr, char side, char uplo, char trans, char diag, i64 m, i64 n, double alpha,
              const double *arf, double *b, i64 ldb)
{
    if (m <= 0 || n <= 0) return;
    int left = up(side) == 'L';
    i64 k = left ? m : n;
    if (alpha == 0.0) {
        for (i64 j = 0; j < n; j++)
            for (i64 i = 0; i < m; i++) b[i + j * ldb] = 0.0;
        return;
    }
    double *T = (double *)malloc(sizeof(double) * (size_t)(k * k));
    double *O = (double *)malloc(sizeof(double) * (size_t)(k * k));
    double *v = (double *)malloc(sizeof(double) * (size_t)k);
    if (!T || !O || !v) { free(T); free(O); free(v); return; }
    unpack_tri(transr, uplo, diag, k, arf, T);
    /* O = op(A), dense row-major */
    for (i64 i = 0; i < k; i++)
        for (i64 j = 0; j < k; j++) O[i * k + j] = (up(trans) == 'N') ? T[i * k + j] : T[j * k + i];
    /* op(A) lower or upper */
    int olow = (up(uplo) == 'L') == (up(trans) == 'N');
    i64 nsys = left ? n : m;
    for (i64 q = 0; q < nsys; q++) {
        /* right-hand side q: column q of B (left) or row q of B (right) */
        for (i64 i = 0; i < k; i++) v[i] = alpha * (left ? b[i + q * ldb] : b[q + i * ldb]);
        if (left) {
            /* op(A) x = v */
            if (olow) {
                for (i64 i = 0; i < k; i++) {
                    double t = v[i];
                    for (i64 c = 0; c < i; c++) t -= O[i * k + c] * v[c];
                    v[i] = t / O[i * k + i];
                }
            } else {
                for (i64 i = k - 1; i >= 0; i--) {
                    double t = v[i];
                    for (i64 c = i + 1; c < k; c++) t -= O[i * k + c] * v[c];
                    v[i] = t / O[i * k + i];
                }
            }
        } else {
            /* x op(A) = v, i.e. op(A)^T x = v: column c of op(A) gives equation c */
            if (olow) {
                for (i64 c = k - 1; c >= 0; c--) {
                    double t = v[c];
                    for (i64 r = c + 1; r < k; r++) t -= O[r * k + c] * v[r];
                    v[c] = t / O[c * k + c];
                }
            } else {
                for (i64 c = 0; c < k; c++) {
                    double t = v[c];
                    for (i64 r = 0; r < c; r++) t -= O[r * k + c] * v[r];
                    v[c] = t / O[c * k + c];
                }
            }
        }
        for (i64 i = 0; i < k; i++) {
            if (left) b[i + q * ldb] = v[i];
            else b[q + i * ldb] = v[i];
        }
    }
    free(T);
    free(O);
    free(v);
}

/* SFRK (the routine table, "Sym rank-k update"): C = alpha op(A) op(A)^T +
 * beta C on the stored triangle of the symmetric C (order n) in RFP, with
 * op(A) = A (n x k, TRANS='N') or A^T (A k x n, TRANS='T'), A column-major
 * with leading dimension lda.  beta = 0 does not read C; alpha = 0 (or
 * k = 0) does not read A.  Every stored entry is the plain dot product. */
void orc_sfrk(char transr, char uplo, char trans, i64 n, i64 k, double alpha, const double *a, i64 lda,
              double beta, double *c)
{
    int notr = up(trans) == 'N';
    for (i64 j = 0; j < n; j++)
        for (i64 i = j; i < n; i++) {
            i64 p = orc_rfp_pos(transr, uplo, n, i, j);
            double t = 0.0;
            if (alpha != 0.0)
                for (i64 l = 0; l < k; l++) {
                    double ail = notr ? a[i + l * lda] : a[l + i * lda];
                    double ajl = notr ? a[j + l * lda] : a[l + j * lda];
                    t += ail * ajl;
                }
            double v = alpha * t;
            if (beta != 0.0) v += beta * c[p];
            c[p] = v;
        }
}

/* Normwise backward error of a solve, max over columns:
 *   eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf).
 * A is the original matrix in RFP; residuals accumulate in long double. */
double orc_backward_error(char transr, char uplo, i64 n, i64 nrhs, const double *arf,
                          const double *b, i64 ldb, const double *x, i64 ldx)
{
    if (n <= 0 || nrhs <= 0) return 0.0;
    double anorm = orc_norm_inf(transr, uplo, n, arf);
    double *F = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!F) return -1.0;
    unpack_lower(transr, uplo, n, arf, F);
    double worst = 0.0;
    for (i64 c = 0; c < nrhs; c++) {
        const double *bc = b + c * ldb, *xc = x + c * ldx;
        long double rmax = 0.0L, xmax = 0.0L, bmax = 0.0L;
        for (i64 i = 0; i < n; i++) {
            long double r = bc[i];
            for (i64 j = 0; j < n; j++) {
                double aij = (i >= j) ? F[i * n + j] : F[j * n + i];
                r -= (long double)aij * (long double)xc[j];
            }
            if (fabsl(r) > rmax) rmax = fabsl(r);
            if (fabsl((long double)xc[i]) > xmax) xmax = fabsl((long double)xc[i]);
            if (fabsl((long double)bc[i]) > bmax) bmax = fabsl((long double)bc[i]);
        }
        long double den = (long double)anorm * xmax + bmax;
        double eta = den > 0 ? (double)(rmax / den) : (double)rmax;
        if (eta > worst) worst = eta;
    }
    free(F);
    return worst;
}

/* Normwise forward error of a solve against a reference solution, max over
 * columns: ||x - x_ref||_inf / ||x_ref||_inf (an exact zero column of x_ref
 * gives ||x||_inf).  Differences accumulate in long double. */
double orc_forward_error(i64 n, i64 nrhs, const double *x, i64 ldx, const double *xr, i64 ldr)
{
    double worst = 0.0;
    for (i64 c = 0; c < nrhs; c++) {
        long double dmax = 0.0L, rmax = 0.0L;
        for (i64 i = 0; i < n; i++) {
            long double d = fabsl((long double)x[i + c * ldx] - (long double)xr[i + c * ldr]);
            long double r = fabsl((long double)xr[i + c * ldr]);
            if (d > dmax) dmax = d;
            if (r > rmax) rmax = r;
        }
        double e = rmax > 0 ? (double)(dmax / rmax) : (double)dmax;
        if (e > worst) worst = e;
    }
    return worst;
}

/* ||L L^T - A||_F / ||A||_F, with L the PFTRF output for A (same layout). */
double orc_factor_residual(char transr, char uplo, i64 n, const double *arf_a, const double *arf_l)
{
    if (n <= 0) return 0.0;
    double *L = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!L) return -1.0;
    unpack_lower(transr, uplo, n, arf_l, L);
    long double num = 0.0L, den = 0.0L;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) {
            long double t = 0.0L;
            for (i64 k = 0; k <= j; k++) t += (long double)L[i * n + k] * L[j * n + k];
            long double a = sym_at(transr, uplo, n, arf_a, i, j);
            long double w = (i == j) ? 1.0L : 2.0L; /* both triangles */
            num += w * (t - a) * (t - a);
            den += w * a * a;
        }
    free(L);
    return (double)sqrtl(num / den);
}

/* ||I - A A^{-1}||_F / (||A||_F ||A^{-1}||_F), both in RFP (same layout). */
double orc_inverse_residual(char transr, char uplo, i64 n, const double *arf_a, const double *arf_inv)
{
    if (n <= 0) return 0.0;
    double *A = (double *)malloc(sizeof(double) * (size_t)(n * n));
    double *V = (double *)malloc(sizeof(double) * (size_t)(n * n));
    if (!A || !V) { free(A); free(V); return -1.0; }
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            A[i * n + j] = sym_at(transr, uplo, n, arf_a, i, j);
            V[i * n + j] = sym_at(transr, uplo, n, arf_inv, i, j);
        }
    long double num = 0.0L, na = 0.0L, nv = 0.0L;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            long double t = 0.0L;
            for (i64 k = 0; k < n; k++) t += (long double)A[i * n + k] * V[k * n + j];
            long double e = ((i == j) ? 1.0L : 0.0L) - t;
            num += e * e;
            na += (long double)A[i * n + j] * A[i * n + j];
            nv += (long double)V[i * n + j] * V[i * n + j];
        }
    free(A);
    free(V);
    return (double)(sqrtl(num) / (sqrtl(na) * sqrtl(nv)));
}
