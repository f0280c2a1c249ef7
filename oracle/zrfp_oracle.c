/*
 * Plain CPU oracle for the complex Hermitian case of RFP Cholesky:
 * factorization, solution and inversion of a Hermitian positive definite
 * matrix (A = L L^H, Section 3 equations (alu)/(lluu), Hermitian rows).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library and never calls it.
 *
 * Format (Section 2 with the closing remark on the complex case beside the
 * routine table): a complex RFP array holds the same n(n+1)/2 positions as
 * the real format of the same TRANSR/UPLO, but wherever the real format keeps
 * a part of the triangle transposed, the complex format keeps its conjugate
 * transpose; TRANSR='C' keeps the conjugate transpose of the whole rectangle
 * (where the real format has TRANSR='T').  The positions are the real
 * oracle's (orc_rfp_pos, read off Figures 4-6); this file adds which stored
 * numbers are conjugates.
 *
 * Numerics (all binary64 complex, metrics accumulated in long double):
 *   - the factor by the textbook definition: l_jj = sqrt(a_jj - sum |l_jk|^2),
 *     l_ij = (a_ij - sum l_ik conj(l_jk)) / l_jj;
 *   - a second path through the paper's four steps on the blocks of the
 *     rectangle (Section 3: POTRF on A11, TRSM L21 = A21 L11^{-H}, HERK
 *     A22 - L21 L21^H, POTRF on A22);
 *   - the solve L Y = B, L^H X = Y (Section 4, Hermitian case);
 *   - the inverse A^{-1} = W^H W with W = L^{-1} (Section 5, Hermitian case).
 * Indices are 0-based.  Complex arrays are interleaved (re, im) doubles.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;
typedef double complex zc;

i64 orc_rfp_pos(char transr, char uplo, i64 n, i64 i, i64 j);

static int zup(char c) { return (c >= 'a' && c <= 'z') ? c - 'a' + 'A' : c; }

/* Stored-triangle element (i,j) (i >= j for UPLO='L', i <= j for 'U'): its
 * offset, and whether the number there is its conjugate.  Reading Figures
 * 4-6: the parts placed transposed are, for 'L', the columns of A22
 * (j >= ceil(n/2)); for 'U', the columns of A11 (j < floor(n/2)). */
i64 orc_zrfp_pos(char transr, char uplo, i64 n, i64 i, i64 j, int *conj)
{
    const int lower = zup(uplo) == 'L';
    const int ctr = zup(transr) == 'C';
    int transposed;
    if (lower)
        transposed = j >= (n + 1) / 2;
    else
        transposed = j < n / 2;
    *conj = transposed != ctr;
    return orc_rfp_pos(ctr ? 'T' : 'N', uplo, n, i, j);
}

/* A(i,j) for any (i,j) of the Hermitian matrix held in arf. */
static zc zget(char transr, char uplo, i64 n, const zc *arf, i64 i, i64 j)
{
    const int lower = zup(uplo) == 'L';
    int flip = 0; /* (i,j) outside the stored triangle: A(i,j) = conj(A(j,i)) */
    if ((lower && i < j) || (!lower && i > j)) {
        i64 t = i; i = j; j = t;
        flip = 1;
    }
    int cj;
    zc v = arf[orc_zrfp_pos(transr, uplo, n, i, j, &cj)];
    if (cj) v = conj(v);
    return flip ? conj(v) : v;
}

/* Store the stored-triangle element (i,j) of the matrix held in arf. */
static void zset(char transr, char uplo, i64 n, zc *arf, i64 i, i64 j, zc v)
{
    int cj;
    i64 p = orc_zrfp_pos(transr, uplo, n, i, j, &cj);
    arf[p] = cj ? conj(v) : v;
}

/* Logical lower triangle L(i,j), i >= j, of the array (the matrix itself, or
 * the factor: for UPLO='U' the array holds U = L^H). */
static zc zgetL(char transr, char uplo, i64 n, const zc *arf, i64 i, i64 j)
{
    return zget(transr, uplo, n, arf, i, j);
}
static void zsetL(char transr, char uplo, i64 n, zc *arf, i64 i, i64 j, zc v)
{
    if (zup(uplo) == 'L')
        zset(transr, uplo, n, arf, i, j, v);
    else
        zset(transr, uplo, n, arf, j, i, conj(v));
}

/* ZTRTTF / ZTFTTR: full (column-major, lda) <-> RFP; only the UPLO triangle
 * of the full array is read / written. */
void orc_ztrttf(char transr, char uplo, i64 n, const zc *a, i64 lda, zc *arf)
{
    const int lower = zup(uplo) == 'L';
    for (i64 j = 0; j < n; j++)
        for (i64 i = lower ? j : 0; i < (lower ? n : j + 1); i++) zset(transr, uplo, n, arf, i, j, a[i + j * lda]);
}

void orc_ztfttr(char transr, char uplo, i64 n, const zc *arf, zc *a, i64 lda)
{
    const int lower = zup(uplo) == 'L';
    for (i64 j = 0; j < n; j++)
        for (i64 i = lower ? j : 0; i < (lower ? n : j + 1); i++) a[i + j * lda] = zget(transr, uplo, n, arf, i, j);
}

/* Textbook Cholesky of the n x n lower triangle F (row-major, F[i*n+j], i >= j),
 * in place; returns 0, or j+1 (plus off) when the j-th pivot is not positive. */
static int zchol_lower(i64 n, zc *F, i64 ld, int off)
{
    for (i64 j = 0; j < n; j++) {
        double d = creal(F[j * ld + j]);
        for (i64 k = 0; k < j; k++) d -= creal(F[j * ld + k]) * creal(F[j * ld + k]) + cimag(F[j * ld + k]) * cimag(F[j * ld + k]);
        if (!(d > 0.0)) return (int)(j + 1 + off);
        const double l = sqrt(d);
        F[j * ld + j] = l;
        for (i64 i = j + 1; i < n; i++) {
            zc s = F[i * ld + j];
            for (i64 k = 0; k < j; k++) s -= F[i * ld + k] * conj(F[j * ld + k]);
            F[i * ld + j] = s / l;
        }
    }
    return 0;
}

/* Definition path: unpack the lower triangle, factor, pack L (UPLO='L') or
 * U = L^H (UPLO='U').  On failure the array is left as given. */
int orc_zpftrf(char transr, char uplo, i64 n, zc *arf)
{
    if (n <= 0) return 0;
    zc *F = (zc *)calloc((size_t)(n * n), sizeof(zc));
    if (!F) return -1;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) F[i * n + j] = zgetL(transr, uplo, n, arf, i, j);
    int info = zchol_lower(n, F, n, 0);
    if (info == 0)
        for (i64 i = 0; i < n; i++)
            for (i64 j = 0; j <= i; j++) zsetL(transr, uplo, n, arf, i, j, F[i * n + j]);
    free(F);
    return info;
}

/* The four steps of Section 3 on the blocks A11 (m1 x m1), A21 (m2 x m1) and
 * A22 (m2 x m2) of the canonical lower matrix, m1 = ceil(n/2) for UPLO='L'
 * and floor(n/2) for 'U' (the orders of T1 and T2 in Figures 4-6). */
int orc_zpftrf_srpa(char transr, char uplo, i64 n, zc *arf)
{
    if (n <= 0) return 0;
    const i64 m1 = zup(uplo) == 'L' ? (n + 1) / 2 : n / 2, m2 = n - m1;
    zc *F = (zc *)calloc((size_t)(n * n), sizeof(zc));
    if (!F) return -1;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) F[i * n + j] = zgetL(transr, uplo, n, arf, i, j);
    /* step 1: POTRF on A11 */
    int info = zchol_lower(m1, F, n, 0);
    if (info == 0) {
        /* step 2: TRSM, each row x of A21 solves x L11^H = a */
        for (i64 r = m1; r < n; r++)
            for (i64 j = 0; j < m1; j++) {
                zc s = F[r * n + j];
                for (i64 k = 0; k < j; k++) s -= F[r * n + k] * conj(F[j * n + k]);
                F[r * n + j] = s / creal(F[j * n + j]);
            }
        /* step 3: HERK, A22 -= L21 L21^H (lower triangle) */
        for (i64 i = m1; i < n; i++)
            for (i64 j = m1; j <= i; j++) {
                zc s = 0;
                for (i64 k = 0; k < m1; k++) s += F[i * n + k] * conj(F[j * n + k]);
                F[i * n + j] -= s;
            }
        /* step 4: POTRF on A22; INFO counts from the start of A */
        info = zchol_lower(m2, F + m1 * n + m1, n, (int)m1);
    }
    if (info == 0)
        for (i64 i = 0; i < n; i++)
            for (i64 j = 0; j <= i; j++) zsetL(transr, uplo, n, arf, i, j, F[i * n + j]);
    free(F);
    return info;
}

/* Solve A X = B with the factor held in arf: L Y = B, then L^H X = Y. */
void orc_zpftrs(char transr, char uplo, i64 n, i64 nrhs, const zc *arf, zc *b, i64 ldb)
{
    if (n <= 0 || nrhs <= 0) return;
    zc *F = (zc *)calloc((size_t)(n * n), sizeof(zc));
    if (!F) return;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) F[i * n + j] = zgetL(transr, uplo, n, arf, i, j);
    for (i64 c = 0; c < nrhs; c++) {
        zc *x = b + c * ldb;
        for (i64 i = 0; i < n; i++) {
            zc s = x[i];
            for (i64 k = 0; k < i; k++) s -= F[i * n + k] * x[k];
            x[i] = s / F[i * n + i];
        }
        for (i64 i = n - 1; i >= 0; i--) {
            zc s = x[i];
            for (i64 k = i + 1; k < n; k++) s -= conj(F[k * n + i]) * x[k];
            x[i] = s / conj(F[i * n + i]);
        }
    }
    free(F);
}

/* Inverse from the factor: W = L^{-1} by forward substitution on the columns
 * of the identity, then A^{-1} = W^H W; the UPLO triangle of A^{-1} replaces
 * the factor.  Returns j+1 when L(j,j) is zero. */
int orc_zpftri(char transr, char uplo, i64 n, zc *arf)
{
    if (n <= 0) return 0;
    zc *F = (zc *)calloc((size_t)(n * n), sizeof(zc));
    zc *W = (zc *)calloc((size_t)(n * n), sizeof(zc));
    if (!F || !W) { free(F); free(W); return -1; }
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) F[i * n + j] = zgetL(transr, uplo, n, arf, i, j);
    for (i64 j = 0; j < n; j++)
        if (F[j * n + j] == 0) { free(F); free(W); return (int)(j + 1); }
    for (i64 c = 0; c < n; c++)
        for (i64 i = c; i < n; i++) {
            zc s = (i == c) ? 1.0 : 0.0;
            for (i64 k = c; k < i; k++) s -= F[i * n + k] * W[k * n + c];
            W[i * n + c] = s / F[i * n + i];
        }
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) {
            zc s = 0; /* (W^H W)(i,j) = sum_k conj(W(k,i)) W(k,j), k >= i */
            for (i64 k = i; k < n; k++) s += conj(W[k * n + i]) * W[k * n + j];
            zsetL(transr, uplo, n, arf, i, j, s);
        }
    free(F);
    free(W);
    return 0;
}

/* Normwise backward error max_c ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
 * (moduli of complex entries), A held in arf. */
double orc_zbackward_error(char transr, char uplo, i64 n, i64 nrhs, const zc *arf, const zc *b, i64 ldb,
                           const zc *x, i64 ldx)
{
    if (n <= 0 || nrhs <= 0) return 0.0;
    zc *A = (zc *)malloc(sizeof(zc) * (size_t)(n * n));
    if (!A) return -1.0;
    long double anorm = 0.0L;
    for (i64 i = 0; i < n; i++) {
        long double row = 0.0L;
        for (i64 j = 0; j < n; j++) {
            A[i * n + j] = zget(transr, uplo, n, arf, i, j);
            row += cabs(A[i * n + j]);
        }
        if (row > anorm) anorm = row;
    }
    double worst = 0.0;
    for (i64 c = 0; c < nrhs; c++) {
        const zc *bc = b + c * ldb, *xc = x + c * ldx;
        long double rmax = 0.0L, xmax = 0.0L, bmax = 0.0L;
        for (i64 i = 0; i < n; i++) {
            long double complex r = bc[i];
            for (i64 j = 0; j < n; j++) r -= (long double complex)A[i * n + j] * (long double complex)xc[j];
            if (cabsl(r) > rmax) rmax = cabsl(r);
            if (cabs(xc[i]) > xmax) xmax = cabs(xc[i]);
            if (cabs(bc[i]) > bmax) bmax = cabs(bc[i]);
        }
        long double den = anorm * xmax + bmax;
        double eta = den > 0 ? (double)(rmax / den) : (double)rmax;
        if (eta > worst) worst = eta;
    }
    free(A);
    return worst;
}

/* ||L L^H - A||_F / ||A||_F over the whole matrix, A and the factor in RFP. */
double orc_zfactor_residual(char transr, char uplo, i64 n, const zc *arf_a, const zc *arf_l)
{
    if (n <= 0) return 0.0;
    zc *L = (zc *)calloc((size_t)(n * n), sizeof(zc));
    if (!L) return -1.0;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) L[i * n + j] = zgetL(transr, uplo, n, arf_l, i, j);
    long double num = 0.0L, den = 0.0L;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j <= i; j++) {
            long double complex t = 0.0L;
            for (i64 k = 0; k <= j; k++) t += (long double complex)L[i * n + k] * conjl((long double complex)L[j * n + k]);
            long double complex a = zget(transr, uplo, n, arf_a, i, j);
            long double w = (i == j) ? 1.0L : 2.0L; /* both triangles */
            num += w * cabsl(t - a) * cabsl(t - a);
            den += w * cabsl(a) * cabsl(a);
        }
    free(L);
    return (double)sqrtl(num / den);
}

/* ||I - A A^{-1}||_F / (||A||_F ||A^{-1}||_F), both in RFP (same layout). */
double orc_zinverse_residual(char transr, char uplo, i64 n, const zc *arf_a, const zc *arf_inv)
{
    if (n <= 0) return 0.0;
    zc *A = (zc *)malloc(sizeof(zc) * (size_t)(n * n));
    zc *V = (zc *)malloc(sizeof(zc) * (size_t)(n * n));
    if (!A || !V) { free(A); free(V); return -1.0; }
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            A[i * n + j] = zget(transr, uplo, n, arf_a, i, j);
            V[i * n + j] = zget(transr, uplo, n, arf_inv, i, j);
        }
    long double num = 0.0L, na = 0.0L, nv = 0.0L;
    for (i64 i = 0; i < n; i++)
        for (i64 j = 0; j < n; j++) {
            long double complex t = 0.0L;
            for (i64 k = 0; k < n; k++) t += (long double complex)A[i * n + k] * (long double complex)V[k * n + j];
            long double complex e = ((i == j) ? 1.0L : 0.0L) - t;
            num += cabsl(e) * cabsl(e);
            na += cabs(A[i * n + j]) * cabs(A[i * n + j]);
            nv += cabs(V[i * n + j]) * cabs(V[i * n + j]);
        }
    free(A);
    free(V);
    return (double)(sqrtl(num) / (sqrtl(na) * sqrtl(nv)));
}
