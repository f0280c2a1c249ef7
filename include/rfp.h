/*
 * rfp.h -- C ABI of the MI355X (gfx950) library for Cholesky factorization,
 * solution and inversion of a symmetric positive definite matrix held in
 * Rectangular Full Packed Format (Gustavson, Wasniewski, Dongarra, Langou,
 * "Rectangular Full Packed Format for Cholesky's Algorithm: Factorization,
 * Solution and Inversion").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - RFP array (arf): n(n+1)/2 entries, device memory, in one of the eight
 *    layouts selected by TRANSR ('N' or 'T') and UPLO ('L' or 'U'), exactly
 *    as defined in Section 2 and drawn in Figures 4-6 (the parity of n is the
 *    third selector).  Characters are case-insensitive.
 *  - Full matrices and right-hand sides are column-major device arrays with a
 *    leading dimension (lda, ldb >= max(1, n)).
 *  - All sizes are int64_t.  n = 0 (or nrhs = 0) returns 0 immediately.
 *  - Ownership: the caller allocates and owns every array.  The handle owns
 *    only scratch memory (leaf inverses, split-K partial sums, low-precision
 *    copies), grown on demand; a grow waits for the device to go idle.
 *  - Streams: work is enqueued on `stream` (NULL = the default stream) and the
 *    call returns without waiting, except where a routine says otherwise.
 *    One handle must not be used by two streams or threads at once.
 *  - Return value: 0 on success; -i when argument i (counted in the paper's
 *    argument order for that routine, given with each routine) is illegal,
 *    in which case nothing is enqueued; RFP_ERR_HANDLE for a bad handle;
 *    RFP_ERR_RUNTIME when the HIP runtime reports an error.
 *  - Numerical status (INFO) is written to a device int so that no call has
 *    to synchronise; read it after the stream has finished.
 */
#ifndef RFP_MI355X_H
#define RFP_MI355X_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RFP_ERR_HANDLE (-101)
#define RFP_ERR_RUNTIME (-102)
#define RFP_ERR_SCRATCH (-103) /* rfp_dpftrs_noalloc: the problem exceeds its fixed scratch */

typedef struct rfp_context* rfp_handle_t;

/* Create a handle bound to HIP device `device` (scratch memory is allocated
 * lazily on that device).  Returns 0, -1 (h is NULL), -2 (bad device) or
 * RFP_ERR_RUNTIME. */
int rfp_create(rfp_handle_t* h, int device);

/* Release the handle and its scratch memory (waits for the device). */
int rfp_destroy(rfp_handle_t h);

/* TRTTF (the paper's table of LAPACK 3.2 RFP routines, "Conv. from TR to
 * TF"): copy the UPLO triangle of the full n x n matrix a (column-major,
 * lda >= max(1,n)) into the RFP array arf of layout (transr, uplo).  The other
 * triangle of a is not read.  Argument order: TRANSR=1, UPLO=2, N=3, A=4,
 * LDA=5, ARF=6. */
int rfp_dtrttf(rfp_handle_t h, char transr, char uplo, int64_t n, const double* a, int64_t lda, double* arf,
               hipStream_t stream);

/* TFTTR ("Conv. from TF to TR"): copy the RFP array into the UPLO triangle of
 * the full matrix a; the other triangle of a is left untouched.  Argument
 * order: TRANSR=1, UPLO=2, N=3, ARF=4, A=5, LDA=6. */
int rfp_dtfttr(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, double* a, int64_t lda,
               hipStream_t stream);

/* PFTRF (Section 3, Figure 4 "Cholesky Factorization Algorithm"): A = L L^T
 * (UPLO='L') or A = U^T U (UPLO='U'); the factor overwrites arf in the same
 * layout.  *info (device int) becomes 0 on success or p > 0 when the leading
 * minor of order p (in the order of A) is not positive definite; the
 * factorization then stops and arf is partly overwritten.  Argument order:
 * TRANSR=1, UPLO=2, N=3, A=4, INFO=5. */
int rfp_dpftrf(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream);

/* PFTRS (Section 4, Figure 4 "Cholesky Solution Algorithm"): solve A X = B
 * with the PFTRF factor in arf; X overwrites b (n x nrhs, column-major,
 * ldb >= max(1,n)).  arf is only read.  Argument order: TRANSR=1, UPLO=2,
 * N=3, NR=4, A=5, B=6, LDB=7. */
int rfp_dpftrs(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf, double* b,
               int64_t ldb, hipStream_t stream);

/* PFTRI (Section 5, Figure 4 "Cholesky Inversion Algorithm"): from the PFTRF
 * factor, overwrite arf with the same triangle of A^{-1} in the same layout
 * (W = L^{-1} by TRTRI/TRMM on the three blocks, then W^T W by LAUUM, SYRK and
 * TRMM).  *info (device int) becomes 0, or i > 0 when the factor's diagonal
 * entry i is exactly zero.  Argument order: TRANSR=1, UPLO=2, N=3, A=4,
 * INFO=5. */
int rfp_dpftri(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Complex Hermitian positive definite matrices (the Hermitian case of
 * Sections 3-5 and the complex rows of the routine table: ZPFTRF, ZPFTRS,
 * ZPFTRI; A = L L^H or U^H U).
 *  - Complex arrays are interleaved (re, im) pairs of doubles: element k
 *    of a complex array p is (p[2k], p[2k+1]); leading dimensions and sizes
 *    count complex elements.  A torch.complex128 tensor has this layout.
 *  - TRANSR is 'N' or 'C'.  The RFP array has the positions of the real
 *    format of the same layout (TRANSR 'C' where the real one has 'T');
 *    every part that the real format keeps transposed is kept conjugate-
 *    transposed here (the paper's convention for the complex case).
 *  - Scratch comes from the handle: leaf inverses of the 64-row diagonal
 *    blocks plus 64 x max(n, nrhs) complex temporaries.
 * --------------------------------------------------------------------- */

/* ZTRTTF: the UPLO triangle of the full Hermitian matrix a (column-major,
 * lda >= max(1,n)) into the RFP array arf.  Argument order: TRANSR=1,
 * UPLO=2, N=3, A=4, LDA=5, ARF=6. */
int rfp_ztrttf(rfp_handle_t h, char transr, char uplo, int64_t n, const double* a, int64_t lda, double* arf,
               hipStream_t stream);

/* ZTFTTR: the RFP array into the UPLO triangle of a (the other triangle is
 * left untouched).  Argument order: TRANSR=1, UPLO=2, N=3, ARF=4, A=5,
 * LDA=6. */
int rfp_ztfttr(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, double* a, int64_t lda,
               hipStream_t stream);

/* ZPFTRF (Section 3, Hermitian case): A = L L^H (UPLO='L') or U^H U ('U')
 * by the four steps on the blocks of the rectangle (POTRF on T1, TRSM
 * S <- S L11^{-H}, HERK T2 <- T2 - S S^H, POTRF on T2).  *info (device int)
 * becomes 0, or p > 0 when the leading minor of order p is not positive
 * definite (the factorization then stops; arf is partly overwritten).
 * Argument order: TRANSR=1, UPLO=2, N=3, A=4, INFO=5. */
int rfp_zpftrf(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream);

/* ZPFTRS (Section 4, Hermitian case): solve A X = B with the ZPFTRF factor
 * (L Y = B, then L^H X = Y); X overwrites b (n x nrhs complex, column-major,
 * ldb >= max(1,n)).  Argument order: TRANSR=1, UPLO=2, N=3, NR=4, A=5, B=6,
 * LDB=7. */
int rfp_zpftrs(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf, double* b,
               int64_t ldb, hipStream_t stream);

/* ZPFTRI (Section 5, Hermitian case): from the ZPFTRF factor, the same
 * triangle of A^{-1} = W^H W, W = L^{-1}, overwrites arf.  *info (device
 * int) becomes 0, or i > 0 when the factor's diagonal entry i is zero.
 * Argument order: TRANSR=1, UPLO=2, N=3, A=4, INFO=5. */
int rfp_zpftri(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream);

/* TFTRI (the paper's routine table, "Triangular inversion"): the inverse of
 * the triangular matrix T held in arf (UPLO='L' lower, 'U' upper) overwrites
 * it in the same layout, by the inversion stage of PFTRI (Section 5, Figure 4
 * "Cholesky Inversion Algorithm" steps 1-4).  DIAG='U': T has a unit diagonal;
 * the stored diagonal is not used and is left as it was.  *info (device int)
 * becomes 0, or i > 0 when T(i,i) is exactly zero (DIAG='N').  Argument order:
 * TRANSR=1, UPLO=2, DIAG=3, N=4, A=5, INFO=6. */
int rfp_dtftri(rfp_handle_t h, char transr, char uplo, char diag, int64_t n, double* arf, int* info,
               hipStream_t stream);

/* TFSM (the paper's routine table, "Triangular solve"; Section 4 uses it as
 * POTRS uses TRSM): B (m x n, column-major, ldb >= max(1,m)) is overwritten by
 *   SIDE='L': X with op(A) X = alpha B (A of order m);
 *   SIDE='R': X with X op(A) = alpha B (A of order n);
 * op(A) = A (TRANS='N') or A^T ('T'); A triangular in arf (UPLO, DIAG as for
 * rfp_dtftri).  alpha = 0 sets B to zero and does not read A.  Argument
 * order: TRANSR=1, SIDE=2, UPLO=3, TRANS=4, DIAG=5, M=6, N=7, ALPHA=8, A=9,
 * B=10, LDB=11. */
int rfp_dtfsm(rfp_handle_t h, char transr, char side, char uplo, char trans, char diag, int64_t m, int64_t n,
              double alpha, const double* arf, double* b, int64_t ldb, hipStream_t stream);

/* SFRK (the paper's routine table, "Sym rank-k update"): C = alpha op(A)
 * op(A)^T + beta C for the symmetric C of order n held in c (RFP), with
 * op(A) = A (TRANS='N', A n x k) or A^T (TRANS='T', A k x n), A column-major
 * with leading dimension lda (>= max(1, n) for 'N', >= max(1, k) for 'T').
 * alpha = 0 or k = 0 does not read A; beta = 0 does not read C.  Argument
 * order: TRANSR=1, UPLO=2, TRANS=3, N=4, K=5, ALPHA=6, A=7, LDA=8, BETA=9,
 * C=10. */
int rfp_dsfrk(rfp_handle_t h, char transr, char uplo, char trans, int64_t n, int64_t k, double alpha,
              const double* a, int64_t lda, double beta, double* c, hipStream_t stream);

/* TPTTF / TFTTP (the paper's routine table, "Conv. from TP to TF" and back):
 * the standard packed array ap (n(n+1)/2 entries, Figure 2: the UPLO
 * triangle column by column) to the RFP array arf of layout (TRANSR, UPLO),
 * and back.  Argument order: TRANSR=1, UPLO=2, N=3, AP=4, ARF=5 (TPTTF);
 * TRANSR=1, UPLO=2, N=3, ARF=4, AP=5 (TFTTP). */
int rfp_dtpttf(rfp_handle_t h, char transr, char uplo, int64_t n, const double* ap, double* arf, hipStream_t stream);
int rfp_dtfttp(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, double* ap, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): PFTRS
 * exactly as rfp_dpftrs (same arguments and argument codes, same kernels,
 * bit-identical results), without a handle.  Its scratch -- the inverses of
 * the factor's 64-row diagonal blocks, the fused solves' ready flags and
 * control words -- lives in a fixed 32 MiB device array of the library, one
 * copy per GPU held until the process ends; the call allocates and frees
 * nothing.  Limits: ceil(m1/64) + ceil(m2/64) <= 991 diagonal blocks (n up to
 * about 63000) and (that count) x ceil(nrhs/16) <= 262144 ready flags;
 * beyond them it returns RFP_ERR_SCRATCH and enqueues nothing.  Runs on the
 * current device and `stream`.  All calls on one GPU share its scratch, so
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must not be issued; consecutive calls on one stream are safe.  The
 * scratch keeps the last call's contents; the ready flags are told apart by
 * an epoch kept in the scratch, so nothing needs clearing between calls.
 * Argument order: TRANSR=1, UPLO=2, N=3, NR=4, A=5, B=6, LDB=7. */
int rfp_dpftrs_noalloc(char transr, char uplo, int64_t n, int64_t nrhs, const double* arf, double* b, int64_t ldb,
                       hipStream_t stream);

/* Single-precision counterparts (SPFTRF / SPFTRS / STRTTF / STFTTR in the
 * paper's routine table); same arguments and semantics with float arrays. */
int rfp_strttf(rfp_handle_t h, char transr, char uplo, int64_t n, const float* a, int64_t lda, float* arf,
               hipStream_t stream);
int rfp_stfttr(rfp_handle_t h, char transr, char uplo, int64_t n, const float* arf, float* a, int64_t lda,
               hipStream_t stream);
int rfp_spftrf(rfp_handle_t h, char transr, char uplo, int64_t n, float* arf, int* info, hipStream_t stream);
int rfp_spftrs(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, const float* arf, float* b,
               int64_t ldb, hipStream_t stream);
int rfp_spftri(rfp_handle_t h, char transr, char uplo, int64_t n, float* arf, int* info, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Mixed precision with iterative refinement (not in the paper: the FP32
 * counterparts above are the paper's; the refinement follows the classical
 * mixed-precision iterative refinement of a Cholesky solve, as in LAPACK's
 * DSPOSV, over the RFP format).
 */
enum { RFP_PREC_FP32 = 0, RFP_PREC_FP16 = 1, RFP_PREC_BF16 = 2, RFP_PREC_FP64 = 3 };

/* PFTRF on an FP32 RFP array with the bulk trailing updates (the GEMM, SYRK
 * and TRSM-update products of every step, not the diagonal-block leaves and
 * their in-place panel products) computed with operands rounded to fprec:
 * RFP_PREC_FP32 (same as rfp_spftrf), RFP_PREC_FP16 or RFP_PREC_BF16, with
 * FP32 accumulation on the matrix cores.  Argument order: FPREC=1, TRANSR=2,
 * UPLO=3, N=4, A=5, INFO=6. */
int rfp_spftrf_mp(rfp_handle_t h, int fprec, char transr, char uplo, int64_t n, float* arf, int* info,
                  hipStream_t stream);

/* Scaled cast: s[i] = 1/sqrt(a_ii) when scale != 0 (else 1), and
 * arf32 = (float)(((a_ij * s_i) * s_j) * mu) on every stored off-diagonal
 * entry, (float)((((a_ii * s_i) * s_i) + shift) * mu) on the diagonal, in the
 * same RFP layout (so diag(s) A diag(s) has a unit diagonal before the shift
 * and mu).  Each operation is rounded in FP64 in that order, then the result
 * once to FP32.  A diagonal entry that is not positive gives s_i = NaN.  s is
 * a device array of n doubles.  Argument order: TRANSR=1, UPLO=2, N=3,
 * ARF=4, SCALE=5, MU=6 (positive, finite), SHIFT=7 (>= 0, finite), S=8,
 * ARF32=9. */
int rfp_dpfcast_s(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, int scale, double mu,
                  double shift, double* s, float* arf32, hipStream_t stream);

/* Diagonal shift of the low-precision factors of rfp_dpfsv_ir and
 * rfp_pfsv_vbatched (not in the paper; the shift of Higham and Pranesh's
 * low-precision Cholesky, SIAM J. Sci. Comput. 43 (2021)): they factor
 * mu (D^{-1/2} A D^{-1/2} + c u I), u the unit roundoff of the factor's
 * precision (2^-24 FP32, 2^-11 FP16, 2^-8 BF16), so that the factor's
 * rounding cannot make an ill-conditioned matrix lose positive
 * definiteness; refinement against the unshifted FP64 matrix removes the
 * shift from the solution.  One c per precision FPREC (RFP_PREC_FP32,
 * RFP_PREC_FP16 or RFP_PREC_BF16), c >= 0 (0: no shift; defaults 64 for
 * FP32, 4 for FP16 and BF16).  Argument order: FPREC=2, C=3. */
int rfp_set_lowp_shift(rfp_handle_t h, int fprec, double c);
int rfp_get_lowp_shift(rfp_handle_t h, int fprec, double* c);

/* LANSF (the paper's routine table, "Norm"): *out (device double) = the norm
 * of the symmetric matrix held in arf: 'M' max |a_ij|, '1', 'O' or 'I' the
 * one-norm (= infinity-norm), 'F' or 'E' Frobenius.  The one-norm and
 * Frobenius sums are accumulated with atomics (order not fixed).  Argument
 * order: NORM=1, TRANSR=2, UPLO=3, N=4, A=5, OUT=6. */
int rfp_dlansf(rfp_handle_t h, char norm, char transr, char uplo, int64_t n, const double* arf, double* out,
               hipStream_t stream);

/* Symmetric product with a thin matrix (not in the paper's routine table;
 * the residual and conjugate-gradient product of rfp_dpfsv_ir):
 * Y = alpha A X + beta Y for the symmetric A of order n held in arf (RFP,
 * only the stored triangle is read, each entry once), X and Y n x nrhs
 * column-major (ldx, ldy >= max(1, n)); Y must not overlap X.  beta = 0 does
 * not read Y.  The summation order is fixed, so the result is the same on
 * every call.  Uses handle scratch (about 3 (n/256) n 16 doubles).  Argument
 * order: TRANSR=1, UPLO=2, N=3, NRHS=4, ALPHA=5, A=6, X=7, LDX=8, BETA=9,
 * Y=10, LDY=11. */
int rfp_dsfmv(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, double alpha, const double* arf,
              const double* x, int64_t ldx, double beta, double* y, int64_t ldy, hipStream_t stream);

/* Solve A X = B for the FP64 SPD matrix in arf (left untouched) by a
 * low-precision Cholesky factor and FP64 iterative refinement:
 *   As = mu (D^{-1/2} A D^{-1/2} + c u I) rounded to FP32 (rfp_dpfcast_s
 *   with scale = 1 and the shift c u of rfp_set_lowp_shift; mu = 2^25 for
 *   FPREC = RFP_PREC_FP16, so that the factor's entries and those of its
 *   diagonal blocks' inverses both stay in the FP16 range, else 1);
 *   Ls = PFTRF(As) with the bulk
 *   updates in precision fprec (as rfp_spftrf_mp); the preconditioner is
 *   M^{-1} = mu D^{-1/2} (Ls Ls^T)^{-1} D^{-1/2} (solves in FP32).
 *   X = 0, R = B; each sweep corrects X from R in FP64, then R = B - A X
 *   (FP64, from arf), until the normwise backward error
 *   max_c ||R_c||_inf / (||A||_inf ||X_c||_inf + ||B_c||_inf) is <= tol.
 *   A sweep is X += M^{-1} R (classical refinement) until one fails to cut
 *   the backward error fourfold; later sweeps run 8 steps of conjugate
 *   gradients on A X = B preconditioned by M^{-1}, in FP64, one recurrence
 *   continued from sweep to sweep and restarted from the true residual R at
 *   each sweep (refinement with a CG inner solver; M^{-1} is then applied in
 *   FP64 arithmetic from an FP64 copy of Ls, so that it is symmetric to FP64
 *   rounding), which converges where kappa(A) u_low is not small.
 * Falls back to the FP64 PFTRF + PFTRS on a copy of A when the scaled copy
 * is not finite, when the low-precision factor is not positive definite,
 * when 3 conjugate-gradient sweeps in a row fail to bring the backward error
 * below 0.9 times its best value (conjugate gradients minimise the error's
 * A-norm, so the residual need not fall every sweep), or after max_iter
 * sweeps.
 * Every decision is taken on the device: the call enqueues the setup,
 * max_iter sweeps and the fall-back without waiting, and what is not needed
 * exits at once.  It never synchronises; once the handle's workspace has been
 * sized by an earlier call of the same n and nrhs, it allocates nothing and
 * can be captured in a HIP graph (a later call that grows the workspace
 * invalidates graphs captured before it).
 * Device outputs (ints): *iter = number of sweeps when refinement converged,
 * or the fall-back reason: -1 max_iter reached, -2 stalled, -3 low-precision
 * factor not positive definite, -4 the scaled low-precision copy of A is not
 * finite (a diagonal entry <= 0, or an entry out of range); *info = the FP64
 * PFTRF INFO of a fall-back (0 otherwise).  X (n x nrhs, ldx) receives the
 * solution; b is only read.  Argument order: FPREC=1, TRANSR=2, UPLO=3, N=4,
 * NRHS=5, A=6, B=7, LDB=8, X=9, LDX=10, TOL=11 (positive), MAX_ITER=12
 * (>= 1), ITER=13, INFO=14. */
int rfp_dpfsv_ir(rfp_handle_t h, int fprec, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf,
                 const double* b, int64_t ldb, double* x, int64_t ldx, double tol, int max_iter, int* iter, int* info,
                 hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched systems (not in the paper): many SPD systems of uneven order, each
 * in its own RFP layout, in one persistent launch.  Each system goes through
 * the paper's factorization (Section 3), solution (Section 4) and, if
 * asked, inversion (Section 5).  A system of order n <= 256 is one task of
 * one workgroup; a larger one is cut into 128-row tiles whose factorization,
 * refinement and inversion steps run as tasks on many workgroups at once.
 */
typedef struct {
    int64_t n;       /* order, n >= 0 */
    int64_t arf_off; /* element offset of the system's RFP array in arf_pool */
    int64_t b_off;   /* element offset of its first right-hand side in b_pool */
    int64_t ldb;     /* leading dimension of its right-hand sides (>= max(1, n)) */
    int64_t nrhs;    /* number of right-hand sides (>= 0) */
    char transr, uplo;
    char pad[6];
} rfp_sys_t;

/* Solve every system of the batch.  sys (device, batch entries) describes
 * the systems; sys_host is the same table in host memory, read to size the
 * handle's workspace for the systems with n > 256 (NULL: such systems are
 * refused with info[i] = -1); arf_pool and b_pool (device) hold the RFP
 * arrays and right-hand sides, which X overwrites.  fprec:
 *   RFP_PREC_FP64: PFTRF in place, then PFTRS (the factor stays in arf);
 *   RFP_PREC_FP32, RFP_PREC_FP16, RFP_PREC_BF16: low-precision factor of
 *     mu (D^{-1/2} A D^{-1/2} + c u I) (D = diag(A); mu = 2^25 for FP16,
 *     else 1; c u as in rfp_set_lowp_shift) with
 *     its bulk updates on operands rounded to fprec (FP32 accumulation), and
 *     FP64 refinement against the untouched FP64 matrix until the normwise
 *     backward error is <= tol, with sweeps as in rfp_dpfsv_ir (classical,
 *     then sweeps of up to 8 preconditioned conjugate-gradient steps in FP64
 *     once a sweep fails to cut the backward error fourfold; stalled after 3
 *     such sweeps in a row that do not bring it below 0.9 times its best
 *     value; at most max_iter sweeps); on failure the FP64 factor and solve
 *     run on arf.
 * With do_pftri != 0, arf ends as the RFP array of A^{-1} (PFTRI after an
 * FP64 factor, in every mode).  Device outputs per system: info[i] = 0 or the
 * FP64 PFTRF INFO (first non-positive pivot, 1-based), -1 for a refused
 * system (bad layout character or ldb, nrhs < 0, or n > 256 without sys_host),
 * which is not touched; iter[i] = 0 (FP64 mode), the number of refinement
 * sweeps, or the reason the FP64 path was taken: -1 max_iter, -2 stalled,
 * -3 low-precision factor not positive definite, -4 scaled copy not finite.
 * No host synchronisation, and no allocation once the handle's workspace has
 * been sized by an earlier call on the same systems, so the call can be
 * captured in a HIP graph.  A later call on the same handle that needs a
 * larger workspace (more systems, or larger ones) replaces it, and a graph
 * captured before then replays into freed memory: capture after the largest
 * call, or give graphs a handle of their own.  Argument order: FPREC=1, BATCH=2, SYS=3,
 * SYS_HOST=4, ARF_POOL=5, B_POOL=6, DO_PFTRI=7, TOL=8, MAX_ITER=9, INFO=10,
 * ITER=11. */
int rfp_pfsv_vbatched(rfp_handle_t h, int fprec, int64_t batch, const rfp_sys_t* sys, const rfp_sys_t* sys_host,
                      double* arf_pool, double* b_pool, int do_pftri, double tol, int max_iter, int* info, int* iter,
                      hipStream_t stream);

/* ------------------------------------------------------------------------
 * Autotuner (not in the paper).  The handle can hold a table of kernel
 * configurations, keyed by shape class (sizes rounded up to powers of two,
 * operand orientation, precision): the GEMM tile (128x128, 64x128, 128x64,
 * 64x64) with its split-K factor, and the right-hand-side slice width of the
 * fused solve.  Without a table the library uses its built-in rules.  Every
 * configuration computes the same result; only speed differs.
 */
enum { RFP_TUNE_FP64 = 1, RFP_TUNE_FP32 = 2, RFP_TUNE_FP16 = 4, RFP_TUNE_BF16 = 8, RFP_TUNE_SCHEDULE = 16 };

/* Time every admissible configuration for the GEMM shapes that PFTRF (and,
 * for FP64, PFTRI) of order n produce in the precisions `precs` (RFP_TUNE_*
 * bits), and the solve's slice widths for nrhs right-hand sides (FP64; nrhs
 * = 0 skips it), on scratch operands on this handle's device; keep the
 * fastest.  With RFP_TUNE_SCHEDULE, also time the FP64 PFTRF of order n
 * under a grid of factorization schedules (256-column panel threshold 3072,
 * 6144, 12288 or never; chunk width 1024, 1536 or 2048; leaf LDS reservation
 * 0 or 24 KB) and keep the fastest for n's size class (sizes rounded up to a
 * power of two); factorizations of that class then use it unless the caller
 * has set a schedule with rfp_set_schedule.  Synchronises the stream; allocates scratch.  Argument order: N=1,
 * NRHS=2, PRECS=3. */
int rfp_autotune(rfp_handle_t h, int64_t n, int64_t nrhs, int precs, hipStream_t stream);
/* Number of tuned entries; drop the table; force one GEMM configuration for
 * every non-tuned shape (tile -1 switches forcing off; split 0 = built-in
 * split-K rule, 1 = none, s = s-way) -- a testing aid. */
int rfp_tune_count(rfp_handle_t h);
int rfp_tune_clear(rfp_handle_t h);
int rfp_tune_force(rfp_handle_t h, int tile, int split);
/* Write / read the table as JSON text (one entry per line).  Load replaces
 * the table; returns -1 when the file cannot be opened, -2 when it is not a
 * table written by rfp_tune_save. */
int rfp_tune_save(rfp_handle_t h, const char* path);
int rfp_tune_load(rfp_handle_t h, const char* path);

/* Fused-solve status (PFTRS and every solve inside the refinement and the
 * FP64 fall-back).  The triangular solves pass solved rows between
 * workgroups through flags; each wait for a flag is bounded (default 2^24
 * polls).  A wait that runs out writes NaN into its block of the solution
 * and sets bit 0 of the handle's device status word.  rfp_solve_status
 * enqueues, on `stream`, a copy of that word into *status (device int) and
 * clears it, so it reports every give-up since the previous call.
 * rfp_set_solve_wait_limit sets the number of polls (0 = give up at the
 * first poll that finds nothing new: a testing aid that makes every kernel
 * still end normally); polls < 0 restores the default.  Argument order:
 * H=1, STATUS=2 / POLLS=2. */
int rfp_solve_status(rfp_handle_t h, int* status, hipStream_t stream);
int rfp_set_solve_wait_limit(rfp_handle_t h, int64_t polls);

/* ------------------------------------------------------------------------
 * Factorization schedule (not in the paper: the paper's four steps run one
 * after the other; here they are overlapped on three streams).  These knobs
 * change only the order and grouping of the same block operations of
 * Section 3 (the 2 x 2 partition of Figure 3 applied to panels of the two
 * diagonal triangles), never the arithmetic each block does, so every
 * setting computes the same factor up to rounding.
 *   wide_panels_above: a diagonal triangle's panels are wide_panel_cols
 *     columns wide while its trailing order exceeds this value, 128 wide
 *     after (default 6144; 0 = always wide; a value >= n = always 128 wide).
 *   chunk_max: the off-diagonal solve (step 2) and its share of step 3 run
 *     by chunks of at most this many columns on a third stream, overlapped
 *     with step 1 (default 1536; at least 512 is used; 0 disables the
 *     overlap, so steps 2 and 3 follow step 1).
 *   lookahead_wait_below: trailing order up to which each bulk trailing
 *     update waits for the critical stream's lookahead product (default
 *     INT64_MAX: always; 0: never).
 *   leaf_lds_pad: bytes of LDS the FP64 128-row diagonal leaf reserves
 *     beyond what it uses, to keep large GEMM workgroups off its compute unit
 *     (default 24576; 0 to 65536).
 *   wide_panel_cols: width of the wide panels, a multiple of 128 (default
 *     256; FP16 and BF16-operand factorizations use 1024 unless a schedule
 *     was set or tuned).  A wide panel's diagonal block is factored by the 2 x 2 partition
 *     down to 128-row leaves; a width at least the triangle's order factors
 *     the whole triangle that way (a fully recursive factorization, whose
 *     trailing updates have the largest inner dimensions and so the least
 *     traffic per flop).
 * rfp_set_schedule(h, NULL) restores the defaults; illegal values return
 * -2 (a field < 0, leaf_lds_pad > 65536, or wide_panel_cols not a positive
 * multiple of 128) and leave the schedule as it was.  The schedule is host state of the handle; calls already enqueued are
 * not affected.  Argument order: H=1, SCHED=2. */
typedef struct {
    int64_t wide_panels_above;
    int64_t chunk_max;
    int64_t lookahead_wait_below;
    int64_t leaf_lds_pad;
    int64_t wide_panel_cols;
} rfp_schedule_t;
int rfp_set_schedule(rfp_handle_t h, const rfp_schedule_t* sched);
int rfp_get_schedule(rfp_handle_t h, rfp_schedule_t* sched);

/* ------------------------------------------------------------------------
 * Kernel timing (introspection, used by the benchmark for its roofline).
 * While enabled, every kernel the handle's calls launch is bracketed by a pair
 * of HIP events on the call's stream.  Enabling creates a pool of 32768 event
 * pairs up front; only when a region launches more kernels than that does a
 * launch wait for the device to fold the finished pairs.  rfp_profile_read
 * waits for the device,
 * folds the finished pairs into one entry per kernel (the kernel's demangled
 * name as rocprofv3 prints it: launches, summed event time, summed
 * algorithmic flops and bytes of those launches), and resets the totals
 * once every entry fits in out (so a first call with cap = 0 only sizes).
 * *count receives the number of kernels (even beyond cap).  Returns 0,
 * RFP_ERR_HANDLE, -4 for bad output arguments or RFP_ERR_RUNTIME. */
typedef struct {
    char name[160];
    int64_t launches;
    double total_ms, flops, bytes;
} rfp_profile_entry;
int rfp_profile_enable(rfp_handle_t h, int on);
int rfp_profile_read(rfp_handle_t h, rfp_profile_entry* out, int cap, int* count);

/* ------------------------------------------------------------------------
 * Plan introspection (host only, touches no device).
 * The drivers are the paper's 2 x 2 block algorithms (Figure 3, Sections 3-5)
 * applied recursively; rfp_plan records the sequence of primitives that
 * rfp_dpftrf ('F'), rfp_dpftrs ('S') or rfp_dpftri ('I') would enqueue for
 * the given arguments and schedule (sched: as rfp_set_schedule; NULL = the
 * defaults), without launching anything, so that the block
 * algebra, the views into the RFP rectangle and the aliasing rules can be
 * checked on a machine without a GPU.  Each record names views as (buffer,
 * element offset, row stride, column stride) with buffer one of the
 * RFP_PLAN_BUF_* values.  Primitive semantics:
 *   RFP_PLAN_GEMM: C(m x n) = alpha * A(m x k) * B(n x k)^T + beta * C, with
 *     A and B masked by tri_a / tri_b (0 none, 1 lower i >= j, 2 upper
 *     i <= j, 3 strictly lower, 4 strictly upper, in the operand's own
 *     indices) and, when c_lower, only C's lower triangle computed.
 *   RFP_PLAN_POTRF_LEAF: Cholesky of the lower triangle of a (order m); the
 *     leaf's inverse goes to view b (row-major, block order = b's row stride);
 *     INFO base info_base.
 *   RFP_PLAN_TRTRI_LEAF: in-place inverse of the lower triangle of a.
 *   RFP_PLAN_TRTRI_LEAVES: inverses of all 64-row diagonal blocks of the lower
 *     triangular a (order m) into consecutive NB x NB row-major blocks at b.
 *   RFP_PLAN_LAUUM_LEAF: lower triangle of W^T W in place (order m).
 *   RFP_PLAN_BLOCK_SOLVE: tri_a 0: L Y = B (forward), 1: L^T X = B
 *     (backward), in place in d (m + k rows, n columns), with L the lower
 *     factor held as a = L11 (order m), b = L21 (k x m), c = L22 (order k);
 *     w holds the inverses of the 64-row diagonal blocks of L11 then of L22,
 *     consecutive NB x NB row-major blocks (as RFP_PLAN_TRTRI_LEAVES writes).
 *   RFP_PLAN_AXPY: C(m x n) += alpha * A (only C's lower triangle when
 *     c_lower).
 *   RFP_PLAN_COPY: C(m x n) = A (A and C do not overlap).
 *   RFP_PLAN_RECORD / RFP_PLAN_WAIT: event m is recorded on / waited for by
 *     stream `stream` (0: the caller's stream, 1 and 2: the handle's two
 *     auxiliary streams).  Every other record carries the stream it runs on;
 *     work on one stream runs in order, across streams only as the events
 *     order it.
 * *count receives the number of records (even beyond cap).  Returns 0, -1 for
 * an unknown routine, -8 for bad output arguments, or the routine's own
 * argument error code. */
enum {
    RFP_PLAN_GEMM = 1,
    RFP_PLAN_POTRF_LEAF = 2,
    RFP_PLAN_TRTRI_LEAF = 3,
    RFP_PLAN_TRTRI_LEAVES = 4,
    RFP_PLAN_LAUUM_LEAF = 5,
    RFP_PLAN_RECORD = 6,
    RFP_PLAN_WAIT = 7,
    RFP_PLAN_BLOCK_SOLVE = 8,
    RFP_PLAN_AXPY = 9,
    RFP_PLAN_COPY = 10
};
enum { RFP_PLAN_BUF_ARF = 0, RFP_PLAN_BUF_B = 1, RFP_PLAN_BUF_WORK = 2, RFP_PLAN_BUF_INFO = 3 };
typedef struct {
    int32_t kind, tri_a, tri_b, c_lower;
    int32_t inplace; /* GEMM: C aliases A or B (one tile spans the aliased dimension) */
    int32_t stream;  /* 0: the caller's stream, 1 and 2: the handle's auxiliary streams */
    int64_t m, n, k;
    double alpha, beta;
    int64_t a[4], b[4], c[4]; /* buffer (-1: unused), offset, row stride, column stride */
    int64_t info_base;
    int64_t d[4], w[4];       /* RFP_PLAN_BLOCK_SOLVE: right-hand sides and block inverses */
} rfp_plan_op;
int rfp_plan(char routine, char transr, char uplo, int64_t n, int64_t nrhs, int64_t ldb,
             const rfp_schedule_t* sched, rfp_plan_op* ops, int64_t cap, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* RFP_MI355X_H */
