// Internal header of the MI355X RFP library: strided views, the RFP block
// descriptor for the eight layouts, and the launchers the drivers call.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>

#include "rfp.h"

namespace rfp {

// A strided 2-D view: element (i, j) lives at p[i * rs + j * cs].  Every view
// the library builds has one unit stride (rs == 1: rows contiguous, i.e. the
// column-major orientation; cs == 1: the row-major orientation).
template <typename T>
struct Mat {
    T* p;
    int64_t rs, cs;
    __host__ __device__ T& at(int64_t i, int64_t j) const { return p[i * rs + j * cs]; }
    __host__ __device__ Mat sub(int64_t i, int64_t j) const { return Mat{p + i * rs + j * cs, rs, cs}; }
    __host__ __device__ Mat tr() const { return Mat{p, cs, rs}; }
    __host__ __device__ operator Mat<const T>() const { return Mat<const T>{p, rs, cs}; }
};

// Operand masks: which entries of an operand (in its own (row, col) indices)
// are read; everything else is taken as zero.  Triangular operands of the
// RFP format must be masked because the complementary triangle of a diagonal
// block holds the other diagonal block's live data.
enum TriMask { TRI_NONE = 0, TRI_LOWER = 1, TRI_UPPER = 2, TRI_SLOWER = 3, TRI_SUPPER = 4 };

// The three blocks of an RFP array seen as the blocks of the lower-triangular
// (canonical) matrix: L11 (m1 x m1, lower), L21 (m2 x m1), L22 (m2 x m2, lower).
// For UPLO='U' the array holds U = L^T, i.e. the same numbers, so the lower
// view of every layout addresses the stored copy of each element.
struct RfpBlocks {
    int64_t n, m1, m2;
    int64_t off11, rs11, cs11;
    int64_t off21, rs21, cs21;
    int64_t off22, rs22, cs22;
};

// Returns false for an illegal TRANSR / UPLO character or n < 0.
// Layout descriptor (Section 2, Figures 4-6).  With n1 = ceil(n/2) columns
// for TRANSR='N' the rectangle AR has LDAR = n (odd n) or n + 1 (even n)
// rows.  For UPLO='L' the first diagonal block has order ceil(n/2): its lower
// triangle sits in the first columns of AR (one row down when n is even, to
// make room for the diagonal of A22), A21 sits under it, and A22's lower
// triangle is stored transposed in the upper part of the top square, shifted
// one column right when n is odd.  For UPLO='U' the first diagonal block has
// order floor(n/2): A12 occupies the top rows of AR, A22's upper triangle
// follows in the same columns, and A11's upper triangle is stored transposed
// below it.  TRANSR='T' stores AR^T with leading dimension n1, which swaps the
// row and column strides of every block.
__host__ __device__ inline bool rfp_blocks(char transr, char uplo, int64_t n, RfpBlocks* o)
{
    const int t = (transr >= 'a' && transr <= 'z') ? transr - 'a' + 'A' : transr;
    const int u = (uplo >= 'a' && uplo <= 'z') ? uplo - 'a' + 'A' : uplo;
    if ((t != 'N' && t != 'T') || (u != 'L' && u != 'U') || n < 0) return false;
    const bool odd = (n & 1) != 0;
    const int64_t ldar = odd ? n : n + 1;
    const int64_t cols = (n + 1) / 2;
    const int64_t sr = (t == 'N') ? 1 : cols;   // stride of one AR row step
    const int64_t sc = (t == 'N') ? ldar : 1;   // stride of one AR column step
    const int64_t extra = odd ? 0 : 1;           // the extra top row of even n
    o->n = n;
    // each block: AR position (row, col) of its (0,0) and whether its row
    // index runs down AR rows (true) or along AR columns (false)
    int64_t r11, c11, r21, c21, r22, c22;
    bool d11, d21, d22;
    if (u == 'L') {
        o->m1 = (n + 1) / 2;
        o->m2 = n - o->m1;
        r11 = extra; c11 = 0; d11 = true;
        r21 = o->m1 + extra; c21 = 0; d21 = true;
        r22 = 0; c22 = 1 - extra; d22 = false;
    } else {
        o->m1 = n / 2;
        o->m2 = n - o->m1;
        r11 = o->m2 + extra; c11 = 0; d11 = true;
        r21 = 0; c21 = 0; d21 = false;
        r22 = o->m1; c22 = 0; d22 = false;
    }
    auto put = [&](int64_t r, int64_t c, bool down, int64_t* off, int64_t* rs, int64_t* cs) {
        *off = r * sr + c * sc;
        *rs = down ? sr : sc;
        *cs = down ? sc : sr;
    };
    put(r11, c11, d11, &o->off11, &o->rs11, &o->cs11);
    put(r21, c21, d21, &o->off21, &o->rs21, &o->cs21);
    put(r22, c22, d22, &o->off22, &o->rs22, &o->cs22);
    return true;
}


template <typename T>
struct RfpView {
    int64_t n, m1, m2;
    Mat<T> t1, s, t2;  // L11, L21, L22
};

template <typename T>
__host__ __device__ inline RfpView<T> rfp_view(const RfpBlocks& b, T* arf)
{
    RfpView<T> v;
    v.n = b.n;
    v.m1 = b.m1;
    v.m2 = b.m2;
    v.t1 = Mat<T>{arf + b.off11, b.rs11, b.cs11};
    v.s = Mat<T>{arf + b.off21, b.rs21, b.cs21};
    v.t2 = Mat<T>{arf + b.off22, b.rs22, b.cs22};
    return v;
}

// Leaf orders of the recursive algorithms: diagonal blocks of at most NB rows
// are handled by one wavefront (solve, inversion), of at most NB2 rows by one
// fused workgroup (factorization).
constexpr int NB = 64;
constexpr int NB2 = 128;

// Default factorization schedule (rfp_schedule_t).  Measured at n = 20000 on
// all eight layouts: 256-column panels above a trailing order of 6144 (best of
// 3072-8192), off-diagonal chunks of at most 1536 columns (of 512-4096), the
// bulk update waiting for the lookahead at every order (better than 0 and
// 2048-6144), and 24 KB of LDS reserved by the FP64 leaf (beside a 128 x 128
// GEMM workgroup the leaf ran 1.5-1.8x slower).
constexpr int64_t DEFAULT_WIDE_PANELS_ABOVE = 6144;
constexpr int64_t DEFAULT_WIDE_PANEL_COLS = 256;
// FP16 / BF16-operand factorizations: their bulk updates are bound by moving
// C rather than by the matrix cores, so wider panels (fewer passes over the
// trailing matrix) pay off (n = 40000: 118 -> 104 ms)
constexpr int64_t DEFAULT_LOWP_WIDE_PANEL_COLS = 1024;
constexpr int64_t DEFAULT_CHUNK_MAX = 1536;
constexpr int64_t DEFAULT_LOOKAHEAD_WAIT_BELOW = INT64_MAX;
constexpr int64_t DEFAULT_LEAF_LDS_PAD = 24 * 1024;
constexpr int64_t MAX_LEAF_LDS_PAD = 64 * 1024;

// Splits of the recursion are multiples of the leaf order measured from the
// root, so the leaves of every sub-problem coincide with the leaves of its root.
inline int64_t rec_split(int64_t n, int nb)
{
    int64_t nblk = (n + nb - 1) / nb;
    return ((nblk + 1) / 2) * nb;
}

struct Profiler;

// Per-call execution context.
// Tuning table (autotuner results): GEMM configurations per shape class and
// right-hand-side slice widths of the fused solve per nrhs class.
struct TuneGemm {
    int tile;    // 0: 128 x 128, 1: 64 x 128, 2: 128 x 64, 3: 64 x 64
    int split;   // 0: built-in rule, 1: no split-K, s > 1: s-way split-K
    float us;    // measured time of the representative shape
};
struct TuneTable {
    std::map<uint64_t, TuneGemm> gemm;
    std::map<uint64_t, int> solve;  // key -> 16-column blocks per slice
    std::map<int, rfp_schedule_t> sched;  // size_bucket(n) -> factorization schedule
    int force_tile = -1, force_split = 0;  // testing: one configuration for every GEMM
};
// Shape classes: sizes by ceil(log2), precision (dt 0 FP64, 1 FP32; lp the
// operand mode), operand orientation bits and the lower-output flag.
__host__ inline int size_bucket(int64_t x)
{
    int b = 0;
    while (b < 40 && ((int64_t)1 << b) < x) b++;
    return b;
}
__host__ inline uint64_t tune_gemm_key(int dt, int lp, int sel, int clower, int64_t m, int64_t n, int64_t k)
{
    return ((uint64_t)dt << 40) | ((uint64_t)lp << 36) | ((uint64_t)sel << 32) | ((uint64_t)clower << 30) |
           ((uint64_t)size_bucket(m) << 20) | ((uint64_t)size_bucket(n) << 10) | (uint64_t)size_bucket(k);
}
__host__ inline uint64_t tune_solve_key(int dt, int64_t n, int64_t nrhs)
{
    return ((uint64_t)dt << 20) | ((uint64_t)size_bucket(n) << 10) | (uint64_t)size_bucket(nrhs);
}

struct Exec {
    hipStream_t stream;
    int* info;          // device; kernels of a factorization exit early when *info != 0
    void* splitk_ws;    // split-K partial sums
    size_t splitk_bytes;
    Profiler* prof;     // optional per-launch event timing
    int lowp = 0;       // FP32 GEMMs: 0 FP32 operands, 1 FP16, 2 BF16 (not for in-place products)
    const TuneTable* tune = nullptr;  // autotuned configurations, if any
    int prio = 0;  // 1: the kernels' waves take the highest issue priority (the critical path, which
                   // shares compute units with bulk work on the other streams)
    int leaf_pad = (int)DEFAULT_LEAF_LDS_PAD;  // LDS bytes the FP64 128-row leaf reserves beyond its own
    const int* gate = nullptr;  // device, or null: the solve-side kernels (fused solve, leaf inverses,
                                // thin symmetric multiply) do nothing while *gate != 0
};

// Brackets one kernel launch with HIP events on the launch stream when
// profiling is enabled; `name` is the kernel's demangled name, `flops` and
// `bytes` its algorithmic work for this launch.
struct ProfScope {
    Profiler* p;
    int slot;
    hipStream_t stream;
    ProfScope(const Exec& ex, const char* name, double flops, double bytes);
    ~ProfScope();
};

// C(m x n) = alpha * A(m x k) * B(n x k)^T + beta * C.
// A(i, kk) = A.at(i, kk) masked by triA; B(j, kk) = B.at(j, kk) masked by triB.
// c_lower: only the entries i >= j of C are computed and written (m >= n).
// inplace: C aliases A (then n <= 128) or B (then m <= 128); the aliased
// dimension is then kept inside one tile, which makes the in-place triangular
// products of the leaves race-free.
// Argument checks shared by the launch and by plan recording.
hipError_t gemm_validate(int64_t m, int64_t n, int64_t a_rs, int64_t a_cs, int64_t b_rs, int64_t b_cs,
                         int64_t c_rs, int64_t c_cs, bool c_lower, bool inplace);
template <typename T>
hipError_t gemm(const Exec& ex, int64_t m, int64_t n, int64_t k, T alpha, Mat<const T> A, int triA,
                Mat<const T> B, int triB, T beta, Mat<T> C, bool c_lower, bool inplace = false);

// Leaf kernels (order nb <= NB, one wavefront per block).
// potrf: in-place Cholesky of the lower triangle of A; writes L^{-1} (NB x NB,
// row-major, zero above the diagonal, identity-padded) to winv; *info = info_base + j + 1 on
// the first non-positive pivot j.
template <typename T>
hipError_t potrf_leaf(const Exec& ex, Mat<T> A, int nb, T* winv, int64_t info_base);
// Batched out-of-place inverses of every NB-leaf of a lower-triangular matrix
// of order n: winv[b] = (diagonal block b)^{-1} (unit: with a unit diagonal,
// which is then not read).
template <typename T>
hipError_t trtri_leaves(const Exec& ex, Mat<const T> A, int64_t n, T* winv, bool unit = false);
// Fused Cholesky of a diagonal block of order nb <= NB2 with the inverse of
// its factor (NB2 x NB2, row-major, zero above the diagonal, identity-padded)
// written to winv; INFO as for potrf_leaf.
template <typename T>
hipError_t potrf128_leaf(const Exec& ex, Mat<T> A, int nb, T* winv, int64_t info_base);
// In-place inverse of a lower-triangular diagonal block of order nb <= 128 by
// one workgroup (MFMA block columns); scratch: 128 x 128 elements of device
// memory owned by the caller's stream.  *ex.info = info_base + i + 1 for the
// first exactly zero diagonal entry i.
template <typename T>
hipError_t trtri128_leaf(const Exec& ex, Mat<T> A, int nb, T* scratch, int64_t info_base);
// In place, the lower triangle of W^T W for a lower-triangular diagonal block
// W of order nb <= 128, by one workgroup on MFMA.
template <typename T>
hipError_t lauum128_leaf(const Exec& ex, Mat<T> A, int nb);

// Fused blocked triangular solve with the whole factor of an RFP matrix
// (Section 4): forward L Y = B, else L^T X = B, over the views L11 (order m1),
// L21 (m2 x m1) and L22 (order m2), in one launch.  winv holds the inverses
// of the 64-row diagonal blocks, those of L11 then those of L22, each NB x NB
// row-major (as trtri_leaves writes them).  b (m1 + m2 rows, nrhs columns,
// column-major, leading dimension ldb) is overwritten by the solution.  flags
// (block_solve_flags ints) are ready flags compared with epoch: every launch
// on the same flags needs an epoch none of them holds.
// epoch (device) is read at launch; status (device, or null) gets bit 0 when a
// bounded wait gives up after spin_limit polls (that block of b becomes NaN).
template <typename T>
hipError_t block_solve(const Exec& ex, bool forward, Mat<const T> t1, Mat<const T> s, Mat<const T> t2, int64_t m1,
                       int64_t m2, const T* winv, T* b, int64_t ldb, int64_t nrhs, int* flags, const int* epoch,
                       int* status, int spin_limit);
int64_t block_solve_flags(int64_t m1, int64_t m2, int64_t nrhs);
// Advance the device epoch of a flag array (clearing the flags when it wraps).
hipError_t epoch_bump(hipStream_t s, int* flags, int64_t nflags, int* epoch);
constexpr int DEFAULT_SPIN_LIMIT = 1 << 24;
hipError_t fill_int(hipStream_t s, int* p, int64_t n, int v);

// Mixed-precision building blocks.
// s[i] = 1/sqrt(a_ii) (scale) or 1, then o = (float)(((a_ij s_i) s_j) mu) on
// every stored entry (shift added to (a_ii s_i) s_i before mu), o in the same
// RFP layout as a.
hipError_t pf_cast_scale(hipStream_t st, const RfpView<const double>& a, const RfpView<float>& o, int scale, double mu,
                         double shift, double* s, int* nonfinite = nullptr);
// Default multiples c of the factor precision's unit roundoff u added to the
// unit diagonal of the scaled matrix before a low-precision factor: the FP32
// factor's own rounding (FP32 accumulation over long inner products) needs a
// larger multiple of its small u than FP16 / BF16 operands do of theirs.
constexpr double DEFAULT_LOWP_SHIFT_FP32 = 64.0;
constexpr double DEFAULT_LOWP_SHIFT_HALF = 4.0;
inline double unit_roundoff(int fprec)
{
    return fprec == RFP_PREC_FP16 ? 0x1p-11 : fprec == RFP_PREC_BF16 ? 0x1p-8 : 0x1p-24;
}
// Norm of the symmetric matrix held in a: which = 0 max |a_ij|, 1 one- (=
// infinity-) norm, 2 Frobenius; work holds n + 3 doubles; *out on the device.
hipError_t pf_norm(hipStream_t st, const RfpView<const double>& a, int which, double* work, double* out);
hipError_t fill_double(hipStream_t s, double* p, int64_t n, double v);
// Y = beta Y + alpha A X, A symmetric in RFP (FP64), X and Y n x nrhs
// column-major; ws holds symm_thin_workspace(m1, m2) bytes.
size_t symm_thin_workspace(int64_t m1, int64_t m2);
hipError_t symm_thin(const Exec& ex, const RfpView<const double>& v, const double* x, int64_t ldx, double alpha,
                     double beta, double* y, int64_t ldy, int64_t nrhs, double* ws);
hipError_t ir_scale_cast(hipStream_t st, const double* r, int64_t ldr, const double* s, float* out, int64_t ldo,
                         int64_t n, int64_t nrhs, const int* gate = nullptr);
hipError_t ir_update(hipStream_t st, double* x, int64_t ldx, const double* s, double mu, const float* d, int64_t ldd,
                     int64_t n, int64_t nrhs, bool accumulate, const int* gate = nullptr);
hipError_t col_dot(hipStream_t st, const double* u, const double* v, int64_t ld, int64_t n, int64_t nrhs, double* out,
                   const int* gate = nullptr);
hipError_t pcg_step(hipStream_t st, double* d, int64_t ldd, double* r, const double* p, const double* q,
                    const double* rz, const double* pq, int64_t ld, int64_t n, int64_t nrhs, const int* gate = nullptr);
hipError_t pcg_dir(hipStream_t st, double* p, const double* z, const double* rz_new, const double* rz_old, int64_t ld,
                   int64_t n, int64_t nrhs, const int* gate = nullptr);
hipError_t col_max(hipStream_t st, const double* v, int64_t ld, int64_t n, int64_t nrhs, double* out,
                   const int* gate = nullptr);
hipError_t backward_error(hipStream_t st, const double* rmax, const double* xmax, const double* bmax,
                          const double* anorm, int64_t nrhs, double* eta, const int* gate = nullptr);
// Device-side control of the refinement (no host synchronisation): see
// pfsv_ir_impl.  IrCtl lives in device memory.
struct IrCtl {
    int phase;      // IR_CLASSIC, IR_PCG, IR_DONE, IR_FALLBACK
    int code;       // sweeps on convergence, else the fall-back reason (< 0)
    int g_ir, g_pcg, g_run;  // gates (0 = run) of classical sweeps, conjugate-gradient sweeps, any sweep
    int g_fb;       // 0 = run the FP64 fall-back (factor and copy)
    int g_fbsolve;  // 0 = run the fall-back solve (its factor succeeded)
    int lp_info;    // INFO of the low-precision factor
    int nonfinite;  // the scaled low-precision copy holds a non-finite entry
    int fb_info;    // INFO of the fall-back factor (gated as the factor's info word)
    int g_cvt;      // 0 = first conjugate-gradient sweep (widen the factor for the FP64 preconditioner, p = z)
    int g_cont;     // 0 = a conjugate-gradient sweep that continues the previous one's recurrence
    int stale;      // conjugate-gradient sweeps in a row without a new best backward error
    int pad[3];
    double eta, prev, best;
};
// conjugate-gradient sweeps in a row that may fail to bring the backward
// error below 0.9 times its best value before the refinement counts as stalled
constexpr int IR_STALE_SWEEPS = 3;
enum { IR_CLASSIC = 0, IR_PCG = 1, IR_DONE = 2, IR_FALLBACK = 3 };
hipError_t ir_start(hipStream_t st, IrCtl* c);
hipError_t ir_setup_decide(hipStream_t st, IrCtl* c);
hipError_t ir_decide(hipStream_t st, IrCtl* c, int it, int max_iter, double tol);
hipError_t ir_finish(hipStream_t st, IrCtl* c, int* iter, int* info);
// y(i, c) = x(i, c) (n x nrhs), or 0 when x is null; nothing while *gate != 0
hipError_t ir_copy(hipStream_t st, double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, int64_t nrhs,
                   const int* gate);
// 1-D copy of count doubles, nothing while *gate != 0
hipError_t gated_copy(hipStream_t st, double* dst, const double* src, int64_t count, const int* gate);
// dst = (double)src over count entries, nothing while *gate != 0
hipError_t widen_copy(hipStream_t st, double* dst, const float* src, int64_t count, const int* gate);
// y(i, c) = (x(i, c) * s[i]) * mul (n x nrhs), nothing while *gate != 0
hipError_t row_scale(hipStream_t st, double* y, int64_t ldy, const double* x, int64_t ldx, const double* s, double mul,
                     int64_t n, int64_t nrhs, const int* gate);

// Batched systems in one persistent launch (csrc/batched.hip).  mode: 0 FP64,
// 1 FP32, 2 FP16, 3 BF16 factor + FP64 refinement.  wgs_mem holds
// batched_wg_scratch_bytes() per workgroup; sysmem the per-system scratch of
// the systems with n > 256 (their total from batched_plan_host); st
// batched_state_bytes(batch); q a task queue of qcap slots; ctl 4 words;
// wgs persistent workgroups of the kernel built for occ (1 or 2) of them per
// compute unit.
size_t batched_wg_scratch_bytes();
size_t batched_state_bytes(int64_t batch);
int64_t batched_plan_host(const rfp_sys_t* sys_host, int64_t batch, int mode, int pftri, int max_iter,
                          int64_t* tasks);
hipError_t batched_solve(const Exec& ex, const rfp_sys_t* sys, int64_t batch, double* arf, double* b, int mode,
                         int pftri, double tol, double shift, int max_iter, int* info, int* iter, char* wgs_mem,
                         int wgs, int occ, char* sysmem, int64_t sysmem_bytes, void* st, unsigned long long* q,
                         int64_t qcap, unsigned long long* ctl);

// 2-D strided copy dst = src (m x n), optionally only the lower triangle.
template <typename Td, typename Ts>
hipError_t copy2d(hipStream_t s, Mat<Td> dst, Mat<const Ts> src, int64_t m, int64_t n, bool lower);

// Packed <-> RFP copy of every stored entry (to_rfp: packed -> RFP).
template <typename T>
hipError_t packed_copy(hipStream_t s, const RfpView<T>& v, T* ap, bool upper_packed, bool to_rfp);
// X = alpha X on an m x n view (lower triangle only if lower); alpha = 0
// writes zeros without reading X.
template <typename T>
hipError_t scale2d(hipStream_t s, Mat<T> x, int64_t m, int64_t n, T alpha, bool lower);
// C += alpha A on an m x n view (lower triangle only if lower).
template <typename T>
hipError_t axpy2d(hipStream_t s, Mat<T> c, Mat<const T> a, int64_t m, int64_t n, T alpha, bool lower);
// Save the diagonal of T1 and T2 into buf (n entries) and set it to one, or
// (restore) write buf back.
template <typename T>
hipError_t unit_diag(hipStream_t s, const RfpView<T>& v, T* buf, bool restore);

// Small utility kernels.
hipError_t set_int(hipStream_t s, int* p, int v);

// Complex Hermitian path (zpf.hip).  A view reads the canonical lower
// element (i, j) at p[i rs + j cs], conjugated when conj.  Masks: operand
// element (r, c) counts only when r - c >= md; ZMASK_NONE keeps all.
constexpr int64_t ZMASK_NONE = -(int64_t(1) << 62);
struct ZView {
    double2* p;
    int64_t rs, cs;
    bool conj;
};
struct ZRfpViews {
    int64_t n, m1, m2;
    ZView t1, s, t2;  // L11, L21, L22
};
// Views of a complex RFP array (TRANSR 'N' or 'C'); false for an illegal
// TRANSR / UPLO.
bool zrfp_views(char transr, char uplo, int64_t n, double2* arf, ZRfpViews* v);
// Scratch (complex elements) of the drivers for order n and nrhs columns.
size_t zwork_elems(int64_t n, int64_t nrhs, bool inverse = false);
hipError_t zconvert(hipStream_t s, const ZRfpViews& v, bool upper, double2* a, int64_t lda, bool to_rfp);
hipError_t zpftrf_run(hipStream_t s, const ZRfpViews& v, double2* work, int* info);
hipError_t zpftrs_run(hipStream_t s, const ZRfpViews& v, double2* b, int64_t ldb, int64_t nrhs, double2* work,
                      int* info);
hipError_t zpftri_run(hipStream_t s, const ZRfpViews& v, double2* work, int* info);

}  // namespace rfp
