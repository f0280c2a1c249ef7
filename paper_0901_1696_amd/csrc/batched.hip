// Batched solver for many SPD systems of uneven order, each in its own RFP
// layout, in one persistent launch: the paper's factorization (Section 3),
// solution (Section 4) and, if asked, inversion (Section 5) for every system,
// or a low-precision factor with FP64 iterative refinement per system.
//
// Work is scheduled through a device queue of tasks.  Every workgroup takes
// the next queue slot, waits until a task has been written into it, runs the
// task and reports it done to its system; the workgroup that finishes the
// last task of a system's current level writes that system's next level
// into the queue.  Tasks never wait for each other, so every wait ends: a
// slot is filled as soon as the tasks before it finish, and once every
// system is complete the waiting workgroups leave.
//
//  * Systems with n <= 256 are one task each: both diagonal blocks are then
//    at most 128 x 128, each one fused LDS leaf (potrf128_block) that also
//    yields the inverse of its factor, and the off-diagonal steps are
//    products of at most 128 x 128 blocks on MFMA (wg_mm) inside the
//    workgroup, with the inverses replacing the triangular solves.
//  * Larger systems are cut into 128-row block rows (those of T1, then those
//    of T2, so a tile never straddles the three blocks of the RFP array) and
//    run as levels of tile tasks, the tasks of one level independent:
//      factorization, right-looking (Section 3's 2 x 2 step on the tiles):
//        P(k) factor + inverse of tile (k,k); T(k) tiles (i,k) <- (i,k) W_kk^T;
//        U(k) tiles (i,j) -= (i,k) (j,k)^T for i >= j > k;
//      solution: one task, forward and backward over the block rows with the
//        tile inverses;
//      refinement: setup, then per sweep one solve task, one residual task
//        per block row and one decision task (the next level is the next
//        sweep or the end of the refinement);
//      inversion (Section 5), W = L^{-1} then W^T W in place: W_kk into tile
//        (k,k); for k from the right, Y_j = L_jk W_kk in place, then
//        X_i = -sum_{j=k+1..i} W_ij Y_j into a scratch column of tiles, then
//        copied over column k; then for each block row i from the top,
//        (W^T W)_ij = sum_{q>=i} W_qi^T W_qj for j < i, then j = i.
//
// Modes: plain FP64 (factor, solve and inverse in place, as PFTRF / PFTRS /
// PFTRI), or a low-precision factor of the diagonally scaled matrix (FP32
// products, or FP16 / BF16 operands with FP32 accumulation for the bulk
// updates) with FP64 iterative refinement against the untouched FP64 matrix,
// falling back to the FP64 factor and solve per system.  PFTRI always works
// from an FP64 factor.  No host synchronisation and no allocation inside the
// call once the workspace is sized: it can be captured in a HIP graph.
#include <algorithm>
#include <cstdio>
#include <type_traits>

#include "leaf128.h"
#include "rfp.h"
#include "tile_mm.h"

namespace rfp {

namespace {

constexpr int BN = 128;   // diagonal block capacity of a one-task system
constexpr int RC = 16;    // right-hand-side columns per pass
constexpr int NMAX = 2 * BN;
constexpr int TB = tile::TB;
constexpr double MU_FP16 = 33554432.0;  // 2^25, as in the single-system refinement

// C(m x n) = alpha A(m x k) B(n x k)^T + beta C on one workgroup, every
// dimension of C at most 128 (n at most 16 * NCB).  Operands are read from
// global memory (L2-resident for these sizes) under band masks; all products
// are formed in registers first and stored after a barrier, so C may alias A
// or B in any way.  Only i >= j is written when c_lower.  LPR rounds both
// operands to FP16 (1) or BF16 (2) before the FP32 products.  A may be held
// in a narrower type TA than the arithmetic (FP32 factors in FP64 products).
template <typename X>
struct NoDeduce {
    typedef X type;
};
template <typename T, int NCB, int LPR = 0, typename TA = T>
__device__ void wg_mm(int m, int n, int k, T alpha, Mat<const typename NoDeduce<TA>::type> A, int triA,
                      Mat<const T> B, int triB, T beta, Mat<T> C, bool c_lower)
{
    typedef typename M16<T>::acc acc_t;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int64_t BIG = (int64_t)1 << 40;
    auto band = [&](int tri, int64_t* lo, int64_t* hi) {
        *lo = -BIG;
        *hi = BIG;
        if (tri == TRI_LOWER) *hi = 0;
        if (tri == TRI_UPPER) *lo = 0;
        if (tri == TRI_SLOWER) *hi = -1;
        if (tri == TRI_SUPPER) *lo = 1;
    };
    int64_t alo, ahi, blo, bhi;
    band(triA, &alo, &ahi);
    band(triB, &blo, &bhi);
    acc_t acc[2][NCB];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int c = 0; c < NCB; c++) acc[s][c] = acc_t{0, 0, 0, 0};
    const int nstrip = (m + 15) / 16, ncb = (n + 15) / 16;
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int strip = w + 4 * s;
        if (strip >= nstrip) continue;
        const int i = strip * 16 + r;
        // Each step's loads are issued together, with no branch around them
        // (an entry outside the masks reads the operand's first element and is
        // replaced by zero), one step ahead of the products that use them.
        TA araw;
        T braw[NCB];
        unsigned oka = 0, okb = 0;
        auto fetch = [&](int kk, TA& a, T (&b)[NCB], unsigned& ma, unsigned& mb) {
            const int ka = kk + g;
            const int64_t da = ka - i;
            const bool ok = i < m && ka < k && da >= alo && da <= ahi;
            a = *(ok ? &A.at(i, ka) : A.p);
            ma = ok ? 1u : 0u;
            mb = 0;
#pragma unroll
            for (int c = 0; c < NCB; c++) {
                const int j = c * 16 + r;
                const int64_t db = ka - j;
                const bool okc = c < ncb && j < n && ka < k && db >= blo && db <= bhi;
                b[c] = *(okc ? &B.at(j, ka) : B.p);
                mb |= (okc ? 1u : 0u) << c;
            }
        };
        fetch(0, araw, braw, oka, okb);
        for (int kk = 0; kk < k; kk += 4) {
            // this step's values are needed here (one wait for all of them) ...
            asm volatile("" : "+v"(araw));
#pragma unroll
            for (int c = 0; c < NCB; c++) asm volatile("" : "+v"(braw[c]));
            const T av = oka ? tile::lp_round<LPR>((T)araw) : T(0);
            T bv[NCB];
#pragma unroll
            for (int c = 0; c < NCB; c++) bv[c] = (okb >> c) & 1 ? tile::lp_round<LPR>(braw[c]) : T(0);
            // ... and the next step's are in flight during the products
            if (kk + 4 < k) fetch(kk + 4, araw, braw, oka, okb);
#pragma unroll
            for (int c = 0; c < NCB; c++) {
                if (c >= ncb) break;
                acc[s][c] = M16<T>::op(av, bv[c], acc[s][c]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int strip = w + 4 * s;
        if (strip >= nstrip) continue;
#pragma unroll
        for (int c = 0; c < NCB; c++) {
            if (c >= ncb) break;
            T cv[4] = {T(0), T(0), T(0), T(0)};
            if (beta != T(0)) {  // the block's reads of C together, then its stores
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int i = strip * 16 + M16<T>::row(lane, e), j = c * 16 + r;
                    const bool ok = i < m && j < n && (!c_lower || i >= j);
                    cv[e] = *(ok ? &C.at(i, j) : C.p);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = strip * 16 + M16<T>::row(lane, e), j = c * 16 + r;
                if (i < m && j < n && (!c_lower || i >= j)) {
                    T v = alpha * acc[s][c][e];
                    if (beta != T(0)) v += beta * cv[e];
                    C.at(i, j) = v;
                }
            }
        }
    }
    __syncthreads();
}

// Scratch of one workgroup for one-task systems (device memory, 256-byte
// aligned pieces).
struct WgScratch {
    double *w1, *w2;          // FP64 inverses of L11, L22 (128 x 128 row-major)
    float *f1, *fs, *f2;      // FP32 scaled copies of T1, S, T2 (128 x 128 column-major)
    float *w1f, *w2f;         // FP32 inverses
    double *sv;               // diagonal scaling (NMAX)
    double *xv, *rv;          // refinement solution and residual (NMAX x RC, column-major)
    float* rf;                // FP32 correction (NMAX x RC)
    double *pv, *qv;          // conjugate-gradient direction and its product with A (NMAX x RC)
    double* rz;               // conjugate-gradient r . z per column (RC)
};

__host__ __device__ inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

__host__ __device__ inline size_t wg_scratch_bytes()
{
    return 2 * align256(sizeof(double) * BN * BN) + 5 * align256(sizeof(float) * BN * BN) +
           align256(sizeof(double) * NMAX) + 4 * align256(sizeof(double) * NMAX * RC) +
           align256(sizeof(float) * NMAX * RC) + align256(sizeof(double) * RC);
}

__device__ WgScratch wg_scratch(char* base)
{
    WgScratch s;
    size_t o = 0;
    auto take = [&](size_t b) {
        char* p = base + o;
        o += align256(b);
        return p;
    };
    s.w1 = (double*)take(sizeof(double) * BN * BN);
    s.w2 = (double*)take(sizeof(double) * BN * BN);
    s.f1 = (float*)take(sizeof(float) * BN * BN);
    s.fs = (float*)take(sizeof(float) * BN * BN);
    s.f2 = (float*)take(sizeof(float) * BN * BN);
    s.w1f = (float*)take(sizeof(float) * BN * BN);
    s.w2f = (float*)take(sizeof(float) * BN * BN);
    s.sv = (double*)take(sizeof(double) * NMAX);
    s.xv = (double*)take(sizeof(double) * NMAX * RC);
    s.rv = (double*)take(sizeof(double) * NMAX * RC);
    s.rf = (float*)take(sizeof(float) * NMAX * RC);
    s.pv = (double*)take(sizeof(double) * NMAX * RC);
    s.qv = (double*)take(sizeof(double) * NMAX * RC);
    s.rz = (double*)take(sizeof(double) * RC);
    return s;
}

// LDS of the persistent kernel: the leaf, the tile products and the cast's
// scalings never run at the same time.
union BatchSmem {
    Leaf128Smem<double> d;
    Leaf128Smem<float> f;
    tile::Smem<double> gd;
    tile::Smem<float> gf;
    double sdiag[2 * TB];
};

// Symmetric element A(i, j) of a system through its lower views.
__device__ __forceinline__ double sym_at(const RfpView<double>& v, int64_t i, int64_t j)
{
    if (i < j) {
        const int64_t q = i;
        i = j;
        j = q;
    }
    if (i < v.m1) return v.t1.at(i, j);
    if (j < v.m1) return v.s.at(i - v.m1, j);
    return v.t2.at(i - v.m1, j - v.m1);
}

// Factor in FP64 in place (Section 3's four steps) and keep both inverses in
// the scratch.  Returns 0 or the failing global pivot (1-based).
__device__ int factor64(BatchSmem& sm, const RfpView<double>& v, const WgScratch& ws)
{
    const int m1 = (int)v.m1, m2 = (int)v.m2;
    int f = potrf128_block<double>(sm.d, v.t1, m1, ws.w1, nullptr, 0);
    if (f) return f;
    if (m2 > 0) {
        wg_mm<double, 8>(m2, m1, m1, 1.0, v.s, TRI_NONE, Mat<const double>{ws.w1, BN, 1}, TRI_LOWER, 0.0, v.s, false);
        wg_mm<double, 8>(m2, m2, m1, -1.0, v.s, TRI_NONE, v.s, TRI_NONE, 1.0, v.t2, true);
        f = potrf128_block<double>(sm.d, v.t2, m2, ws.w2, nullptr, 0);
        if (f) return m1 + f;
    }
    return 0;
}

// X = A^{-1} B on an r-column slab B (rows m1 + m2, column-major, ld), with
// the factor's inverses W1, W2 and L21 = S (Figure 4's solution steps with
// the triangular solves done by the inverses).  The factor may be held in a
// narrower type TF than the arithmetic T.
template <typename T, typename TF = T>
__device__ void solve_slab(int m1, int m2, Mat<const typename NoDeduce<TF>::type> s, const TF* w1, const TF* w2, T* b,
                           int64_t ld, int r)
{
    Mat<T> B1{b, 1, ld}, B2{b + m1, 1, ld};
    Mat<const TF> W1{w1, BN, 1}, W2{w2, BN, 1};
    wg_mm<T, 1, 0, TF>(m1, r, m1, T(1), W1, TRI_LOWER, Mat<const T>(B1).tr(), TRI_NONE, T(0), B1, false);
    if (m2 > 0) {
        wg_mm<T, 1, 0, TF>(m2, r, m1, T(-1), s, TRI_NONE, Mat<const T>(B1).tr(), TRI_NONE, T(1), B2, false);
        wg_mm<T, 1, 0, TF>(m2, r, m2, T(1), W2, TRI_LOWER, Mat<const T>(B2).tr(), TRI_NONE, T(0), B2, false);
        wg_mm<T, 1, 0, TF>(m2, r, m2, T(1), W2.tr(), TRI_UPPER, Mat<const T>(B2).tr(), TRI_NONE, T(0), B2, false);
        wg_mm<T, 1, 0, TF>(m1, r, m2, T(-1), s.tr(), TRI_NONE, Mat<const T>(B2).tr(), TRI_NONE, T(1), B1, false);
    }
    wg_mm<T, 1, 0, TF>(m1, r, m1, T(1), W1.tr(), TRI_UPPER, Mat<const T>(B1).tr(), TRI_NONE, T(0), B1, false);
}

// A^{-1} in place from the FP64 factor (Section 5): W21 = -W22 L21 W11 into
// S, then T1 = W11^T W11 + W21^T W21, S = W22^T W21, T2 = W22^T W22.
__device__ void invert64(const RfpView<double>& v, const WgScratch& ws)
{
    const int m1 = (int)v.m1, m2 = (int)v.m2;
    Mat<const double> W1{ws.w1, BN, 1}, W2{ws.w2, BN, 1};
    if (m2 > 0) {
        wg_mm<double, 8>(m2, m1, m1, 1.0, v.s, TRI_NONE, W1.tr(), TRI_UPPER, 0.0, v.s, false);
        wg_mm<double, 8>(m2, m1, m2, -1.0, W2, TRI_LOWER, Mat<const double>(v.s).tr(), TRI_NONE, 0.0, v.s, false);
    }
    wg_mm<double, 8>(m1, m1, m1, 1.0, W1.tr(), TRI_UPPER, W1.tr(), TRI_UPPER, 0.0, v.t1, true);
    if (m2 > 0) {
        wg_mm<double, 8>(m1, m1, m2, 1.0, Mat<const double>(v.s).tr(), TRI_NONE, Mat<const double>(v.s).tr(),
                         TRI_NONE, 1.0, v.t1, true);
        wg_mm<double, 8>(m2, m1, m2, 1.0, W2.tr(), TRI_UPPER, Mat<const double>(v.s).tr(), TRI_NONE, 0.0, v.s,
                         false);
        wg_mm<double, 8>(m2, m2, m2, 1.0, W2.tr(), TRI_UPPER, W2.tr(), TRI_UPPER, 0.0, v.t2, true);
    }
}

// max over the block's threads (non-negative values; NaN wins): wavefront
// reductions, then the four wavefront results through red[0..3].
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }
__device__ double wg_max(double v, double* red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double out = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
    __syncthreads();
    return out;
}

// sum over the block's threads (same reduction tree as wg_max)
__device__ double wg_sum(double v, double* red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double out = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return out;
}

// Refinement: sweeps apply M^{-1} once (classical refinement) until one
// fails to cut the backward error fourfold; later sweeps run PCG_STEPS steps
// of preconditioned conjugate gradients in FP64, one recurrence continued
// from sweep to sweep with the true residual replacing the recursive one at
// each sweep's start; the refinement stalls after IR_STALE_SWEEPS such
// sweeps in a row that fail to bring the backward error below 0.9 times its
// best value (conjugate gradients minimise the error's A-norm, so the
// residual need not fall every sweep).
constexpr int PCG_STEPS = 8;

// normwise backward error of one column from its maxima (NaN anywhere: NaN)
__device__ __forceinline__ double col_eta(double rm, double xm, double bm, double anorm)
{
    const double den = anorm * xm + bm;
    return (den != den || rm != rm) ? __builtin_nan("") : den > 0.0 ? rm / den : rm > 0.0 ? __builtin_inf() : 0.0;
}

}  // namespace

// ------------------------------------------------------------- task model
// Per-system state (device).  Flags: the low-precision factor failed, the
// scaled copy is not finite, the FP64 factor is needed (fall-back), the
// FP64 factor failed.
enum { F_LPFAIL = 1, F_NONFINITE = 2, F_NEED64 = 4, F_F64FAIL = 8 };
enum { K_NONE = 0, K_SMALL = 1, K_TILED = 2, K_DONE = 3 };
struct SysState {
    int64_t off;      // byte offset of its scratch in the per-system area
    int kind;         // K_*
    int nb1, nb2;     // block rows of T1 and T2
    int level;        // current level
    int ntask;        // tasks of the current level
    int done;         // tasks of the current level finished
    int flags;
    int info, code;   // FP64 INFO; refinement sweeps or fall-back reason
    int cfail;        // first right-hand side left to the FP64 solve
    int jump;         // refinement: local level that follows setup, a decision or a CG update
    int sweep;        // refinement: sweeps done
    int pcg;          // refinement: sweeps run conjugate gradients
    int cgstep;       // refinement: conjugate-gradient steps of the current sweep
    int cgcont;       // refinement: the conjugate-gradient recurrence has started
    int stale;        // refinement: conjugate-gradient sweeps in a row without a new best
    double best;      // refinement: best backward error since the switch to conjugate gradients
    double prev;      // refinement: previous backward error
    double anorm;     // refinement: ||A||_inf
};

// Stages of a tiled system, in order.
enum { ST_CAST = 0, ST_LPFAC, ST_IR, ST_F64FAC, ST_SOLVE, ST_TRTRI, ST_LAUUM, ST_END };
// refinement stage, local levels: 0 setup; a classical sweep is 1 solve,
// 2 residual, 3 decision; a conjugate-gradient sweep repeats 4 (z = M^{-1} r,
// new direction p), 5 (q = A p, one task per block row), 6 (update of x and
// r), then 2 and 3
enum { IR_SETUP = 0, IR_SOLVE = 1, IR_RESID = 2, IR_DECIDE = 3, CG_Z = 4, CG_Q = 5, CG_UPD = 6, IR_LEVELS = 7 };

struct BatchArgs {
    const rfp_sys_t* sys;
    int64_t batch;
    double* arf;
    double* b;
    int mode;       // 0 FP64; 1 FP32, 2 FP16, 3 BF16 factor + FP64 refinement
    int pftri;
    double tol;
    double shift;   // added to the unit diagonal of the scaled matrix before the low-precision factor
    int max_iter;
    int* info;
    int* iter;
    char* wgs;               // per-workgroup scratch (one-task systems)
    char* sysmem;            // per-system scratch (tiled systems)
    int64_t sysmem_bytes;
    SysState* st;            // [batch]
    unsigned long long* q;   // task queue: slot = task + 1, 0 while empty
    int64_t qcap;
    unsigned long long* ctl; // [0] head, [1] tail, [2] systems not finished, [3] error
    int64_t spin_limit;
};

// ----------------------------------------------------- level structure
__host__ __device__ inline int64_t fac_levels(int nb) { return nb > 0 ? 3 * (int64_t)nb - 2 : 0; }
__host__ __device__ inline int64_t trtri_levels(int nb) { return nb > 0 ? 3 * (int64_t)nb - 2 : 0; }
__host__ __device__ inline int64_t lauum_levels(int nb) { return nb > 0 ? 2 * (int64_t)nb - 1 : 0; }
__host__ __device__ inline int64_t stage_levels(int stage, int nb, int mode)
{
    switch (stage) {
        case ST_CAST: return mode ? 1 : 0;
        case ST_LPFAC: return mode ? fac_levels(nb) : 0;
        case ST_IR: return mode ? IR_LEVELS : 0;
        case ST_F64FAC: return fac_levels(nb);
        case ST_SOLVE: return 1;
        case ST_TRTRI: return trtri_levels(nb);
        case ST_LAUUM: return lauum_levels(nb);
        default: return 0;
    }
}
// (stage, local level) of level ell >= 0; false past the end
__host__ __device__ inline bool locate(int64_t ell, int nb, int mode, int* stage, int64_t* loc)
{
    if (ell < 0) return false;
    for (int s = ST_CAST; s < ST_END; s++) {
        const int64_t L = stage_levels(s, nb, mode);
        if (ell < L) {
            *stage = s;
            *loc = ell;
            return true;
        }
        ell -= L;
    }
    return false;
}
__host__ __device__ inline int64_t stage_start(int stage, int nb, int mode)
{
    int64_t o = 0;
    for (int s = ST_CAST; s < stage; s++) o += stage_levels(s, nb, mode);
    return o;
}
// tasks of (stage, local level)
__host__ __device__ inline int64_t level_tasks(int stage, int64_t loc, int nb)
{
    switch (stage) {
        case ST_CAST: return (int64_t)nb * (nb + 1) / 2;
        case ST_LPFAC:
        case ST_F64FAC: {
            const int64_t k = loc / 3, sub = loc % 3, rest = nb - 1 - k;
            return sub == 0 ? 1 : sub == 1 ? rest : rest * (rest + 1) / 2;
        }
        case ST_IR: return (loc == IR_RESID || loc == CG_Q) ? nb : 1;
        case ST_SOLVE: return 1;
        case ST_TRTRI: {
            if (loc == 0) return nb;
            const int64_t k = nb - 2 - (loc - 1) / 3;
            return nb - 1 - k;
        }
        case ST_LAUUM: {
            if (loc == 0) return 1;
            const int64_t i = (loc + 1) / 2;
            return ((loc + 1) % 2 == 0) ? i : 1;
        }
        default: return 0;
    }
}

// Scratch of a tiled system (256-byte aligned pieces).
struct TileScratch {
    double* w64;     // nb inverses of the FP64 diagonal tiles (TB x TB row-major)
    float* lpt;      // low-precision tiles, tile (i,j) at tile index i (i+1)/2 + j (TB x TB row-major)
    float* w32;      // nb inverses of the low-precision diagonal tiles
    double* sv;      // diagonal scaling (n)
    double* rs;      // row sums of |A| (n)
    double *xv, *rv; // refinement solution and residual (n x nrhs, leading dimension n)
    float* rf;       // low-precision correction (n x nrhs)
    double *pv, *qv; // conjugate-gradient direction and its product with A (n x nrhs)
    double* rz;      // conjugate-gradient r . z per right-hand side
    double* bm;      // max |b| per right-hand side
    double* tmp;     // inversion: one column of tiles (nb x TB x TB)
    size_t bytes;
};
__host__ __device__ inline TileScratch tile_scratch(char* base, int64_t n, int64_t nrhs, int nb, int mode, int pftri)
{
    TileScratch s;
    size_t o = 0;
    auto take = [&](size_t b) {
        char* p = base + o;
        o += align256(b);
        return p;
    };
    const size_t t2 = (size_t)TB * TB;
    const size_t ntiles = (size_t)nb * (nb + 1) / 2;
    const size_t nr = (size_t)(nrhs > 0 ? nrhs : 1);
    s.w64 = (double*)take(sizeof(double) * nb * t2);
    s.lpt = mode ? (float*)take(sizeof(float) * ntiles * t2) : nullptr;
    s.w32 = mode ? (float*)take(sizeof(float) * nb * t2) : nullptr;
    s.sv = mode ? (double*)take(sizeof(double) * n) : nullptr;
    s.rs = mode ? (double*)take(sizeof(double) * n) : nullptr;
    s.xv = mode ? (double*)take(sizeof(double) * n * nr) : nullptr;
    s.rv = mode ? (double*)take(sizeof(double) * n * nr) : nullptr;
    s.rf = mode ? (float*)take(sizeof(float) * n * nr) : nullptr;
    s.pv = mode ? (double*)take(sizeof(double) * n * nr) : nullptr;
    s.qv = mode ? (double*)take(sizeof(double) * n * nr) : nullptr;
    s.rz = mode ? (double*)take(sizeof(double) * nr) : nullptr;
    s.bm = mode ? (double*)take(sizeof(double) * nr) : nullptr;
    s.tmp = pftri ? (double*)take(sizeof(double) * nb * t2) : nullptr;
    s.bytes = o;
    return s;
}

// Plan of one system: kind, block rows, scratch bytes, an upper bound of its
// tasks (for the queue's capacity).
struct SysPlan {
    int kind, nb1, nb2;
    int64_t bytes, tasks;
};
__host__ __device__ inline SysPlan plan_of(const rfp_sys_t& sd, int mode, int pftri, int max_iter)
{
    SysPlan p{K_NONE, 0, 0, 0, 0};
    RfpBlocks blk;
    if (!rfp_blocks(sd.transr, sd.uplo, sd.n, &blk) || sd.n == 0 || sd.nrhs < 0 || sd.ldb < (sd.n > 0 ? sd.n : 1))
        return p;
    if (sd.n <= NMAX) {
        p.kind = K_SMALL;
        p.tasks = 1;
        return p;
    }
    p.kind = K_TILED;
    p.nb1 = (int)((blk.m1 + TB - 1) / TB);
    p.nb2 = (int)((blk.m2 + TB - 1) / TB);
    const int nb = p.nb1 + p.nb2;
    p.bytes = (int64_t)tile_scratch(nullptr, sd.n, sd.nrhs, nb, mode, pftri).bytes;
    int64_t tasks = 0;
    for (int s = ST_CAST; s < ST_END; s++) {
        if (s == ST_IR) {
            // setup, then per sweep at most PCG_STEPS conjugate-gradient
            // steps (1 + nb + 1 tasks each), the residual and the decision
            if (mode) tasks += 1 + (int64_t)(max_iter > 0 ? max_iter : 1) * (PCG_STEPS * (nb + 2) + nb + 1);
            continue;
        }
        const int64_t L = stage_levels(s, nb, mode);
        for (int64_t l = 0; l < L; l++) tasks += level_tasks(s, l, nb);
    }
    p.tasks = tasks;
    return p;
}

#ifndef RFP_BATCHED_X2
size_t batched_wg_scratch_bytes() { return wg_scratch_bytes(); }
size_t batched_state_bytes(int64_t batch) { return align256(sizeof(SysState) * (size_t)batch); }

int64_t batched_plan_host(const rfp_sys_t* sys_host, int64_t batch, int mode, int pftri, int max_iter,
                          int64_t* tasks)
{
    int64_t bytes = 0, t = 0;
    for (int64_t i = 0; i < batch; i++) {
        const SysPlan p = plan_of(sys_host[i], mode, pftri, max_iter);
        bytes += p.bytes;
        t += p.tasks;
    }
    *tasks = t;
    return bytes;
}
#endif

namespace {

// ------------------------------------------------------------ tile views
struct Tiles {
    RfpView<double> v;   // the system's FP64 array
    int nb1, nb;
    int64_t m1, n;
    __device__ int64_t r0(int b) const { return b < nb1 ? (int64_t)b * TB : m1 + (int64_t)(b - nb1) * TB; }
    __device__ int cnt(int b) const
    {
        const int64_t len = b < nb1 ? m1 : n - m1, o = b < nb1 ? (int64_t)b * TB : (int64_t)(b - nb1) * TB;
        return (int)(len - o < TB ? len - o : TB);
    }
    // FP64 tile (i, j), i >= j, of the lower view
    __device__ Mat<double> t64(int i, int j) const
    {
        if (i < nb1) return v.t1.sub(r0(i), r0(j));
        if (j < nb1) return v.s.sub(r0(i) - m1, r0(j));
        return v.t2.sub(r0(i) - m1, r0(j) - m1);
    }
};
__device__ __forceinline__ int64_t tid(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }
__device__ __forceinline__ Mat<float> lp_tile(const TileScratch& s, int i, int j)
{
    return Mat<float>{s.lpt + tid(i, j) * TB * TB, TB, 1};
}
__device__ __forceinline__ void tri_decode(int64_t t, int* i, int* j)
{
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(r + 1) * (r + 2) / 2 <= t) r++;
    while ((int64_t)r * (r + 1) / 2 > t) r--;
    *i = r;
    *j = (int)(t - (int64_t)r * (r + 1) / 2);
}
template <typename T>
__device__ __forceinline__ Mat<T> diag_inv(T* w, int k)
{
    return Mat<T>{w + (int64_t)k * TB * TB, TB, 1};
}

// device-scope fences around the data of tasks run by other workgroups
// (the L2 caches of different XCDs are not coherent with each other)
__device__ __forceinline__ void release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// --------------------------------------------------------- one-task systems
// R (m1 + m2 rows, r <= RC columns, leading dimension NMAX) += alpha A X, A
// the system's FP64 matrix through its lower views, its strict upper
// triangle mirrored.
__device__ void small_symm(const RfpView<double>& v, const double* x, double* rr, int r, double alpha)
{
    const int m1 = (int)v.m1, m2 = (int)v.m2;
    Mat<const double> X1{x, 1, NMAX}, X2{x + m1, 1, NMAX};
    Mat<double> R1{rr, 1, NMAX}, R2{rr + m1, 1, NMAX};
    wg_mm<double, 1>(m1, r, m1, alpha, v.t1, TRI_LOWER, X1.tr(), TRI_NONE, 1.0, R1, false);
    wg_mm<double, 1>(m1, r, m1, alpha, Mat<const double>(v.t1).tr(), TRI_SUPPER, X1.tr(), TRI_NONE, 1.0, R1, false);
    if (m2 > 0) {
        wg_mm<double, 1>(m1, r, m2, alpha, Mat<const double>(v.s).tr(), TRI_NONE, X2.tr(), TRI_NONE, 1.0, R1, false);
        wg_mm<double, 1>(m2, r, m1, alpha, v.s, TRI_NONE, X1.tr(), TRI_NONE, 1.0, R2, false);
        wg_mm<double, 1>(m2, r, m2, alpha, v.t2, TRI_LOWER, X2.tr(), TRI_NONE, 1.0, R2, false);
        wg_mm<double, 1>(m2, r, m2, alpha, Mat<const double>(v.t2).tr(), TRI_SUPPER, X2.tr(), TRI_NONE, 1.0, R2,
                         false);
    }
}

// z = mu D^{-1/2} (Ls Ls^T)^{-1} D^{-1/2} r on an r-column slab (leading
// dimension NMAX): the low-precision preconditioner, solved with the factor's
// FP32 values and inverses, in FP32 (added into z when add) or, for the
// conjugate-gradient steps, in FP64 (so that the operator it applies is
// symmetric to FP64 rounding: an FP32 solve's rounding would swamp the small
// eigenvalues of the preconditioned matrix of an ill-conditioned system).
__device__ void small_prec(int n, int m1, int m2, Mat<const float> FS, const WgScratch& ws, const double* rin,
                           double* z, int r, double mu, bool add, bool fp64 = false)
{
    const int t = threadIdx.x;
    if (fp64) {
        for (int idx = t; idx < n * RC; idx += 256) {
            const int i = idx % n, c = idx / n;
            z[i + c * NMAX] = ws.sv[i] * rin[i + c * NMAX];
        }
        __syncthreads();
        solve_slab<double, float>(m1, m2, FS, ws.w1f, ws.w2f, z, NMAX, r);
        for (int idx = t; idx < n * RC; idx += 256) {
            const int i = idx % n, c = idx / n;
            z[i + c * NMAX] = (z[i + c * NMAX] * ws.sv[i]) * mu;
        }
        __syncthreads();
        return;
    }
    for (int idx = t; idx < n * RC; idx += 256) {
        const int i = idx % n, c = idx / n;
        ws.rf[i + c * NMAX] = (float)(ws.sv[i] * rin[i + c * NMAX]);
    }
    __syncthreads();
    solve_slab<float>(m1, m2, FS, ws.w1f, ws.w2f, ws.rf, NMAX, r);
    for (int idx = t; idx < n * RC; idx += 256) {
        const int i = idx % n, c = idx / n;
        const double d = ((double)ws.rf[i + c * NMAX] * ws.sv[i]) * mu;
        z[i + c * NMAX] = add ? z[i + c * NMAX] + d : d;
    }
    __syncthreads();
}

// PCG_STEPS steps of preconditioned conjugate gradients on A x = b (FP64
// throughout) from the true residual r of x (in ws.rv, updated to the
// recursive residual), x in ws.xv; the recurrence starts (p = z) unless cont,
// when it continues the previous sweep's (p = z + beta p).
__device__ void small_pcg(const RfpView<double>& v, Mat<const float> FS, const WgScratch& ws, int r, double mu,
                          double* red, bool cont)
{
    const int t = threadIdx.x, m1 = (int)v.m1, m2 = (int)v.m2, n = m1 + m2;
    for (int k = 0; k < PCG_STEPS; k++) {
        small_prec(n, m1, m2, FS, ws, ws.rv, ws.qv, r, mu, false, true);  // z into qv
        const bool first = k == 0 && !cont;
        for (int c = 0; c < r; c++) {
            double s = 0.0;
            for (int i = t; i < n; i += 256) s += ws.rv[i + c * NMAX] * ws.qv[i + c * NMAX];
            s = wg_sum(s, red);
            const double rz = ws.rz[c];
            const double beta = (!first && rz != 0.0) ? s / rz : 0.0;
            for (int i = t; i < n; i += 256) {
                const int o = i + c * NMAX;
                ws.pv[o] = first ? ws.qv[o] : ws.qv[o] + beta * ws.pv[o];
            }
            __syncthreads();
            if (t == 0) ws.rz[c] = s;
        }
        for (int idx = t; idx < n * RC; idx += 256) ws.qv[idx % n + (idx / n) * NMAX] = 0.0;
        __syncthreads();
        small_symm(v, ws.pv, ws.qv, r, 1.0);  // q = A p
        for (int c = 0; c < r; c++) {
            double s = 0.0;
            for (int i = t; i < n; i += 256) s += ws.pv[i + c * NMAX] * ws.qv[i + c * NMAX];
            s = wg_sum(s, red);
            const double al = s != 0.0 ? ws.rz[c] / s : 0.0;
            for (int i = t; i < n; i += 256) {
                const int o = i + c * NMAX;
                ws.xv[o] += al * ws.pv[o];
                ws.rv[o] -= al * ws.qv[o];
            }
        }
        __syncthreads();
    }
}

// Everything for a system with n <= 256 in this workgroup.
__device__ __attribute__((noinline)) void small_system(const BatchArgs& a, int64_t id, BatchSmem& sm, double* red, const WgScratch& ws)
{
    const int t = threadIdx.x;
    const rfp_sys_t sd = a.sys[id];
    RfpBlocks blk;
    rfp_blocks(sd.transr, sd.uplo, sd.n, &blk);
    double* arf = a.arf + sd.arf_off;
    const RfpView<double> v = rfp_view(blk, arf);
    const int n = (int)sd.n, m1 = (int)blk.m1, m2 = (int)blk.m2;
    int code = 0, finfo = 0;
    bool need64 = a.mode == 0;
    int64_t c_fail = 0;  // first right-hand side left to the FP64 solve
    const double mu = a.mode == 2 ? MU_FP16 : 1.0;

    if (a.mode != 0 && n > 0) {
        // ---- low-precision factor of mu D^{-1/2} A D^{-1/2}
        for (int i = t; i < n; i += 256) {
            const double d = sym_at(v, i, i);
            ws.sv[i] = d > 0.0 ? 1.0 / sqrt(d) : __builtin_nan("");
        }
        __syncthreads();
        int nonfinite = 0;
        for (int idx = t; idx < BN * BN; idx += 256) {
            const int i = idx % BN, j = idx / BN;
            float f;
            const double dg = i == j ? a.shift : 0.0;
            if (i < m1 && j <= i) {
                ws.f1[idx] = f = (float)((((v.t1.at(i, j) * ws.sv[i]) * ws.sv[j]) + dg) * mu);
                nonfinite |= !__builtin_isfinite(f);
            }
            if (i < m2 && j < m1) {
                ws.fs[idx] = f = (float)(((v.s.at(i, j) * ws.sv[m1 + i]) * ws.sv[j]) * mu);
                nonfinite |= !__builtin_isfinite(f);
            }
            if (i < m2 && j <= i) {
                ws.f2[idx] = f = (float)((((v.t2.at(i, j) * ws.sv[m1 + i]) * ws.sv[m1 + j]) + dg) * mu);
                nonfinite |= !__builtin_isfinite(f);
            }
        }
        nonfinite = __syncthreads_or(nonfinite);
        const Mat<float> F1{ws.f1, 1, BN}, FS{ws.fs, 1, BN}, F2{ws.f2, 1, BN};
        int f = 0;
        if (!nonfinite) {
            f = potrf128_block<float>(sm.f, F1, m1, ws.w1f, nullptr, 0);
            if (!f && m2 > 0) {
                wg_mm<float, 8>(m2, m1, m1, 1.f, FS, TRI_NONE, Mat<const float>{ws.w1f, BN, 1}, TRI_LOWER, 0.f, FS,
                                false);
                if (a.mode == 2) wg_mm<float, 8, 1>(m2, m2, m1, -1.f, FS, TRI_NONE, FS, TRI_NONE, 1.f, F2, true);
                else if (a.mode == 3) wg_mm<float, 8, 2>(m2, m2, m1, -1.f, FS, TRI_NONE, FS, TRI_NONE, 1.f, F2, true);
                else wg_mm<float, 8>(m2, m2, m1, -1.f, FS, TRI_NONE, FS, TRI_NONE, 1.f, F2, true);
                f = potrf128_block<float>(sm.f, F2, m2, ws.w2f, nullptr, 0);
            }
        }
        if (nonfinite || f) {
            code = nonfinite ? -4 : -3;
            need64 = true;
        } else {
            // ||A||_inf once per system (row sums of |A|)
            double rsm = 0.0;
            for (int i = t; i < n; i += 256) {
                double s = 0.0;
                for (int j = 0; j < n; j++) s += fabs(sym_at(v, i, j));
                rsm = nanmax(rsm, s);
            }
            const double anorm = wg_max(rsm, red);
            // refinement, one slab of up to RC right-hand sides at a time
            int worst = 0;
            for (int64_t c0 = 0; c0 < sd.nrhs && code == 0; c0 += RC) {
                const int r = (int)((sd.nrhs - c0) < RC ? (sd.nrhs - c0) : RC);
                double* bb = a.b + sd.b_off + c0 * sd.ldb;
                for (int idx = t; idx < n * RC; idx += 256) {
                    const int i = idx % n, c = idx / n;
                    const double bv = c < r ? bb[i + c * sd.ldb] : 0.0;
                    ws.xv[i + c * NMAX] = 0.0;
                    ws.rv[i + c * NMAX] = bv;
                }
                __syncthreads();
                double prev = 0.0, best = 0.0;
                int done = -1, stale = 0, pcg_sweeps = 0;
                bool pcg = false;
                for (int it = 1; it <= a.max_iter; it++) {
                    if (pcg) small_pcg(v, FS, ws, r, mu, red, pcg_sweeps++ > 0);
                    else small_prec(n, m1, m2, FS, ws, ws.rv, ws.xv, r, mu, true);
                    // r = b - A x in FP64 from the untouched RFP matrix
                    for (int idx = t; idx < n * RC; idx += 256) {
                        const int i = idx % n, c = idx / n;
                        ws.rv[i + c * NMAX] = c < r ? bb[i + c * sd.ldb] : 0.0;
                    }
                    __syncthreads();
                    small_symm(v, ws.xv, ws.rv, r, -1.0);
                    // normwise backward error, max over the slab's columns
                    double eta = 0.0;
                    for (int c = 0; c < r; c++) {
                        double rm = 0.0, xm = 0.0, bmx = 0.0;
                        for (int i = t; i < n; i += 256) {
                            rm = nanmax(rm, fabs(ws.rv[i + c * NMAX]));
                            xm = nanmax(xm, fabs(ws.xv[i + c * NMAX]));
                            bmx = nanmax(bmx, fabs(bb[i + c * sd.ldb]));
                        }
                        rm = wg_max(rm, red);
                        xm = wg_max(xm, red);
                        bmx = wg_max(bmx, red);
                        eta = nanmax(eta, col_eta(rm, xm, bmx, anorm));
                    }
                    if (eta <= a.tol) {
                        done = it;
                        break;
                    }
                    if (pcg) {
                        if (eta < 0.9 * best) {
                            best = eta;
                            stale = 0;
                        } else if (++stale >= IR_STALE_SWEEPS) {
                            done = -2;
                            break;
                        }
                    }
                    if (it > 1 && !pcg && !(eta < 0.25 * prev)) {
                        pcg = true;
                        best = eta < prev ? eta : prev;
                    }
                    prev = eta;
                }
                if (done < 0) {
                    code = done;  // -1 max_iter, -2 stalled; earlier slabs are already solved
                    need64 = true;
                    c_fail = c0;
                    break;
                }
                worst = done > worst ? done : worst;
                for (int idx = t; idx < n * r; idx += 256) {
                    const int i = idx % n, c = idx / n;
                    bb[i + c * sd.ldb] = ws.xv[i + c * NMAX];
                }
                __syncthreads();
            }
            if (code == 0) code = worst;
        }
    }
    if (need64 || a.pftri) {
        // FP64 factor in place (plain mode, fall-back, or for the inverse)
        finfo = n > 0 ? factor64(sm, v, ws) : 0;
        if (finfo == 0 && need64) {
            for (int64_t c0 = c_fail; c0 < sd.nrhs; c0 += RC) {
                const int r = (int)((sd.nrhs - c0) < RC ? (sd.nrhs - c0) : RC);
                solve_slab<double>(m1, m2, v.s, ws.w1, ws.w2, a.b + sd.b_off + c0 * sd.ldb, sd.ldb, r);
            }
        }
        if (finfo == 0 && a.pftri) invert64(v, ws);
    }
    if (t == 0) {
        a.info[id] = finfo;
        a.iter[id] = a.mode == 0 ? 0 : code;
    }
    __syncthreads();
}

// ------------------------------------------------------------ tile tasks
// Factorization tasks on FP64 tiles (LP = false) or low-precision tiles:
// P(k), the leaf of tile (k,k) with its inverse.
template <bool LP>
__device__ __attribute__((noinline)) void fac_p_task(SysState& S, const Tiles& tl, const TileScratch& ts, int k,
                                                     BatchSmem& sm)
{
    int f;
    if constexpr (LP) f = potrf128_block<float>(sm.f, lp_tile(ts, k, k), tl.cnt(k), diag_inv(ts.w32, k).p, nullptr, 0);
    else f = potrf128_block<double>(sm.d, tl.t64(k, k), tl.cnt(k), diag_inv(ts.w64, k).p, nullptr, 0);
    if (f && threadIdx.x == 0) {
        if (LP) {
            S.flags |= F_LPFAIL;
        } else {
            S.flags |= F_F64FAIL;
            S.info = (int)(tl.r0(k) + f);
        }
    }
}

// T(k): tile (i,k) <- tile (i,k) W_kk^T (in place; FP32 products for the
// low-precision factor); U(k): tile (i,j) -= tile (i,k) tile (j,k)^T
// (operands rounded to the mode's precision for the low-precision factor).
template <bool LP>
__device__ __attribute__((noinline)) void fac_gemm_task(const BatchArgs& a, const Tiles& tl, const TileScratch& ts,
                                                        int k, int sub, int64_t t, BatchSmem& sm)
{
    typedef typename std::conditional<LP, float, double>::type T;
    auto tileT = [&](int i, int j) -> Mat<T> {
        if constexpr (LP) return lp_tile(ts, i, j);
        else return tl.t64(i, j);
    };
    T* w;
    if constexpr (LP) w = ts.w32;
    else w = ts.w64;
    tile::Acc<T> acc;
    acc.zero();
    tile::Smem<T>& gs = *reinterpret_cast<tile::Smem<T>*>(&sm);
    if (sub == 1) {
        const int i = k + 1 + (int)t;
        const Mat<T> X = tileT(i, k);
        tile::mma<T, 0>(gs, acc, tl.cnt(i), tl.cnt(k), tl.cnt(k), X, TRI_NONE, diag_inv(w, k), TRI_LOWER);
        tile::store<T>(acc, tl.cnt(i), tl.cnt(k), T(1), T(0), X, false);
        return;
    }
    int i, j;
    tri_decode(t, &i, &j);
    i += k + 1;
    j += k + 1;
    const Mat<T> C = tileT(i, j);
    if constexpr (LP) {
        if (a.mode == 2)
            tile::mma<float, 1>(gs, acc, tl.cnt(i), tl.cnt(j), tl.cnt(k), tileT(i, k), TRI_NONE, tileT(j, k), TRI_NONE);
        else if (a.mode == 3)
            tile::mma<float, 2>(gs, acc, tl.cnt(i), tl.cnt(j), tl.cnt(k), tileT(i, k), TRI_NONE, tileT(j, k), TRI_NONE);
        else
            tile::mma<float, 0>(gs, acc, tl.cnt(i), tl.cnt(j), tl.cnt(k), tileT(i, k), TRI_NONE, tileT(j, k), TRI_NONE);
    } else {
        tile::mma<double, 0>(gs, acc, tl.cnt(i), tl.cnt(j), tl.cnt(k), tileT(i, k), TRI_NONE, tileT(j, k), TRI_NONE);
    }
    tile::store<T>(acc, tl.cnt(i), tl.cnt(j), T(-1), T(1), C, i == j);
}

// Low-precision tile (i,j) = (float)(((a_ij s_i) s_j) mu), lower triangle of
// the diagonal tiles; a non-finite value flags the system.
__device__ __attribute__((noinline)) void cast_task(const BatchArgs& a, SysState& S, const Tiles& tl, const TileScratch& ts, int64_t t,
                          double* sdiag)
{
    int i, j;
    tri_decode(t, &i, &j);
    const int ci = tl.cnt(i), cj = tl.cnt(j);
    const double mu = a.mode == 2 ? MU_FP16 : 1.0;
    const int th = threadIdx.x;
    // scalings of the tile's rows (sdiag[0..127]) and columns (sdiag[128..255])
    {
        const int q = th & 127, c = th >> 7;
        const int blkq = c ? j : i, cnt = c ? cj : ci;
        double v = 1.0;
        if (q < cnt) {
            const double d = tl.t64(blkq, blkq).at(q, q);
            v = d > 0.0 ? 1.0 / sqrt(d) : __builtin_nan("");
        }
        sdiag[c * TB + q] = v;
    }
    __syncthreads();
    const Mat<double> A = tl.t64(i, j);
    const Mat<float> L = lp_tile(ts, i, j);
    int bad = 0;
    const bool rfast = A.rs == 1;
    for (int e = th; e < TB * TB; e += 256) {
        const int r = rfast ? e % TB : e / TB, c = rfast ? e / TB : e % TB;
        if (r < ci && c < cj && (i != j || r >= c)) {
            double v = (A.at(r, c) * sdiag[r]) * sdiag[TB + c];
            if (i == j && r == c) v = v + a.shift;
            const float f = (float)(v * mu);
            L.at(r, c) = f;
            bad |= !__builtin_isfinite(f);
        }
    }
    bad = __syncthreads_or(bad);
    if (bad && th == 0) atomicOr(&S.flags, F_NONFINITE);
}

// Forward (L Y = B) then backward (L^T X = Y) substitution over the block
// rows with the tile inverses, on an n x r slab (column-major, ld): with the
// FP64 tiles (T = double, LPT false) or the low-precision tiles (LPT), in
// FP32 or FP64 arithmetic.
template <typename T, bool LPT>
__device__ void tile_solve(const Tiles& tl, const TileScratch& ts, T* b, int64_t ld, int r)
{
    // TF: the factor's storage (the low-precision tiles for an FP32 solve or
    // an FP64 solve with FP32 tiles, else the FP64 array)
    typedef typename std::conditional<LPT, float, T>::type TF;
    const int nb = tl.nb;
    TF* w;
    if constexpr (LPT) w = ts.w32;
    else w = ts.w64;
    auto tileT = [&](int i, int j) -> Mat<const TF> {
        if constexpr (LPT) return lp_tile(ts, i, j);
        else return tl.t64(i, j);
    };
    auto slab = [&](int k) { return Mat<T>{b + tl.r0(k), 1, ld}; };
    for (int k = 0; k < nb; k++) {
        const Mat<T> Bk = slab(k);
        for (int j = 0; j < k; j++)
            wg_mm<T, 1, 0, TF>(tl.cnt(k), r, tl.cnt(j), T(-1), tileT(k, j), TRI_NONE, Mat<const T>(slab(j)).tr(),
                               TRI_NONE, T(1), Bk, false);
        wg_mm<T, 1, 0, TF>(tl.cnt(k), r, tl.cnt(k), T(1), diag_inv(w, k), TRI_LOWER, Mat<const T>(Bk).tr(), TRI_NONE,
                           T(0), Bk, false);
    }
    for (int k = nb - 1; k >= 0; k--) {
        const Mat<T> Bk = slab(k);
        for (int j = k + 1; j < nb; j++)
            wg_mm<T, 1, 0, TF>(tl.cnt(k), r, tl.cnt(j), T(-1), tileT(j, k).tr(), TRI_NONE,
                               Mat<const T>(slab(j)).tr(), TRI_NONE, T(1), Bk, false);
        wg_mm<T, 1, 0, TF>(tl.cnt(k), r, tl.cnt(k), T(1), Mat<const TF>(diag_inv(w, k)).tr(), TRI_UPPER,
                           Mat<const T>(Bk).tr(), TRI_NONE, T(0), Bk, false);
    }
}

// Block row i of R += alpha A X (n x nrhs pairs, leading dimension n): the
// tiles (i, j), j <= i, and the mirrored (j, i)^T, j > i, of the FP64 array.
__device__ void rowblock_symm(const Tiles& tl, int i, const double* x, double* rr, int64_t n, int64_t nrhs,
                              double alpha)
{
    const int ci = tl.cnt(i);
    for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
        const int r = (int)(nrhs - c0 < RC ? nrhs - c0 : RC);
        const Mat<double> R{rr + tl.r0(i) + c0 * n, 1, n};
        for (int j = 0; j < tl.nb; j++) {
            const Mat<const double> X{x + tl.r0(j) + c0 * n, 1, n};
            if (j < i) {
                wg_mm<double, 1>(ci, r, tl.cnt(j), alpha, tl.t64(i, j), TRI_NONE, X.tr(), TRI_NONE, 1.0, R, false);
            } else if (j == i) {
                wg_mm<double, 1>(ci, r, ci, alpha, tl.t64(i, i), TRI_LOWER, X.tr(), TRI_NONE, 1.0, R, false);
                wg_mm<double, 1>(ci, r, ci, alpha, Mat<const double>(tl.t64(i, i)).tr(), TRI_SUPPER, X.tr(),
                                 TRI_NONE, 1.0, R, false);
            } else {
                wg_mm<double, 1>(ci, r, tl.cnt(j), alpha, Mat<const double>(tl.t64(j, i)).tr(), TRI_NONE, X.tr(),
                                 TRI_NONE, 1.0, R, false);
            }
        }
    }
}

// z = mu D^{-1/2} (Ls Ls^T)^{-1} D^{-1/2} r over all right-hand sides (the
// low-precision preconditioner, solved with the FP32 tiles and tile
// inverses), in FP32 into z or added into it, or (fp64, for the
// conjugate-gradient steps) in FP64 arithmetic, which keeps the operator it
// applies symmetric to FP64 rounding.
__device__ void tile_prec(const BatchArgs& a, const Tiles& tl, const TileScratch& ts, int64_t n, int64_t nrhs,
                          const double* rin, double* z, bool add, bool fp64 = false)
{
    const int th = threadIdx.x;
    const double mu = a.mode == 2 ? MU_FP16 : 1.0;
    if (fp64) {
        for (int64_t e = th; e < n * nrhs; e += 256) z[e] = ts.sv[e % n] * rin[e];
        __syncthreads();
        for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
            const int r = (int)(nrhs - c0 < RC ? nrhs - c0 : RC);
            tile_solve<double, true>(tl, ts, z + c0 * n, n, r);
        }
        for (int64_t e = th; e < n * nrhs; e += 256) z[e] = (z[e] * ts.sv[e % n]) * mu;
        __syncthreads();
        return;
    }
    for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
        const int r = (int)(nrhs - c0 < RC ? nrhs - c0 : RC);
        for (int64_t e = th; e < n * r; e += 256) {
            const int64_t i = e % n, c = c0 + e / n;
            ts.rf[i + c * n] = (float)(ts.sv[i] * rin[i + c * n]);
        }
        __syncthreads();
        tile_solve<float, true>(tl, ts, ts.rf + c0 * n, n, r);
        for (int64_t e = th; e < n * r; e += 256) {
            const int64_t i = e % n, c = c0 + e / n;
            const double d = ((double)ts.rf[i + c * n] * ts.sv[i]) * mu;
            z[i + c * n] = add ? z[i + c * n] + d : d;
        }
        __syncthreads();
    }
}

// Refinement tasks of a tiled system.
__device__ __attribute__((noinline)) void ir_task(const BatchArgs& a, SysState& S, const Tiles& tl, const TileScratch& ts, const rfp_sys_t& sd,
                        int64_t loc, int64_t t, double* red)
{
    const int th = threadIdx.x;
    const int64_t n = sd.n, nrhs = sd.nrhs;
    double* b = a.b + sd.b_off;
    if (loc == IR_SETUP) {
        if (S.flags & (F_LPFAIL | F_NONFINITE)) {
            if (th == 0) {
                S.code = (S.flags & F_NONFINITE) ? -4 : -3;
                S.flags |= F_NEED64;
                S.cfail = 0;
                S.jump = IR_LEVELS;
            }
            return;
        }
        for (int64_t i = th; i < n; i += 256) {
            const int bi = i < tl.m1 ? (int)(i / TB) : tl.nb1 + (int)((i - tl.m1) / TB);
            const int64_t q = i - tl.r0(bi);
            const double d = tl.t64(bi, bi).at(q, q);
            ts.sv[i] = d > 0.0 ? 1.0 / sqrt(d) : __builtin_nan("");
            ts.rs[i] = 0.0;
        }
        __syncthreads();
        // row sums of |A| over the tiles: each tile adds to its rows and, off
        // the diagonal, to its columns (the mirrored entries)
        for (int i = 0; i < tl.nb; i++)
            for (int j = 0; j <= i; j++) {
                const Mat<double> A = tl.t64(i, j);
                const int ci = tl.cnt(i), cj = tl.cnt(j);
                if (th < ci) {
                    double s = 0.0;
                    for (int c = 0; c < cj; c++)
                        if (i != j || c <= th) s += fabs(A.at(th, c));
                    ts.rs[tl.r0(i) + th] += s;
                }
                __syncthreads();
                if (th < cj) {
                    double s = 0.0;
                    for (int r = 0; r < ci; r++)
                        if (i != j || r > th) s += fabs(A.at(r, th));
                    ts.rs[tl.r0(j) + th] += s;
                }
                __syncthreads();
            }
        double m = 0.0;
        for (int64_t i = th; i < n; i += 256) m = nanmax(m, ts.rs[i]);
        m = wg_max(m, red);
        for (int64_t e = th; e < n * nrhs; e += 256) {
            const int64_t i = e % n, c = e / n;
            ts.xv[e] = 0.0;
            ts.rv[e] = b[i + c * sd.ldb];
        }
        for (int64_t c = th; c < nrhs; c += 256) {
            double bmx = 0.0;
            for (int64_t i = 0; i < n; i++) bmx = nanmax(bmx, fabs(b[i + c * sd.ldb]));
            ts.bm[c] = bmx;
        }
        if (th == 0) {
            S.anorm = m;
            S.sweep = 0;
            S.pcg = 0;
            S.cgstep = 0;
            S.cgcont = 0;
            S.stale = 0;
            S.best = 0.0;
            S.prev = 0.0;
            S.code = 0;
            S.jump = nrhs > 0 ? IR_SOLVE : IR_LEVELS;
        }
        return;
    }
    if (loc == IR_SOLVE) {
        // x += mu D^{-1/2} (Ls Ls^T)^{-1} D^{-1/2} r
        tile_prec(a, tl, ts, n, nrhs, ts.rv, ts.xv, true);
        return;
    }
    if (loc == IR_RESID || loc == CG_Q) {
        // block row i of r = b - A x, or of q = A p
        const int i = (int)t;
        const int ci = tl.cnt(i);
        const bool res = loc == IR_RESID;
        double* out = res ? ts.rv : ts.qv;
        for (int64_t e = th; e < ci * nrhs; e += 256) {
            const int64_t q = e % ci, c = e / ci;
            out[tl.r0(i) + q + c * n] = res ? b[tl.r0(i) + q + c * sd.ldb] : 0.0;
        }
        __syncthreads();
        rowblock_symm(tl, i, res ? ts.xv : ts.pv, out, n, nrhs, res ? -1.0 : 1.0);
        return;
    }
    if (loc == CG_Z) {
        // z = M^{-1} r into q's storage; rz' = r . z; p = z + (rz' / rz) p
        // (p = z when the recurrence starts)
        tile_prec(a, tl, ts, n, nrhs, ts.rv, ts.qv, false, true);
        const bool first = S.cgcont == 0;
        for (int64_t c = 0; c < nrhs; c++) {
            double s = 0.0;
            for (int64_t i = th; i < n; i += 256) s += ts.rv[i + c * n] * ts.qv[i + c * n];
            s = wg_sum(s, red);
            const double rz = ts.rz[c];
            const double beta = (!first && rz != 0.0) ? s / rz : 0.0;
            for (int64_t i = th; i < n; i += 256) {
                const int64_t o = i + c * n;
                ts.pv[o] = first ? ts.qv[o] : ts.qv[o] + beta * ts.pv[o];
            }
            __syncthreads();
            if (th == 0) ts.rz[c] = s;
        }
        if (th == 0) S.cgcont = 1;
        return;
    }
    if (loc == CG_UPD) {
        // alpha = rz / (p . q); x += alpha p; r -= alpha q (the recursive
        // residual); a sweep ends after PCG_STEPS steps, or earlier once the
        // recursive residual meets the tolerance
        double eta = 0.0;
        for (int64_t c = 0; c < nrhs; c++) {
            double s = 0.0;
            for (int64_t i = th; i < n; i += 256) s += ts.pv[i + c * n] * ts.qv[i + c * n];
            s = wg_sum(s, red);
            const double al = s != 0.0 ? ts.rz[c] / s : 0.0;
            double rm = 0.0, xm = 0.0;
            for (int64_t i = th; i < n; i += 256) {
                const int64_t o = i + c * n;
                ts.xv[o] += al * ts.pv[o];
                ts.rv[o] -= al * ts.qv[o];
                rm = nanmax(rm, fabs(ts.rv[o]));
                xm = nanmax(xm, fabs(ts.xv[o]));
            }
            rm = wg_max(rm, red);
            xm = wg_max(xm, red);
            eta = nanmax(eta, col_eta(rm, xm, ts.bm[c], S.anorm));
        }
        if (th == 0) {
            S.cgstep++;
            S.jump = (S.cgstep >= PCG_STEPS || eta <= a.tol) ? IR_RESID : CG_Z;
        }
        return;
    }
    // IR_DECIDE: normwise backward error over all right-hand sides
    double eta = 0.0;
    for (int64_t c = 0; c < nrhs; c++) {
        double rm = 0.0, xm = 0.0;
        for (int64_t i = th; i < n; i += 256) {
            rm = nanmax(rm, fabs(ts.rv[i + c * n]));
            xm = nanmax(xm, fabs(ts.xv[i + c * n]));
        }
        rm = wg_max(rm, red);
        xm = wg_max(xm, red);
        eta = nanmax(eta, col_eta(rm, xm, ts.bm[c], S.anorm));
    }
    const int it = S.sweep + 1;
    const bool swept_pcg = S.pcg != 0;
    const bool better = eta < 0.9 * S.best;
    const int stale = swept_pcg ? (better ? 0 : S.stale + 1) : 0;
    int done = 0;  // 1 converged, -1 max_iter, -2 stalled
    if (eta <= a.tol) done = 1;
    else if (swept_pcg && stale >= IR_STALE_SWEEPS) done = -2;
    else if (it >= a.max_iter) done = -1;
    if (done == 1) {
        for (int64_t e = th; e < n * nrhs; e += 256) {
            const int64_t i = e % n, c = e / n;
            b[i + c * sd.ldb] = ts.xv[e];
        }
    }
    __syncthreads();
    if (th == 0) {
        const double prev = S.prev;
        S.sweep = it;
        S.prev = eta;
        if (done == 1) {
            S.code = it;
            S.jump = IR_LEVELS;
        } else if (done < 0) {
            S.code = done;
            S.flags |= F_NEED64;
            S.cfail = 0;
            S.jump = IR_LEVELS;
        } else {
            if (swept_pcg) {
                S.stale = stale;
                if (better) S.best = eta;
            } else if (it > 1 && !(eta < 0.25 * prev)) {
                S.pcg = 1;
                S.best = eta < prev ? eta : prev;
                S.stale = 0;
            }
            S.cgstep = 0;
            S.jump = S.pcg ? CG_Z : IR_SOLVE;
        }
    }
}

// Inversion tasks (FP64 tiles, after the FP64 factor).
// Y(k): tile (j,k) <- L_jk W_kk (in place)
__device__ __attribute__((noinline)) void trtri_y(const Tiles& tl, const TileScratch& ts, int k, int j, BatchSmem& sm)
{
    tile::Acc<double> acc;
    acc.zero();
    const Mat<double> Y = tl.t64(j, k);
    tile::mma<double, 0>(sm.gd, acc, tl.cnt(j), tl.cnt(k), tl.cnt(k), Y, TRI_NONE,
                         Mat<const double>(diag_inv(ts.w64, k)).tr(), TRI_UPPER);
    tile::store<double>(acc, tl.cnt(j), tl.cnt(k), 1.0, 0.0, Y, false);
}

// A(k): X_i = -sum_{j=k+1..i} W_ij Y_j into the scratch column
__device__ __attribute__((noinline)) void trtri_x(const Tiles& tl, const TileScratch& ts, int k, int i, BatchSmem& sm)
{
    tile::Acc<double> acc;
    acc.zero();
    for (int j = k + 1; j <= i; j++)
        tile::mma<double, 0>(sm.gd, acc, tl.cnt(i), tl.cnt(k), tl.cnt(j), tl.t64(i, j), j == i ? TRI_LOWER : TRI_NONE,
                             Mat<const double>(tl.t64(j, k)).tr(), TRI_NONE);
    tile::store<double>(acc, tl.cnt(i), tl.cnt(k), -1.0, 0.0, Mat<double>{ts.tmp + (int64_t)i * TB * TB, TB, 1},
                        false);
}

__device__ __attribute__((noinline)) void trtri_task(const Tiles& tl, const TileScratch& ts, int64_t loc, int64_t t,
                                                     BatchSmem& sm)
{
    const int nb = tl.nb, th = threadIdx.x;
    if (loc == 0) {
        // tile (k,k) <- W_kk (its lower triangle)
        const int k = (int)t, c = tl.cnt(k);
        const Mat<double> D = tl.t64(k, k);
        const double* w = ts.w64 + (int64_t)k * TB * TB;
        const bool rfast = D.rs == 1;
        for (int e = th; e < TB * TB; e += 256) {
            const int r = rfast ? e % TB : e / TB, q = rfast ? e / TB : e % TB;
            if (r < c && q <= r) D.at(r, q) = w[r * TB + q];
        }
        return;
    }
    const int k = nb - 2 - (int)((loc - 1) / 3), sub = (int)((loc - 1) % 3);
    const int i = k + 1 + (int)t;
    if (sub == 0) {
        trtri_y(tl, ts, k, i, sm);
        return;
    }
    if (sub == 1) {
        trtri_x(tl, ts, k, i, sm);
        return;
    }
    // tile (i,k) <- X_i
    const Mat<double> X{ts.tmp + (int64_t)i * TB * TB, TB, 1};
    const Mat<double> D = tl.t64(i, k);
    const int ci = tl.cnt(i), ck = tl.cnt(k);
    const bool rfast = D.rs == 1;
    for (int e = th; e < TB * TB; e += 256) {
        const int r = rfast ? e % TB : e / TB, q = rfast ? e / TB : e % TB;
        if (r < ci && q < ck) D.at(r, q) = X.at(r, q);
    }
}

__device__ __attribute__((noinline)) void lauum_task(const Tiles& tl, int64_t loc, int64_t t, BatchSmem& sm)
{
    const int nb = tl.nb;
    int i, j;
    if (loc == 0) {
        i = 0;
        j = 0;
    } else {
        i = (int)((loc + 1) / 2);
        j = ((loc + 1) % 2 == 0) ? (int)t : i;
    }
    // (W^T W)_ij = sum_{q >= i} W_qi^T W_qj
    tile::Acc<double> acc;
    acc.zero();
    for (int q = i; q < nb; q++)
        tile::mma<double, 0>(sm.gd, acc, tl.cnt(i), tl.cnt(j), tl.cnt(q), Mat<const double>(tl.t64(q, i)).tr(),
                             q == i ? TRI_UPPER : TRI_NONE, Mat<const double>(tl.t64(q, j)).tr(),
                             q == j ? TRI_UPPER : TRI_NONE);
    tile::store<double>(acc, tl.cnt(i), tl.cnt(j), 1.0, 0.0, tl.t64(i, j), i == j);
}

// The FP64 solve of a tiled system (columns cfail .. nrhs - 1).
__device__ __attribute__((noinline)) void solve_task(const BatchArgs& a, const SysState& S, const Tiles& tl, const TileScratch& ts,
                           const rfp_sys_t& sd)
{
    for (int64_t c0 = S.cfail; c0 < sd.nrhs; c0 += RC) {
        const int r = (int)(sd.nrhs - c0 < RC ? sd.nrhs - c0 : RC);
        tile_solve<double, false>(tl, ts, a.b + sd.b_off + c0 * sd.ldb, sd.ldb, r);
    }
}

// Is a level of this stage skipped, given the system's flags?
__device__ bool skipped(const BatchArgs& a, const SysState& S, const rfp_sys_t& sd, int stage)
{
    switch (stage) {
        case ST_LPFAC: return (S.flags & (F_LPFAIL | F_NONFINITE)) != 0;
        case ST_F64FAC: return (a.mode != 0 && !(S.flags & F_NEED64) && !a.pftri) || (S.flags & F_F64FAIL);
        case ST_SOLVE:
            return (a.mode != 0 && !(S.flags & F_NEED64)) || (S.flags & F_F64FAIL) || sd.nrhs == 0;
        case ST_TRTRI:
        case ST_LAUUM: return !a.pftri || (S.flags & F_F64FAIL);
        default: return false;
    }
}

// Queue entry: system (26 bits) | level (18 bits) | task (20 bits).
__device__ __forceinline__ unsigned long long entry(int64_t s, int64_t level, int64_t t)
{
    return ((unsigned long long)s << 38) | ((unsigned long long)level << 20) | (unsigned long long)t;
}

// count tasks from entry base into the queue; false when the queue is full
__device__ bool push(const BatchArgs& a, unsigned long long base, int64_t count)
{
    const unsigned long long p0 = atomicAdd(&a.ctl[1], (unsigned long long)count);
    for (int64_t c = 0; c < count; c++) {
        const unsigned long long p = p0 + (unsigned long long)c;
        if ((int64_t)p >= a.qcap) return false;
        __hip_atomic_store(&a.q[p], base + (unsigned long long)c + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

__device__ void finish(const BatchArgs& a, int64_t s, SysState& S)
{
    a.info[s] = S.info;
    a.iter[s] = a.mode == 0 ? 0 : S.code;
    S.kind = K_DONE;
    release();
    __hip_atomic_fetch_add(&a.ctl[2], ~0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// After the current level of system s is complete (or at the start): queue
// its next level that is not skipped, or finish the system.  One thread.
__device__ void advance(const BatchArgs& a, int64_t s, SysState& S, const rfp_sys_t& sd)
{
    const int nb = S.nb1 + S.nb2;
    int stage;
    int64_t loc;
    int64_t ell = S.level + 1;
    if (locate(S.level, nb, a.mode, &stage, &loc) && stage == ST_IR &&
        (loc == IR_SETUP || loc == IR_DECIDE || loc == CG_UPD))
        ell = stage_start(ST_IR, nb, a.mode) + S.jump;
    for (;; ell++) {
        if (!locate(ell, nb, a.mode, &stage, &loc)) {
            finish(a, s, S);
            return;
        }
        if (skipped(a, S, sd, stage)) continue;
        const int64_t cnt = level_tasks(stage, loc, nb);
        if (cnt == 0) continue;
        S.level = (int)ell;
        S.ntask = (int)cnt;
        S.done = 0;
        release();
        if (!push(a, entry(s, ell, 0), cnt)) __hip_atomic_store(&a.ctl[3], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
}

}  // namespace

#ifndef RFP_BATCHED_X2
// Setup: per-system plan and scratch offsets (one workgroup, scan over the
// systems in chunks of 256); the control words.
__global__ __launch_bounds__(256) void batched_setup_kernel(BatchArgs a)
{
    __shared__ int64_t part[256];
    __shared__ int64_t base_sh;
    const int t = threadIdx.x;
    if (t == 0) base_sh = 0;
    __syncthreads();
    int64_t remaining = 0;
    for (int64_t c0 = 0; c0 < a.batch; c0 += 256) {
        const int64_t id = c0 + t;
        SysPlan p{K_NONE, 0, 0, 0, 0};
        if (id < a.batch) p = plan_of(a.sys[id], a.mode, a.pftri, a.max_iter);
        part[t] = p.bytes;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int64_t v = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        const int64_t off = base_sh + part[t] - p.bytes;
        if (id < a.batch) {
            SysState& S = a.st[id];
            S.off = off;
            S.kind = p.kind;
            if (p.kind == K_TILED && off + p.bytes > a.sysmem_bytes) S.kind = K_NONE;  // no room: refused
            S.nb1 = p.nb1;
            S.nb2 = p.nb2;
            S.level = -1;
            S.ntask = 0;
            S.done = 0;
            S.flags = 0;
            S.info = 0;
            S.code = 0;
            S.cfail = 0;
            S.jump = 0;
            S.sweep = 0;
            S.pcg = 0;
            S.cgstep = 0;
            S.cgcont = 0;
            S.stale = 0;
            S.best = 0.0;
            S.prev = 0.0;
            S.anorm = 0.0;
            if (S.kind == K_NONE) {
                // n = 0 with a legal layout is a quick return; anything else is refused
                RfpBlocks blk;
                const rfp_sys_t sd = a.sys[id];
                const bool empty = sd.n == 0 && rfp_blocks(sd.transr, sd.uplo, 0, &blk);
                a.info[id] = empty ? 0 : -1;
                a.iter[id] = 0;
                S.kind = K_DONE;
            } else {
                remaining++;
            }
        }
        __syncthreads();
        if (t == 255) base_sh += part[255];
        __syncthreads();
    }
    part[t] = remaining;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) part[t] += part[t + o];
        __syncthreads();
    }
    if (t == 0) {
        a.ctl[0] = 0;
        a.ctl[1] = 0;
        a.ctl[2] = (unsigned long long)part[0];
        a.ctl[3] = 0;
    }
}

__global__ void zero_u64_kernel(unsigned long long* p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

// The first level of every system into the queue.
__global__ __launch_bounds__(256) void batched_queue_kernel(BatchArgs a)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.batch) return;
    SysState& S = a.st[id];
    if (S.kind == K_SMALL) {
        S.level = 0;
        S.ntask = 1;
        if (!push(a, entry(id, 0, 0), 1)) __hip_atomic_store(&a.ctl[3], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (S.kind == K_TILED) {
        advance(a, id, S, a.sys[id]);
    }
}

// Systems the persistent kernel did not finish (queue full, a wait that ran
// out): info = -2.
__global__ void batched_finish_kernel(BatchArgs a)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.batch) return;
    if (a.st[id].kind != K_DONE) {
        a.info[id] = -2;
        a.iter[id] = 0;
    }
}

#endif

// The persistent loop, built twice: batched_kernel runs one workgroup per
// compute unit, which leaves the tile tasks of systems with n > 256 their
// full register budget; batched_kernel_x2 runs two (at most 256 registers a
// lane, some spilled, and two 78 KB LDS blocks per CU), which hides more of
// the per-system latency of a batch that holds only one-task systems.  The
// second is built in its own translation unit (batched_x2.hip includes this
// file with RFP_BATCHED_X2 defined): the loop's callees are compiled once
// per unit, and only there do they all get the smaller register budget.
__device__ __forceinline__ void batched_loop(const BatchArgs& a)
{
    __shared__ BatchSmem sm;
    __shared__ double red[4];
    __shared__ unsigned long long slot;
    __shared__ int go;
    const int t = threadIdx.x;
    const WgScratch ws = wg_scratch(a.wgs + (size_t)blockIdx.x * wg_scratch_bytes());
    for (;;) {
        if (t == 0) {
            const unsigned long long p = atomicAdd(&a.ctl[0], 1ull);
            go = 0;
            if ((int64_t)p < a.qcap) {
                int64_t spins = 0;
                for (;;) {
                    const unsigned long long v = __hip_atomic_load(&a.q[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    if (v) {
                        slot = v - 1;
                        go = 1;
                        break;
                    }
                    if (__hip_atomic_load(&a.ctl[2], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
                    if (__hip_atomic_load(&a.ctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                    if (++spins > a.spin_limit) {
                        __hip_atomic_store(&a.ctl[3], 2ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            acquire();
        }
        __syncthreads();
        if (!go) break;
        const unsigned long long e = slot;
        __syncthreads();
        const int64_t s = (int64_t)(e >> 38), ell = (int64_t)((e >> 20) & 0x3ffff), tk = (int64_t)(e & 0xfffff);
        SysState& S = a.st[s];
        if (S.kind == K_SMALL) {
            small_system(a, s, sm, red, ws);
            if (t == 0) {
                S.kind = K_DONE;
                release();
                __hip_atomic_fetch_add(&a.ctl[2], ~0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            continue;
        }
        const rfp_sys_t sd = a.sys[s];
        RfpBlocks blk;
        rfp_blocks(sd.transr, sd.uplo, sd.n, &blk);
        Tiles tl;
        tl.v = rfp_view(blk, a.arf + sd.arf_off);
        tl.nb1 = S.nb1;
        tl.nb = S.nb1 + S.nb2;
        tl.m1 = blk.m1;
        tl.n = sd.n;
        const TileScratch ts = tile_scratch(a.sysmem + S.off, sd.n, sd.nrhs, tl.nb, a.mode, a.pftri);
        int stage = ST_END;
        int64_t loc = 0;
        locate(ell, tl.nb, a.mode, &stage, &loc);
        switch (stage) {
            case ST_CAST: cast_task(a, S, tl, ts, tk, sm.sdiag); break;
            case ST_LPFAC:
                if (loc % 3 == 0) fac_p_task<true>(S, tl, ts, (int)(loc / 3), sm);
                else fac_gemm_task<true>(a, tl, ts, (int)(loc / 3), (int)(loc % 3), tk, sm);
                break;
            case ST_IR: ir_task(a, S, tl, ts, sd, loc, tk, red); break;
            case ST_F64FAC:
                if (loc % 3 == 0) fac_p_task<false>(S, tl, ts, (int)(loc / 3), sm);
                else fac_gemm_task<false>(a, tl, ts, (int)(loc / 3), (int)(loc % 3), tk, sm);
                break;
            case ST_SOLVE: solve_task(a, S, tl, ts, sd); break;
            case ST_TRTRI: trtri_task(tl, ts, loc, tk, sm); break;
            case ST_LAUUM: lauum_task(tl, loc, tk, sm); break;
            default: break;
        }
        __syncthreads();
        if (t == 0) {
            release();
            const int prev = __hip_atomic_fetch_add(&S.done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (prev + 1 == S.ntask) {
                acquire();
                advance(a, s, S, sd);
            }
        }
        __syncthreads();
    }
}

#ifdef RFP_BATCHED_X2
__global__ __launch_bounds__(256, 2) void batched_kernel_x2(BatchArgs a) { batched_loop(a); }

hipError_t launch_batched_x2(unsigned wgs, hipStream_t stream, const BatchArgs& a)
{
    hipLaunchKernelGGL(batched_kernel_x2, dim3(wgs), dim3(256), 0, stream, a);
    return hipGetLastError();
}
#else
__global__ __launch_bounds__(256, 1) void batched_kernel(BatchArgs a) { batched_loop(a); }

// batched_x2.hip: the same loop built for two workgroups per compute unit
hipError_t launch_batched_x2(unsigned wgs, hipStream_t stream, const BatchArgs& a);

hipError_t batched_solve(const Exec& ex, const rfp_sys_t* sys, int64_t batch, double* arf, double* b, int mode,
                         int pftri, double tol, double shift, int max_iter, int* info, int* iter, char* wgs_mem,
                         int wgs, int occ, char* sysmem, int64_t sysmem_bytes, void* st, unsigned long long* q,
                         int64_t qcap, unsigned long long* ctl)
{
    if (batch <= 0) return hipSuccess;
    BatchArgs a{sys, batch, arf, b, mode, pftri, tol, shift, max_iter, info, iter, wgs_mem, sysmem, sysmem_bytes,
                (SysState*)st, q, qcap, ctl, (int64_t)1 << 26};
    hipLaunchKernelGGL(batched_setup_kernel, dim3(1), dim3(256), 0, ex.stream, a);
    const int64_t zb = std::min<int64_t>((qcap + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)std::max<int64_t>(zb, 1)), dim3(256), 0, ex.stream, q, qcap);
    const unsigned sb = (unsigned)((batch + 255) / 256);
    hipLaunchKernelGGL(batched_queue_kernel, dim3(sb), dim3(256), 0, ex.stream, a);
    if (occ == 2) {
        ProfScope ps(ex, "rfp::batched_kernel_x2(rfp::BatchArgs)", 0.0, 0.0);
        const hipError_t e = launch_batched_x2((unsigned)wgs, ex.stream, a);
        if (e != hipSuccess) return e;
    } else {
        ProfScope ps(ex, "rfp::batched_kernel(rfp::BatchArgs)", 0.0, 0.0);
        hipLaunchKernelGGL(batched_kernel, dim3((unsigned)wgs), dim3(256), 0, ex.stream, a);
    }
    hipLaunchKernelGGL(batched_finish_kernel, dim3(sb), dim3(256), 0, ex.stream, a);
    return hipGetLastError();
}
#endif

}  // namespace rfp
