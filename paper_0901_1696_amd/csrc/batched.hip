// Batched solver for many small SPD systems of uneven order (n <= 256), each
// in its own RFP layout: one persistent launch in which every workgroup takes
// systems from a work counter and runs, for each, the paper's four-step
// factorization (Section 3: POTRF of T1, TRSM of S, SYRK of T2, POTRF of T2),
// the solve (Section 4) and optionally the inversion (Section 5), all inside
// the workgroup.  With n <= 256 both diagonal blocks have order <= 128, so
// every diagonal block is one fused LDS leaf (potrf128_block) that also
// yields the inverse of its factor; the off-diagonal steps are products of
// at most 128 x 128 blocks on MFMA (wg_mm), with the inverses replacing the
// triangular solves.
//
// Two modes: plain FP64 (factor, solve and inverse in place, as PFTRF /
// PFTRS / PFTRI), and an FP32 factor of the diagonally scaled matrix with
// FP64 iterative refinement (the FP64 matrix stays untouched unless the
// refinement falls back to the FP64 factor).  No host synchronisation and no
// allocation inside: the call can be captured in a HIP graph.
#include <cstdio>

#include "leaf128.h"
#include "rfp.h"

namespace rfp {

namespace {

constexpr int BN = 128;   // diagonal block capacity
constexpr int RC = 16;    // right-hand-side columns per pass
constexpr int NMAX = 2 * BN;

// C(m x n) = alpha A(m x k) B(n x k)^T + beta C on one workgroup, every
// dimension of C at most 128 (n at most 16 * NCB).  Operands are read from
// global memory (L2-resident for these sizes) under band masks; all products
// are formed in registers first and stored after a barrier, so C may alias A
// or B in any way.  Only i >= j is written when c_lower.
template <typename T, int NCB>
__device__ void wg_mm(int m, int n, int k, T alpha, Mat<const T> A, int triA, Mat<const T> B, int triB, T beta,
                      Mat<T> C, bool c_lower)
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
        for (int kk = 0; kk < k; kk += 4) {
            const int ka = kk + g;
            const int64_t da = ka - i;
            const T av = (i < m && ka < k && da >= alo && da <= ahi) ? A.at(i, ka) : T(0);
#pragma unroll
            for (int c = 0; c < NCB; c++) {
                if (c >= ncb) break;
                const int j = c * 16 + r;
                const int64_t db = ka - j;
                const T bv = (j < n && ka < k && db >= blo && db <= bhi) ? B.at(j, ka) : T(0);
                acc[s][c] = M16<T>::op(av, bv, acc[s][c]);
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
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = strip * 16 + M16<T>::row(lane, e), j = c * 16 + r;
                if (i < m && j < n && (!c_lower || i >= j)) {
                    T v = alpha * acc[s][c][e];
                    if (beta != T(0)) v += beta * C.at(i, j);
                    C.at(i, j) = v;
                }
            }
        }
    }
    __syncthreads();
}

// Scratch of one workgroup (device memory, 256-byte aligned pieces).
struct WgScratch {
    double *w1, *w2;          // FP64 inverses of L11, L22 (128 x 128 row-major)
    float *f1, *fs, *f2;      // FP32 scaled copies of T1, S, T2 (128 x 128 column-major)
    float *w1f, *w2f;         // FP32 inverses
    double *sv;               // diagonal scaling (NMAX)
    double *xv, *rv;          // refinement solution and residual (NMAX x RC, column-major)
    float* rf;                // FP32 correction (NMAX x RC)
};

__device__ __forceinline__ size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

__host__ __device__ inline size_t wg_scratch_bytes()
{
    auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 2 * a(sizeof(double) * BN * BN) + 5 * a(sizeof(float) * BN * BN) + a(sizeof(double) * NMAX) +
           2 * a(sizeof(double) * NMAX * RC) + a(sizeof(float) * NMAX * RC);
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
    return s;
}

union BatchSmem {
    Leaf128Smem<double> d;
    Leaf128Smem<float> f;
};

// Symmetric element A(i, j) of a system through its lower views.
__device__ __forceinline__ double sym_at(const RfpView<double>& v, int i, int j)
{
    if (i < j) {
        const int q = i;
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
// the triangular solves done by the inverses).
template <typename T>
__device__ void solve_slab(int m1, int m2, Mat<const T> s, const T* w1, const T* w2, T* b, int64_t ld, int r)
{
    Mat<T> B1{b, 1, ld}, B2{b + m1, 1, ld};
    Mat<const T> W1{w1, BN, 1}, W2{w2, BN, 1};
    wg_mm<T, 1>(m1, r, m1, T(1), W1, TRI_LOWER, Mat<const T>(B1).tr(), TRI_NONE, T(0), B1, false);
    if (m2 > 0) {
        wg_mm<T, 1>(m2, r, m1, T(-1), s, TRI_NONE, Mat<const T>(B1).tr(), TRI_NONE, T(1), B2, false);
        wg_mm<T, 1>(m2, r, m2, T(1), W2, TRI_LOWER, Mat<const T>(B2).tr(), TRI_NONE, T(0), B2, false);
        wg_mm<T, 1>(m2, r, m2, T(1), W2.tr(), TRI_UPPER, Mat<const T>(B2).tr(), TRI_NONE, T(0), B2, false);
        wg_mm<T, 1>(m1, r, m2, T(-1), s.tr(), TRI_NONE, Mat<const T>(B2).tr(), TRI_NONE, T(1), B1, false);
    }
    wg_mm<T, 1>(m1, r, m1, T(1), W1.tr(), TRI_UPPER, Mat<const T>(B1).tr(), TRI_NONE, T(0), B1, false);
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

// max over the block's threads (non-negative values; NaN wins)
__device__ double wg_max(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + s];
            red[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    const double out = red[0];
    __syncthreads();
    return out;
}

}  // namespace

struct BatchArgs {
    const rfp_sys_t* sys;
    int64_t batch;
    double* arf;
    double* b;
    int mode;       // 0 FP64; 1 FP32 factor + FP64 refinement
    int pftri;
    double tol;
    int max_iter;
    int* info;
    int* iter;
    int* counter;   // work counter, zero at launch
    char* scratch;  // per-workgroup scratch, wg_scratch_bytes() each
};

__global__ __launch_bounds__(256) void batched_kernel(BatchArgs a)
{
    __shared__ BatchSmem sm;
    __shared__ double red[256];
    __shared__ int next;
    const int t = threadIdx.x;
    const WgScratch ws = wg_scratch(a.scratch + (size_t)blockIdx.x * wg_scratch_bytes());
    for (;;) {
        if (t == 0) next = atomicAdd(a.counter, 1);
        __syncthreads();
        const int64_t id = next;
        __syncthreads();
        if (id >= a.batch) break;
        const rfp_sys_t sd = a.sys[id];
        RfpBlocks blk;
        if (!rfp_blocks(sd.transr, sd.uplo, sd.n, &blk) || sd.n > NMAX) {
            if (t == 0) a.info[id] = -1;
            continue;
        }
        double* arf = a.arf + sd.arf_off;
        const RfpView<double> v = rfp_view(blk, arf);
        const int n = (int)sd.n, m1 = (int)blk.m1, m2 = (int)blk.m2;
        int code = 0, finfo = 0;
        bool need64 = a.mode == 0;
        int64_t c_fail = 0;  // first right-hand side left to the FP64 solve

        if (a.mode == 1 && n > 0) {
            // ---- FP32 factor of D^{-1/2} A D^{-1/2}
            for (int i = t; i < n; i += 256) {
                const double d = sym_at(v, i, i);
                ws.sv[i] = d > 0.0 ? 1.0 / sqrt(d) : __builtin_nan("");
            }
            __syncthreads();
            for (int idx = t; idx < BN * BN; idx += 256) {
                const int i = idx % BN, j = idx / BN;
                if (i < m1 && j <= i) ws.f1[idx] = (float)((v.t1.at(i, j) * ws.sv[i]) * ws.sv[j]);
                if (i < m2 && j < m1) ws.fs[idx] = (float)((v.s.at(i, j) * ws.sv[m1 + i]) * ws.sv[j]);
                if (i < m2 && j <= i) ws.f2[idx] = (float)((v.t2.at(i, j) * ws.sv[m1 + i]) * ws.sv[m1 + j]);
            }
            __syncthreads();
            const Mat<float> F1{ws.f1, 1, BN}, FS{ws.fs, 1, BN}, F2{ws.f2, 1, BN};
            int f = potrf128_block<float>(sm.f, F1, m1, ws.w1f, nullptr, 0);
            if (!f && m2 > 0) {
                wg_mm<float, 8>(m2, m1, m1, 1.f, FS, TRI_NONE, Mat<const float>{ws.w1f, BN, 1}, TRI_LOWER, 0.f, FS,
                                false);
                wg_mm<float, 8>(m2, m2, m1, -1.f, FS, TRI_NONE, FS, TRI_NONE, 1.f, F2, true);
                f = potrf128_block<float>(sm.f, F2, m2, ws.w2f, nullptr, 0);
            }
            if (f) {
                code = -3;
                need64 = true;
            } else {
                // ||A||_inf once per system (row sums of |A|)
                double rs = 0.0;
                for (int i = t; i < n; i += 256) {
                    double s = 0.0;
                    for (int j = 0; j < n; j++) s += fabs(sym_at(v, i, j));
                    rs = s > rs ? s : rs;
                }
                const double anorm = wg_max(rs, red);
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
                    double prev = 0.0;
                    int done = -1;
                    for (int it = 1; it <= a.max_iter; it++) {
                        for (int idx = t; idx < n * RC; idx += 256) {
                            const int i = idx % n, c = idx / n;
                            ws.rf[i + c * NMAX] = (float)(ws.sv[i] * ws.rv[i + c * NMAX]);
                        }
                        __syncthreads();
                        solve_slab<float>(m1, m2, FS, ws.w1f, ws.w2f, ws.rf, NMAX, r);
                        for (int idx = t; idx < n * RC; idx += 256) {
                            const int i = idx % n, c = idx / n;
                            ws.xv[i + c * NMAX] += (double)ws.rf[i + c * NMAX] * ws.sv[i];
                        }
                        __syncthreads();
                        // r = b - A x in FP64 from the untouched RFP matrix
                        for (int idx = t; idx < n * RC; idx += 256) {
                            const int i = idx % n, c = idx / n;
                            ws.rv[i + c * NMAX] = c < r ? bb[i + c * sd.ldb] : 0.0;
                        }
                        __syncthreads();
                        Mat<const double> X1{ws.xv, 1, NMAX}, X2{ws.xv + m1, 1, NMAX};
                        Mat<double> R1{ws.rv, 1, NMAX}, R2{ws.rv + m1, 1, NMAX};
                        wg_mm<double, 1>(m1, r, m1, -1.0, v.t1, TRI_LOWER, X1.tr(), TRI_NONE, 1.0, R1, false);
                        wg_mm<double, 1>(m1, r, m1, -1.0, Mat<const double>(v.t1).tr(), TRI_SUPPER, X1.tr(), TRI_NONE,
                                         1.0, R1, false);
                        if (m2 > 0) {
                            wg_mm<double, 1>(m1, r, m2, -1.0, Mat<const double>(v.s).tr(), TRI_NONE, X2.tr(),
                                             TRI_NONE, 1.0, R1, false);
                            wg_mm<double, 1>(m2, r, m1, -1.0, v.s, TRI_NONE, X1.tr(), TRI_NONE, 1.0, R2, false);
                            wg_mm<double, 1>(m2, r, m2, -1.0, v.t2, TRI_LOWER, X2.tr(), TRI_NONE, 1.0, R2, false);
                            wg_mm<double, 1>(m2, r, m2, -1.0, Mat<const double>(v.t2).tr(), TRI_SUPPER, X2.tr(),
                                             TRI_NONE, 1.0, R2, false);
                        }
                        // normwise backward error, max over the slab's columns
                        double eta = 0.0;
                        for (int c = 0; c < r; c++) {
                            double rm = 0.0, xm = 0.0, bmx = 0.0;
                            for (int i = t; i < n; i += 256) {
                                const double q = fabs(ws.rv[i + c * NMAX]), x = fabs(ws.xv[i + c * NMAX]);
                                const double bq = fabs(bb[i + c * sd.ldb]);
                                rm = (q > rm || q != q) ? q : rm;
                                xm = (x > xm || x != x) ? x : xm;
                                bmx = (bq > bmx || bq != bq) ? bq : bmx;
                            }
                            rm = wg_max(rm, red);
                            xm = wg_max(xm, red);
                            bmx = wg_max(bmx, red);
                            const double den = anorm * xm + bmx;
                            const double e = (den != den || rm != rm) ? __builtin_nan("")
                                             : den > 0.0              ? rm / den
                                             : rm > 0.0               ? __builtin_inf()
                                                                      : 0.0;
                            eta = (e > eta || e != e) ? e : eta;
                        }
                        if (eta <= a.tol) {
                            done = it;
                            break;
                        }
                        if (it > 1 && !(eta < 0.5 * prev)) {
                            done = -2;
                            break;
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
}

size_t batched_scratch_bytes(int wgs) { return (size_t)wgs * wg_scratch_bytes(); }

hipError_t batched_solve(const Exec& ex, const rfp_sys_t* sys, int64_t batch, double* arf, double* b, int mode,
                         int pftri, double tol, int max_iter, int* info, int* iter, int* counter, char* scratch,
                         int wgs)
{
    if (batch <= 0) return hipSuccess;
    hipError_t e = fill_int(ex.stream, counter, 1, 0);
    if (e != hipSuccess) return e;
    BatchArgs a{sys, batch, arf, b, mode, pftri, tol, max_iter, info, iter, counter, scratch};
    ProfScope ps(ex, "rfp::batched_kernel(rfp::BatchArgs)", 0.0, 0.0);
    hipLaunchKernelGGL(batched_kernel, dim3((unsigned)wgs), dim3(256), 0, ex.stream, a);
    return hipGetLastError();
}

}  // namespace rfp
