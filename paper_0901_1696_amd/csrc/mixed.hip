// Kernels of the mixed-precision solve with iterative refinement: the
// scaled cast of the FP64 RFP matrix to an FP32 RFP workspace, norms of a
// symmetric matrix held in RFP, and the elementwise steps of a refinement
// sweep (scaled cast of the residual, FP64 update of the solution, column
// maxima for the backward error).
//
// Every RFP kernel walks the three blocks T1, S and T2 through their
// canonical lower views; each view has one unit stride, and the 64 x 64 tile
// of a workgroup is read with the fast thread index along it.
#include <algorithm>
#include <cstdio>

#include "rfp_common.h"

namespace rfp {

namespace {
constexpr int TT = 64;  // tile edge of the RFP block kernels
}

// s[i] = 1 / sqrt(a_ii) (scale != 0) or 1; NaN for a diagonal entry that is
// not positive, so that the scaled matrix cannot be factored.
__global__ void diag_scale_kernel(Mat<const double> t1, int64_t m1, Mat<const double> t2, int64_t m2, int scale,
                                  double* s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m1 + m2) return;
    const double d = i < m1 ? t1.at(i, i) : t2.at(i - m1, i - m1);
    double v = 1.0;
    if (scale) v = d > 0.0 ? 1.0 / sqrt(d) : __builtin_nan("");
    s[i] = v;
}

// dst(i, j) = (float)(((src(i, j) * sr[i]) * sc[j]) * mu) over an m x n block
// (lower triangle only if lower, a diagonal block: then shift is added to
// each diagonal entry before mu); src and dst have the same strides.
__global__ __launch_bounds__(256) void cast_block_kernel(Mat<const double> src, Mat<float> dst, int64_t m, int64_t n,
                                                         int lower, const double* sr, const double* sc, double mu,
                                                         double shift, int64_t tiles_m, int* nonfinite)
{
    const int64_t ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
    const int64_t i0 = ti * TT, j0 = tj * TT;
    if (lower && j0 > i0 + TT - 1) return;
    const int t = threadIdx.x, fast = t % TT, slow = t / TT;
    const bool rows = src.rs == 1;
#pragma unroll 4
    for (int r = 0; r < TT / 4; r++) {
        const int li = rows ? fast : slow + 4 * r;
        const int lj = rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) {
            double v = src.at(i, j) * sr[i];
            v = v * sc[j];
            if (lower && i == j) v = v + shift;
            v = v * mu;
            const float f = (float)v;
            dst.at(i, j) = f;
            if (nonfinite && !__builtin_isfinite(f)) *nonfinite = 1;
        }
    }
}

hipError_t pf_cast_scale(hipStream_t st, const RfpView<const double>& a, const RfpView<float>& o, int scale, double mu,
                         double shift, double* s, int* nonfinite)
{
    const int64_t n = a.m1 + a.m2;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(diag_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a.t1, a.m1, a.t2, a.m2,
                       scale, s);
    auto blk = [&](Mat<const double> src, Mat<float> dst, int64_t m, int64_t nn, bool lower, const double* sr,
                   const double* sc) {
        if (m <= 0 || nn <= 0) return;
        const int64_t tm = (m + TT - 1) / TT, tn = (nn + TT - 1) / TT;
        hipLaunchKernelGGL(cast_block_kernel, dim3((unsigned)(tm * tn)), dim3(256), 0, st, src, dst, m, nn,
                           lower ? 1 : 0, sr, sc, mu, shift, tm, nonfinite);
    };
    blk(a.t1, o.t1, a.m1, a.m1, true, s, s);
    blk(a.s, o.s, a.m2, a.m1, false, s + a.m1, s);
    blk(a.t2, o.t2, a.m2, a.m2, true, s + a.m1, s + a.m1);
    return hipGetLastError();
}

// ---------------------------------------------------------------- norms
// Per 64 x 64 tile of a block with global row / column offsets gi0 / gj0
// (symmetric matrix: an off-diagonal stored entry also stands for its mirror):
//   rowsum[g] += |a| for both rows it belongs to, maxabs = max |a|,
//   sumsq += a^2 (twice off the diagonal).
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(256) void sym_norm_kernel(Mat<const double> a, int64_t m, int64_t n, int lower,
                                                       int64_t gi0, int64_t gj0, int64_t tiles_m, double* rowsum,
                                                       double* maxabs, double* sumsq)
{
    __shared__ double rs[TT], cs[TT];
    __shared__ double red[256];
    __shared__ double redm[256];
    const int64_t ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
    const int64_t i0 = ti * TT, j0 = tj * TT;
    if (lower && j0 > i0 + TT - 1) return;
    const int t = threadIdx.x, fast = t % TT, slow = t / TT;
    if (t < TT) rs[t] = cs[t] = 0.0;
    __syncthreads();
    const bool rows = a.rs == 1;
    double sq = 0.0, mx = 0.0;
    // all loads of a thread in flight together (an element outside the block
    // or its triangle reads the view's first element and is skipped)
    double av[TT / 4];
#pragma unroll
    for (int r = 0; r < TT / 4; r++) {
        const int li = rows ? fast : slow + 4 * r;
        const int lj = rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        av[r] = *((i < m && j < n && (!lower || i >= j)) ? &a.at(i, j) : a.p);
    }
#pragma unroll
    for (int r = 0; r < TT / 4; r++) {
        const int li = rows ? fast : slow + 4 * r;
        const int lj = rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) {
            const double v = fabs(av[r]);
            const bool diag = gi0 + i == gj0 + j;
            atomicAdd(&rs[li], v);
            if (!diag) atomicAdd(&cs[lj], v);
            sq += diag ? v * v : 2.0 * v * v;
            mx = v > mx ? v : mx;
        }
    }
    red[t] = sq;
    redm[t] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[t] += red[t + w];
            redm[t] = redm[t] > redm[t + w] ? redm[t] : redm[t + w];
        }
        __syncthreads();
    }
    if (t < TT) {
        if (i0 + t < m && rs[t] != 0.0) atomicAdd(&rowsum[gi0 + i0 + t], rs[t]);
        if (j0 + t < n && cs[t] != 0.0) atomicAdd(&rowsum[gj0 + j0 + t], cs[t]);
    }
    if (t == 0) {
        atomicAdd(sumsq, red[0]);
        atomic_max_nonneg(maxabs, redm[0]);
    }
}

__global__ void fill_double_kernel(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t fill_double(hipStream_t s, double* p, int64_t n, double v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_double_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// out = max_i v[i] (non-negative entries), one workgroup
__global__ __launch_bounds__(256) void max_reduce_kernel(const double* v, int64_t n, double* out)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = v[i] > m ? v[i] : m;
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x]
                                                                                          : red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void norm_finish_kernel(int which, const double* inf, const double* maxabs, const double* sumsq,
                                   double* out)
{
    if (threadIdx.x != 0) return;
    *out = which == 0 ? *maxabs : which == 1 ? *inf : sqrt(*sumsq);
}

// work: n + 3 doubles.  which: 0 max-abs, 1 one/infinity norm, 2 Frobenius.
hipError_t pf_norm(hipStream_t st, const RfpView<const double>& a, int which, double* work, double* out)
{
    const int64_t n = a.m1 + a.m2;
    double* rowsum = work;
    double* inf = work + n;
    double* maxabs = work + n + 1;
    double* sumsq = work + n + 2;
    hipError_t e = fill_double(st, work, n + 3, 0.0);
    if (e != hipSuccess) return e;
    auto blk = [&](Mat<const double> v, int64_t m, int64_t nn, bool lower, int64_t gi0, int64_t gj0) {
        if (m <= 0 || nn <= 0) return;
        const int64_t tm = (m + TT - 1) / TT, tn = (nn + TT - 1) / TT;
        hipLaunchKernelGGL(sym_norm_kernel, dim3((unsigned)(tm * tn)), dim3(256), 0, st, v, m, nn, lower ? 1 : 0,
                           gi0, gj0, tm, rowsum, maxabs, sumsq);
    };
    blk(a.t1, a.m1, a.m1, true, 0, 0);
    blk(a.s, a.m2, a.m1, false, a.m1, 0);
    blk(a.t2, a.m2, a.m2, true, a.m1, a.m1);
    if (n > 0) hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, st, rowsum, n, inf);
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(64), 0, st, which, inf, maxabs, sumsq, out);
    return hipGetLastError();
}

// ------------------------------------------------------- refinement sweep
// out(i, c) = (float)(s[i] * r(i, c))
__global__ void ir_scale_cast_kernel(const double* r, int64_t ldr, const double* s, float* out, int64_t ldo, int64_t n,
                                     int64_t nrhs, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n && c < nrhs) out[i + c * ldo] = (float)(s[i] * r[i + c * ldr]);
}

// x(i, c) += (double)d(i, c) * s[i] * mu   (or x = ..., accumulate == 0)
__global__ void ir_update_kernel(double* x, int64_t ldx, const double* s, double mu, const float* d, int64_t ldd,
                                 int64_t n, int64_t nrhs, int accumulate, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n && c < nrhs) {
        const double v = ((double)d[i + c * ldd] * s[i]) * mu;
        x[i + c * ldx] = accumulate ? x[i + c * ldx] + v : v;
    }
}

// out[c] = sum_i u(i, c) v(i, c), one workgroup per column (fixed order)
__global__ __launch_bounds__(256) void col_dot_kernel(const double* u, const double* v, int64_t ld, int64_t n,
                                                      double* out, const int* gate)
{
    if (gate && *gate) return;
    __shared__ double red[256];
    const int64_t c = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += u[i + c * ld] * v[i + c * ld];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// alpha_c = rz[c] / pq[c] (0 when pq[c] = 0); d += alpha p; r -= alpha q
__global__ void pcg_step_kernel(double* d, int64_t ldd, double* r, const double* p, const double* q, const double* rz,
                                const double* pq, int64_t ld, int64_t n, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    const double a = pq[c] != 0.0 ? rz[c] / pq[c] : 0.0;
    const int64_t o = i + c * ld;
    d[i + c * ldd] += a * p[o];
    r[o] -= a * q[o];
}

// beta_c = rz_new[c] / rz_old[c] (0 when rz_old[c] = 0); p = z + beta p
__global__ void pcg_dir_kernel(double* p, const double* z, const double* rz_new, const double* rz_old, int64_t ld,
                               int64_t n, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    const double b = rz_old[c] != 0.0 ? rz_new[c] / rz_old[c] : 0.0;
    const int64_t o = i + c * ld;
    p[o] = z[o] + b * p[o];
}

// out[c] = max_i |v(i, c)|, one workgroup per column
__global__ __launch_bounds__(256) void colmax_kernel(const double* v, int64_t ld, int64_t n, double* out,
                                                     const int* gate)
{
    if (gate && *gate) return;
    __shared__ double red[256];
    const int64_t c = blockIdx.x;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double a = fabs(v[i + c * ld]);
        m = (a > m || a != a) ? a : m;  // a NaN wins
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + w];
            red[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// eta = max_c rmax[c] / (anorm * xmax[c] + bmax[c])  (normwise backward error)
__global__ __launch_bounds__(256) void eta_kernel(const double* rmax, const double* xmax, const double* bmax,
                                                  const double* anorm, int64_t nrhs, double* eta, const int* gate)
{
    if (gate && *gate) return;
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t c = threadIdx.x; c < nrhs; c += 256) {
        const double den = *anorm * xmax[c] + bmax[c];
        // a NaN anywhere (residual, solution, right-hand side, norm) gives NaN
        const double e = (den != den || rmax[c] != rmax[c]) ? __builtin_nan("")
                         : den > 0.0                        ? rmax[c] / den
                         : rmax[c] > 0.0                    ? __builtin_inf()
                                                            : 0.0;
        m = (e > m || e != e) ? e : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + w];
            red[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *eta = red[0];
}

hipError_t ir_scale_cast(hipStream_t st, const double* r, int64_t ldr, const double* s, float* out, int64_t ldo,
                         int64_t n, int64_t nrhs, const int* gate)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(ir_scale_cast_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, r,
                       ldr, s, out, ldo, n, nrhs, gate);
    return hipGetLastError();
}

hipError_t ir_update(hipStream_t st, double* x, int64_t ldx, const double* s, double mu, const float* d, int64_t ldd,
                     int64_t n, int64_t nrhs, bool accumulate, const int* gate)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(ir_update_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, x, ldx,
                       s, mu, d, ldd, n, nrhs, accumulate ? 1 : 0, gate);
    return hipGetLastError();
}

hipError_t col_dot(hipStream_t st, const double* u, const double* v, int64_t ld, int64_t n, int64_t nrhs, double* out,
                   const int* gate)
{
    if (nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_dot_kernel, dim3((unsigned)nrhs), dim3(256), 0, st, u, v, ld, n, out, gate);
    return hipGetLastError();
}

hipError_t pcg_step(hipStream_t st, double* d, int64_t ldd, double* r, const double* p, const double* q,
                    const double* rz, const double* pq, int64_t ld, int64_t n, int64_t nrhs, const int* gate)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pcg_step_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, d, ldd, r,
                       p, q, rz, pq, ld, n, gate);
    return hipGetLastError();
}

hipError_t pcg_dir(hipStream_t st, double* p, const double* z, const double* rz_new, const double* rz_old, int64_t ld,
                   int64_t n, int64_t nrhs, const int* gate)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pcg_dir_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, p, z,
                       rz_new, rz_old, ld, n, gate);
    return hipGetLastError();
}

hipError_t col_max(hipStream_t st, const double* v, int64_t ld, int64_t n, int64_t nrhs, double* out, const int* gate)
{
    if (nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)nrhs), dim3(256), 0, st, v, ld, n, out, gate);
    return hipGetLastError();
}

hipError_t backward_error(hipStream_t st, const double* rmax, const double* xmax, const double* bmax,
                          const double* anorm, int64_t nrhs, double* eta, const int* gate)
{
    hipLaunchKernelGGL(eta_kernel, dim3(1), dim3(256), 0, st, rmax, xmax, bmax, anorm, nrhs, eta, gate);
    return hipGetLastError();
}

// ------------------------------------------------- refinement control
// The refinement's decisions are taken on the device, by one-thread kernels
// between the sweeps, and every sweep kernel reads a gate word: the host
// enqueues the setup, max_iter sweeps and the fall-back once, without
// waiting, and the sweeps after convergence (or the fall-back when it is not
// needed) exit at their first instruction.
__device__ __forceinline__ void ir_gates(IrCtl* c)
{
    c->g_cvt = 1;
    c->g_cont = 1;
    c->g_ir = c->phase != IR_CLASSIC;
    c->g_pcg = c->phase != IR_PCG;
    c->g_run = c->phase >= IR_DONE;
    c->g_fb = c->phase != IR_FALLBACK;
    // the fall-back factor's INFO word doubles as its gate: nonzero skips it
    c->fb_info = c->phase == IR_FALLBACK ? 0 : -1;
}

__global__ void ir_start_kernel(IrCtl* c)
{
    if (threadIdx.x != 0) return;
    c->phase = IR_CLASSIC;
    c->code = 0;
    c->lp_info = 0;
    c->nonfinite = 0;
    c->eta = 0.0;
    c->prev = 0.0;
    c->best = 0.0;
    c->stale = 0;
    ir_gates(c);
}

// after the scaled cast and the low-precision factor
__global__ void ir_setup_decide_kernel(IrCtl* c)
{
    if (threadIdx.x != 0) return;
    if (c->nonfinite) {
        c->phase = IR_FALLBACK;
        c->code = -4;
    } else if (c->lp_info != 0) {
        c->phase = IR_FALLBACK;
        c->code = -3;
    }
    ir_gates(c);
}

// after sweep `it` (1-based) has left its backward error in c->eta: converged
// at eta <= tol; a classical sweep that does not cut eta fourfold switches to
// conjugate-gradient sweeps, which continue one recurrence from sweep to
// sweep (each restarts it from the true residual); conjugate gradients
// minimise the error's A-norm, so the residual need not fall every sweep,
// and the refinement stalls (-2) only after IR_STALE_SWEEPS of them in a row
// that do not bring eta below 0.9 times its best value; max_iter sweeps
// without convergence give -1.  NaN compares false everywhere, so it ends in
// a stall.
__global__ void ir_decide_kernel(IrCtl* c, int it, int max_iter, double tol)
{
    if (threadIdx.x != 0 || c->phase >= IR_DONE) return;
    const int before = c->phase;
    const double eta = c->eta;
    if (eta <= tol) {
        c->phase = IR_DONE;
        c->code = it;
    } else {
        const bool swept_pcg = c->phase == IR_PCG;
        if (swept_pcg) {
            if (eta < 0.9 * c->best) {
                c->best = eta;
                c->stale = 0;
            } else {
                c->stale++;
            }
        }
        if (swept_pcg && c->stale >= IR_STALE_SWEEPS) {
            c->phase = IR_FALLBACK;
            c->code = -2;
        } else if (it >= max_iter) {
            c->phase = IR_FALLBACK;
            c->code = -1;
        } else if (it > 1 && !swept_pcg && !(eta < 0.25 * c->prev)) {
            c->phase = IR_PCG;
            c->best = eta < c->prev ? eta : c->prev;
            c->stale = 0;
        }
        c->prev = eta;
    }
    ir_gates(c);
    // open exactly when this decision starts, or continues, the
    // conjugate-gradient sweeps
    c->g_cvt = !(before == IR_CLASSIC && c->phase == IR_PCG);
    c->g_cont = !(before == IR_PCG && c->phase == IR_PCG);
}

__global__ void ir_finish_kernel(const IrCtl* c, int* iter, int* info)
{
    if (threadIdx.x != 0) return;
    *iter = c->code;
    *info = c->phase == IR_FALLBACK ? c->fb_info : 0;
}

hipError_t ir_start(hipStream_t st, IrCtl* c)
{
    hipLaunchKernelGGL(ir_start_kernel, dim3(1), dim3(64), 0, st, c);
    return hipGetLastError();
}

hipError_t ir_setup_decide(hipStream_t st, IrCtl* c)
{
    hipLaunchKernelGGL(ir_setup_decide_kernel, dim3(1), dim3(64), 0, st, c);
    return hipGetLastError();
}

hipError_t ir_decide(hipStream_t st, IrCtl* c, int it, int max_iter, double tol)
{
    hipLaunchKernelGGL(ir_decide_kernel, dim3(1), dim3(64), 0, st, c, it, max_iter, tol);
    return hipGetLastError();
}

hipError_t ir_finish(hipStream_t st, IrCtl* c, int* iter, int* info)
{
    hipLaunchKernelGGL(ir_finish_kernel, dim3(1), dim3(64), 0, st, (const IrCtl*)c, iter, info);
    return hipGetLastError();
}

__global__ void ir_copy_kernel(double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) y[i + c * ldy] = x ? x[i + c * ldx] : 0.0;
}

hipError_t ir_copy(hipStream_t st, double* y, int64_t ldy, const double* x, int64_t ldx, int64_t n, int64_t nrhs,
                   const int* gate)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(ir_copy_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, y, ldy, x,
                       ldx, n, gate);
    return hipGetLastError();
}

// grid-stride 1-D copy (two doubles per thread and step)
__global__ __launch_bounds__(256) void gated_copy_kernel(double* dst, const double* src, int64_t count,
                                                         const int* gate)
{
    if (gate && *gate) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

hipError_t gated_copy(hipStream_t st, double* dst, const double* src, int64_t count, const int* gate)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(gated_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, count, gate);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void widen_copy_kernel(double* dst, const float* src, int64_t count,
                                                         const int* gate)
{
    if (gate && *gate) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = (double)src[i];
}

hipError_t widen_copy(hipStream_t st, double* dst, const float* src, int64_t count, const int* gate)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(widen_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, count, gate);
    return hipGetLastError();
}

// y(i, c) = (x(i, c) * s[i]) * mul
__global__ void row_scale_kernel(double* y, int64_t ldy, const double* x, int64_t ldx, const double* s, double mul,
                                 int64_t n, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) y[i + c * ldy] = (x[i + c * ldx] * s[i]) * mul;
}

hipError_t row_scale(hipStream_t st, double* y, int64_t ldy, const double* x, int64_t ldx, const double* s, double mul,
                     int64_t n, int64_t nrhs, const int* gate)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(row_scale_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, y, ldy,
                       x, ldx, s, mul, n, gate);
    return hipGetLastError();
}

}  // namespace rfp

