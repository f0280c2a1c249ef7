// Full <-> RFP conversion (TRTTF / TFTTR, the paper's LAPACK routine table)
// as three 2-D strided block copies: T1 <-> A11, S <-> A21, T2 <-> A22, each
// block addressed through the canonical lower view.  The copy is tiled
// 64 x 64 through LDS so that both the load and the store run along the
// contiguous direction of their own array, whichever orientation each side
// has; triangular blocks are copied under a lower-triangle mask so the seam
// between T1 and T2 is never overwritten.
#include "rfp_common.h"

namespace rfp {

constexpr int CT = 64;

template <typename Td, typename Ts>
__global__ __launch_bounds__(256) void copy2d_kernel(Mat<Td> dst, Mat<const Ts> src, int64_t m, int64_t n,
                                                      int lower, int64_t tiles_m)
{
    __shared__ Ts tile[CT][CT + 1];
    const int64_t ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
    const int64_t i0 = ti * CT, j0 = tj * CT;
    if (lower && j0 > i0 + CT - 1) return;
    const int t = threadIdx.x;
    const int fast = t % CT, slow = t / CT;
    const bool src_rows = src.rs == 1;  // source row index contiguous
    // all loads of a thread in flight together: an element outside the block
    // (or its triangle) reads the view's first element and is not kept
    Ts v[CT / 4];
#pragma unroll
    for (int r = 0; r < CT / 4; r++) {
        const int li = src_rows ? fast : slow + 4 * r;
        const int lj = src_rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        const bool ok = i < m && j < n && (!lower || i >= j);
        v[r] = *(ok ? &src.at(i, j) : src.p);
    }
#pragma unroll
    for (int r = 0; r < CT / 4; r++) {
        const int li = src_rows ? fast : slow + 4 * r;
        const int lj = src_rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) tile[li][lj] = v[r];
    }
    __syncthreads();
    const bool dst_rows = dst.rs == 1;
#pragma unroll
    for (int r = 0; r < CT / 4; r++) {
        const int li = dst_rows ? fast : slow + 4 * r;
        const int lj = dst_rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) dst.at(i, j) = (Td)tile[li][lj];
    }
}

template <typename Td, typename Ts>
hipError_t copy2d(hipStream_t s, Mat<Td> dst, Mat<const Ts> src, int64_t m, int64_t n, bool lower)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t tm = (m + CT - 1) / CT, tn = (n + CT - 1) / CT;
    hipLaunchKernelGGL((copy2d_kernel<Td, Ts>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, dst, src, m, n,
                       lower ? 1 : 0, tm);
    return hipGetLastError();
}

template hipError_t copy2d<double, double>(hipStream_t, Mat<double>, Mat<const double>, int64_t, int64_t, bool);
template hipError_t copy2d<float, float>(hipStream_t, Mat<float>, Mat<const float>, int64_t, int64_t, bool);

// Packed <-> RFP (TPTTF / TFTTP, the paper's routine table): every stored
// entry of one RFP block (canonical lower view, global offset gi0 / gj0) is
// exchanged with its place in the packed array of order N: for UPLO='L'
// column gj holds rows gj..N-1, (gi, gj) at gi - gj + gj N - gj (gj - 1) / 2;
// for UPLO='U' the same entry is (gj, gi) of the upper triangle, at
// gj + gi (gi + 1) / 2.  The RFP side is read or written along its unit
// stride.
template <typename T>
__global__ __launch_bounds__(256) void packed_copy_kernel(Mat<T> v, int64_t m, int64_t n, int lower, int64_t gi0,
                                                          int64_t gj0, T* ap, int64_t N, int upper_packed, int to_rfp,
                                                          int64_t tiles_m)
{
    const int64_t ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
    const int64_t i0 = ti * CT, j0 = tj * CT;
    if (lower && j0 > i0 + CT - 1) return;
    const int t = threadIdx.x, fast = t % CT, slow = t / CT;
    const bool rows = v.rs == 1;
#pragma unroll 4
    for (int r = 0; r < CT / 4; r++) {
        const int li = rows ? fast : slow + 4 * r;
        const int lj = rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) {
            const int64_t gi = gi0 + i, gj = gj0 + j;
            const int64_t p = upper_packed ? gj + gi * (gi + 1) / 2 : gi - gj + gj * N - gj * (gj - 1) / 2;
            if (to_rfp) v.at(i, j) = ap[p];
            else ap[p] = v.at(i, j);
        }
    }
}

template <typename T>
hipError_t packed_copy(hipStream_t s, const RfpView<T>& v, T* ap, bool upper_packed, bool to_rfp)
{
    const int64_t N = v.m1 + v.m2;
    auto blk = [&](Mat<T> b, int64_t m, int64_t n, bool lower, int64_t gi0, int64_t gj0) {
        if (m <= 0 || n <= 0) return;
        const int64_t tm = (m + CT - 1) / CT, tn = (n + CT - 1) / CT;
        hipLaunchKernelGGL((packed_copy_kernel<T>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, b, m, n,
                           lower ? 1 : 0, gi0, gj0, ap, N, upper_packed ? 1 : 0, to_rfp ? 1 : 0, tm);
    };
    blk(v.t1, v.m1, v.m1, true, 0, 0);
    blk(v.s, v.m2, v.m1, false, v.m1, 0);
    blk(v.t2, v.m2, v.m2, true, v.m1, v.m1);
    return hipGetLastError();
}
template hipError_t packed_copy<double>(hipStream_t, const RfpView<double>&, double*, bool, bool);
template hipError_t packed_copy<float>(hipStream_t, const RfpView<float>&, float*, bool, bool);

// X = alpha X on an m x n view (lower triangle only if lower); alpha = 0
// writes zeros without reading X.
template <typename T>
__global__ __launch_bounds__(256) void scale2d_kernel(Mat<T> x, int64_t m, int64_t n, T alpha, int lower,
                                                      int64_t tiles_m)
{
    const int64_t ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
    const int64_t i0 = ti * CT, j0 = tj * CT;
    if (lower && j0 > i0 + CT - 1) return;
    const int t = threadIdx.x, fast = t % CT, slow = t / CT;
    const bool rows = x.rs == 1;
#pragma unroll 4
    for (int r = 0; r < CT / 4; r++) {
        const int li = rows ? fast : slow + 4 * r;
        const int lj = rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) x.at(i, j) = alpha == T(0) ? T(0) : alpha * x.at(i, j);
    }
}

template <typename T>
hipError_t scale2d(hipStream_t s, Mat<T> x, int64_t m, int64_t n, T alpha, bool lower)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t tm = (m + CT - 1) / CT, tn = (n + CT - 1) / CT;
    hipLaunchKernelGGL((scale2d_kernel<T>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, x, m, n, alpha,
                       lower ? 1 : 0, tm);
    return hipGetLastError();
}
template hipError_t scale2d<double>(hipStream_t, Mat<double>, int64_t, int64_t, double, bool);
template hipError_t scale2d<float>(hipStream_t, Mat<float>, int64_t, int64_t, float, bool);

// C += alpha A on an m x n view (lower triangle only if lower).
template <typename T>
__global__ __launch_bounds__(256) void axpy2d_kernel(Mat<T> c, Mat<const T> a, int64_t m, int64_t n, T alpha,
                                                     int lower, int64_t tiles_m)
{
    const int64_t ti = blockIdx.x % tiles_m, tj = blockIdx.x / tiles_m;
    const int64_t i0 = ti * CT, j0 = tj * CT;
    if (lower && j0 > i0 + CT - 1) return;
    const int t = threadIdx.x, fast = t % CT, slow = t / CT;
    const bool rows = c.rs == 1;
    // in groups of four rows: the group's loads issued together (an element
    // outside the block or its triangle reads the first element of each view
    // and is not stored)
#pragma unroll
    for (int r0 = 0; r0 < CT / 4; r0 += 4) {
        T av[4], cv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int r = r0 + u;
            const int li = rows ? fast : slow + 4 * r;
            const int lj = rows ? slow + 4 * r : fast;
            const int64_t i = i0 + li, j = j0 + lj;
            const bool ok = i < m && j < n && (!lower || i >= j);
            av[u] = *(ok ? &a.at(i, j) : a.p);
            cv[u] = *(ok ? &c.at(i, j) : c.p);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int r = r0 + u;
            const int li = rows ? fast : slow + 4 * r;
            const int lj = rows ? slow + 4 * r : fast;
            const int64_t i = i0 + li, j = j0 + lj;
            if (i < m && j < n && (!lower || i >= j)) c.at(i, j) = cv[u] + alpha * av[u];
        }
    }
}

template <typename T>
hipError_t axpy2d(hipStream_t s, Mat<T> c, Mat<const T> a, int64_t m, int64_t n, T alpha, bool lower)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t tm = (m + CT - 1) / CT, tn = (n + CT - 1) / CT;
    hipLaunchKernelGGL((axpy2d_kernel<T>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, c, a, m, n, alpha,
                       lower ? 1 : 0, tm);
    return hipGetLastError();
}
template hipError_t axpy2d<double>(hipStream_t, Mat<double>, Mat<const double>, int64_t, int64_t, double, bool);
template hipError_t axpy2d<float>(hipStream_t, Mat<float>, Mat<const float>, int64_t, int64_t, float, bool);

// The diagonal of the two diagonal blocks: save it to buf and set it to one
// (restore = 0), or write buf back (restore = 1).
template <typename T>
__global__ void unit_diag_kernel(Mat<T> t1, int64_t m1, Mat<T> t2, int64_t m2, T* buf, int restore)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m1 + m2) return;
    T& d = i < m1 ? t1.at(i, i) : t2.at(i - m1, i - m1);
    if (restore) {
        d = buf[i];
    } else {
        buf[i] = d;
        d = T(1);
    }
}

template <typename T>
hipError_t unit_diag(hipStream_t s, const RfpView<T>& v, T* buf, bool restore)
{
    const int64_t n = v.m1 + v.m2;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((unit_diag_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v.t1, v.m1, v.t2,
                       v.m2, buf, restore ? 1 : 0);
    return hipGetLastError();
}
template hipError_t unit_diag<double>(hipStream_t, const RfpView<double>&, double*, bool);
template hipError_t unit_diag<float>(hipStream_t, const RfpView<float>&, float*, bool);

__global__ void set_int_kernel(int* p, int v)
{
    if (threadIdx.x == 0) *p = v;
}

hipError_t set_int(hipStream_t s, int* p, int v)
{
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace rfp
