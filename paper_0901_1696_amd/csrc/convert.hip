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
#pragma unroll
    for (int r = 0; r < CT / 4; r++) {
        const int li = src_rows ? fast : slow + 4 * r;
        const int lj = src_rows ? slow + 4 * r : fast;
        const int64_t i = i0 + li, j = j0 + lj;
        if (i < m && j < n && (!lower || i >= j)) tile[li][lj] = src.at(i, j);
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
