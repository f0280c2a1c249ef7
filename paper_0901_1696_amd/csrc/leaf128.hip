// Leaf kernel of the blocked factorization: one workgroup factors a diagonal
// block of order <= 128 and inverts its factor (potrf128_block).
#include <cstdio>

#include "leaf128.h"

namespace rfp {

template <typename T>
__global__ __launch_bounds__(256) void potrf128_kernel(Mat<T> A, int nb, T* winv, int* info, int64_t info_base)
{
    if (info && *info) return;
    // always on the critical path: first in issue when sharing a compute unit with bulk work
    __builtin_amdgcn_s_setprio(3);
    __shared__ Leaf128Smem<T> sm;
    (void)potrf128_block<T>(sm, A, nb, winv, info, info_base);
}

template <typename T>
hipError_t potrf128_leaf(const Exec& ex, Mat<T> A, int nb, T* winv, int64_t info_base)
{
    static char name[2][96];
    const int ti = sizeof(T) == 8 ? 0 : 1;
    if (!name[ti][0])
        snprintf(name[ti], sizeof name[ti], "rfp::potrf128_kernel<%s>(rfp::Mat<%s>, int, %s*, int*, long)",
                 ti ? "float" : "double", ti ? "float" : "double", ti ? "float" : "double");
    ProfScope ps(ex, name[ti], 2.0 * nb * nb * nb / 3.0, sizeof(T) * (double)nb * nb * 2.0);
    // The FP64 leaf reserves LDS it does not use (ex.leaf_pad bytes, 24 KB by
    // default), so that no 128 x 128 GEMM workgroup (64-72 KB) of the bulk
    // updates can share its compute unit (the smaller panel products still
    // can): it is on the critical path.
    const unsigned pad = sizeof(T) == 8 ? (unsigned)ex.leaf_pad : 0;
    hipLaunchKernelGGL((potrf128_kernel<T>), dim3(1), dim3(256), pad, ex.stream, A, nb, winv, ex.info, info_base);
    return hipGetLastError();
}

template hipError_t potrf128_leaf<double>(const Exec&, Mat<double>, int, double*, int64_t);
template hipError_t potrf128_leaf<float>(const Exec&, Mat<float>, int, float*, int64_t);

template <typename T>
__global__ __launch_bounds__(256) void trtri128_kernel(Mat<T> A, int nb, T* scratch, int* info, int64_t info_base)
{
    if (info && *info) return;
    // on the critical path of the inversion: first in issue on a shared compute unit
    __builtin_amdgcn_s_setprio(3);
    __shared__ Leaf128Smem<T> sm;
    (void)trtri128_block<T>(sm, A, nb, scratch, info, info_base);
}

template <typename T>
hipError_t trtri128_leaf(const Exec& ex, Mat<T> A, int nb, T* scratch, int64_t info_base)
{
    static char name[2][96];
    const int ti = sizeof(T) == 8 ? 0 : 1;
    if (!name[ti][0])
        snprintf(name[ti], sizeof name[ti], "rfp::trtri128_kernel<%s>(rfp::Mat<%s>, int, %s*, int*, long)",
                 ti ? "float" : "double", ti ? "float" : "double", ti ? "float" : "double");
    ProfScope ps(ex, name[ti], (double)nb * nb * nb / 3.0, sizeof(T) * (double)nb * nb);
    hipLaunchKernelGGL((trtri128_kernel<T>), dim3(1), dim3(256), 0, ex.stream, A, nb, scratch, ex.info, info_base);
    return hipGetLastError();
}

template hipError_t trtri128_leaf<double>(const Exec&, Mat<double>, int, double*, int64_t);
template hipError_t trtri128_leaf<float>(const Exec&, Mat<float>, int, float*, int64_t);

template <typename T>
__global__ __launch_bounds__(256) void lauum128_kernel(Mat<T> A, int nb, const int* info)
{
    if (info && *info) return;
    __builtin_amdgcn_s_setprio(3);
    __shared__ Leaf128Smem<T> sm;
    lauum128_block<T>(sm, A, nb);
}

template <typename T>
hipError_t lauum128_leaf(const Exec& ex, Mat<T> A, int nb)
{
    static char name[2][96];
    const int ti = sizeof(T) == 8 ? 0 : 1;
    if (!name[ti][0])
        snprintf(name[ti], sizeof name[ti], "rfp::lauum128_kernel<%s>(rfp::Mat<%s>, int, int const*)",
                 ti ? "float" : "double", ti ? "float" : "double");
    ProfScope ps(ex, name[ti], (double)nb * nb * nb / 3.0, sizeof(T) * (double)nb * nb);
    hipLaunchKernelGGL((lauum128_kernel<T>), dim3(1), dim3(256), 0, ex.stream, A, nb, (const int*)ex.info);
    return hipGetLastError();
}

template hipError_t lauum128_leaf<double>(const Exec&, Mat<double>, int);
template hipError_t lauum128_leaf<float>(const Exec&, Mat<float>, int);

}  // namespace rfp
