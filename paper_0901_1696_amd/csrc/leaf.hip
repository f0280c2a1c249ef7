// 64-row diagonal-block ("leaf") kernels: Cholesky with the inverse of the
// factor (POTRF, Section 3) and the batched inverses of every diagonal block
// of a triangle (the fused solves, TFSM), on blocks of order at most NB = 64.
// One wavefront handles one block; rows or columns live in
// lanes and the block is broadcast through LDS, so the only synchronisation
// is within the wavefront.  Every store back into the RFP array is masked to
// the block's own lower triangle: the other triangle of a diagonal block is
// the other diagonal block's data.
#include <cstdio>

#include "rfp_common.h"

namespace rfp {

// Cholesky of one leaf.  Lane i holds row i of the block in registers; at step
// j the pivot column is published in LDS and every lane updates its row:
// l_jj = sqrt(a_jj), l_ij = a_ij / l_jj, a_ik -= l_ij l_kj (k > j).
// Then W = L^{-1} by forward substitution, lane c building column c, and W is
// stored row-major (W(r, c) at winv[r * NB + c]) for the panel TRSM.
template <typename T>
__global__ __launch_bounds__(64) void potrf_leaf_kernel(Mat<T> A, int nb, T* winv, int* info, int64_t info_base)
{
    if (info && *info) return;
    const int i = threadIdx.x;
    __shared__ T col[NB];
    __shared__ T Ls[NB][NB + 1];
    __shared__ T rdiag[NB];

    T a[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) a[j] = (i < nb && j <= i) ? A.at(i, j) : (i == j ? T(1) : T(0));

    int fail = 0;
#pragma unroll
    for (int j = 0; j < NB; j++) {
        T d = T(1);
        if (j < nb && !fail) {
            col[i] = a[j];
            __syncthreads();
            d = col[j];
            if (!(d > T(0))) fail = j + 1;
        }
        if (j < nb && !fail) {
            const T l = sqrt(d);
            const T rl = T(1) / l;
            const T lij = (i > j) ? a[j] * rl : (i == j ? l : T(0));
            a[j] = lij;
            const T t = lij * rl;
#pragma unroll
            for (int k = j + 1; k < NB; k++) a[k] -= t * col[k];
            __syncthreads();
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (fail) {
        if (i == 0) *info = (int)(info_base + fail);
        return;
    }
    if (i < nb) {
#pragma unroll
        for (int j = 0; j < NB; j++)
            if (j <= i) A.at(i, j) = a[j];
    }
    if (!winv) return;
#pragma unroll
    for (int j = 0; j < NB; j++) Ls[i][j] = (j <= i) ? a[j] : T(0);
    __syncthreads();
    rdiag[i] = T(1) / Ls[i][i];
    __syncthreads();
    // lane c: column c of W, rows r = 0..NB-1
    const int c = i;
    T w[NB];
#pragma unroll
    for (int r = 0; r < NB; r++) {
        T s = (r == c) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < r; q++) s -= Ls[r][q] * w[q];
        w[r] = s * rdiag[r];
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < NB; r++) winv[r * NB + c] = w[r];
}

// Forward substitution for W = L^{-1} of a block already in LDS; lane c
// returns column c.  Diagonal entries are inverted once per row.
template <typename T>
__device__ __forceinline__ void inv_columns(const T (*Ls)[NB + 1], const T* rdiag, int c, T* w)
{
#pragma unroll
    for (int r = 0; r < NB; r++) {
        T s = (r == c) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < r; q++) s -= Ls[r][q] * w[q];
        w[r] = s * rdiag[r];
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Out-of-place inverses of all leaves of a lower-triangular matrix of order n
// (one wavefront per leaf, blockIdx.x = leaf).  Used by PFTRS and TFSM.
// unit: the diagonal is taken as ones (not read).  Does nothing while
// *gate != 0 (gate may be null).
template <typename T>
__global__ __launch_bounds__(64) void trtri_leaves_kernel(Mat<const T> A, int64_t n, T* winv, const int* gate,
                                                          int unit)
{
    if (gate && *gate) return;
    const int64_t b = blockIdx.x;
    const int64_t o = b * NB;
    const int nb = (int)((n - o) < NB ? (n - o) : NB);
    const int i = threadIdx.x;
    __shared__ T Ls[NB][NB + 1];
    __shared__ T rdiag[NB];
    // row i of the block, sixteen loads in flight at a time (an entry that is
    // not read takes the block's first element and is replaced)
#pragma unroll
    for (int j0 = 0; j0 < NB; j0 += 16) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int j = j0 + u;
            const bool rd = i < nb && (j < i || (j == i && !unit));
            v[u] = *(rd ? &A.at(o + i, o + j) : &A.at(o, o));
        }
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int j = j0 + u;
            Ls[i][j] = (i < nb && j < i) ? v[u] : (i == j ? ((i < nb && !unit) ? v[u] : T(1)) : T(0));
        }
    }
    __syncthreads();
    rdiag[i] = T(1) / Ls[i][i];
    __syncthreads();
    T w[NB];
    inv_columns<T>(Ls, rdiag, i, w);
    T* out = winv + b * NB * NB;
#pragma unroll
    for (int r = 0; r < NB; r++) out[r * NB + i] = w[r];
}

template <typename T>
static const char* lname(const char* kern, const char* args)
{
    // demangled name as rocprofv3 prints it, e.g. "rfp::potrf_leaf_kernel<double>(...)"
    static thread_local char buf[160];
    snprintf(buf, sizeof buf, "rfp::%s<%s>(%s)", kern, sizeof(T) == 8 ? "double" : "float", args);
    return buf;
}

template <typename T>
hipError_t potrf_leaf(const Exec& ex, Mat<T> A, int nb, T* winv, int64_t info_base)
{
    ProfScope ps(ex, lname<T>("potrf_leaf_kernel", sizeof(T) == 8 ? "rfp::Mat<double>, int, double*, int*, long"
                                                                  : "rfp::Mat<float>, int, float*, int*, long"),
                 (double)nb * nb * nb / 3.0 + (double)nb * nb * nb / 3.0, sizeof(T) * (double)nb * nb * 1.5);
    hipLaunchKernelGGL((potrf_leaf_kernel<T>), dim3(1), dim3(64), 0, ex.stream, A, nb, winv, ex.info, info_base);
    return hipGetLastError();
}

template <typename T>
hipError_t trtri_leaves(const Exec& ex, Mat<const T> A, int64_t n, T* winv, bool unit)
{
    if (n <= 0) return hipSuccess;
    const int64_t nl = (n + NB - 1) / NB;
    ProfScope ps(ex, lname<T>("trtri_leaves_kernel", sizeof(T) == 8 ? "rfp::Mat<double const>, long, double*, int const*, int"
                                                                    : "rfp::Mat<float const>, long, float*, int const*, int"),
                 (double)nl * NB * NB * NB / 3.0, sizeof(T) * (double)nl * NB * NB * 1.5);
    hipLaunchKernelGGL((trtri_leaves_kernel<T>), dim3((unsigned)nl), dim3(64), 0, ex.stream, A, n, winv, ex.gate,
                       unit ? 1 : 0);
    return hipGetLastError();
}

#define RFP_LEAF_INST(T)                                                               \
    template hipError_t potrf_leaf<T>(const Exec&, Mat<T>, int, T*, int64_t);          \
    template hipError_t trtri_leaves<T>(const Exec&, Mat<const T>, int64_t, T*, bool);
RFP_LEAF_INST(double)
RFP_LEAF_INST(float)

}  // namespace rfp
