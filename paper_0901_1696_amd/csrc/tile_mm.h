// Workgroup-level tile products for the batched solver's tile tasks:
// acc (a 128 x 128 tile held in registers by 256 threads) += A B^T with A
// (m x k) and B (n x k) strided views, m, n <= 128, any k, staged through LDS
// in 16-wide k slabs (the next slab is loaded into registers while the
// current one is multiplied).  Operands may be masked to a triangle; entries
// outside the mask, and rows or columns past m, n or k, are read as zero.
// The LDS buffers are the caller's, so that they can share storage with the
// diagonal-block leaf of the same kernel.
//
// Layout: the four wavefronts form a 2 x 2 grid, wave (wm, wn) owning rows
// 64 wm .. 64 wm + 63 and columns 64 wn .. 64 wn + 63 as 4 x 4 MFMA blocks of
// 16 x 16.  LPR (FP32 tiles only) rounds each operand to FP16 (1) or BF16 (2)
// when it is staged: the products of rounded operands are exact in FP32, so
// the result equals that of low-precision-operand MFMA with FP32
// accumulation.
#pragma once
#include "rfp_common.h"

namespace rfp {

namespace tile {

constexpr int TB = 128;  // tile order
constexpr int KS = 16;   // k slab
constexpr int KP = KS + 2;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc op(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of register e of lane l in a 16 x 16 result block (column l % 16)
    static __device__ __forceinline__ int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <>
struct Mfma<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc op(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

template <typename T>
struct Smem {
    __attribute__((aligned(16))) T A[TB][KP];
    __attribute__((aligned(16))) T B[TB][KP];
};

template <typename T>
struct Acc {
    typename Mfma<T>::acc v[4][4];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) v[a][b] = typename Mfma<T>::acc{0, 0, 0, 0};
    }
};

// mask (in the operand's own indices): TRI_NONE, TRI_LOWER (r >= c),
// TRI_UPPER (r <= c), TRI_SLOWER (r > c), TRI_SUPPER (r < c)
__device__ __forceinline__ bool keep(int tri, int64_t r, int64_t c)
{
    switch (tri) {
        case TRI_LOWER: return r >= c;
        case TRI_UPPER: return r <= c;
        case TRI_SLOWER: return r > c;
        case TRI_SUPPER: return r < c;
        default: return true;
    }
}

template <int LPR>
__device__ __forceinline__ float lp_round(float v)
{
    if constexpr (LPR == 1) return (float)(_Float16)v;
    if constexpr (LPR == 2) {
        // round to nearest even in the upper 16 bits (bfloat16), NaN kept
        unsigned u = __float_as_uint(v);
        if ((u & 0x7f800000u) == 0x7f800000u) return v;
        u += 0x7fffu + ((u >> 16) & 1u);
        return __uint_as_float(u & 0xffff0000u);
    }
    return v;
}
template <int LPR>
__device__ __forceinline__ double lp_round(double v)
{
    return v;
}

// Each thread stages 8 elements of each operand per slab: the 128 x 16 slab
// is read along the operand's unit stride (rows when rs == 1, k otherwise).
// Every lane loads (an entry outside the slab or the mask reads the operand's
// first element, always valid) and keeps the mask in bit e of `mk`; the mask
// and the rounding are applied when the slab is stored, so the loads stay in
// flight during the previous slab's products.
template <typename T>
__device__ __forceinline__ void load_slab(const Mat<const T>& X, int rows, int64_t k0, int64_t K, int tri, T (&r)[8],
                                          unsigned& mk)
{
    const int t = threadIdx.x;
    const bool rfast = X.rs == 1;
    mk = 0;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int idx = t + 256 * e;
        const int i = rfast ? idx % TB : idx / KS, kk = rfast ? idx / TB : idx % KS;
        const int64_t k = k0 + kk;
        const bool ok = i < rows && k < K && keep(tri, i, k);
        r[e] = *(ok ? &X.at(i, k) : X.p);
        mk |= (ok ? 1u : 0u) << e;
    }
}
template <typename T, int LPR>
__device__ __forceinline__ void store_slab(const Mat<const T>& X, T (&S)[TB][KP], const T (&r)[8], unsigned mk)
{
    const int t = threadIdx.x;
    const bool rfast = X.rs == 1;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int idx = t + 256 * e;
        const int i = rfast ? idx % TB : idx / KS, kk = rfast ? idx / TB : idx % KS;
        S[i][kk] = (mk >> e) & 1 ? lp_round<LPR>(r[e]) : T(0);
    }
}

// acc += A(m x K) B(n x K)^T.  All 256 threads call it; it ends with a barrier.
template <typename T, int LPR = 0>
__device__ void mma(Smem<T>& sm, Acc<T>& acc, int m, int n, int64_t K, Mat<const T> A, int triA, Mat<const T> B,
                    int triB)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int r = lane & 15, g = lane >> 4;
    T ra[8], rb[8];
    unsigned ma = 0, mb = 0;
    if (K > 0) {
        load_slab<T>(A, m, 0, K, triA, ra, ma);
        load_slab<T>(B, n, 0, K, triB, rb, mb);
    }
    for (int64_t k0 = 0; k0 < K; k0 += KS) {
        __syncthreads();  // the previous slab's products are done with the LDS
        store_slab<T, LPR>(A, sm.A, ra, ma);
        store_slab<T, LPR>(B, sm.B, rb, mb);
        __syncthreads();
        if (k0 + KS < K) {
            load_slab<T>(A, m, k0 + KS, K, triA, ra, ma);
            load_slab<T>(B, n, k0 + KS, K, triB, rb, mb);
        }
#pragma unroll
        for (int kk = 0; kk < KS; kk += 4) {
            T av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; a++) av[a] = sm.A[64 * wm + 16 * a + r][kk + g];
#pragma unroll
            for (int b = 0; b < 4; b++) bv[b] = sm.B[64 * wn + 16 * b + r][kk + g];
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) acc.v[a][b] = Mfma<T>::op(av[a], bv[b], acc.v[a][b]);
        }
    }
    __syncthreads();
}

// C = alpha acc + beta C on the m x n tile (only i >= j when c_lower);
// beta = 0 does not read C.  Every thread's operand reads are finished
// (mma ends with a barrier), so C may alias A or B.
template <typename T>
__device__ void store(const Acc<T>& acc, int m, int n, T alpha, T beta, Mat<T> C, bool c_lower)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
            T cv[4] = {T(0), T(0), T(0), T(0)};
            if (beta != T(0)) {  // the block's reads of C together, then its stores
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int i = 64 * wm + 16 * a + Mfma<T>::row(lane, e);
                    const int j = 64 * wn + 16 * b + (lane & 15);
                    const bool ok = i < m && j < n && (!c_lower || i >= j);
                    cv[e] = *(ok ? &C.at(i, j) : C.p);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = 64 * wm + 16 * a + Mfma<T>::row(lane, e);
                const int j = 64 * wn + 16 * b + (lane & 15);
                if (i < m && j < n && (!c_lower || i >= j)) {
                    T v = alpha * acc.v[a][b][e];
                    if (beta != T(0)) v += beta * cv[e];
                    C.at(i, j) = v;
                }
            }
        }
}

}  // namespace tile

}  // namespace rfp
