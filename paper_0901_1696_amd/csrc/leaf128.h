// Fused Cholesky of one diagonal block of order <= 128 with the inverse of
// its factor, as a workgroup-level device routine (256 threads): used by the
// leaf kernel of the blocked factorization and by the batched solver.
//
// The workgroup keeps the lower triangle of the block in LDS, packed by
// 16-row block rows (75.8 KB: small enough to share a CU with one workgroup
// of the bulk-update GEMM, so that a leaf on a second stream starts as soon
// as one GEMM workgroup retires instead of waiting for a whole CU).  For
// each 16-column block column:
//   1. one wavefront factors the 16 x 16 diagonal block and forms its
//      inverse in the same register sweep (readlane broadcasts);
//   2. all four wavefronts solve the panel below with MFMA, X = A_p W^T;
//   3. all four wavefronts update the trailing lower triangle, A -= X X^T.
// The factor is stored back (masked to the block's own lower triangle), then
// W = L^{-1} is formed in place, block column by block column from the right:
// W_RR is already inverted, so W_Rj = -(W_RR L_Rj) W_jj (the diagonal
// inverses wait in the output array between the two phases).
#pragma once
#include "rfp_common.h"

#ifndef RFP_LEAF_STAMP
#define RFP_LEAF_STAMP(k)
#endif

namespace rfp {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct M16;
template <>
struct M16<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc op(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct M16<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc op(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// D: width of the block columns whose diagonal blocks are factored and
// inverted by one wavefront.
constexpr int N = 128, D = 16, DP = D + 2;

// Packed lower-triangle layout: block row b (rows 16b .. 16b + 15) keeps
// columns 0 .. 16b + 15 of each row, with a row pitch of 16b + 18 elements
// (the padding shifts consecutive rows by 4 or 36 banks, so the 16 rows that
// feed one MFMA operand hit distinct banks).  prow(i) is the offset of row i.
__device__ __forceinline__ int prow(int i)
{
    const int b = i >> 4;
    return 128 * b * b + 160 * b + (i & 15) * (16 * b + 18);
}
constexpr int NPACK = 128 * 8 * 8 + 160 * 8;  // prow(N): 9472 elements

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Broadcast of lane l's value to the whole wavefront (l uniform).
__device__ __forceinline__ double bcast(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bcast(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1 / sqrt(d) and sqrt(d) of a positive pivot: the hardware reciprocal
// square root estimate refined by two coupled Newton (Goldschmidt) steps on
// g ~ sqrt(d) and h ~ 1 / (2 sqrt(d)) (each squares the relative error), then
// one residual correction of the root; both results come out within about
// one unit in the last place.  Pivots too small for the hardware estimate
// take the library routines.
__device__ __forceinline__ void rsqrt_sqrt(double d, double& rl, double& l)
{
    if (d < 1e-280) {
        l = sqrt(d);
        rl = 1.0 / l;
        return;
    }
    const double y = __builtin_amdgcn_rsq(d);
    double g = d * y, h = 0.5 * y;
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const double r = __builtin_fma(-g, h, 0.5);
        g = __builtin_fma(g, r, g);
        h = __builtin_fma(h, r, h);
    }
    const double e = __builtin_fma(-g, g, d);
    l = __builtin_fma(e, h, g);
    rl = 2.0 * h;
}
__device__ __forceinline__ void rsqrt_sqrt(float d, float& rl, float& l)
{
    if (d < 1e-30f) {
        l = sqrtf(d);
        rl = 1.0f / l;
        return;
    }
    const float y = __builtin_amdgcn_rsqf(d);
    const float h = 0.5f * y, g = d * y;
    const float r = __builtin_fmaf(-g, h, 0.5f);
    rl = 2.0f * __builtin_fmaf(h, r, h);
    l = __builtin_fmaf(g, r, g);
}

// Cholesky factor and its inverse of the D x D diagonal block at (o, o) of
// the LDS matrix, by one wavefront in registers, both right-looking.  Lane
// i < D holds row i of the block (a), and lane c < D the running column c of
// W = L^{-1} (s).  At column j: the pivot a_jj is broadcast (readlane),
// l_jj = sqrt(a_jj), the column becomes l_ij = a_ij / l_jj; row j of W is
// final, W(j, c) = s_j / l_jj; then every later row c takes the broadcast
// l_cj = L(c, j) into both recurrences, a_ck -= l_cj l_kj for the factor and
// s_c -= L(c, j) W(j, .) for the inverse (forward substitution of L W = I,
// accumulated as the columns of L appear).  Entries above the diagonal are
// never read.  Returns 0, or j + 1 for the first pivot that is not positive
// (uniform; nothing is stored then).  On success the factor goes back to L
// and the inverse to Wd (row-major, zero above the diagonal).
template <typename T>
__device__ __forceinline__ int chol_inv(T* L, int o, T (*Wd)[DP], int lane)
{
    const int i = lane;
    T a[D], s[D];
#pragma unroll
    for (int j = 0; j < D; j++) {
        a[j] = (i < D && j <= i) ? L[prow(o + i) + o + j] : T(0);
        s[j] = (j == i) ? T(1) : T(0);
    }
    int fail = 0;
#pragma unroll
    for (int j = 0; j < D; j++) {
        T d = bcast(a[j], j);
        if (!(d > T(0)) && !fail) fail = j + 1;
        if (fail) d = T(1);  // keep the remaining steps finite; the result is discarded
        T rl, l;
        rsqrt_sqrt(d, rl, l);
        a[j] = (i == j) ? l : a[j] * rl;
        const T wj = (j >= i) ? s[j] * rl : T(0);
        s[j] = wj;
#pragma unroll
        for (int c = j + 1; c < D; c++) {
            const T lcj = bcast(a[j], c);
            a[c] -= a[j] * lcj;
            s[c] -= lcj * wj;
        }
    }
    if (fail) return fail;
    if (i < D) {
#pragma unroll
        for (int j = 0; j < D; j++) {
            if (j <= i) L[prow(o + i) + o + j] = a[j];
            Wd[j][i] = s[j];
        }
    }
    wave_sync();
    return 0;
}

template <typename T>
struct Leaf128Smem {
    __attribute__((aligned(16))) T L[NPACK];
    __attribute__((aligned(16))) T Wd[D][DP];  // inverse of the current diagonal block
    int fail;
};

}  // namespace

// Factor the lower triangle of A (order nb <= 128) in place; when winv is not
// null, write W = L^{-1} to it (128 x 128 row-major, zero above the diagonal,
// identity on the padding).  Returns 0, or j + 1 for the first pivot j that
// is not positive (then *info = info_base + j + 1 when info is not null and
// A is left partly updated).  All 256 threads must call it; it ends with a
// barrier.
template <typename T>
__device__ int potrf128_block(Leaf128Smem<T>& sm, Mat<T> A, int nb, T* winv, int* info, int64_t info_base)
{
    T* L = sm.L;
    T(&Wd)[D][DP] = sm.Wd;  // Wd[r][c] = (L_jj^{-1})(r, c)
    int& fail = sm.fail;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = lane & 15, g = lane >> 4;  // MFMA operand row and k offset of the lane
    if (t == 0) fail = 0;
    const bool colmajor = A.rs == 1;
    // the packed triangle (and the rest of each diagonal block, as zeros);
    // rows past nb are the identity
#pragma unroll 16
    for (int it = 0; it < N * N / 256; it++) {
        const int idx = t + it * 256;
        const int i = colmajor ? idx % N : idx / N;
        const int j = colmajor ? idx / N : idx % N;
        if (j < 16 * ((i >> 4) + 1)) {
            T v = (i == j) ? T(1) : T(0);
            if (i < nb && j <= i) v = A.at(i, j);
            L[prow(i) + j] = v;
        }
    }
    __syncthreads();
    RFP_LEAF_STAMP(0);

    const int nblk = (nb + D - 1) / D;
    typedef typename M16<T>::acc acc_t;

    // ---------------------------------------------------------------- factor
    for (int kb = 0; kb < nblk; kb++) {
        const int o = kb * D;
        // wavefront 0 factors and inverts the diagonal block (a failing pivot
        // is recorded in `fail`); the inverse is parked in its final place in
        // winv, where the inversion phase picks it up again
        if (w == 0) {
            const int f = chol_inv<T>(L, o, Wd, lane);
            if (f) {
                if (lane == 0) fail = o + f;
            } else if (winv && lane < D) {
                for (int q = 0; q < D; q++) winv[(o + q) * N + o + lane] = Wd[q][lane];
            }
            RFP_LEAF_STAMP(40 + 2 * kb);
        }
        __syncthreads();
        RFP_LEAF_STAMP(1 + 3 * kb);
        if (fail) break;
        const int r0 = o + D, nrb = (N - r0) / 16;  // 16-row blocks below
        // panel: X(i, c) = sum_k L(i, o + k) W(c, k), i.e. X = A_p W^T; a wave
        // owns whole row blocks, so reading and overwriting them is race-free
        for (int rb = w; rb < nrb; rb += 4) {
            acc_t x0 = acc_t{0, 0, 0, 0};
            const T* Lr = L + prow(r0 + rb * 16 + r) + o;
#pragma unroll
            for (int kk = 0; kk < D; kk += 4) x0 = M16<T>::op(Lr[kk + g], Wd[r][kk + g], x0);
#pragma unroll
            for (int q = 0; q < 4; q++) L[prow(r0 + rb * 16 + M16<T>::row(lane, q)) + o + r] = x0[q];
        }
        __syncthreads();
        RFP_LEAF_STAMP(2 + 3 * kb);
        // trailing update of the lower triangle of 16 x 16 blocks below/right
        const int nt = nrb * (nrb + 1) / 2;
        for (int b = w; b < nt; b += 4) {
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= b) bi++;
            const int bj = b - bi * (bi + 1) / 2;
            acc_t s = acc_t{0, 0, 0, 0};
            const T* X = L + prow(r0 + bi * 16 + r) + o;
            const T* Y = L + prow(r0 + bj * 16 + r) + o;
#pragma unroll
            for (int kk = 0; kk < D; kk += 4) s = M16<T>::op(X[kk + g], Y[kk + g], s);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = bi * 16 + M16<T>::row(lane, q), j = bj * 16 + r;
                if (i >= j) L[prow(r0 + i) + r0 + j] -= s[q];
            }
        }
        __syncthreads();
        RFP_LEAF_STAMP(3 + 3 * kb);
    }
    if (fail) {
        const int f = fail;
        __syncthreads();
        if (t == 0 && info) *info = (int)(info_base + f);
        return f;
    }
    // store the factor: its own lower triangle only
#pragma unroll 16
    for (int idx = t; idx < N * N; idx += 256) {
        const int i = colmajor ? idx % N : idx / N;
        const int j = colmajor ? idx / N : idx % N;
        if (i < nb && j <= i) A.at(i, j) = L[prow(i) + j];
    }
    RFP_LEAF_STAMP(30);
    if (!winv) {
        __syncthreads();
        return 0;
    }

    // --------------------------------------------------------------- inverse
    for (int kb = nblk - 1; kb >= 0; kb--) {
        const int o = kb * D;
        __syncthreads();
        for (int idx = t; idx < D * D; idx += 256) Wd[idx / D][idx % D] = winv[(o + idx / D) * N + o + idx % D];
        __syncthreads();
        const int r0 = o + D, nrb = (N - r0) / 16;
        // T = W_RR L_Rj  (W_RR already in place, lower triangular).  A wave owns
        // the row blocks w and w + 4 (at most seven row blocks exist).
        acc_t tacc[2];
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = w + 4 * q2;
            tacc[q2] = acc_t{0, 0, 0, 0};
            if (rb < nrb) {
                const T* Xr = L + prow(r0 + rb * 16 + r) + r0;
                const int kend = (rb + 1) * 16;  // W_RR(i, k) = 0 for k > i
                for (int kk = 0; kk < kend; kk += 4)
                    tacc[q2] = M16<T>::op(Xr[kk + g], L[prow(r0 + kk + g) + o + r], tacc[q2]);
            }
        }
        __syncthreads();  // every wave has read L_Rj
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = w + 4 * q2;
            if (rb < nrb) {
#pragma unroll
                for (int q = 0; q < 4; q++) L[prow(r0 + rb * 16 + M16<T>::row(lane, q)) + o + r] = tacc[q2][q];
            }
        }
        // W_Rj = -T W_jj, in place on the wave's own rows
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = w + 4 * q2;
            if (rb < nrb) {
                acc_t y0 = acc_t{0, 0, 0, 0};
                const T* Lr = L + prow(r0 + rb * 16 + r) + o;
                wave_sync();
#pragma unroll
                for (int kk = 0; kk < D; kk += 4) y0 = M16<T>::op(Lr[kk + g], Wd[kk + g][r], y0);
                wave_sync();
#pragma unroll
                for (int q = 0; q < 4; q++) L[prow(r0 + rb * 16 + M16<T>::row(lane, q)) + o + r] = -y0[q];
            }
        }
        // the diagonal block becomes its inverse
        if (w == 0 && lane < D) {
#pragma unroll
            for (int q = 0; q < D; q++)
                if (q >= lane) L[prow(o + q) + o + lane] = Wd[q][lane];
        }
    }
    __syncthreads();
    RFP_LEAF_STAMP(31);
    // W row-major into winv (zero above the diagonal, identity on padding)
    for (int idx = t; idx < N * N; idx += 256) {
        const int i = idx / N, j = idx % N;
        winv[idx] = (j <= i) ? L[prow(i) + j] : T(0);
    }
    __syncthreads();
    return 0;
}

}  // namespace rfp
