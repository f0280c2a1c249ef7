// Fused Cholesky of one diagonal block of order <= 128 with the inverse of
// its factor, as a workgroup-level device routine (256 threads): used by the
// leaf kernel of the blocked factorization and by the batched solver.
//
// The workgroup keeps the whole block in LDS (128 x 130 elements, rows
// k-contiguous).  For each 32-column block column:
//   1. one wavefront factors the 32 x 32 diagonal block (row per lane, the
//      pivot column broadcast through LDS) and inverts it;
//   2. all four wavefronts solve the panel below with MFMA, X = A_p W^T;
//   3. all four wavefronts update the trailing lower triangle, A -= X X^T.
// The factor is stored back (masked to the block's own lower triangle), then
// W = L^{-1} is formed in place, block column by block column from the right:
// W_RR is already inverted, so W_Rj = -(W_RR L_Rj) W_jj.
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
// inverted by one wavefront (16 or 32; the sequential work per leaf grows
// with D, the MFMA panel and trailing work does not).
constexpr int N = 128, LP = N + 2, D = 16, DP = D + 2;
constexpr bool TWO_HALVES = D > 16;

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// acc(16 x 16) += sum_k X(xr + i, xk + k) * Y(yr + j, yk + k), k < K (multiple of 4),
// X and Y rows k-contiguous in LDS with pitch P.  Lane l supplies k = kk + l/16.
template <typename T, int P>
__device__ __forceinline__ void mma_rows(typename M16<T>::acc& acc, const T (*X)[P], int xr, int xk,
                                         const T (*Y)[P], int yr, int yk, int K, int lane)
{
    const int r = lane & 15, g = lane >> 4;
    for (int kk = 0; kk < K; kk += 4)
        acc = M16<T>::op(X[xr + r][xk + kk + g], Y[yr + r][yk + kk + g], acc);
}

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

// Cholesky of the 32 x 32 diagonal block at (o, o) of the LDS matrix by one
// wavefront, right-looking in registers: lane i < 32 holds row i; at column
// j the pivot and the column entries l_cj are broadcast from their lanes
// (readlane), l_jj = sqrt(a_jj), l_ij = a_ij / l_jj, and every row updates
// a_ic -= l_ij l_cj for c > j.  Entries above the diagonal are never read.
// Returns 0, or j + 1 for the first pivot that is not positive (uniform);
// on success the factor is stored back to LDS.
template <typename T>
__device__ __forceinline__ int chol32(T (*L)[LP], int o, int lane)
{
    const int i = lane;
    T a[D];
#pragma unroll
    for (int j = 0; j < D; j++) a[j] = (i < D && j <= i) ? L[o + i][o + j] : T(0);
#pragma unroll
    for (int j = 0; j < D; j++) {
        const T d = bcast(a[j], j);
        if (!(d > T(0))) return j + 1;
        const T l = sqrt(d), rl = T(1) / l;
        a[j] = (i == j) ? l : a[j] * rl;
#pragma unroll
        for (int c = j + 1; c < D; c++) a[c] -= a[j] * bcast(a[j], c);
    }
#pragma unroll
    for (int j = 0; j < D; j++)
        if (i < D && j <= i) L[o + i][o + j] = a[j];
    wave_sync();
    return 0;
}

// Inverse of the lower-triangular 32 x 32 block at (o, o): lane c < 32 forms
// column c by forward substitution in registers, W(r, c) = (delta_rc -
// sum_{q<r} L(r, q) W(q, c)) / L(r, r), with each L(r, q) broadcast from
// lane r's copy of row r; the result goes to Wd (row-major, zero above the
// diagonal).  rdg is unused (kept for the call signature).
template <typename T>
__device__ __forceinline__ void inv32(T (*L)[LP], int o, T (*Wd)[DP], T* rdg, int lane)
{
    (void)rdg;
    const int c = lane;
    T a[D], w[D];
#pragma unroll
    for (int j = 0; j < D; j++) a[j] = (c < D && j <= c) ? L[o + c][o + j] : T(0);
#pragma unroll
    for (int r = 0; r < D; r++) {
        T s = (r == c) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < r; q++) s -= bcast(a[q], r) * w[q];
        const T rr = T(1) / bcast(a[r], r);
        w[r] = (r >= c) ? s * rr : T(0);
    }
    if (c < D) {
#pragma unroll
        for (int r = 0; r < D; r++) Wd[r][c] = w[r];
    }
    wave_sync();
}

template <typename T>
struct Leaf128Smem {
    __attribute__((aligned(16))) T L[N][LP];
    __attribute__((aligned(16))) T Wd[D][DP];
    T rdg[D];
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
    T(&L)[N][LP] = sm.L;
    T(&Wd)[D][DP] = sm.Wd;  // Wd[r][c] = (L_jj^{-1})(r, c)
    T* rdg = sm.rdg;
    int& fail = sm.fail;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) fail = 0;
    const bool colmajor = A.rs == 1;
#pragma unroll 16
    for (int it = 0; it < N * N / 256; it++) {
        const int idx = t + it * 256;
        const int i = colmajor ? idx % N : idx / N;
        const int j = colmajor ? idx / N : idx % N;
        T v = (i == j) ? T(1) : T(0);
        if (i < nb && j <= i) v = A.at(i, j);
        L[i][j] = v;
    }
    __syncthreads();
    RFP_LEAF_STAMP(0);

    const int nblk = (nb + D - 1) / D;
    typedef typename M16<T>::acc acc_t;

    // factor the 32 x 32 diagonal block at offset o (wavefront 0) and leave
    // its inverse in Wd; a failing pivot is recorded in `fail`
    // (the inverse of each diagonal block is also parked in its final place in
    // winv, where the inversion phase picks it up again)
    auto diag = [&](int o, bool factor) {
        if (factor) {
            if (w == 0) {
                const int f = chol32<T>(L, o, lane);
                if (f) {
                    if (lane == 0) fail = o + f;
                    return;
                }
                RFP_LEAF_STAMP(40 + 2 * (o / D));
                inv32<T>(L, o, Wd, rdg, lane);
                RFP_LEAF_STAMP(41 + 2 * (o / D));
                if (winv && lane < D) {
                    for (int r = 0; r < D; r++) winv[(o + r) * N + o + lane] = Wd[r][lane];
                }
            }
        } else {
            for (int idx = t; idx < D * D; idx += 256) Wd[idx / D][idx % D] = winv[(o + idx / D) * N + o + idx % D];
        }
    };

    // ---------------------------------------------------------------- factor
    for (int kb = 0; kb < nblk; kb++) {
        const int o = kb * D;
        diag(o, true);
        __syncthreads();
        RFP_LEAF_STAMP(1 + 3 * kb);
        if (fail) break;
        const int r0 = o + D, nrb = (N - r0) / 16;  // 16-row blocks below
        // panel: X(i, c) = sum_k L(i, o + k) W(c, k), i.e. X = A_p W^T; a wave
        // owns whole row blocks, so reading and overwriting them is race-free
        for (int rb = w; rb < nrb; rb += 4) {
            acc_t x0 = acc_t{0, 0, 0, 0}, x1 = acc_t{0, 0, 0, 0};
            (void)x1;
            {
                const int r = lane & 15, g = lane >> 4;
#pragma unroll
                for (int kk = 0; kk < D; kk += 4) {
                    const T av = L[r0 + rb * 16 + r][o + kk + g];
                    x0 = M16<T>::op(av, Wd[r][kk + g], x0);
                    if constexpr (TWO_HALVES) x1 = M16<T>::op(av, Wd[16 + r][kk + g], x1);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = r0 + rb * 16 + M16<T>::row(lane, q);
                L[i][o + (lane & 15)] = x0[q];
                if constexpr (TWO_HALVES) L[i][o + 16 + (lane & 15)] = x1[q];
            }
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
            mma_rows<T, LP>(s, L, r0 + bi * 16, o, L, r0 + bj * 16, o, D, lane);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = bi * 16 + M16<T>::row(lane, q), j = bj * 16 + (lane & 15);
                if (i >= j) L[r0 + i][r0 + j] -= s[q];
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
        if (i < nb && j <= i) A.at(i, j) = L[i][j];
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
        diag(o, false);  // Wd = L_jj^{-1}, as parked in winv by the factor phase
        __syncthreads();
        const int r0 = o + D, nrb = (N - r0) / 16;
        // T = W_RR L_Rj  (W_RR already in place, lower triangular).  A wave owns
        // the row blocks w and w + 4 (at most seven row blocks exist).
        acc_t tacc[2][2];
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = w + 4 * q2;
            tacc[q2][0] = acc_t{0, 0, 0, 0};
            tacc[q2][1] = acc_t{0, 0, 0, 0};
            if (rb < nrb) {
                const int r = lane & 15, g = lane >> 4;
                const int kend = (rb + 1) * 16;  // W_RR(i, k) = 0 for k > i
                for (int kk = 0; kk < kend; kk += 4) {
                    const T av = L[r0 + rb * 16 + r][r0 + kk + g];
                    tacc[q2][0] = M16<T>::op(av, L[r0 + kk + g][o + r], tacc[q2][0]);
                    if constexpr (TWO_HALVES)
                        tacc[q2][1] = M16<T>::op(av, L[r0 + kk + g][o + 16 + r], tacc[q2][1]);
                }
            }
        }
        __syncthreads();  // every wave has read L_Rj
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = w + 4 * q2;
            if (rb < nrb) {
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int i = r0 + rb * 16 + M16<T>::row(lane, q);
                    L[i][o + (lane & 15)] = tacc[q2][0][q];
                    if constexpr (TWO_HALVES) L[i][o + 16 + (lane & 15)] = tacc[q2][1][q];
                }
            }
        }
        // W_Rj = -T W_jj, in place on the wave's own rows
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = w + 4 * q2;
            if (rb < nrb) {
                acc_t y0 = acc_t{0, 0, 0, 0}, y1 = acc_t{0, 0, 0, 0};
                const int r = lane & 15, g = lane >> 4;
                wave_sync();
#pragma unroll
                for (int kk = 0; kk < D; kk += 4) {
                    const T av = L[r0 + rb * 16 + r][o + kk + g];
                    y0 = M16<T>::op(av, Wd[kk + g][r], y0);
                    if constexpr (TWO_HALVES) y1 = M16<T>::op(av, Wd[kk + g][16 + r], y1);
                }
                wave_sync();
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int i = r0 + rb * 16 + M16<T>::row(lane, q);
                    L[i][o + (lane & 15)] = -y0[q];
                    if constexpr (TWO_HALVES) L[i][o + 16 + (lane & 15)] = -y1[q];
                }
            }
        }
        // the diagonal block becomes its inverse
        if (w == 0 && lane < D) {
#pragma unroll
            for (int r = 0; r < D; r++)
                if (r >= lane) L[o + r][o + lane] = Wd[r][lane];
        }
    }
    __syncthreads();
    RFP_LEAF_STAMP(31);
    // W row-major into winv (zero above the diagonal, identity on padding)
    for (int idx = t; idx < N * N; idx += 256) {
        const int i = idx / N, j = idx % N;
        winv[idx] = (j <= i) ? L[i][j] : T(0);
    }
    __syncthreads();
    return 0;
}


}  // namespace rfp
