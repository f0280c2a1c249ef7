// Fused Cholesky of one diagonal block of order <= 128 with the inverse of
// its factor, as a workgroup-level device routine (256 threads): used by the
// leaf kernel of the blocked factorization and by the batched solver.
//
// The workgroup keeps the lower triangle of the block in LDS, packed by
// 16-row block rows (75.8 KB: small enough to share a CU with one workgroup
// of the bulk-update GEMM, so that a leaf on a second stream starts as soon
// as one GEMM workgroup retires instead of waiting for a whole CU).  For
// each 16-column block column:
//   1. one wavefront factors the 16 x 16 diagonal block (left-looking, rows
//      in lanes) and inverts it (columns in lanes);
//   2. all four wavefronts solve the panel below with MFMA, X = A_p W^T;
//   3. the trailing lower triangle is updated, A -= X X^T: block column k + 1
//      at once by all four wavefronts, the columns beyond it by wavefronts
//      1-3 while wavefront 0 factors diagonal block k + 1.
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
// the packed LDS matrix, by one wavefront (lane i = lane % 16 works on row i;
// lanes 16..63 repeat lanes 0..15 and store nothing).
//
// Factor, left-looking: at column j every row forms
//   t_i = a_ij - sum_{q<j} l_iq l_jq
// from its own earlier entries l_iq (registers) and row j of L, which lane j
// has written to LDS column by column (broadcast reads, issued ahead of
// need); only the newest entry l_{j,j-1} comes by readlane from lane j, so
// the step-to-step chain is that product, the pivot broadcast t_j and the
// refined reciprocal square root: l_jj = sqrt(t_j), l_ij = t_i / l_jj.
//
// Inverse W = L^{-1}, by columns: lane c forms column c by forward
// substitution, W(r, c) = (delta_rc - sum_{q<r} L(r, q) W(q, c)) / l_rr, with
// L(r, q) read from LDS (broadcast) and 1 / l_rr kept from the factor.
//
// Entries above the diagonal are never read.  Returns 0, or j + 1 for the
// first pivot that is not positive (uniform; the block is left partly
// written then).  On success the factor is in L and the inverse in Wd
// (row-major, zero above the diagonal).
template <typename T>
__device__ __forceinline__ int chol_inv(T* L, int o, T (*Wd)[DP], int lane)
{
    const int i = lane & 15;
    const bool owner = lane < 16;
    T* Lrow = L + prow(o + i) + o;  // row i of the block
    T a[D], rl[D];
#pragma unroll
    for (int j = 0; j < D; j++) a[j] = (j <= i) ? Lrow[j] : T(0);
    int fail = 0;
    // part = a_ij - sum_{q<j-1} l_iq l_jq, formed one column ahead (its
    // operands are final one step early), so that it overlaps the previous
    // pivot
    T part = a[0];
#pragma unroll
    for (int j = 0; j < D; j++) {
        // the pivot lane finishes its own t with its own l_{j,j-1}; the other
        // rows need that entry by broadcast, off the pivot's chain
        T d, t;
        if (j > 0) {
            d = bcast(part - a[j - 1] * a[j - 1], j);
            t = part - a[j - 1] * bcast(a[j - 1], j);
        } else {
            d = bcast(part, 0);
            t = part;
        }
        if (!(d > T(0)) && !fail) fail = j + 1;  // a failed block is discarded
        T nxt = T(0);
        if (j + 1 < D) {
            const T* Ln = L + prow(o + j + 1) + o;
            nxt = a[j + 1];
#pragma unroll
            for (int q = 0; q < j; q++) nxt -= a[q] * Ln[q];
        }
        T r, l;
        rsqrt_sqrt(d, r, l);
        rl[j] = r;
        a[j] = (i == j) ? l : t * r;  // rows above j: unused values, never stored
        if (owner && i >= j) Lrow[j] = a[j];
        part = nxt;
    }
    if (fail) return fail;
    // inverse, column c = i
    T w[D];
#pragma unroll
    for (int rr = 0; rr < D; rr++) {
        const T* Lr = L + prow(o + rr) + o;
        T s = (rr == i) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < rr; q++) s -= Lr[q] * w[q];
        w[rr] = (rr >= i) ? s * rl[rr] : T(0);
    }
    if (owner) {
#pragma unroll
        for (int rr = 0; rr < D; rr++) Wd[rr][i] = w[rr];
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

// The packed lower triangle of A (order nb <= 128) into L (and the rest of
// each diagonal block, as zeros); rows past nb are the identity.  All 256
// threads; no barrier at the end.
template <typename T>
__device__ __forceinline__ void leaf128_load(T* L, Mat<T> A, int nb)
{
    const int t = threadIdx.x;
    const bool colmajor = A.rs == 1;
    // In two batches of 32 per thread: all loads first (each lane from its
    // element clamped into the stored lower triangle, a valid address), then
    // the LDS stores.  A's pointer is generic, so a load written after an LDS
    // store could not be moved ahead of it: interleaved, every element would
    // wait for its own load.
    for (int it0 = 0; it0 < N * N / 256; it0 += 32) {
        T a[32];
#pragma unroll
        for (int u = 0; u < 32; u++) {
            const int idx = t + (it0 + u) * 256;
            const int i = colmajor ? idx % N : idx / N;
            const int j = colmajor ? idx / N : idx % N;
            const int ic = i < nb ? i : nb - 1, jc = j < ic ? j : ic;
            a[u] = nb > 0 ? A.at(ic, jc) : T(0);
        }
#pragma unroll
        for (int u = 0; u < 32; u++) {
            const int idx = t + (it0 + u) * 256;
            const int i = colmajor ? idx % N : idx / N;
            const int j = colmajor ? idx / N : idx % N;
            if (j < 16 * ((i >> 4) + 1)) {
                T v = (i == j) ? T(1) : T(0);
                if (i < nb && j <= i) v = a[u];
                L[prow(i) + j] = v;
            }
        }
    }
}

// L's own lower triangle (order nb) back into A (the other triangle of A is
// another block's data).  All 256 threads; no barrier.
template <typename T>
__device__ __forceinline__ void leaf128_store(const T* L, Mat<T> A, int nb)
{
    const int t = threadIdx.x;
    const bool colmajor = A.rs == 1;
    // its own lower triangle only, with stepped addresses
    // (column-major: each thread one row, every other column; row-major: one
    // row per wave and step, one column per lane)
    // (LDS reads batched ahead of the stores, as for the load; reads past a
    // packed row stay inside L and are not stored)
    if (colmajor) {
        const int i = t & (N - 1), j0 = t >> 7;
        if (i < nb) {
            T* a = A.p + i + (int64_t)j0 * A.cs;
            const T* l = L + prow(i) + j0;
            for (int u0 = 0; u0 < N / 2 && j0 + 2 * u0 <= i; u0 += 16) {
                T v[16];
#pragma unroll
                for (int u = 0; u < 16; u++) v[u] = l[2 * (u0 + u)];
#pragma unroll
                for (int u = 0; u < 16; u++)
                    if (j0 + 2 * (u0 + u) <= i) a[2 * (int64_t)(u0 + u) * A.cs] = v[u];
            }
        }
    } else {
        const int j = t & (N - 1);
        const int64_t jo = (int64_t)j * A.cs;
        for (int i0 = t >> 7; i0 < nb; i0 += 32) {
            T v[16];
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int i = i0 + 2 * u;
                v[u] = L[prow(i < N ? i : N - 1) + j];
            }
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int i = i0 + 2 * u;
                if (i < nb && j <= i) A.p[(int64_t)i * A.rs + jo] = v[u];
            }
        }
    }
}

// W = L^{-1} in place in L, from the factor in L and the inverses W_jj of its
// nblk diagonal 16 x 16 blocks parked in winv (128 x 128 row-major, at their
// final places); with write_winv the whole W then goes to winv (zero above
// the diagonal).  All 256 threads; ends with a barrier.
template <typename T>
__device__ __forceinline__ void leaf128_invert(Leaf128Smem<T>& sm, int nblk, T* winv, bool write_winv)
{
    T* L = sm.L;
    T(&Wd)[D][DP] = sm.Wd;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = lane & 15, g = lane >> 4;
    typedef typename M16<T>::acc acc_t;
    // --------------------------------------------------------------- inverse
    // Step kb (right to left): T = W_RR L_Rj, then W_Rj = -T W_jj.  T is
    // formed transposed (operands swapped), which leaves each lane holding
    // T(lane % 16, kappa_q) with kappa_q the accumulator row index of
    // register q: exactly the A operand of the second product when its B
    // operand is read at the same kappa_q, so T never goes through LDS.  The
    // parked W_jj is fetched one step ahead (one element per thread).  Row
    // blocks per wave: {w, 6 - w} for w < 3, {3} for wave 3 (at most seven).
    T wnext = nblk > 0 ? winv[((nblk - 1) * D + t / 16) * N + (nblk - 1) * D + t % 16] : T(0);
    for (int kb = nblk - 1; kb >= 0; kb--) {
        const int o = kb * D;
        __syncthreads();  // the previous step is done with Wd and with L
        Wd[t / 16][t % 16] = wnext;
        if (kb > 0) wnext = winv[(o - D + t / 16) * N + o - D + t % 16];
        const int r0 = o + D, nrb = (N - r0) / 16;
        const int rbs[2] = {w, w < 3 ? 6 - w : 7};
        // W_RR(i, k) = 0 for k past row i's block, so row block rb needs
        // k < 16 (rb + 1).  The two row blocks share the L_Rj operand, and
        // each sum is split over even and odd k steps: four independent
        // accumulation chains instead of one or two long ones.
        const int ke0 = rbs[0] < nrb ? (rbs[0] + 1) * 16 : 0, ke1 = rbs[1] < nrb ? (rbs[1] + 1) * 16 : 0;
        const T* Wr0 = L + prow(r0 + rbs[0] * 16 + r) + r0;  // W_RR, row r of each block
        const T* Wr1 = L + prow(r0 + rbs[1] * 16 + r) + r0;
        acc_t t00 = acc_t{0, 0, 0, 0}, t01 = t00, t10 = t00, t11 = t00;
        const int kboth = ke0 < ke1 ? ke0 : ke1;
        int kk = 0;
#pragma unroll 2
        for (; kk < kboth; kk += 8) {
            const T l0 = L[prow(r0 + kk + g) + o + r], l1 = L[prow(r0 + kk + 4 + g) + o + r];
            t00 = M16<T>::op(l0, Wr0[kk + g], t00);
            t10 = M16<T>::op(l0, Wr1[kk + g], t10);
            t01 = M16<T>::op(l1, Wr0[kk + 4 + g], t01);
            t11 = M16<T>::op(l1, Wr1[kk + 4 + g], t11);
        }
        for (int k2 = kk; k2 < ke0; k2 += 8) {
            t00 = M16<T>::op(L[prow(r0 + k2 + g) + o + r], Wr0[k2 + g], t00);
            t01 = M16<T>::op(L[prow(r0 + k2 + 4 + g) + o + r], Wr0[k2 + 4 + g], t01);
        }
#pragma unroll 2
        for (int k2 = kk; k2 < ke1; k2 += 8) {
            t10 = M16<T>::op(L[prow(r0 + k2 + g) + o + r], Wr1[k2 + g], t10);
            t11 = M16<T>::op(L[prow(r0 + k2 + 4 + g) + o + r], Wr1[k2 + 4 + g], t11);
        }
        const acc_t tacc[2] = {t00 + t01, t10 + t11};
        __syncthreads();  // every wave has read L_Rj; W_jj is in Wd
#pragma unroll
        for (int q2 = 0; q2 < 2; q2++) {
            const int rb = rbs[q2];
            if (rb < nrb) {
                acc_t y = acc_t{0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; q++) y = M16<T>::op(tacc[q2][q], Wd[M16<T>::row(lane, q)][r], y);
#pragma unroll
                for (int q = 0; q < 4; q++) L[prow(r0 + rb * 16 + M16<T>::row(lane, q)) + o + r] = -y[q];
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
    // W row-major into winv (zero above the diagonal, identity on padding),
    // LDS reads batched ahead of the stores
    for (int it0 = 0; write_winv && it0 < N * N / 256; it0 += 16) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int idx = t + (it0 + u) * 256, i = idx / N, j = idx % N;
            v[u] = (j <= i) ? L[prow(i) + j] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 16; u++) winv[t + (it0 + u) * 256] = v[u];
    }
    __syncthreads();
}

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
    RFP_LEAF_STAMP(32);
    if (t == 0) fail = 0;
    leaf128_load<T>(L, A, nb);
    __syncthreads();
    RFP_LEAF_STAMP(0);

    const int nblk = (nb + D - 1) / D;
    typedef typename M16<T>::acc acc_t;

    // Trailing update of step k, A -= X X^T over the 16 x 16 blocks (bi, bj),
    // bi >= bj, of the lower triangle below diagonal block k (indices
    // relative to block k + 1).  It is split by block column: column bj = 0
    // (the next diagonal block and the panel below it) is needed at once;
    // the columns bj >= 1 only one step later, so they are applied by
    // wavefronts 1-3 while wavefront 0 factors the next diagonal block.  Each
    // element still receives the updates of steps 0, 1, ... in order.
    auto update_block = [&](int o, int bi, int bj) {
        const int r0 = o + D;
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
    };

    // ---------------------------------------------------------------- factor
    for (int kb = 0; kb < nblk; kb++) {
        const int o = kb * D;
        if (w == 0) {
            // wavefront 0 factors and inverts the diagonal block (a failing
            // pivot is recorded in `fail`); the inverse is parked in its final
            // place in winv, where the inversion phase picks it up again
            const int f = chol_inv<T>(L, o, Wd, lane);
            if (f) {
                if (lane == 0) fail = o + f;
            } else if (winv && lane < D) {
                for (int q = 0; q < D; q++) winv[(o + q) * N + o + lane] = Wd[q][lane];
            }
            RFP_LEAF_STAMP(40 + 2 * kb);
        } else if (kb > 0) {
            // the rest of step kb - 1's update: block columns bj >= 1 (the
            // columns beyond diagonal block kb), as a triangle of
            // (nrb - 1) x (nrb - 1) blocks
            const int op = o - D, nrb = (N - o) / 16, cnt = nrb * (nrb - 1) / 2;
            for (int b = w - 1; b < cnt; b += 3) {
                int bi = 0;
                while ((bi + 1) * (bi + 2) / 2 <= b) bi++;
                const int bj = b - bi * (bi + 1) / 2;
                update_block(op, bi + 1, bj + 1);
            }
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
        // step kb's update of block column 0 (the next diagonal block and the
        // blocks below it)
        for (int bi = w; bi < nrb; bi += 4) update_block(o, bi, 0);
        __syncthreads();
        RFP_LEAF_STAMP(3 + 3 * kb);
    }
    if (fail) {
        const int f = fail;
        __syncthreads();
        if (t == 0 && info) *info = (int)(info_base + f);
        return f;
    }
    leaf128_store<T>(L, A, nb);
    RFP_LEAF_STAMP(30);
    if (!winv) {
        __syncthreads();
        return 0;
    }

    leaf128_invert<T>(sm, nblk, winv, true);
    RFP_LEAF_STAMP(33);
    __syncthreads();
    return 0;
}

// In-place inverse W = L^{-1} of the lower-triangular A (order nb <= 128):
// the four wavefronts invert the diagonal 16 x 16 blocks (two each, lane c
// forming column c by forward substitution) and park them in scratch (128 x
// 128 row-major), then the block columns are formed from the right as in the
// factorization leaf (W_Rj = -(W_RR L_Rj) W_jj on MFMA).  Returns 0, or i + 1
// for the first exactly zero diagonal entry i (then *info = info_base + i + 1
// when info is not null, and A is unchanged).  All 256 threads must call it;
// it ends with a barrier.
template <typename T>
__device__ int trtri128_block(Leaf128Smem<T>& sm, Mat<T> A, int nb, T* scratch, int* info, int64_t info_base)
{
    T* L = sm.L;
    int& fail = sm.fail;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) fail = 1 << 30;
    leaf128_load<T>(L, A, nb);
    __syncthreads();
    if (t < nb && L[prow(t) + t] == T(0)) atomicMin(&fail, t + 1);
    __syncthreads();
    if (fail < (1 << 30)) {
        const int f = fail;
        __syncthreads();
        if (t == 0 && info) *info = (int)(info_base + f);
        return f;
    }
    const int nblk = (nb + D - 1) / D;
    for (int kb = w; kb < nblk; kb += 4) {
        const int o = kb * D;
        if (lane < D) {
            const int c = lane;
            T wv[D];
#pragma unroll
            for (int rr = 0; rr < D; rr++) {
                const T* Lr = L + prow(o + rr) + o;
                T sum = (rr == c) ? T(1) : T(0);
#pragma unroll
                for (int q = 0; q < rr; q++) sum -= Lr[q] * wv[q];
                wv[rr] = (rr >= c) ? sum / Lr[rr] : T(0);
            }
#pragma unroll
            for (int rr = 0; rr < D; rr++) scratch[(o + rr) * N + o + c] = wv[rr];
        }
    }
    __syncthreads();  // the parked inverses are visible to the whole workgroup
    leaf128_invert<T>(sm, nblk, scratch, false);
    leaf128_store<T>(L, A, nb);
    __syncthreads();
    return 0;
}

// In place, the lower triangle of W^T W for the lower-triangular A = W of
// order nb <= 128 (the LAUUM step of the inversion): the 36 output blocks
// C_ij = sum_{k >= i} W_ki^T W_kj (i >= j, 16 x 16 each) are shared out over
// the four wavefronts and formed on MFMA from W in LDS (rows past nb are the
// identity and add nothing to the stored part), then written over W.  All
// 256 threads must call it; it ends with a barrier.
template <typename T>
__device__ void lauum128_block(Leaf128Smem<T>& sm, Mat<T> A, int nb)
{
    T* L = sm.L;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = lane & 15, g = lane >> 4;
    typedef typename M16<T>::acc acc_t;
    leaf128_load<T>(L, A, nb);
    __syncthreads();
    const int nblk = (nb + D - 1) / D, nout = nblk * (nblk + 1) / 2;
    constexpr int PER = (8 * 9 / 2 + 3) / 4;  // output blocks per wavefront at most
    acc_t c[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        c[q] = acc_t{0, 0, 0, 0};
        const int b = w + 4 * q;
        if (b < nout) {
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= b) bi++;
            const int bj = b - bi * (bi + 1) / 2;
            // A operand: W_ki^T (row r, k index); B operand: W_kj (k index, column r)
            for (int bk = bi; bk < nblk; bk++) {
#pragma unroll
                for (int kk = 0; kk < D; kk += 4) {
                    const T* row = L + prow(bk * D + kk + g);
                    c[q] = M16<T>::op(row[bi * D + r], row[bj * D + r], c[q]);
                }
            }
        }
    }
    __syncthreads();  // every wavefront is done reading W
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int b = w + 4 * q;
        if (b < nout) {
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= b) bi++;
            const int bj = b - bi * (bi + 1) / 2;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = bi * D + M16<T>::row(lane, e), j = bj * D + r;
                if (i >= j) L[prow(i) + j] = c[q][e];
            }
        }
    }
    __syncthreads();
    leaf128_store<T>(L, A, nb);
    __syncthreads();
}

}  // namespace rfp
