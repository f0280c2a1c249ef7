// Strided, masked GEMM on CDNA4 matrix cores: the Level-3 update behind every
// TRSM, SYRK, TRMM and GEMM step of the RFP Cholesky factorization, solution
// and inversion (Sections 3-5).  One kernel template serves all of them:
//   C(m x n) = alpha * A(m x k) * B(n x k)^T + beta * C
// with every operand a strided view straight into the RFP rectangle (either
// orientation), optional triangular masks on A and B, and an optional
// lower-triangle-only output for the symmetric rank-k updates.
//
// Work decomposition: a 256-thread workgroup (four wave64s in a 2 x 2 grid)
// computes a 128 x 128 tile of C; each wave owns 64 x 64 = 4 x 4 MFMA blocks
// of 16 x 16 held in accumulation registers.  K advances in slabs of 16
// staged through LDS (double buffered, one barrier per slab); the next slab's
// global loads are issued before the current slab's MFMAs.
#include "rfp_common.h"

namespace rfp {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Operand layout of both 16x16x4 instructions: lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16).  Result layout differs (measured on gfx950): lane l,
// register r holds D(row, l % 16) with row = l/16 + 4r for FP64 and
// row = 4(l/16) + r for FP32.
template <>
struct Mfma<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc op(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc op(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int BM = 128, BN = 128, BK = 16, NTH = 256;
constexpr int LPAD = 1;  // LDS row padding (elements)

template <typename T>
struct GemmParams {
    int64_t m, n, k;
    const T* A;
    int64_t lda;
    const T* B;
    int64_t ldb;
    T* C;
    int64_t ldc;
    T alpha, beta;
    int triA, triB;
    int c_lower;
    int tiles_m;
    int64_t kchunk;
    T* W;  // split-K partials, [split][n][m], or null
    const int* info;
};

__device__ __forceinline__ bool keep(int tri, int64_t i, int64_t j)
{
    switch (tri) {
        case TRI_LOWER: return i >= j;
        case TRI_UPPER: return i <= j;
        case TRI_SLOWER: return i > j;
        case TRI_SUPPER: return i < j;
        default: return true;
    }
}

// AMC: A's row index is contiguous (column-major A); else A's k index is.
// BNC: B's row index (the n index of C) is contiguous; else its k index is.
// CMC: C's row index is contiguous.
template <typename T, bool AMC, bool BNC, bool CMC>
__global__ __launch_bounds__(NTH) void gemm_kernel(GemmParams<T> p)
{
    if (p.info && *p.info) return;

    int64_t ti, tj;
    const int bid = blockIdx.x;
    if (p.c_lower) {
        // bid enumerates the lower triangle of tiles row by row
        int r = (int)((sqrtf(8.0f * (float)bid + 1.0f) - 1.0f) * 0.5f);
        while ((r + 1) * (r + 2) / 2 <= bid) r++;
        while (r * (r + 1) / 2 > bid) r--;
        ti = r;
        tj = bid - r * (r + 1) / 2;
    } else {
        ti = bid % p.tiles_m;
        tj = bid / p.tiles_m;
    }
    const int64_t i0 = ti * BM, j0 = tj * BN;
    const int64_t m = p.m, n = p.n;

    int64_t kb = (int64_t)blockIdx.z * p.kchunk;
    int64_t ke = kb + p.kchunk < p.k ? kb + p.kchunk : p.k;
    // skip k slabs that a triangular operand zeroes for this whole tile
    if (p.triA == TRI_LOWER || p.triA == TRI_SLOWER) ke = ke < i0 + BM ? ke : i0 + BM;
    if (p.triA == TRI_UPPER || p.triA == TRI_SUPPER) kb = kb > i0 ? kb : i0;
    if (p.triB == TRI_LOWER || p.triB == TRI_SLOWER) ke = ke < j0 + BN ? ke : j0 + BN;
    if (p.triB == TRI_UPPER || p.triB == TRI_SUPPER) kb = kb > j0 ? kb : j0;

    __shared__ T As[2][BK][BM + LPAD];
    __shared__ T Bs[2][BK][BN + LPAD];

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;

    constexpr int EA = BM * BK / NTH;  // elements of each operand tile per thread
    // per-thread coordinates inside a tile
    const int a_i = AMC ? (t % BM) : (t / BK);
    const int a_k = AMC ? (t / BM) : (t % BK);
    const int b_j = BNC ? (t % BN) : (t / BK);
    const int b_k = BNC ? (t / BN) : (t % BK);
    constexpr int A_STEP = AMC ? NTH / BM : NTH / BK;  // along k (AMC) or i
    constexpr int B_STEP = BNC ? NTH / BN : NTH / BK;

    T ra[EA], rb[EA];

    auto load = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < EA; r++) {
            int64_t i = i0 + (AMC ? a_i : a_i + r * A_STEP);
            int64_t kk = k0 + (AMC ? a_k + r * A_STEP : a_k);
            bool ok = i < m && kk < ke && keep(p.triA, i, kk);
            ra[r] = ok ? (AMC ? p.A[i + kk * p.lda] : p.A[i * p.lda + kk]) : T(0);
        }
#pragma unroll
        for (int r = 0; r < EA; r++) {
            int64_t j = j0 + (BNC ? b_j : b_j + r * B_STEP);
            int64_t kk = k0 + (BNC ? b_k + r * B_STEP : b_k);
            bool ok = j < n && kk < ke && keep(p.triB, j, kk);
            rb[r] = ok ? (BNC ? p.B[j + kk * p.ldb] : p.B[j * p.ldb + kk]) : T(0);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < EA; r++) {
            if (AMC) As[buf][a_k + r * A_STEP][a_i] = ra[r];
            else As[buf][a_k][a_i + r * A_STEP] = ra[r];
        }
#pragma unroll
        for (int r = 0; r < EA; r++) {
            if (BNC) Bs[buf][b_k + r * B_STEP][b_j] = rb[r];
            else Bs[buf][b_k][b_j + r * B_STEP] = rb[r];
        }
    };

    typedef typename Mfma<T>::acc acc_t;
    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = acc_t{0, 0, 0, 0};

    const int64_t nslab = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    if (nslab > 0) {
        load(kb);
        store(0);
        __syncthreads();
        for (int64_t s = 0; s < nslab; s++) {
            const int buf = (int)(s & 1);
            if (s + 1 < nslab) load(kb + (s + 1) * BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                T af[4], bf[4];
                const int kr = kk + (lane >> 4);
#pragma unroll
                for (int x = 0; x < 4; x++) af[x] = As[buf][kr][wm * 64 + x * 16 + (lane & 15)];
#pragma unroll
                for (int x = 0; x < 4; x++) bf[x] = Bs[buf][kr][wn * 64 + x * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < 4; a++)
#pragma unroll
                    for (int b = 0; b < 4; b++) acc[a][b] = Mfma<T>::op(af[a], bf[b], acc[a][b]);
            }
            if (s + 1 < nslab) store(buf ^ 1);
            __syncthreads();
        }
    }

    // accumulator (a, b)[r] holds C(row, col) with
    // row = wm*64 + a*16 + Mfma<T>::row(lane, r), col = wn*64 + b*16 + lane%16
    const int cl = lane & 15;
    if (p.W) {
        T* W = p.W + (int64_t)blockIdx.z * m * n;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const int64_t j = j0 + wn * 64 + b * 16 + cl;
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int64_t i = i0 + wm * 64 + a * 16 + Mfma<T>::row(lane, r);
                    if (i < m && j < n) W[j * m + i] = acc[a][b][r];
                }
            }
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int64_t j = j0 + wn * 64 + b * 16 + cl;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t i = i0 + wm * 64 + a * 16 + Mfma<T>::row(lane, r);
                if (i < m && j < n && (!p.c_lower || i >= j)) {
                    T* c = CMC ? &p.C[i + j * p.ldc] : &p.C[i * p.ldc + j];
                    T v = p.alpha * acc[a][b][r];
                    if (p.beta != T(0)) v += p.beta * *c;
                    *c = v;
                }
            }
        }
}

// C = alpha * sum_z W[z] + beta * C over the (masked) m x n output.
template <typename T, bool CMC>
__global__ __launch_bounds__(256) void splitk_reduce(GemmParams<T> p, int nsplit)
{
    if (p.info && *p.info) return;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = p.m * p.n;
    if (idx >= total) return;
    int64_t i, j;
    if (CMC) { i = idx % p.m; j = idx / p.m; }
    else { j = idx % p.n; i = idx / p.n; }
    if (p.c_lower && i < j) return;
    T s = 0;
    for (int z = 0; z < nsplit; z++) s += p.W[(int64_t)z * total + j * p.m + i];
    T* c = CMC ? &p.C[i + j * p.ldc] : &p.C[i * p.ldc + j];
    T v = p.alpha * s;
    if (p.beta != T(0)) v += p.beta * *c;
    *c = v;
}

template <typename T, bool AMC, bool BNC, bool CMC>
static void launch(const GemmParams<T>& p, dim3 grid, hipStream_t s)
{
    hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC>), grid, dim3(NTH), 0, s, p);
}

template <typename T>
hipError_t gemm(const Exec& ex, int64_t m, int64_t n, int64_t k, T alpha, Mat<const T> A, int triA,
                Mat<const T> B, int triB, T beta, Mat<T> C, bool c_lower)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    if (c_lower && m != n) return hipErrorInvalidValue;
    GemmParams<T> p{};
    p.m = m;
    p.n = n;
    p.k = k < 0 ? 0 : k;
    const bool amc = A.rs == 1;
    if (!amc && A.cs != 1) return hipErrorInvalidValue;
    const bool bnc = B.rs == 1;
    if (!bnc && B.cs != 1) return hipErrorInvalidValue;
    const bool cmc = C.rs == 1;
    if (!cmc && C.cs != 1) return hipErrorInvalidValue;
    p.A = A.p;
    p.lda = amc ? A.cs : A.rs;
    p.B = B.p;
    p.ldb = bnc ? B.cs : B.rs;
    p.C = C.p;
    p.ldc = cmc ? C.cs : C.rs;
    p.alpha = alpha;
    p.beta = beta;
    p.triA = triA;
    p.triB = triB;
    p.c_lower = c_lower ? 1 : 0;
    p.info = ex.info;
    const int64_t tm = (m + BM - 1) / BM, tn = (n + BN - 1) / BN;
    const int64_t ntiles = c_lower ? tm * (tm + 1) / 2 : tm * tn;
    p.tiles_m = (int)tm;

    // split K when the tile grid cannot fill the chip and K is long
    int64_t nsplit = 1;
    if (ntiles < 256 && p.k >= 1024 && ex.splitk_ws) {
        nsplit = (512 + ntiles - 1) / ntiles;
        int64_t kmax = p.k / 256;
        if (nsplit > kmax) nsplit = kmax;
        if (nsplit > 32) nsplit = 32;
        while (nsplit > 1 && (size_t)(nsplit * m * n) * sizeof(T) > ex.splitk_bytes) nsplit--;
    }
    if (nsplit > 1) {
        int64_t chunk = (p.k + nsplit - 1) / nsplit;
        chunk = (chunk + BK - 1) / BK * BK;
        nsplit = (p.k + chunk - 1) / chunk;
        p.kchunk = chunk;
        p.W = (T*)ex.splitk_ws;
    } else {
        p.kchunk = p.k;
        p.W = nullptr;
    }
    dim3 grid((unsigned)ntiles, 1, (unsigned)nsplit);
    const int sel = (amc ? 4 : 0) | (bnc ? 2 : 0) | (cmc ? 1 : 0);
    switch (sel) {
        case 0: launch<T, false, false, false>(p, grid, ex.stream); break;
        case 1: launch<T, false, false, true>(p, grid, ex.stream); break;
        case 2: launch<T, false, true, false>(p, grid, ex.stream); break;
        case 3: launch<T, false, true, true>(p, grid, ex.stream); break;
        case 4: launch<T, true, false, false>(p, grid, ex.stream); break;
        case 5: launch<T, true, false, true>(p, grid, ex.stream); break;
        case 6: launch<T, true, true, false>(p, grid, ex.stream); break;
        default: launch<T, true, true, true>(p, grid, ex.stream); break;
    }
    if (nsplit > 1) {
        const int64_t total = m * n;
        dim3 g((unsigned)((total + 255) / 256));
        if (cmc) hipLaunchKernelGGL((splitk_reduce<T, true>), g, dim3(256), 0, ex.stream, p, (int)nsplit);
        else hipLaunchKernelGGL((splitk_reduce<T, false>), g, dim3(256), 0, ex.stream, p, (int)nsplit);
    }
    return hipGetLastError();
}

template hipError_t gemm<double>(const Exec&, int64_t, int64_t, int64_t, double, Mat<const double>, int,
                                 Mat<const double>, int, double, Mat<double>, bool);
template hipError_t gemm<float>(const Exec&, int64_t, int64_t, int64_t, float, Mat<const float>, int,
                                Mat<const float>, int, float, Mat<float>, bool);

}  // namespace rfp
