// Y = beta Y + alpha A X for the symmetric matrix A held in RFP and a thin X
// (n x r, r small): the residual and the conjugate-gradient products of the
// mixed-precision solve.  HBM-bound: the work is reading A.
//
// Through the canonical lower views (T1 = L11, S = L21, T2 = L22),
//   Y1 = tril(T1) X1 + stril(T1)^T X1 + S^T X2
//   Y2 = S X1 + tril(T2) X2 + stril(T2)^T X2.
// Each of the six products is one launch of a skinny kernel: a workgroup
// takes 64 rows of the (masked, possibly transposed) block and one chunk of
// its k range, stages 64 x 64 tiles of the block and 64-row slabs of X in LDS
// (both loaded along their unit stride), accumulates on FP64 MFMA and writes
// its 64 x r partial product to a workspace slice.  One reduction then adds
// all slices of a row in a fixed order (deterministic result) and applies
// alpha and beta.  The grid splits k so that every product has enough
// workgroups in flight to stream the block at full bandwidth.
#include <algorithm>

#include "rfp_common.h"

namespace rfp {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int TM = 64;      // rows per workgroup
constexpr int TK = 64;      // k per LDS slab
constexpr int SP = TK + 4;  // LDS pitch
constexpr int RMAX = 32;    // columns of X per launch

struct SkinnyArgs {
    Mat<const double> a;  // m x k view
    int64_t m, k;
    int64_t lo, hi;       // keep a(i, kk) when lo <= kk - i <= hi
    const double* x;      // k x r, column-major
    int64_t ldx;
    int r;
    int64_t kc;           // k per chunk
    double* w;            // this product's first slice; chunk c writes slice c (w + c * wslice)
    int64_t wslice;       // doubles per slice
    int64_t wld;          // leading dimension of a slice (rows of the output half)
    int64_t row0;         // first output row of this product inside the slice
    const int* gate;      // device, or null: nothing is done while *gate != 0
};

}  // namespace

template <int NCB>
__global__ __launch_bounds__(256) void skinny_kernel(SkinnyArgs p)
{
    __shared__ __attribute__((aligned(16))) double As[TM][SP];
    __shared__ __attribute__((aligned(16))) double Xs[16 * NCB][SP];
    if (p.gate && *p.gate) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * TM;
    const int chunk = blockIdx.y;
    int64_t kb = (int64_t)chunk * p.kc, ke = std::min<int64_t>(kb + p.kc, p.k);
    // the band mask bounds k for the whole tile: lo <= kk - i <= hi
    kb = std::max<int64_t>(kb, i0 + p.lo);
    ke = std::min<int64_t>(ke, i0 + TM - 1 + p.hi + 1);
    const bool rows_fast = p.a.rs == 1;

    v4d acc[NCB];
#pragma unroll
    for (int c = 0; c < NCB; c++) acc[c] = v4d{0, 0, 0, 0};

    constexpr int AE = TM * TK / 256, XE = 16 * NCB * TK / 256;
    double ra[AE], rx[XE];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < AE; e++) {
            const int idx = t + 256 * e;
            const int li = rows_fast ? idx % TM : idx / TK, lk = rows_fast ? idx / TM : idx % TK;
            const int64_t i = i0 + li, kk = k0 + lk;
            const int64_t d = kk - i;
            const bool ok = i < p.m && kk < ke && d >= p.lo && d <= p.hi;
            ra[e] = ok ? p.a.at(i, kk) : 0.0;
        }
#pragma unroll
        for (int e = 0; e < XE; e++) {
            const int idx = t + 256 * e;
            const int lk = idx % TK, c = idx / TK;
            const int64_t kk = k0 + lk;
            rx[e] = (kk < ke && c < p.r) ? p.x[kk + c * p.ldx] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < AE; e++) {
            const int idx = t + 256 * e;
            const int li = rows_fast ? idx % TM : idx / TK, lk = rows_fast ? idx / TM : idx % TK;
            As[li][lk] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < XE; e++) {
            const int idx = t + 256 * e;
            Xs[idx / TK][idx % TK] = rx[e];
        }
    };
    if (kb < ke) {
        load(kb);
        for (int64_t k0 = kb; k0 < ke; k0 += TK) {
            store();
            __syncthreads();
            if (k0 + TK < ke) load(k0 + TK);  // next slab in flight during the products
#pragma unroll 4
            for (int kk = 0; kk < TK; kk += 4) {
                const double av = As[16 * w + r][kk + g];
#pragma unroll
                for (int c = 0; c < NCB; c++)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xs[c * 16 + r][kk + g], acc[c], 0, 0, 0);
            }
            __syncthreads();
        }
    }
    // result layout of the FP64 MFMA: lane, register e -> row lane/16 + 4e, column lane % 16
    double* out = p.w + (int64_t)chunk * p.wslice;
#pragma unroll
    for (int c = 0; c < NCB; c++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int64_t i = i0 + 16 * w + (lane >> 4) + 4 * e;
            const int col = c * 16 + r;
            if (i < p.m && col < p.r) out[(p.row0 + i) + (int64_t)col * p.wld] = acc[c][e];
        }
}

// y(i, c) = beta y(i, c) + alpha sum_q w[q](i, c), q in slice order
__global__ void skinny_reduce_kernel(const double* w, int nslices, int64_t wslice, int64_t wld, int64_t m, int r,
                                     double alpha, double beta, double* y, int64_t ldy, const int* gate)
{
    if (gate && *gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= m || c >= r) return;
    double s = 0.0;
    for (int q = 0; q < nslices; q++) s += w[q * wslice + i + (int64_t)c * wld];
    double v = alpha * s;
    if (beta != 0.0) v += beta * y[i + c * ldy];
    y[i + c * ldy] = v;
}

namespace {

constexpr int MAX_CHUNKS = 8;

int chunks_for(int64_t m, int64_t k)
{
    const int64_t tiles = (m + TM - 1) / TM;
    int64_t c = (2048 + tiles - 1) / std::max<int64_t>(tiles, 1);
    c = std::min<int64_t>(c, (k + 255) / 256);
    return (int)std::max<int64_t>(1, std::min<int64_t>(c, MAX_CHUNKS));
}

struct Product {
    Mat<const double> a;
    int64_t m, k, lo, hi;
    int half;      // 0: Y1, 1: Y2
    int64_t xoff;  // first row of X it reads
};

}  // namespace

size_t symm_thin_workspace(int64_t m1, int64_t m2)
{
    return sizeof(double) * (size_t)(3 * MAX_CHUNKS) * RMAX * (size_t)(m1 + m2);
}

hipError_t symm_thin(const Exec& ex, const RfpView<const double>& v, const double* x, int64_t ldx, double alpha,
                     double beta, double* y, int64_t ldy, int64_t nrhs, double* ws)
{
    const int64_t m1 = v.m1, m2 = v.m2, n = m1 + m2;
    if (n == 0 || nrhs <= 0) return hipSuccess;
    const int64_t BIG = (int64_t)1 << 62;
    const Product prods[6] = {
        {v.t1, m1, m1, -BIG, 0, 0, 0},        // tril(T1) X1
        {v.t1.tr(), m1, m1, 1, BIG, 0, 0},    // stril(T1)^T X1
        {v.s.tr(), m1, m2, -BIG, BIG, 0, m1}, // S^T X2
        {v.s, m2, m1, -BIG, BIG, 1, 0},       // S X1
        {v.t2, m2, m2, -BIG, 0, 1, m1},       // tril(T2) X2
        {v.t2.tr(), m2, m2, 1, BIG, 1, m1},   // stril(T2)^T X2
    };
    // slices of half h: sum over its products of their chunk counts
    const int64_t half_rows[2] = {m1, m2};
    double* half_ws[2] = {ws, ws + (size_t)(3 * MAX_CHUNKS) * RMAX * m1};
    for (int64_t c0 = 0; c0 < nrhs; c0 += RMAX) {
        const int r = (int)std::min<int64_t>(RMAX, nrhs - c0);
        int nsl[2] = {0, 0};
        for (const Product& pr : prods) {
            if (pr.m <= 0) continue;
            const int h = pr.half;
            const int64_t wslice = half_rows[h] * RMAX;
            SkinnyArgs a;
            a.a = pr.a;
            a.m = pr.m;
            a.k = pr.k;
            a.lo = pr.lo;
            a.hi = pr.hi;
            a.x = x + pr.xoff + c0 * ldx;
            a.ldx = ldx;
            a.r = r;
            int nch = pr.k > 0 ? chunks_for(pr.m, pr.k) : 1;
            a.kc = pr.k > 0 ? ((pr.k + nch - 1) / nch + TK - 1) / TK * TK : TK;
            nch = pr.k > 0 ? (int)((pr.k + a.kc - 1) / a.kc) : 1;
            a.w = half_ws[h] + (int64_t)nsl[h] * wslice;
            a.wslice = wslice;
            a.wld = half_rows[h];
            a.row0 = 0;
            a.gate = ex.gate;
            nsl[h] += nch;
            const dim3 grid((unsigned)((pr.m + TM - 1) / TM), (unsigned)nch);
            ProfScope ps(ex, r > 16 ? "rfp::skinny_kernel<2>(rfp::(anonymous namespace)::SkinnyArgs)"
                                    : "rfp::skinny_kernel<1>(rfp::(anonymous namespace)::SkinnyArgs)",
                         2.0 * (double)pr.m * (double)pr.k * r, 8.0 * (double)pr.m * (double)pr.k);
            if (r > 16) hipLaunchKernelGGL(skinny_kernel<2>, grid, dim3(256), 0, ex.stream, a);
            else hipLaunchKernelGGL(skinny_kernel<1>, grid, dim3(256), 0, ex.stream, a);
        }
        for (int h = 0; h < 2; h++) {
            if (half_rows[h] <= 0) continue;
            double* yh = y + (h ? m1 : 0) + c0 * ldy;
            const dim3 grid((unsigned)((half_rows[h] + 255) / 256), (unsigned)r);
            hipLaunchKernelGGL(skinny_reduce_kernel, grid, dim3(256), 0, ex.stream, half_ws[h], nsl[h],
                               half_rows[h] * RMAX, half_rows[h], half_rows[h], r, alpha, beta, yh, ldy, ex.gate);
        }
    }
    return hipGetLastError();
}

}  // namespace rfp
