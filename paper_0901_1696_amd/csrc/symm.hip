// Y = beta Y + alpha A X for the symmetric matrix A held in RFP and a thin X
// (n x r, r small): the residual and the conjugate-gradient products of the
// mixed-precision solve.  HBM-bound: the work is reading A, and every stored
// entry is read once.
//
// Through the canonical lower views (T1 = L11, S = L21, T2 = L22),
//   Y1 = tril(T1) X1 + stril(T1)^T X1 + S^T X2
//   Y2 = S X1 + tril(T2) X2 + stril(T2)^T X2.
// Each stored block B (T1 and T2 through their lower triangles, S whole)
// gives a row product B X_cols and a column product B^T X_rows from the same
// load.  One launch per block: a workgroup owns a 256 x 256 region of the
// block (4 x 4 tiles of 64; on a triangle only the regions on or below the
// diagonal, and there only the tiles on or below it), stages each tile in
// LDS once and applies it twice on FP64 MFMA: to the X rows of the region's
// columns (the row product of its tile row) and, transposed, to the X rows of
// its rows (the column product of its tile column; the diagonal excluded on a
// triangle).  Row products are summed over a region's tile columns in
// registers and written as the region's partial for its rows (one slice per
// region column); column products are summed over the region's tile rows and
// written as its partial for its columns (one slice per region row).  One
// reduction then adds, for every output row, the slices that cover it in a
// fixed order (deterministic result) and applies alpha and beta.
#include <algorithm>

#include "rfp_common.h"

namespace rfp {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int TT = 64;       // tile edge
constexpr int RG = 4;        // tiles per region edge
constexpr int RS = TT * RG;  // region edge
constexpr int SP = TT + 4;   // LDS pitch of a tile or an X slab
constexpr int RX = 16;       // columns of X per pass

struct RegionArgs {
    Mat<const double> a;  // m x k block
    int64_t m, k;
    int lower;            // a diagonal block: only its lower triangle is stored (m == k)
    const double* xc;     // X rows for the row product (k rows), column-major
    const double* xr;     // X rows for the column product (m rows)
    int64_t ldx;
    int r;                // columns in this pass (<= RX)
    int nbi, nbj;         // regions along m and along k
    double* rowpart;      // slice bj at rowpart + bj * rp_slice: m x RX, leading dimension m
    int64_t rp_slice;
    double* colpart;      // slice bi at colpart + bi * cp_slice: k x RX, leading dimension k
    int64_t cp_slice;
    const int* gate;      // device, or null: nothing is done while *gate != 0
};

inline int64_t regions(int64_t len) { return (len + RS - 1) / RS; }

}  // namespace

__device__ double g_symv_zero = 0.0;  // never written

__global__ __launch_bounds__(256) void symv_region_kernel(RegionArgs p)
{
    __shared__ __attribute__((aligned(16))) double As[TT][SP];       // tile, As[row][col]
    __shared__ __attribute__((aligned(16))) double Xr[RX][RS + 4];   // X rows of the region, [column][row]
    __shared__ __attribute__((aligned(16))) double Xc[RX][SP];       // X rows of one tile column, [column][k]
    if (p.gate && *p.gate) return;
    int bi, bj;
    if (p.lower) {
        const int b = (int)blockIdx.x;
        int q = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
        while ((q + 1) * (q + 2) / 2 <= b) q++;
        while (q * (q + 1) / 2 > b) q--;
        bi = q;
        bj = b - q * (q + 1) / 2;
    } else {
        bi = (int)blockIdx.x % p.nbi;
        bj = (int)blockIdx.x / p.nbi;
    }
    const int64_t i0 = (int64_t)bi * RS, j0 = (int64_t)bj * RS;
    const bool diag_region = p.lower && bi == bj;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const bool rows_fast = p.a.rs == 1;

    for (int idx = t; idx < RS * RX; idx += 256) {
        const int row = idx % RS, c = idx / RS;
        const int64_t i = i0 + row;
        Xr[c][row] = (i < p.m && c < p.r) ? p.xr[i + (int64_t)c * p.ldx] : 0.0;
    }

    // tiles of the region in order (tile column major), present when they
    // hold stored entries inside the block
    auto present = [&](int it, int jt) {
        return (!diag_region || it >= jt) && i0 + (int64_t)it * TT < p.m && j0 + (int64_t)jt * TT < p.k;
    };
    constexpr int AE = TT * TT / 256;
    double ra[AE];
    auto load = [&](int it, int jt) {
        const int64_t ti = i0 + (int64_t)it * TT, tj = j0 + (int64_t)jt * TT;
        const bool dtile = diag_region && it == jt;
#pragma unroll
        for (int e = 0; e < AE; e++) {
            const int idx = t + 256 * e;
            const int li = rows_fast ? idx % TT : idx / TT, lk = rows_fast ? idx / TT : idx % TT;
            const int64_t i = ti + li, kk = tj + lk;
            const bool ok = i < p.m && kk < p.k && (!dtile || li >= lk);
            // a masked-off element is loaded from a zero in device memory:
            // every load is issued (no branch), so the wait for this tile
            // does not wait for the loads issued after it
            ra[e] = *(ok ? &p.a.at(i, kk) : &g_symv_zero);
        }
    };
    auto next_of = [&](int q) {  // first present tile at or after position q, else RG * RG
        for (; q < RG * RG; q++)
            if (present(q % RG, q / RG)) return q;
        return RG * RG;
    };

    v4d racc[RG];
#pragma unroll
    for (int x = 0; x < RG; x++) racc[x] = v4d{0, 0, 0, 0};
    int q = next_of(0);
    if (q < RG * RG) load(q % RG, q / RG);
    int cur_jt = -1;
    v4d cacc = v4d{0, 0, 0, 0};
    while (q < RG * RG) {
        const int it = q % RG, jt = q / RG;
        const int qn = next_of(q + 1);
        __syncthreads();  // the previous tile's products are done with As (and Xc)
        if (jt != cur_jt) {
            // X rows of the new tile column
            for (int idx = t; idx < TT * RX; idx += 256) {
                const int kk = idx % TT, c = idx / TT;
                const int64_t j = j0 + (int64_t)jt * TT + kk;
                Xc[c][kk] = (j < p.k && c < p.r) ? p.xc[j + (int64_t)c * p.ldx] : 0.0;
            }
            cur_jt = jt;
            cacc = v4d{0, 0, 0, 0};
        }
#pragma unroll
        for (int e = 0; e < AE; e++) {
            const int idx = t + 256 * e;
            const int li = rows_fast ? idx % TT : idx / TT, lk = rows_fast ? idx / TT : idx % TT;
            As[li][lk] = ra[e];
        }
        __syncthreads();
        if (qn < RG * RG) load(qn % RG, qn / RG);  // next tile in flight during the products
        // row product: rows 16 w .. of the tile against the tile column's X
        v4d racc_t = v4d{0, 0, 0, 0};
#pragma unroll 4
        for (int kk = 0; kk < TT; kk += 4)
            racc_t = __builtin_amdgcn_mfma_f64_16x16x4f64(As[16 * w + r16][kk + g], Xc[r16][kk + g], racc_t, 0, 0, 0);
        // column product: columns 16 w .. of the tile (rows of A^T) against the
        // tile row's X; the diagonal of a diagonal tile is excluded
        const bool dtile = diag_region && it == jt;
        const int col = 16 * w + r16;
#pragma unroll 4
        for (int kk = 0; kk < TT; kk += 4) {
            const int row = kk + g;
            const double av = (!dtile || row > col) ? As[row][col] : 0.0;
            cacc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xr[r16][it * TT + row], cacc, 0, 0, 0);
        }
#pragma unroll
        for (int x = 0; x < RG; x++)
            if (x == it) racc[x] += racc_t;
        // the tile column is complete: its partial for the region's columns
        if (qn >= RG * RG || qn / RG != jt) {
            double* out = p.colpart + (int64_t)bi * p.cp_slice;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int64_t j = j0 + (int64_t)jt * TT + 16 * w + g + 4 * e;
                if (j < p.k && r16 < p.r) out[j + (int64_t)r16 * p.k] = cacc[e];
            }
        }
        q = qn;
    }
    // row partials of the region's tile rows (every tile row of the region
    // that lies inside the block, including those whose tiles were absent)
    double* out = p.rowpart + (int64_t)bj * p.rp_slice;
#pragma unroll
    for (int x = 0; x < RG; x++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int64_t i = i0 + (int64_t)x * TT + 16 * w + g + 4 * e;
            if (i < p.m && r16 < p.r) out[i + (int64_t)r16 * p.m] = racc[x][e];
        }
}

namespace {

// Slices of one output half, in summation order: a range of slices of one
// partial array is added for row i when lo(i) <= slice <= hi(i).
struct SliceSet {
    const double* base;
    int64_t slice, ld;  // doubles per slice; leading dimension
    int kind;           // 0: all slices [0, count); 1: slices 0 .. i / RS; 2: slices i / RS .. count - 1
    int count;
};

struct ReduceArgs {
    SliceSet s[3];
    int nsets;
    int64_t m;
    int r;
    double alpha, beta;
    double* y;
    int64_t ldy;
    const int* gate;
};

}  // namespace

__global__ void symv_reduce_kernel(ReduceArgs p)
{
    if (p.gate && *p.gate) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= p.m || c >= p.r) return;
    const int ri = (int)(i / RS);
    double sum = 0.0;
    for (int q = 0; q < p.nsets; q++) {
        const SliceSet& s = p.s[q];
        const int lo = s.kind == 2 ? ri : 0, hi = s.kind == 1 ? ri : s.count - 1;
        for (int k = lo; k <= hi; k++) sum += s.base[k * s.slice + i + (int64_t)c * s.ld];
    }
    double v = p.alpha * sum;
    if (p.beta != 0.0) v += p.beta * p.y[i + (int64_t)c * p.ldy];
    p.y[i + (int64_t)c * p.ldy] = v;
}

namespace {

// Partial arrays of the three blocks: T1 row and column, S row and column, T2
// row and column, each regions x rows x RX doubles.
struct PartLayout {
    int64_t off[6], slice[6];
    int64_t total;
};
PartLayout part_layout(int64_t m1, int64_t m2)
{
    PartLayout L;
    const int64_t rows[6] = {m1, m1, m2, m1, m2, m2};           // rows of each partial slice
    const int64_t count[6] = {regions(m1), regions(m1), regions(m1), regions(m2), regions(m2), regions(m2)};
    int64_t o = 0;
    for (int q = 0; q < 6; q++) {
        L.off[q] = o;
        L.slice[q] = rows[q] * RX;
        o += count[q] * L.slice[q];
    }
    L.total = o;
    return L;
}

}  // namespace

size_t symm_thin_workspace(int64_t m1, int64_t m2)
{
    // either block may be the larger one
    return sizeof(double) * (size_t)std::max(part_layout(m1, m2).total, part_layout(m2, m1).total);
}

hipError_t symm_thin(const Exec& ex, const RfpView<const double>& v, const double* x, int64_t ldx, double alpha,
                     double beta, double* y, int64_t ldy, int64_t nrhs, double* ws)
{
    const int64_t m1 = v.m1, m2 = v.m2, n = m1 + m2;
    if (n == 0 || nrhs <= 0) return hipSuccess;
    const PartLayout L = part_layout(m1, m2);
    const int nb1 = (int)regions(m1), nb2 = (int)regions(m2);
    for (int64_t c0 = 0; c0 < nrhs; c0 += RX) {
        const int r = (int)std::min<int64_t>(RX, nrhs - c0);
        const double* x1 = x + c0 * ldx;
        const double* x2 = x1 + m1;
        struct Blk {
            Mat<const double> a;
            int64_t m, k;
            int lower;
            const double *xc, *xr;
            int rowq, colq;  // partial arrays
        };
        const Blk blks[3] = {
            {v.t1, m1, m1, 1, x1, x1, 0, 1},  // T1: rows and columns in half 1
            {v.s, m2, m1, 0, x1, x2, 2, 3},   // S: rows in half 2, columns in half 1
            {v.t2, m2, m2, 1, x2, x2, 4, 5},  // T2: rows and columns in half 2
        };
        for (const Blk& b : blks) {
            if (b.m <= 0 || b.k <= 0) continue;
            RegionArgs a;
            a.a = b.a;
            a.m = b.m;
            a.k = b.k;
            a.lower = b.lower;
            a.xc = b.xc;
            a.xr = b.xr;
            a.ldx = ldx;
            a.r = r;
            a.nbi = (int)regions(b.m);
            a.nbj = (int)regions(b.k);
            a.rowpart = ws + L.off[b.rowq];
            a.rp_slice = L.slice[b.rowq];
            a.colpart = ws + L.off[b.colq];
            a.cp_slice = L.slice[b.colq];
            a.gate = ex.gate;
            const int64_t nreg = b.lower ? (int64_t)a.nbi * (a.nbi + 1) / 2 : (int64_t)a.nbi * a.nbj;
            ProfScope ps(ex, "rfp::symv_region_kernel(rfp::(anonymous namespace)::RegionArgs)",
                         2.0 * (double)b.m * (double)b.k * r * (b.lower ? 1.0 : 2.0),
                         8.0 * (double)b.m * (double)b.k * (b.lower ? 0.5 : 1.0));
            hipLaunchKernelGGL(symv_region_kernel, dim3((unsigned)nreg), dim3(256), 0, ex.stream, a);
        }
        // half 1: T1 rows (slices 0 .. i/RS), T1 columns (i/RS ..), S columns (all)
        // half 2: S rows (all), T2 rows (0 .. i/RS), T2 columns (i/RS ..)
        for (int h = 0; h < 2; h++) {
            const int64_t mh = h ? m2 : m1;
            if (mh <= 0) continue;
            ReduceArgs p{};
            if (h == 0) {
                p.s[0] = SliceSet{ws + L.off[0], L.slice[0], m1, 1, nb1};
                p.s[1] = SliceSet{ws + L.off[1], L.slice[1], m1, 2, nb1};
                p.s[2] = SliceSet{ws + L.off[3], L.slice[3], m1, 0, m2 > 0 ? nb2 : 0};
            } else {
                p.s[0] = SliceSet{ws + L.off[2], L.slice[2], m2, 0, nb1};
                p.s[1] = SliceSet{ws + L.off[4], L.slice[4], m2, 1, nb2};
                p.s[2] = SliceSet{ws + L.off[5], L.slice[5], m2, 2, nb2};
            }
            p.nsets = 3;
            p.m = mh;
            p.r = r;
            p.alpha = alpha;
            p.beta = beta;
            p.y = y + (h ? m1 : 0) + c0 * ldy;
            p.ldy = ldy;
            p.gate = ex.gate;
            const dim3 grid((unsigned)((mh + 255) / 256), (unsigned)r);
            hipLaunchKernelGGL(symv_reduce_kernel, grid, dim3(256), 0, ex.stream, p);
        }
    }
    return hipGetLastError();
}

}  // namespace rfp
