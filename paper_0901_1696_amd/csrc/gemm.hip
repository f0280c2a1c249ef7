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
#include <cstdio>
#include <type_traits>

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

constexpr int BK = 16, NTH = 256;
// global and LDS address spaces, for the global-to-LDS transfer builtin
typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;
constexpr int KP = BK + 2;  // LDS row pitch (elements): k-contiguous rows, 16-byte aligned, conflict-free

// Low-precision operand modes of the FP32 GEMM (LP): 0 FP32 MFMA; 1 operands
// rounded to FP16 and 2 to BF16 when staged in LDS, products on gfx950's
// 16x16x32 MFMA with FP32 accumulation.  Each lane supplies eight k values of
// its row of A (row l % 16) and the same eight k values of its column of B
// (column l % 16), the k group 8 (l / 16) .. 8 (l / 16) + 7 of a 32-deep
// slab; since A and B use the same assignment every k of the slab is summed
// exactly once, whatever order the instruction takes its k slots in.  The
// result layout is the FP32 one.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
template <typename T, int LP>
struct Lds {
    typedef T type;
    static constexpr int pitch = KP;
};
template <>
struct Lds<float, 1> {
    typedef _Float16 type;
    static constexpr int pitch = 40;  // 32-deep slabs in 80-byte rows: 16-byte aligned k groups
};
template <>
struct Lds<float, 2> {
    typedef short type;  // BF16 bit pattern
    static constexpr int pitch = 40;
};
// FP32 -> BF16, round to nearest even (a NaN stays a quiet NaN)
__device__ __forceinline__ short f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
template <int LP, typename T>
__device__ __forceinline__ typename Lds<T, LP>::type to_lds(T v)
{
    if constexpr (LP == 1) return (_Float16)v;
    else if constexpr (LP == 2) return f32_to_bf16(v);
    else return v;  // native precision: no conversion
}

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
    // With one triangular operand the k-range of a tile splits into slabs
    // that cross the operand's diagonal next to the tile and slabs it keeps
    // whole: part 0 runs all of them, part 1 only the whole ones (no masks),
    // part 2 only the crossing ones (masked).
    int part;
    int band;  // the tile's extent along the triangular operand's rows (parts 1, 2; work accounting)
    // Tile order (not with tri_enum): 0 deals GROUP tile rows at a time;
    // otherwise (bit 3 set) `group` tile rows (bit 0 clear) or columns (bit 0
    // set) at a time, and bits 1 and 2 reverse the tile rows and columns.  With one
    // triangular operand the tiles' k-ranges vary along one direction of the
    // grid: the groups run across it, and there are at least as many groups
    // as XCDs, so that each XCD's contiguous range of groups holds an even
    // share of the work, longest tiles first.
    int order, group;
    int c_lower;   // write only C(i, j) with i >= j
    int tri_enum;  // square lower output: the grid enumerates lower tiles only
    int tiles_m, tiles_n;
    int64_t kchunk;
    T* W;  // split-K partials, [split][n][m], or null
    const int* info;
    int prio;  // raise the waves' issue priority
};

// A mask keeps (i, kk) when lo <= kk - i <= hi.
struct Band {
    int64_t lo, hi;
};
__device__ __forceinline__ Band band_of(int tri)
{
    const int64_t BIG = (int64_t)1 << 62;
    switch (tri) {
        case TRI_LOWER: return Band{-BIG, 0};
        case TRI_UPPER: return Band{0, BIG};
        case TRI_SLOWER: return Band{-BIG, -1};
        case TRI_SUPPER: return Band{1, BIG};
        default: return Band{-BIG, BIG};
    }
}

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec2<float> {
    typedef float __attribute__((ext_vector_type(2))) type;
};

// Map the launch index to a tile.  Workgroups are dealt round-robin to the
// eight XCDs, so consecutive launch indices are first regrouped into one
// contiguous range per XCD (each XCD has its own L2); within that order,
// tiles go column-group by column-group, GROUP tile rows at a time, so the
// tiles resident at once share A row panels and B column panels.
constexpr int NXCD = 8, GROUP = 8;
__device__ __forceinline__ int xcd_remap(int bid, int total)
{
    const int per = total / NXCD, rem = total % NXCD;
    const int x = bid % NXCD, q = bid / NXCD;
    return x * per + (x < rem ? x : rem) + q;
}

// One tile of C per workgroup: four waves in a 2 x 2 grid, each owning
// WMB x WNB MFMA blocks of 16 x 16, so the tile is (32 WMB) x (32 WNB).
// AMC: A's row index is contiguous (column-major A); else A's k index is.
// BNC: B's row index (the n index of C) is contiguous; else its k index is.
// CMC: C's row index is contiguous.
template <typename T, bool AMC, bool BNC, bool CMC, int WMB, int WNB, int LP = 0, bool DMA = false>
__global__ __launch_bounds__(NTH, (WMB * WNB >= 16) ? 1 : 2) void gemm_kernel(GemmParams<T> p)
{
    constexpr int BM = 32 * WMB, BN = 32 * WNB;
    if (p.info && *p.info) return;
    if (p.prio) __builtin_amdgcn_s_setprio(3);

    int64_t ti, tj;
    {
        const int total = p.tri_enum ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
        const int bid = xcd_remap((int)blockIdx.x, total);
        if (p.tri_enum) {
            // lower triangle of tiles, row by row
            int r = (int)((sqrtf(8.0f * (float)bid + 1.0f) - 1.0f) * 0.5f);
            while ((r + 1) * (r + 2) / 2 <= bid) r++;
            while (r * (r + 1) / 2 > bid) r--;
            ti = r;
            tj = bid - r * (r + 1) / 2;
        } else if (!(p.order & 1)) {
            const int G = p.order ? p.group : GROUP;
            const int per_group = G * p.tiles_n;
            const int g = bid / per_group;
            const int first = g * G;
            const int rows = (p.tiles_m - first) < G ? (p.tiles_m - first) : G;
            const int in = bid - g * per_group;
            ti = first + in % rows;
            tj = in / rows;
        } else {
            // p.group tile columns at a time
            const int G = p.group;
            const int per_group = G * p.tiles_m;
            const int g = bid / per_group;
            const int first = g * G;
            const int cols = (p.tiles_n - first) < G ? (p.tiles_n - first) : G;
            const int in = bid - g * per_group;
            tj = first + in % cols;
            ti = in / cols;
        }
        if (p.order & 2) ti = p.tiles_m - 1 - ti;
        if (p.order & 4) tj = p.tiles_n - 1 - tj;
    }
    const int64_t i0 = ti * BM, j0 = tj * BN;
    const int64_t m = p.m, n = p.n;
    if (p.c_lower && j0 >= i0 + BM) return;  // tile entirely above the diagonal

    int64_t kb = (int64_t)blockIdx.z * p.kchunk;
    int64_t ke = kb + p.kchunk < p.k ? kb + p.kchunk : p.k;
    // skip k slabs that a triangular operand zeroes for this whole tile
    if (p.part == 0) {
        if (p.triA == TRI_LOWER || p.triA == TRI_SLOWER) ke = ke < i0 + BM ? ke : i0 + BM;
        if (p.triA == TRI_UPPER || p.triA == TRI_SUPPER) kb = kb > i0 ? kb : i0;
        if (p.triB == TRI_LOWER || p.triB == TRI_SLOWER) ke = ke < j0 + BN ? ke : j0 + BN;
        if (p.triB == TRI_UPPER || p.triB == TRI_SUPPER) kb = kb > j0 ? kb : j0;
    } else {
        // the crossing slabs [lo, hi): the tile's own rows of the operand;
        // below them a lower operand keeps every entry, above them an upper one
        const bool onA = p.triA != TRI_NONE;
        const int tri = onA ? p.triA : p.triB;
        const int64_t lo = onA ? i0 : j0, hi = lo + (onA ? BM : BN);
        const bool lower = tri == TRI_LOWER || tri == TRI_SLOWER;
        if (p.part == 2) {
            kb = kb > lo ? kb : lo;
            ke = ke < hi ? ke : hi;
        } else if (lower) {
            ke = ke < lo ? ke : lo;
        } else {
            kb = kb > hi ? kb : hi;
        }
    }

    typedef typename Lds<T, LP>::type LT;
    constexpr int KPL = Lds<T, LP>::pitch;
    __shared__ __attribute__((aligned(16))) LT As[2][BM][KPL];
    __shared__ __attribute__((aligned(16))) LT Bs[2][BN][KPL];

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;

    // slab depth of the register-staged path: 32 k values for FP16/BF16
    // operands (one 16x16x32 MFMA per fragment pair), 16 otherwise
    constexpr int SK = LP != 0 ? 32 : BK;
    constexpr int EA = BM * SK / NTH;  // elements of each operand tile per thread
    constexpr int EB = BN * SK / NTH;
    const int a_i = AMC ? (t % BM) : (t / SK);
    const int a_k = AMC ? (t / BM) : (t % SK);
    const int b_j = BNC ? (t % BN) : (t / SK);
    const int b_k = BNC ? (t / BN) : (t % SK);
    constexpr int A_STEP = AMC ? NTH / BM : NTH / SK;  // along k (AMC) or i
    constexpr int B_STEP = BNC ? NTH / BN : NTH / SK;

    const Band ba = band_of(p.triA), bb = band_of(p.triB);
    const int64_t kmax = p.k > 0 ? p.k - 1 : 0;
    const bool a_nomask = p.triA == TRI_NONE || p.part == 1, b_nomask = p.triB == TRI_NONE || p.part == 1;
    // Rows past the edge of a ragged tile are clamped to the last row of the
    // operand (a valid address; the value is zeroed when the slab is stored).
    // A column-major operand keeps one pointer per thread (its clamped row);
    // a k-contiguous one recomputes each row's address at every load from an
    // opaque copy of the thread's row, so that no per-row pointer (two
    // registers each) stays live across the main loop.  With the scheduling
    // fence between the two k groups of a slab (at most eight LDS fragments
    // in flight), every FP64 tile fits two workgroups per CU, which the MFMA
    // needs to hide HBM latency.
    const int a_lim = (int)((m - 1 - i0) < (BM - 1) ? (m - 1 - i0) : (BM - 1));
    const int b_lim = (int)((n - 1 - j0) < (BN - 1) ? (n - 1 - j0) : (BN - 1));
    const T* a_org = AMC ? p.A + i0 + (a_i < a_lim ? a_i : a_lim) : p.A + i0 * p.lda;
    const T* b_org = BNC ? p.B + j0 + (b_j < b_lim ? b_j : b_lim) : p.B + j0 * p.ldb;
    const bool a_all_rows = i0 + BM <= m, b_all_rows = j0 + BN <= n;

    T ra[EA], rb[EB];

    // Element (row ai + r A_STEP or ai, k index kk) of each operand's tile.
    auto ld_a = [&](int r, int ai, int64_t kk) -> T {
        if constexpr (AMC) return a_org[kk * p.lda];
        const int row = ai + r * A_STEP;
        const int64_t i = row < a_lim ? row : a_lim;
        return a_org[i * p.lda + kk];
    };
    auto ld_b = [&](int r, int bj, int64_t kk) -> T {
        if constexpr (BNC) return b_org[kk * p.ldb];
        const int row = bj + r * B_STEP;
        const int64_t j = row < b_lim ? row : b_lim;
        return b_org[j * p.ldb + kk];
    };
    // k offset within the slab of element r of a column-major operand's
    // thread (row fixed, k varying).  FP16/BF16 operands take runs of eight
    // consecutive k (group g + STEP (r / 8), element r % 8), so that a run
    // goes to LDS as one 16-byte store along its row; FP32/FP64 ones take
    // every STEP-th k.
    constexpr bool PACK = LP != 0;
    static_assert(!PACK || ((!AMC || EA % 8 == 0) && (!BNC || EB % 8 == 0)), "runs of eight k per thread");
    auto kofs = [&](int g, int step, int r) -> int { return PACK ? 8 * (g + step * (r / 8)) + (r % 8) : g + r * step; };
    // Full slab [k0, k0 + SK) inside [kb, ke): no k bounds.
    auto load_fast = [&](int64_t k0) {
        int ai = a_i, ak = a_k, bj = b_j, bk = b_k;
        asm volatile("" : "+v"(ai), "+v"(bj));
#pragma unroll
        for (int r = 0; r < EA; r++) ra[r] = ld_a(r, ai, k0 + (AMC ? kofs(ak, A_STEP, r) : ak));
#pragma unroll
        for (int r = 0; r < EB; r++) rb[r] = ld_b(r, bj, k0 + (BNC ? kofs(bk, B_STEP, r) : bk));
    };
    // Ragged last slab: k clamped into the operand (entries at or past ke are
    // zeroed by the store).
    auto load_tail = [&](int64_t k0) {
        int ai = a_i, ak = a_k, bj = b_j, bk = b_k;
        asm volatile("" : "+v"(ai), "+v"(bj));
#pragma unroll
        for (int r = 0; r < EA; r++) {
            const int64_t kk = k0 + (AMC ? kofs(ak, A_STEP, r) : ak);
            ra[r] = ld_a(r, ai, kk < kmax ? kk : kmax);
        }
#pragma unroll
        for (int r = 0; r < EB; r++) {
            const int64_t kk = k0 + (BNC ? kofs(bk, B_STEP, r) : bk);
            rb[r] = ld_b(r, bj, kk < kmax ? kk : kmax);
        }
    };
    auto mask_a = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < EA; r++) {
            const int64_t i = i0 + a_i + (AMC ? 0 : r * A_STEP);
            const int64_t kk = k0 + (AMC ? kofs(a_k, A_STEP, r) : a_k);
            const int64_t d = kk - i;
            const bool ok = i < m && kk < ke && d >= ba.lo && d <= ba.hi;
            ra[r] = ok ? ra[r] : T(0);
        }
    };
    auto mask_b = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < EB; r++) {
            const int64_t j = j0 + b_j + (BNC ? 0 : r * B_STEP);
            const int64_t kk = k0 + (BNC ? kofs(b_k, B_STEP, r) : b_k);
            const int64_t d = kk - j;
            const bool ok = j < n && kk < ke && d >= bb.lo && d <= bb.hi;
            rb[r] = ok ? rb[r] : T(0);
        }
    };
    auto store = [&](int buf, int64_t k0, bool tail) {
        // uniform per workgroup: the masks run only where a tile needs them
        if (tail || !a_all_rows || !a_nomask) mask_a(k0);
        if (tail || !b_all_rows || !b_nomask) mask_b(k0);
        if constexpr (PACK && AMC) {
            typedef LT v8t __attribute__((ext_vector_type(8)));
#pragma unroll
            for (int q = 0; q < EA / 8; q++) {
                v8t v;
#pragma unroll
                for (int e = 0; e < 8; e++) v[e] = to_lds<LP>(ra[8 * q + e]);
                *reinterpret_cast<v8t*>(&As[buf][a_i][8 * (a_k + A_STEP * q)]) = v;
            }
        } else {
#pragma unroll
            for (int r = 0; r < EA; r++) {
                if (AMC) As[buf][a_i][a_k + r * A_STEP] = to_lds<LP>(ra[r]);
                else As[buf][a_i + r * A_STEP][a_k] = to_lds<LP>(ra[r]);
            }
        }
        if constexpr (PACK && BNC) {
            typedef LT v8t __attribute__((ext_vector_type(8)));
#pragma unroll
            for (int q = 0; q < EB / 8; q++) {
                v8t v;
#pragma unroll
                for (int e = 0; e < 8; e++) v[e] = to_lds<LP>(rb[8 * q + e]);
                *reinterpret_cast<v8t*>(&Bs[buf][b_j][8 * (b_k + B_STEP * q)]) = v;
            }
        } else {
#pragma unroll
            for (int r = 0; r < EB; r++) {
                if (BNC) Bs[buf][b_j][b_k + r * B_STEP] = to_lds<LP>(rb[r]);
                else Bs[buf][b_j + r * B_STEP][b_k] = to_lds<LP>(rb[r]);
            }
        }
    };

    typedef typename Mfma<T>::acc acc_t;
    typedef typename Vec2<T>::type v2_t;
    acc_t acc[WMB][WNB];
#pragma unroll
    for (int a = 0; a < WMB; a++)
#pragma unroll
        for (int b = 0; b < WNB; b++) acc[a][b] = acc_t{0, 0, 0, 0};

    // Each ds_read_b128 brings two k values (2g, 2g+1 of an 8-wide k group,
    // g = lane / 16) for two MFMA k-steps; A and B use the same assignment, so
    // every k of the group is summed exactly once.
    const int lrow = lane & 15, lk = 2 * (lane >> 4);
    auto compute = [&](int buf) {
        if constexpr (LP != 0) {
            typedef typename std::conditional<LP == 1, v8h, v8s>::type v8l;
            const int lk8 = 8 * (lane >> 4);
            v8l af[WMB], bf[WNB];
#pragma unroll
            for (int x = 0; x < WMB; x++)
                af[x] = *reinterpret_cast<const v8l*>(&As[buf][wm * (BM / 2) + x * 16 + lrow][lk8]);
#pragma unroll
            for (int x = 0; x < WNB; x++)
                bf[x] = *reinterpret_cast<const v8l*>(&Bs[buf][wn * (BN / 2) + x * 16 + lrow][lk8]);
#pragma unroll
            for (int a = 0; a < WMB; a++)
#pragma unroll
                for (int b = 0; b < WNB; b++) {
                    if constexpr (LP == 1)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(CMC ? bf[b] : af[a], CMC ? af[a] : bf[b],
                                                                           acc[a][b], 0, 0, 0);
                    else
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(v8bf, CMC ? bf[b] : af[a]), __builtin_bit_cast(v8bf, CMC ? af[a] : bf[b]),
                            acc[a][b], 0, 0, 0);
                }
            return;
        } else {
#pragma unroll
        for (int kg = 0; kg < BK; kg += 8) {
            v2_t af[WMB], bf[WNB];
#pragma unroll
            for (int x = 0; x < WMB; x++)
                af[x] = *reinterpret_cast<const v2_t*>(&As[buf][wm * (BM / 2) + x * 16 + lrow][kg + lk]);
#pragma unroll
            for (int x = 0; x < WNB; x++)
                bf[x] = *reinterpret_cast<const v2_t*>(&Bs[buf][wn * (BN / 2) + x * 16 + lrow][kg + lk]);
#pragma unroll
            for (int a = 0; a < WMB; a++)
#pragma unroll
                for (int b = 0; b < WNB; b++)
                    acc[a][b] = Mfma<T>::op(CMC ? bf[b].x : af[a].x, CMC ? af[a].x : bf[b].x, acc[a][b]);
#pragma unroll
            for (int a = 0; a < WMB; a++)
#pragma unroll
                for (int b = 0; b < WNB; b++)
                    acc[a][b] = Mfma<T>::op(CMC ? bf[b].y : af[a].y, CMC ? af[a].y : bf[b].y, acc[a][b]);
            __builtin_amdgcn_sched_barrier(0);
        }
        }
    };

    const int64_t span = ke > kb ? ke - kb : 0;
    if constexpr (DMA) {
        // Direct staging (FP64, unmasked operands, whole slabs): each slab of
        // A and B goes from global memory straight into LDS, four bytes per
        // lane and instruction (any 8-byte-aligned pitch), with no register
        // copy; the registers this frees hold a second set of MFMA fragments,
        // so the next k group's LDS reads overlap the current one's products.
        // A k-contiguous operand keeps 128-byte rows whose 16-byte chunks are
        // permuted (chunk c of row r in slot c ^ (r & 7), and rows 8-15 of
        // every 16 swapped in pairs), which makes the fragment reads
        // conflict-free; an i-contiguous one keeps k rows padded by 64 bytes.
        // Separate arrays per buffer let the compiler see that a transfer into
        // one does not alias reads of the other.
        static_assert(sizeof(T) == 8 && LP == 0, "direct staging is FP64 only");
        constexpr int PA = AMC ? BM + 8 : BK, PB = BNC ? BN + 8 : BK;  // pitch (elements)
        constexpr int SA = AMC ? BK * PA : BM * BK, SB = BNC ? BK * PB : BN * BK;
        constexpr int QA = BM / 8, QB = BN / 8;  // transfers per thread and slab
        __shared__ __attribute__((aligned(16))) double A0[SA], A1[SA], B0[SB], B1[SB];
        const int wu = __builtin_amdgcn_readfirstlane(w);
        // Source of each transfer, in bytes from the slab origin.  Rows past a
        // ragged edge read the last row (their products are never stored).
        // Only a few per-lane parts stay live; the offsets themselves are
        // formed again at every slab (the parts are made opaque so that the
        // compiler does not keep one register per transfer across the loop).
        // i-contiguous: transfer q covers 32 rows of k column kq(q); the lane
        // part is the row's byte offset.  k-contiguous: transfer q covers two
        // rows, 8q + (rb ^ (q & 1)); the lane parts are rb and the chunk
        // offset for even and odd q.
        auto parts = [&](auto mc, auto bmx, int lim, int* rb, uint32_t* cb) {
            constexpr bool MC = decltype(mc)::value;
            constexpr int BX = decltype(bmx)::value;
            if constexpr (MC) {
                const int i = (BX == 128 ? wu : (wu & 1)) * 32 + (lane >> 1);
                cb[0] = (uint32_t)((i < lim ? i : lim) * 8 + (lane & 1) * 4);
            } else {
#pragma unroll
                for (int par = 0; par < 2; par++) {
                    rb[par] = (2 * wu + (lane >> 5)) ^ par;
                    const int c = ((lane & 31) >> 2) ^ (rb[par] & 7);
                    cb[par] = (uint32_t)((2 * c + ((lane & 3) >> 1)) * 8 + (lane & 1) * 4);
                }
            }
        };
        int rba[2] = {0, 0}, rbb[2] = {0, 0};
        uint32_t cba[2] = {0, 0}, cbb[2] = {0, 0};
        parts(std::integral_constant<bool, AMC>{}, std::integral_constant<int, BM>{}, a_lim, rba, cba);
        parts(std::integral_constant<bool, BNC>{}, std::integral_constant<int, BN>{}, b_lim, rbb, cbb);
        auto issue = [&](auto mc, auto bmx, double* X, const char* src, int64_t ld, int lim, int* rb0,
                         uint32_t* cb0) {
            constexpr bool MC = decltype(mc)::value;
            constexpr int BX = decltype(bmx)::value;
            constexpr int P = MC ? BX + 8 : BK;
            int rb[2] = {rb0[0], rb0[1]};
            uint32_t cb[2] = {cb0[0], cb0[1]};
            asm volatile("" : "+v"(rb[0]), "+v"(rb[1]), "+v"(cb[0]), "+v"(cb[1]));
            // likewise the uniform parts (each transfer's LDS base and column),
            // which would otherwise take one scalar register each
            int wq = wu;
            int64_t ldq = ld;
            asm volatile("" : "+s"(wq), "+s"(ldq));
            ld = ldq;
            if constexpr (MC) {
                // transfer q of wave w: k column KS q + kq0, rows 32 part .. + 31
                constexpr int KS = BX == 128 ? 1 : 2;
                const int kq0 = BX == 128 ? 0 : (wq >> 1), part = BX == 128 ? wq : (wq & 1);
                const uint32_t step = (uint32_t)(KS * ld * 8);
                uint32_t o = (uint32_t)(kq0 * ld * 8) + cb[0];
                double* d = X + kq0 * P + part * 32;
#pragma unroll
                for (int q = 0; q < BX / 8; q++) {
                    __builtin_amdgcn_global_load_lds((gvoid_t*)(src + o), (lvoid_t*)d, 4, 0, 0);
                    o += step;
                    d += KS * P;
                }
            } else {
                // row offsets in bytes: rb ld 8 per lane, 8 q ld 8 per transfer,
                // clamped at the last row with one min
                const uint32_t ld8 = (uint32_t)ld * 8u, last = (uint32_t)lim * ld8;
                const uint32_t ro[2] = {(uint32_t)rb[0] * ld8, (uint32_t)rb[1] * ld8};
#pragma unroll
                for (int q = 0; q < BX / 8; q++) {
                    uint32_t o = ro[q & 1] + (uint32_t)(8 * q) * ld8;
                    o = (o < last ? o : last) + cb[q & 1];
                    __builtin_amdgcn_global_load_lds((gvoid_t*)(src + o), (lvoid_t*)(X + (4 * q + wq) * 32), 4, 0, 0);
                }
            }
        };
        auto dma = [&](double* XA, double* XB, int64_t k0) {
            const char* sa = (const char*)(p.A + (AMC ? i0 + k0 * p.lda : i0 * p.lda + k0));
            const char* sb = (const char*)(p.B + (BNC ? j0 + k0 * p.ldb : j0 * p.ldb + k0));
            issue(std::integral_constant<bool, AMC>{}, std::integral_constant<int, BM>{}, XA, sa, p.lda, a_lim, rba,
                  cba);
            issue(std::integral_constant<bool, BNC>{}, std::integral_constant<int, BN>{}, XB, sb, p.ldb, b_lim, rbb,
                  cbb);
        };
        // fragments of k group kg: lane (lrow, g) holds k = kg + 2g (.x) and kg + 2g + 1 (.y)
        const int g = lane >> 4;
        const int rsw = lrow ^ ((lrow >> 3) & 1);
        const int sl0 = 2 * (g ^ (lrow & 7)), sl1 = 2 * ((4 + g) ^ (lrow & 7));
        auto frag = [&](const double* XA, const double* XB, auto kgc, v2_t(&af)[WMB], v2_t(&bf)[WNB]) {
            constexpr int kg = decltype(kgc)::value;
#pragma unroll
            for (int x = 0; x < WMB; x++) {
                const int r = wm * (BM / 2) + x * 16;
                if constexpr (AMC) {
                    const double* c = XA + (kg + 2 * g) * PA + r + lrow;
                    af[x] = v2_t{c[0], c[PA]};
                } else {
                    af[x] = *reinterpret_cast<const v2_t*>(XA + (r + rsw) * BK + (kg ? sl1 : sl0));
                }
            }
#pragma unroll
            for (int x = 0; x < WNB; x++) {
                const int r = wn * (BN / 2) + x * 16;
                if constexpr (BNC) {
                    const double* c = XB + (kg + 2 * g) * PB + r + lrow;
                    bf[x] = v2_t{c[0], c[PB]};
                } else {
                    bf[x] = *reinterpret_cast<const v2_t*>(XB + (r + rsw) * BK + (kg ? sl1 : sl0));
                }
            }
        };
        auto mma = [&](const v2_t(&af)[WMB], const v2_t(&bf)[WNB]) {
#pragma unroll
            for (int a = 0; a < WMB; a++)
#pragma unroll
                for (int b = 0; b < WNB; b++)
                    acc[a][b] = Mfma<T>::op(CMC ? bf[b].x : af[a].x, CMC ? af[a].x : bf[b].x, acc[a][b]);
#pragma unroll
            for (int a = 0; a < WMB; a++)
#pragma unroll
                for (int b = 0; b < WNB; b++)
                    acc[a][b] = Mfma<T>::op(CMC ? bf[b].y : af[a].y, CMC ? af[a].y : bf[b].y, acc[a][b]);
        };
        using K0 = std::integral_constant<int, 0>;
        using K8 = std::integral_constant<int, 8>;
        const int64_t ns = span / BK;  // whole slabs only (checked by the host)
        v2_t fa[WMB], fb[WNB], ga[WMB], gb[WNB];
        auto sync = [] {
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this thread's transfers have landed
            __syncthreads();
        };
        // One pass per slab s (buffer s % 2), entered after a barrier with k
        // group 1 of slab s in (ga, gb) and slab s + 1 complete in the other
        // buffer: start slab s + 2 into this buffer (slab s is no longer read;
        // near the end the last slab again, never read from here), read k
        // group 0 of slab s + 1, finish slab s, start slab s + 1, read its k
        // group 1, and meet at the barrier with no transfer outstanding.  The
        // transfers and LDS reads are spread over the products.
        auto pass = [&](double* CA, double* CB, double* NA, double* NB, int64_t s) {
            dma(CA, CB, kb + (s + 2 < ns ? s + 2 : ns - 1) * BK);
            frag(NA, NB, K0{}, fa, fb);
            mma(ga, gb);
            mma(fa, fb);
            frag(NA, NB, K8{}, ga, gb);
            constexpr int NT = (BM + BN) / 8, NM = 2 * WMB * WNB, NF = WMB + WNB;
            constexpr int M1 = NT / 2 < NM - NF ? NT / 2 : NM - NF;  // products carrying transfers
#pragma unroll
            for (int x = 0; x < M1; x++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x010, (NT + M1 - 1) / M1, 0);
            }
#pragma unroll
            for (int x = 0; x < NF; x++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            if constexpr (NM - M1 - NF > 0) __builtin_amdgcn_sched_group_barrier(0x008, NM - M1 - NF, 0);
#pragma unroll
            for (int x = 0; x < NF; x++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, NM - NF, 0);
            sync();
        };
        if (ns > 0) {
            dma(A0, B0, kb);
            if (ns > 1) dma(A1, B1, kb + BK);
            sync();
            frag(A0, B0, K0{}, fa, fb);
            mma(fa, fb);
            frag(A0, B0, K8{}, ga, gb);
            sync();
            int64_t s = 0;
            while (s + 1 < ns) {
                pass(A0, B0, A1, B1, s++);
                if (s + 1 >= ns) break;
                pass(A1, B1, A0, B0, s++);
            }
            mma(ga, gb);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // the spare transfers of the last passes
        }
    } else {
        const int64_t nfull = span / SK, nslab = (span + SK - 1) / SK;
        if (nslab > 0) {
            if (nfull > 0) load_fast(kb);
            else load_tail(kb);
            store(0, kb, nfull == 0);
            __syncthreads();
            int64_t s = 0;
            // steady state: the slab being prefetched is a full one.  The
            // scheduling fence keeps the next slab's LDS stores (and the wait for
            // its global loads that they imply) after this slab's products.
            for (; s + 1 < nfull; s++) {
                load_fast(kb + (s + 1) * SK);
                compute((int)(s & 1));
                __builtin_amdgcn_sched_barrier(0);
                store((int)((s + 1) & 1), kb + (s + 1) * SK, false);
                __syncthreads();
            }
            if (s + 1 < nslab) {  // a ragged slab follows the last full one
                load_tail(kb + (s + 1) * SK);
                compute((int)(s & 1));
                __builtin_amdgcn_sched_barrier(0);
                store((int)((s + 1) & 1), kb + (s + 1) * SK, true);
                __syncthreads();
                s++;
            }
            compute((int)(s & 1));
        }
    }

    // accumulator (a, b)[r] holds C(row, col) with row = wm*BM/2 + a*16 + x,
    // col = wn*BN/2 + b*16 + y, where (x, y) = (Mfma<T>::row(lane, r), lane%16);
    // for column-major C the products are formed transposed (operands swapped)
    // and (x, y) = (lane%16, Mfma<T>::row(lane, r)), so that the 16 lanes of a
    // row group store 16 consecutive elements of a column
    const int cl = lane & 15;
    if (p.W) {
        T* W = p.W + (int64_t)blockIdx.z * m * n;
#pragma unroll
        for (int a = 0; a < WMB; a++)
#pragma unroll
            for (int b = 0; b < WNB; b++) {
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int64_t i = i0 + wm * (BM / 2) + a * 16 + (CMC ? cl : Mfma<T>::row(lane, r));
                    const int64_t j = j0 + wn * (BN / 2) + b * 16 + (CMC ? Mfma<T>::row(lane, r) : cl);
                    if (i < m && j < n) W[j * m + i] = acc[a][b][r];
                }
            }
        return;
    }
    // Element (a, b, r) of this thread's share of the tile: its address, and
    // whether it is stored at all.
    auto c_at = [&](int a, int b, int r, bool& ok) -> T* {
        const int64_t i = i0 + wm * (BM / 2) + a * 16 + (CMC ? cl : Mfma<T>::row(lane, r));
        const int64_t j = j0 + wn * (BN / 2) + b * 16 + (CMC ? Mfma<T>::row(lane, r) : cl);
        ok = i < m && j < n && (!p.c_lower || i >= j);
        return CMC ? &p.C[i + j * p.ldc] : &p.C[i * p.ldc + j];
    };
    if (p.beta == T(0)) {
#pragma unroll
        for (int a = 0; a < WMB; a++)
#pragma unroll
            for (int b = 0; b < WNB; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    bool ok;
                    T* c = c_at(a, b, r, ok);
                    if (ok) *c = p.alpha * acc[a][b][r];
                }
        return;
    }
    // C = alpha acc + beta C by block rows of 16: a block row's reads are all
    // issued before any of its results is stored (written element by element,
    // read-then-store would serialise one memory latency per element, since
    // the compiler cannot prove the addresses distinct), and for row-major C
    // the next block row's reads before this one's stores.
    T cv[CMC ? 1 : 2][WNB][4];
    auto fetch = [&](int a, auto buf) {
        constexpr int q = decltype(buf)::value;
#pragma unroll
        for (int b = 0; b < WNB; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                bool ok;
                const T* c = c_at(a, b, r, ok);
                cv[q][b][r] = ok ? *c : T(0);
            }
    };
    auto finish = [&](int a, auto buf) {
        constexpr int q = decltype(buf)::value;
#pragma unroll
        for (int b = 0; b < WNB; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                bool ok;
                T* c = c_at(a, b, r, ok);
                if (ok) *c = p.alpha * acc[a][b][r] + p.beta * cv[q][b][r];
            }
    };
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;
    if constexpr (CMC) {
        // (one buffer: the column-major address arithmetic leaves no room for two)
#pragma unroll
        for (int a = 0; a < WMB; a++) {
            fetch(a, B0{});
            finish(a, B0{});
        }
    } else {
        fetch(0, B0{});
#pragma unroll
        for (int a = 0; a < WMB; a += 2) {
            if (a + 1 < WMB) fetch(a + 1, B1{});
            finish(a, B0{});
            if (a + 1 < WMB) {
                if (a + 2 < WMB) fetch(a + 2, B0{});
                finish(a + 1, B1{});
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

template <typename T>
static constexpr const char* tname() { return sizeof(T) == 8 ? "double" : "float"; }

// Demangled kernel names as rocprofv3 prints them.
template <typename T, bool AMC, bool BNC, bool CMC, int WMB, int WNB, int LP = 0, bool DMA = false>
static const char* kname()
{
    static char buf[120];
    if (!buf[0])
        snprintf(buf, sizeof buf, "rfp::gemm_kernel<%s, %s, %s, %s, %d, %d, %d, %s>(rfp::GemmParams<%s>)", tname<T>(),
                 AMC ? "true" : "false", BNC ? "true" : "false", CMC ? "true" : "false", WMB, WNB, LP,
                 DMA ? "true" : "false", tname<T>());
    return buf;
}

// Algorithmic work of one launch: multiply-adds over the entries of C that
// are computed and the k-range each one needs once triangular operands are
// taken into account (zero entries of a masked operand are not work).
static double tri_pairs(int tri, int64_t rows, int64_t k)
{
    // number of kept (row, kk) pairs of an operand of `rows` x `k` under mask tri
    auto lower = [](int64_t r, int64_t c, int64_t d) {  // #(i,j): i - j >= d
        double s = 0;
        for (int64_t i = 0; i < r; i++) {
            int64_t hi = i - d + 1;
            s += hi <= 0 ? 0 : (double)(hi < c ? hi : c);
        }
        return s;
    };
    switch (tri) {
        case TRI_LOWER: return lower(rows, k, 0);
        case TRI_SLOWER: return lower(rows, k, 1);
        case TRI_UPPER: return (double)rows * k - lower(rows, k, 1);
        case TRI_SUPPER: return (double)rows * k - lower(rows, k, 0);
        default: return (double)rows * k;
    }
}

template <typename T>
static double out_cells(const GemmParams<T>& p)
{
    // entries of C computed: all, or those with i >= j (m >= n)
    return p.c_lower ? (double)p.m * p.n - 0.5 * (double)p.n * (double)(p.n - 1) : (double)p.m * (double)p.n;
}

// Kept (row, kk) pairs of a triangular operand inside the slabs that cross
// its diagonal next to each row's tile (tiles of `band` rows).
static double band_pairs(int tri, int64_t rows, int64_t k, int band)
{
    double s = 0;
    for (int64_t i = 0; i < rows; i++) {
        const int64_t t0 = i / band * band, t1 = t0 + band < k ? t0 + band : k;
        int64_t lo = t0, hi = t1;  // kept kk in [lo, hi)
        switch (tri) {
            case TRI_LOWER: hi = hi < i + 1 ? hi : i + 1; break;
            case TRI_SLOWER: hi = hi < i ? hi : i; break;
            case TRI_UPPER: lo = lo > i ? lo : i; break;
            case TRI_SUPPER: lo = lo > i + 1 ? lo : i + 1; break;
            default: break;
        }
        if (hi > lo) s += (double)(hi - lo);
    }
    return s;
}

template <typename T>
static double gemm_flops(const GemmParams<T>& p)
{
    double cells = out_cells(p);
    double kfrac = 1.0;
    if (p.k > 0) {
        if (p.part != 0) {
            const bool onA = p.triA != TRI_NONE;
            const int tri = onA ? p.triA : p.triB;
            const int64_t rows = onA ? p.m : p.n;
            const double band = band_pairs(tri, rows, p.k, p.band);
            const double kept = p.part == 2 ? band : tri_pairs(tri, rows, p.k) - band;
            kfrac = kept / ((double)rows * p.k);
        } else {
            if (p.triA) kfrac *= tri_pairs(p.triA, p.m, p.k) / ((double)p.m * p.k);
            if (p.triB) kfrac *= tri_pairs(p.triB, p.n, p.k) / ((double)p.n * p.k);
        }
    }
    return 2.0 * cells * (double)p.k * kfrac;
}

template <typename T>
static double gemm_bytes(const GemmParams<T>& p)
{
    double cells = out_cells(p);
    return sizeof(T) * ((double)p.m * p.k + (double)p.n * p.k + cells * (p.beta != T(0) ? 2.0 : 1.0));
}

template <typename T, bool AMC, bool BNC, bool CMC>
static void launch(const GemmParams<T>& p, dim3 grid, int tile, const Exec& ex, int lp, bool dma)
{
    if constexpr (sizeof(T) == 4) {
        // low-precision operand kernels: square tiles only (128 or 64)
        if (lp == 1 || lp == 2) {
            const bool big = tile == 0;
            if (lp == 1 && big) {
                ProfScope ps(ex, kname<T, AMC, BNC, CMC, 4, 4, 1>(), gemm_flops(p), gemm_bytes(p));
                hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 4, 4, 1>), grid, dim3(NTH), 0, ex.stream, p);
            } else if (lp == 1) {
                ProfScope ps(ex, kname<T, AMC, BNC, CMC, 2, 2, 1>(), gemm_flops(p), gemm_bytes(p));
                hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 2, 2, 1>), grid, dim3(NTH), 0, ex.stream, p);
            } else if (big) {
                ProfScope ps(ex, kname<T, AMC, BNC, CMC, 4, 4, 2>(), gemm_flops(p), gemm_bytes(p));
                hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 4, 4, 2>), grid, dim3(NTH), 0, ex.stream, p);
            } else {
                ProfScope ps(ex, kname<T, AMC, BNC, CMC, 2, 2, 2>(), gemm_flops(p), gemm_bytes(p));
                hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 2, 2, 2>), grid, dim3(NTH), 0, ex.stream, p);
            }
            return;
        }
    }
    if constexpr (sizeof(T) == 8) {
        if (dma) {
            switch (tile) {
                case 0: {
                    ProfScope ps(ex, kname<T, AMC, BNC, CMC, 4, 4, 0, true>(), gemm_flops(p), gemm_bytes(p));
                    hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 4, 4, 0, true>), grid, dim3(NTH), 0, ex.stream, p);
                } break;
                case 1: {
                    ProfScope ps(ex, kname<T, AMC, BNC, CMC, 2, 4, 0, true>(), gemm_flops(p), gemm_bytes(p));
                    hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 2, 4, 0, true>), grid, dim3(NTH), 0, ex.stream, p);
                } break;
                case 2: {
                    ProfScope ps(ex, kname<T, AMC, BNC, CMC, 4, 2, 0, true>(), gemm_flops(p), gemm_bytes(p));
                    hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 4, 2, 0, true>), grid, dim3(NTH), 0, ex.stream, p);
                } break;
                default: {
                    ProfScope ps(ex, kname<T, AMC, BNC, CMC, 2, 2, 0, true>(), gemm_flops(p), gemm_bytes(p));
                    hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 2, 2, 0, true>), grid, dim3(NTH), 0, ex.stream, p);
                } break;
            }
            return;
        }
    }
    switch (tile) {
        case 0: {
            ProfScope ps(ex, kname<T, AMC, BNC, CMC, 4, 4>(), gemm_flops(p), gemm_bytes(p));
            hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 4, 4>), grid, dim3(NTH), 0, ex.stream, p);
        } break;
        case 1: {
            ProfScope ps(ex, kname<T, AMC, BNC, CMC, 2, 4>(), gemm_flops(p), gemm_bytes(p));
            hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 2, 4>), grid, dim3(NTH), 0, ex.stream, p);
        } break;
        case 2: {
            ProfScope ps(ex, kname<T, AMC, BNC, CMC, 4, 2>(), gemm_flops(p), gemm_bytes(p));
            hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 4, 2>), grid, dim3(NTH), 0, ex.stream, p);
        } break;
        default: {
            ProfScope ps(ex, kname<T, AMC, BNC, CMC, 2, 2>(), gemm_flops(p), gemm_bytes(p));
            hipLaunchKernelGGL((gemm_kernel<T, AMC, BNC, CMC, 2, 2>), grid, dim3(NTH), 0, ex.stream, p);
        } break;
    }
}

// Tile shapes (BM x BN): 0 = 128 x 128, 1 = 64 x 128, 2 = 128 x 64, 3 = 64 x 64.
static const int TILE_BM[4] = {128, 64, 128, 64};
static const int TILE_BN[4] = {128, 128, 64, 64};

// Pick the largest tile that still gives the chip enough workgroups.  For an
// in-place product a dimension of at most 128 is covered by a single tile, so
// each workgroup owns whole rows (C aliasing A) or columns (C aliasing B).
static int pick_tile(int64_t m, int64_t n, bool c_lower, bool inplace, int64_t* tm, int64_t* tn,
                     bool square_only = false)
{
    const int64_t want = 512;  // two workgroups per CU on 256 CUs
    int best = -1;
    int64_t best_tiles = -1;
    for (int t = 0; t < 4; t++) {
        const int bm = TILE_BM[t], bn = TILE_BN[t];
        if (square_only && bm != bn) continue;
        if (c_lower && m == n && bm != bn) continue;
        if (inplace && m <= 128 && bm < m) continue;
        if (inplace && n <= 128 && bn < n) continue;
        const int64_t a = (m + bm - 1) / bm, b = (n + bn - 1) / bn;
        const int64_t tiles = (c_lower && m == n) ? a * (a + 1) / 2 : a * b;
        if (tiles >= want) {
            best = t;
            best_tiles = tiles;
            break;
        }
        if (tiles > best_tiles) {
            best = t;
            best_tiles = tiles;
        }
    }
    *tm = (m + TILE_BM[best] - 1) / TILE_BM[best];
    *tn = (n + TILE_BN[best] - 1) / TILE_BN[best];
    return best;
}

hipError_t gemm_validate(int64_t m, int64_t n, int64_t a_rs, int64_t a_cs, int64_t b_rs, int64_t b_cs,
                         int64_t c_rs, int64_t c_cs, bool c_lower, bool inplace)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    if (inplace && m > 128 && n > 128) return hipErrorInvalidValue;
    if (c_lower && m < n) return hipErrorInvalidValue;
    if (a_rs != 1 && a_cs != 1) return hipErrorInvalidValue;
    if (b_rs != 1 && b_cs != 1) return hipErrorInvalidValue;
    if (c_rs != 1 && c_cs != 1) return hipErrorInvalidValue;
    return hipSuccess;
}

template <typename T>
hipError_t gemm(const Exec& ex, int64_t m, int64_t n, int64_t k, T alpha, Mat<const T> A, int triA,
                Mat<const T> B, int triB, T beta, Mat<T> C, bool c_lower, bool inplace)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    {
        const hipError_t v = gemm_validate(m, n, A.rs, A.cs, B.rs, B.cs, C.rs, C.cs, c_lower, inplace);
        if (v != hipSuccess) return v;
    }
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
    p.prio = ex.prio;
    int64_t tm, tn;
    // low-precision operands for the bulk updates only: in-place products
    // (the leaf-level panel solves) stay in FP32
    const int lp = (sizeof(T) == 4 && !inplace) ? ex.lowp : 0;
    const bool amc0 = A.rs == 1, bnc0 = B.rs == 1, cmc0 = C.rs == 1;
    // an autotuned (or forced) configuration for this shape class, if admissible
    int tile = -1, tsplit = 0;
    if (ex.tune && !inplace) {
        const int sel0 = (amc0 ? 4 : 0) | (bnc0 ? 2 : 0) | (cmc0 ? 1 : 0);
        auto it = ex.tune->gemm.find(
            tune_gemm_key(sizeof(T) == 8 ? 0 : 1, lp, sel0, c_lower ? 1 : 0, m, n, k < 0 ? 0 : k));
        if (it != ex.tune->gemm.end()) {
            tile = it->second.tile;
            tsplit = it->second.split;
        } else if (ex.tune->force_tile >= 0) {
            tile = ex.tune->force_tile;
            tsplit = ex.tune->force_split;
        }
        if (tile < 0 || tile > 3 || (c_lower && m == n && TILE_BM[tile] != TILE_BN[tile]) ||
            (lp && TILE_BM[tile] != TILE_BN[tile]))
            tile = -1;
    }
    if (tile >= 0) {
        tm = (m + TILE_BM[tile] - 1) / TILE_BM[tile];
        tn = (n + TILE_BN[tile] - 1) / TILE_BN[tile];
    } else {
        tile = pick_tile(m, n, c_lower, inplace, &tm, &tn, lp != 0);
    }
    p.tri_enum = (c_lower && m == n) ? 1 : 0;
    if (!p.tri_enum && (triA != TRI_NONE) != (triB != TRI_NONE)) {
        const bool lowA = triA == TRI_LOWER || triA == TRI_SLOWER, lowB = triB == TRI_LOWER || triB == TRI_SLOWER;
        p.order = 8 | (triA != TRI_NONE ? (1 | (lowA ? 2 : 0)) : (lowB ? 4 : 0));
        const int64_t across = (p.order & 1) ? tn : tm;  // tiles the groups are cut from
        p.group = (int)std::min<int64_t>(GROUP, std::max<int64_t>(1, across / NXCD));
    }
    const int64_t ntiles = p.tri_enum ? tm * (tm + 1) / 2 : tm * tn;
    p.tiles_m = (int)tm;
    p.tiles_n = (int)tn;

    // split K when the tile grid cannot fill the chip and K is long (or as tuned)
    int64_t nsplit = 1;
    if (tsplit > 1 && ex.splitk_ws) {
        nsplit = tsplit;
        if (nsplit > p.k / BK) nsplit = p.k / BK;
        while (nsplit > 1 && (size_t)(nsplit * m * n) * sizeof(T) > ex.splitk_bytes) nsplit--;
        if (nsplit < 1) nsplit = 1;
    } else if (tsplit == 0 && ntiles < 256 && p.k >= 1024 && ex.splitk_ws) {
        nsplit = (512 + ntiles - 1) / ntiles;
        int64_t kmax = p.k / 256;
        if (nsplit > kmax) nsplit = kmax;
        if (nsplit > 32) nsplit = 32;
        while (nsplit > 1 && (size_t)(nsplit * m * n) * sizeof(T) > ex.splitk_bytes) nsplit--;
    }
    if (nsplit > 1) {
        const int64_t sk = lp != 0 ? 32 : BK;  // the kernel's slab depth
        int64_t chunk = (p.k + nsplit - 1) / nsplit;
        chunk = (chunk + sk - 1) / sk * sk;
        nsplit = (p.k + chunk - 1) / chunk;
        p.kchunk = chunk;
        p.W = (T*)ex.splitk_ws;
    } else {
        p.kchunk = p.k;
        p.W = nullptr;
    }
    dim3 grid((unsigned)ntiles, 1, (unsigned)nsplit);
    // direct global-to-LDS staging: FP64, unmasked operands, whole slabs, one
    // pass over k, row offsets within 32 bits (the in-place leaf products
    // keep the register path)
#ifndef RFP_GEMM_DIRECT
#define RFP_GEMM_DIRECT 1
#endif
    const bool direct_ok = RFP_GEMM_DIRECT && sizeof(T) == 8 && lp == 0 && !inplace && nsplit == 1 &&
                           p.k % BK == 0 && p.lda < (1 << 22) && p.ldb < (1 << 22);
    const bool dma = direct_ok && triA == TRI_NONE && triB == TRI_NONE;
    const int sel = (amc ? 4 : 0) | (bnc ? 2 : 0) | (cmc ? 1 : 0);
    // One triangular operand and a long k-range: the slabs the operand keeps
    // whole go through the direct-staging kernel without masks, then the
    // slabs crossing its diagonal (one tile's worth of k) are added by the
    // masked kernel.
    if (direct_ok && (triA != TRI_NONE) != (triB != TRI_NONE) && p.k > 2 * TILE_BM[0]) {
        GemmParams<T> q = p;
        q.part = 1;
        q.band = triA != TRI_NONE ? TILE_BM[tile] : TILE_BN[tile];
        auto go = [&](const GemmParams<T>& g, bool direct) {
            switch (sel) {
                case 0: launch<T, false, false, false>(g, grid, tile, ex, lp, direct); break;
                case 1: launch<T, false, false, true>(g, grid, tile, ex, lp, direct); break;
                case 2: launch<T, false, true, false>(g, grid, tile, ex, lp, direct); break;
                case 3: launch<T, false, true, true>(g, grid, tile, ex, lp, direct); break;
                case 4: launch<T, true, false, false>(g, grid, tile, ex, lp, direct); break;
                case 5: launch<T, true, false, true>(g, grid, tile, ex, lp, direct); break;
                case 6: launch<T, true, true, false>(g, grid, tile, ex, lp, direct); break;
                default: launch<T, true, true, true>(g, grid, tile, ex, lp, direct); break;
            }
        };
        go(q, true);
        q.part = 2;
        q.beta = T(1);
        go(q, false);
        return hipGetLastError();
    }
    switch (sel) {
        case 0: launch<T, false, false, false>(p, grid, tile, ex, lp, dma); break;
        case 1: launch<T, false, false, true>(p, grid, tile, ex, lp, dma); break;
        case 2: launch<T, false, true, false>(p, grid, tile, ex, lp, dma); break;
        case 3: launch<T, false, true, true>(p, grid, tile, ex, lp, dma); break;
        case 4: launch<T, true, false, false>(p, grid, tile, ex, lp, dma); break;
        case 5: launch<T, true, false, true>(p, grid, tile, ex, lp, dma); break;
        case 6: launch<T, true, true, false>(p, grid, tile, ex, lp, dma); break;
        default: launch<T, true, true, true>(p, grid, tile, ex, lp, dma); break;
    }
    if (nsplit > 1) {
        const int64_t total = m * n;
        dim3 g((unsigned)((total + 255) / 256));
        static char rn[2][80];
        const int ci = cmc ? 1 : 0;
        if (!rn[ci][0])
            snprintf(rn[ci], sizeof rn[ci], "rfp::splitk_reduce<%s, %s>(rfp::GemmParams<%s>, int)", tname<T>(),
                     cmc ? "true" : "false", tname<T>());
        ProfScope ps(ex, rn[ci], (double)nsplit * total, sizeof(T) * (double)(nsplit + 1) * total);
        if (cmc) hipLaunchKernelGGL((splitk_reduce<T, true>), g, dim3(256), 0, ex.stream, p, (int)nsplit);
        else hipLaunchKernelGGL((splitk_reduce<T, false>), g, dim3(256), 0, ex.stream, p, (int)nsplit);
    }
    return hipGetLastError();
}

template hipError_t gemm<double>(const Exec&, int64_t, int64_t, int64_t, double, Mat<const double>, int,
                                 Mat<const double>, int, double, Mat<double>, bool, bool);
template hipError_t gemm<float>(const Exec&, int64_t, int64_t, int64_t, float, Mat<const float>, int,
                                Mat<const float>, int, float, Mat<float>, bool, bool);

}  // namespace rfp
