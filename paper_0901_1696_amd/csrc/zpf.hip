// Complex Hermitian (Z) RFP Cholesky: factorization, solution and inversion
// of a Hermitian positive definite matrix held in complex Rectangular Full
// Packed Format (Section 3, A = L L^H; Section 4, L Y = B and L^H X = Y;
// Section 5, A^{-1} = W^H W with W = L^{-1}; the complex rows of the routine
// table: ZPFTRF, ZPFTRS, ZPFTRI with TRANSR = 'N' or 'C').
//
// Format: the element positions are those of the real format of the same
// TRANSR/UPLO; wherever the real format keeps a part transposed, the complex
// one keeps its conjugate transpose, and TRANSR = 'C' keeps the conjugate
// transpose of the whole rectangle.  Each of the three blocks (L11, L21, L22
// of the canonical lower matrix) is therefore a strided view whose numbers
// are either the canonical elements or their conjugates (ZView::conj).
//
// Arithmetic: complex numbers are interleaved (re, im) doubles.  Every block
// product goes through one MFMA kernel: a 64 x 64 tile of C per workgroup,
// operands staged in LDS as separate real and imaginary planes (conjugation,
// transposition and triangular masks applied while staging), and each complex
// multiply-add of a 16 x 16 x 4 step formed by four FP64 MFMAs
// (re += ar br - ai bi, im += ar bi + ai br).  Diagonal blocks of at most 64
// rows are factored and inverted by one workgroup in LDS.  The blocked
// drivers below follow the paper's steps with 64-column blocks.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rfp_common.h"

namespace rfp {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int ZT = 64;  // C tile (rows and columns) and leaf order
constexpr int ZK = 16;  // K step of the product
constexpr int ZQ = ZT * ZK / 256;  // operand elements per thread and K step

__device__ __forceinline__ void wave_sync_z() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ double2 zconj_if(double2 v, bool c)
{
    if (c) v.y = -v.y;
    return v;
}

// C = alpha op(A) op(B) + beta C on views (real alpha, beta).
//   op(A) is M x K: A (ta = 0) or A^H (ta = 1); an element (r, c) of A's view
//   (before op) counts only when r - c >= mda (else it is zero);
//   likewise B (N columns) with tb, mdb; C(i, j) is written only when
//   i - j >= mdc.  beta = 0: C is not read.  gate: nothing runs while *gate.
//   Split K (part != null): workgroup z of a tile sums only K range
//   [z kchunk, (z + 1) kchunk) and stores its raw sums in part (one 64 x 64
//   block per tile and z); zsplit_reduce_kernel then adds the nsplit blocks
//   of a tile in order of z and applies alpha, beta and the mask.
struct ZGemm {
    int64_t M, N, K;
    ZView A, B, C;
    int ta, tb;
    int64_t mda, mdb, mdc;
    double alpha, beta;
    const int* gate;
    int64_t kchunk;
    int nsplit;
    double2* part;
};

__global__ __launch_bounds__(256, 2) void zgemm_kernel(ZGemm g)
{
    if (g.gate && *g.gate) return;
    const int64_t i0 = (int64_t)blockIdx.x * ZT, j0 = (int64_t)blockIdx.y * ZT;
    if (i0 + ZT - 1 - j0 < g.mdc) return;  // the whole tile lies outside C's mask
    constexpr int PA = ZT + 8;
    __shared__ double Ar[ZK][PA], Ai[ZK][PA], Br[ZK][PA], Bi[ZK][PA];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;

    // K range where both operands can be nonzero for this tile
    int64_t klo = 0, khi = g.K;
    if (g.part) {
        klo = (int64_t)blockIdx.z * g.kchunk;
        khi = std::min<int64_t>(khi, klo + g.kchunk);
    }
    if (g.mda > ZMASK_NONE) {
        if (!g.ta) khi = std::min<int64_t>(khi, i0 + ZT - 1 - g.mda + 1);  // A(i, k): k <= i - mda
        else klo = std::max<int64_t>(klo, i0 + g.mda);                     // A(k, i): k >= i + mda
    }
    if (g.mdb > ZMASK_NONE) {
        if (!g.tb) klo = std::max<int64_t>(klo, j0 + g.mdb);               // B(k, j): k >= j + mdb
        else khi = std::min<int64_t>(khi, j0 + ZT - 1 - g.mdb + 1);        // B(j, k): k <= j - mdb
    }

    // staging maps: the element index e = t + 256 q runs along the operand's
    // unit stride (coalesced loads): element q of a thread is (i0 + i, k) with
    // i = i_0 + q di, k = k_0 + q dk (di, dk: 0 and 8, or 4 and 0), so its
    // address is base + q step + k0 times the stride along K.
    const bool a_fast_i = (g.ta ? g.A.cs : g.A.rs) == 1;
    const bool b_fast_j = (g.tb ? g.B.rs : g.B.cs) == 1;
    const bool aconj = g.A.conj != (g.ta != 0), bconj = g.B.conj != (g.tb != 0);
    const int64_t a_is = g.ta ? g.A.cs : g.A.rs, a_ks = g.ta ? g.A.rs : g.A.cs;  // strides along i and K
    const int64_t b_js = g.tb ? g.B.rs : g.B.cs, b_ks = g.tb ? g.B.cs : g.B.rs;  // along j and K
    const int ai_0 = a_fast_i ? (t & (ZT - 1)) : t / ZK, ak_0 = a_fast_i ? t / ZT : (t & (ZK - 1));
    const int a_di = a_fast_i ? 0 : 256 / ZK, a_dk = a_fast_i ? 256 / ZT : 0;
    const int bj_0 = b_fast_j ? (t & (ZT - 1)) : t / ZK, bk_0 = b_fast_j ? t / ZT : (t & (ZK - 1));
    const int b_dj = b_fast_j ? 0 : 256 / ZK, b_dk = b_fast_j ? 256 / ZT : 0;
    const double2* a_base = g.A.p + (i0 + ai_0) * a_is + ak_0 * a_ks;
    const double2* b_base = g.B.p + (j0 + bj_0) * b_js + bk_0 * b_ks;
    const int64_t a_step = a_di * a_is + a_dk * a_ks, b_step = b_dj * b_js + b_dk * b_ks;
    // Raw operand values of the next step and their keep masks (bit q):
    // every lane loads (a masked element reads the view's first element,
    // always valid), and the mask and conjugation are applied only when the
    // values are staged, so the loads stay in flight during the products.
    double2 ra[ZQ], rb[ZQ];
    unsigned ma = 0, mb = 0;
    auto load = [&](int64_t k0) {
        const double2* pa = a_base + k0 * a_ks;
        const double2* pb = b_base + k0 * b_ks;
        ma = mb = 0;
#pragma unroll
        for (int q = 0; q < ZQ; q++) {
            const int64_t gi = i0 + ai_0 + q * a_di, gka = k0 + ak_0 + q * a_dk;
            const int64_t gj = j0 + bj_0 + q * b_dj, gkb = k0 + bk_0 + q * b_dk;
            // masks on the stored (row - column): A(gi, k) or A(k, gi); B(k, gj) or B(gj, k)
            const bool ia = gi < g.M && gka >= klo && gka < khi && (g.ta ? gka - gi : gi - gka) >= g.mda;
            const bool ib = gj < g.N && gkb >= klo && gkb < khi && (g.tb ? gj - gkb : gkb - gj) >= g.mdb;
            ra[q] = *(ia ? pa + q * a_step : g.A.p);
            rb[q] = *(ib ? pb + q * b_step : g.B.p);
            ma |= (ia ? 1u : 0u) << q;
            mb |= (ib ? 1u : 0u) << q;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int q = 0; q < ZQ; q++) {
            const double2 va = (ma >> q) & 1 ? zconj_if(ra[q], aconj) : make_double2(0.0, 0.0);
            const double2 vb = (mb >> q) & 1 ? zconj_if(rb[q], bconj) : make_double2(0.0, 0.0);
            Ar[ak_0 + q * a_dk][ai_0 + q * a_di] = va.x;
            Ai[ak_0 + q * a_dk][ai_0 + q * a_di] = va.y;
            Br[bk_0 + q * b_dk][bj_0 + q * b_dj] = vb.x;
            Bi[bk_0 + q * b_dk][bj_0 + q * b_dj] = vb.y;
        }
    };

    v4d cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) cr[a][b] = ci[a][b] = v4d{0, 0, 0, 0};

    int64_t k0 = klo / ZK * ZK;  // K steps aligned to ZK (elements below klo are masked)
    if (k0 < khi) load(k0);
    for (; k0 < khi; k0 += ZK) {
        __syncthreads();  // the previous step's reads of the planes are done
        stage();
        __syncthreads();
        if (k0 + ZK < khi) load(k0 + ZK);  // in flight during this step's products
#pragma unroll
        for (int kk = 0; kk < ZK; kk += 4) {
            const int k = kk + (lane >> 4);
            double ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int a = 0; a < 2; a++) {
                ar[a] = Ar[k][32 * wr + 16 * a + (lane & 15)];
                ai[a] = Ai[k][32 * wr + 16 * a + (lane & 15)];
            }
#pragma unroll
            for (int b = 0; b < 2; b++) {
                br[b] = Br[k][32 * wc + 16 * b + (lane & 15)];
                bi[b] = Bi[k][32 * wc + 16 * b + (lane & 15)];
            }
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++) {
                    cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], cr[a][b], 0, 0, 0);
                    cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], bi[b], cr[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], ci[a][b], 0, 0, 0);
                    ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], ci[a][b], 0, 0, 0);
                }
        }
    }

    // result element r of a lane: row (lane / 16) + 4 r, column lane % 16
    if (g.part) {
        double2* pb = g.part + (((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * g.nsplit + blockIdx.z) * ZT * ZT;
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int li = 32 * wr + 16 * a + (lane >> 4) + 4 * r, lj = 32 * wc + 16 * b + (lane & 15);
                    pb[li + lj * ZT] = make_double2(cr[a][b][r], ci[a][b][r]);
                }
        return;
    }
    // by halves of the wave's rows: all reads of C first (a masked element
    // reads C's first element), then the stores, so that the reads are not
    // each waited for inside a branch
#pragma unroll
    for (int a = 0; a < 2; a++) {
        double2 o[2][4];
        if (g.beta != 0.0) {
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int64_t i = i0 + 32 * wr + 16 * a + (lane >> 4) + 4 * r;
                    const int64_t j = j0 + 32 * wc + 16 * b + (lane & 15);
                    const bool ok = i < g.M && j < g.N && i - j >= g.mdc;
                    o[b][r] = *(ok ? g.C.p + i * g.C.rs + j * g.C.cs : g.C.p);
                }
        }
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t i = i0 + 32 * wr + 16 * a + (lane >> 4) + 4 * r;
                const int64_t j = j0 + 32 * wc + 16 * b + (lane & 15);
                if (i < g.M && j < g.N && i - j >= g.mdc) {
                    double2 v = make_double2(g.alpha * cr[a][b][r], g.alpha * ci[a][b][r]);
                    if (g.beta != 0.0) {
                        const double2 c = zconj_if(o[b][r], g.C.conj);
                        v.x += g.beta * c.x;
                        v.y += g.beta * c.y;
                    }
                    *(g.C.p + i * g.C.rs + j * g.C.cs) = zconj_if(v, g.C.conj);
                }
            }
    }
}

__global__ __launch_bounds__(256) void zsplit_reduce_kernel(ZGemm g)
{
    if (g.gate && *g.gate) return;
    const int64_t i0 = (int64_t)blockIdx.x * ZT, j0 = (int64_t)blockIdx.y * ZT;
    if (i0 + ZT - 1 - j0 < g.mdc) return;
    const double2* pb = g.part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * g.nsplit * ZT * ZT;
    for (int e = threadIdx.x; e < ZT * ZT; e += 256) {
        const int64_t i = i0 + e % ZT, j = j0 + e / ZT;
        if (i >= g.M || j >= g.N || i - j < g.mdc) continue;
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < g.nsplit; z++) {
            const double2 v = pb[(int64_t)z * ZT * ZT + e];
            sr += v.x;
            si += v.y;
        }
        double2* cp = g.C.p + i * g.C.rs + j * g.C.cs;
        double2 v = make_double2(g.alpha * sr, g.alpha * si);
        if (g.beta != 0.0) {
            const double2 o = zconj_if(*cp, g.C.conj);
            v.x += g.beta * o.x;
            v.y += g.beta * o.y;
        }
        *cp = zconj_if(v, g.C.conj);
    }
}

// C(i, j) = alpha A(i, j) + beta C(i, j) for i - j >= mdc (beta = 0: C not read).
struct ZAxpby {
    int64_t M, N;
    ZView A, C;
    int64_t mdc;
    double alpha, beta;
    const int* gate;
};

__global__ __launch_bounds__(256) void zaxpby_kernel(ZAxpby g)
{
    if (g.gate && *g.gate) return;
    const int64_t i0 = (int64_t)blockIdx.x * ZT, j0 = (int64_t)blockIdx.y * ZT;
    const bool fast_i = g.C.rs == 1;
    for (int e = threadIdx.x; e < ZT * ZT; e += 256) {
        const int64_t i = i0 + (fast_i ? e % ZT : e / ZT), j = j0 + (fast_i ? e / ZT : e % ZT);
        if (i >= g.M || j >= g.N || i - j < g.mdc) continue;
        double2 v = zconj_if(g.A.p[i * g.A.rs + j * g.A.cs], g.A.conj);
        v.x *= g.alpha;
        v.y *= g.alpha;
        double2* cp = g.C.p + i * g.C.rs + j * g.C.cs;
        if (g.beta != 0.0) {
            const double2 o = zconj_if(*cp, g.C.conj);
            v.x += g.beta * o.x;
            v.y += g.beta * o.y;
        }
        *cp = zconj_if(v, g.C.conj);
    }
}

// Diagonal blocks of at most 64 rows, one workgroup each: block b is the
// diagonal block at (b * 64, b * 64) of the view (order min(64, m - 64 b)).
//   ZLEAF_FACTOR: Cholesky in place (lower triangle written back, real
//                 diagonal), then W = L^{-1} into w[b];
//   ZLEAF_INV:    W = L^{-1} of the factor already in the view, into w[b];
//   ZLEAF_INV_INPLACE: as ZLEAF_INV, and W also replaces the block's lower
//                 triangle.
// w[b] is a dense 64 x 64 column-major block (zero above the diagonal).
// INFO: FACTOR, first non-positive pivot p (1-based in the block) ->
// info_off + 64 b + p; INV modes, first zero diagonal entry likewise.
enum { ZLEAF_FACTOR = 0, ZLEAF_INV = 1, ZLEAF_INV_INPLACE = 2 };

// *info = v unless it already holds a smaller nonzero position (blocks may
// report in any order; INFO is the first failing position).
__device__ void info_first(int* info, int v)
{
    int old = __hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (old == 0 || v < old) {
        const int prev = atomicCAS(info, old, v);
        if (prev == old) break;
        old = prev;
    }
}

__global__ __launch_bounds__(256) void zleaf_kernel(ZView A, int64_t m, int mode, double2* w, int* info,
                                                    int64_t info_off, const int* gate)
{
    if (gate && *gate) return;
    constexpr int P = ZT + 1;
    __shared__ double Lr[ZT][P], Li[ZT][P], Wr[ZT][P], Wi[ZT][P];
    __shared__ int fail_sh, zero_sh;
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x, k0 = b * ZT;
    const int nb = (int)std::min<int64_t>(ZT, m - k0);
    if (nb <= 0) return;
    {
        // all 16 loads of a thread in flight together (an element outside the
        // lower triangle reads the block's first element and is dropped)
        constexpr int PER = ZT * ZT / 256;
        double2 v[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int e = t + 256 * u, i = e % ZT, j = e / ZT;
            const bool in = i >= j && i < nb;
            v[u] = *(in ? A.p + (k0 + i) * A.rs + (k0 + j) * A.cs : A.p + k0 * A.rs + k0 * A.cs);
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int e = t + 256 * u, i = e % ZT, j = e / ZT;
            double2 x = (i >= j && i < nb) ? zconj_if(v[u], A.conj) : make_double2(0.0, 0.0);
            if (i == j) x.y = 0.0;  // the diagonal of a Hermitian matrix and of its factor is real
            Lr[i][j] = x.x;
            Li[i][j] = x.y;
        }
    }
    if (t == 0) {
        fail_sh = 0;
        zero_sh = 1 << 30;  // first zero on the diagonal (INV modes)
    }
    __syncthreads();
    const int ti = t & (ZT - 1), tq = t >> 6;  // trailing update: row ti, columns tq, tq + 4, ...
    if (mode == ZLEAF_FACTOR) {
        // right-looking, one column per step, two barriers per step
        for (int j = 0; j < nb; j++) {
            const double d = Lr[j][j];  // final since the previous step's barrier
            if (!(d > 0.0)) {           // uniform: every thread reads the same LDS word
                if (t == 0) {
                    info_first(info, (int)(info_off + k0 + j + 1));
                    fail_sh = 1;
                }
                break;
            }
            const double l = sqrt(d), rl = 1.0 / l;
            if (t > j && t < nb) {
                Lr[t][j] *= rl;
                Li[t][j] *= rl;
            }
            __syncthreads();
            // L(j, j) is not read again in this step (every thread has d)
            if (t == 0) Lr[j][j] = l;
            // trailing lower triangle: L(i, c) -= L(i, j) conj(L(c, j)), j < c <= i
            const int i = j + 1 + ti;
            if (i < nb) {
                const double xr = Lr[i][j], xi = Li[i][j];
                for (int c = j + 1 + tq; c <= i; c += 4) {
                    const double yr = Lr[c][j], yi = Li[c][j];
                    Lr[i][c] -= xr * yr + xi * yi;
                    Li[i][c] -= xi * yr - xr * yi;
                }
            }
            __syncthreads();
        }
        if (fail_sh) return;
        // the factor back into the view (lower triangle of the block)
        for (int e = t; e < ZT * ZT; e += 256) {
            const int i = e % ZT, j = e / ZT;
            if (i >= j && i < nb)
                A.p[(k0 + i) * A.rs + (k0 + j) * A.cs] = zconj_if(make_double2(Lr[i][j], Li[i][j]), A.conj);
        }
    } else {
        if (info && t < nb && Lr[t][t] == 0.0) atomicMin(&zero_sh, t + 1);
        __syncthreads();
        if (zero_sh < (1 << 30)) {
            if (t == 0) info_first(info, (int)(info_off + k0 + zero_sh));
            return;
        }
    }
    // W = L^{-1} by forward substitution down each column,
    // W(i, c) = -(sum_{k = c}^{i-1} L(i, k) W(k, c)) / L(i, i): four lanes of
    // one wavefront per column (lane part p sums k = c + p, c + p + 4, ...),
    // so a column never waits on another wavefront
    {
        const int c = t >> 2, part = t & 3;
        for (int i = part; i < ZT; i += 4) {
            Wr[i][c] = 0.0;
            Wi[i][c] = 0.0;
        }
        wave_sync_z();
        for (int i = 0; i < nb; i++) {
            double sr = 0.0, si = 0.0;
            if (c < i && c < nb)
                for (int k = c + part; k < i; k += 4) {
                    sr += Lr[i][k] * Wr[k][c] - Li[i][k] * Wi[k][c];
                    si += Lr[i][k] * Wi[k][c] + Li[i][k] * Wr[k][c];
                }
            sr += __shfl_xor(sr, 1);
            si += __shfl_xor(si, 1);
            sr += __shfl_xor(sr, 2);
            si += __shfl_xor(si, 2);
            if (part == 0 && c <= i && c < nb) {
                const double rd = 1.0 / Lr[i][i];
                Wr[i][c] = i == c ? rd : -sr * rd;
                Wi[i][c] = i == c ? 0.0 : -si * rd;
            }
            wave_sync_z();  // row i of the column is visible to its four lanes
        }
    }
    __syncthreads();
    double2* wb = w + b * ZT * ZT;
    for (int e = t; e < ZT * ZT; e += 256) {
        const int i = e % ZT, j = e / ZT;
        wb[i + j * ZT] = make_double2(Wr[i][j], Wi[i][j]);
        if (mode == ZLEAF_INV_INPLACE && i >= j && i < nb)
            A.p[(k0 + i) * A.rs + (k0 + j) * A.cs] = zconj_if(make_double2(Wr[i][j], Wi[i][j]), A.conj);
    }
}

// ZTRTTF / ZTFTTR on one block of the RFP array: element (i, j) of the view
// (i >= j on a diagonal block) is canonical element (ro + i, co + j) of A.
__global__ void zconvert_kernel(ZView v, int64_t rows, int64_t cols, bool diag, int64_t ro, int64_t co, bool upper,
                                double2* a, int64_t lda, bool to_rfp)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t i = v.rs == 1 ? idx % rows : idx / cols, j = v.rs == 1 ? idx / rows : idx % cols;
    if (diag && i < j) return;
    const int64_t gi = ro + i, gj = co + j;
    double2* p = v.p + i * v.rs + j * v.cs;
    // canonical lower element L(gi, gj): UPLO='L' A(gi, gj); 'U' conj(A(gj, gi))
    double2* ap = upper ? a + gj + gi * lda : a + gi + gj * lda;
    if (to_rfp) {
        const double2 l = zconj_if(*ap, upper);
        *p = zconj_if(l, v.conj);
    } else {
        const double2 l = zconj_if(*p, v.conj);
        *ap = zconj_if(l, upper);
    }
}

inline unsigned tiles(int64_t x) { return (unsigned)((x + ZT - 1) / ZT); }

}  // namespace

// ---------------------------------------------------------------- launchers

ZView zview_sub(const ZView& v, int64_t i, int64_t j)
{
    return ZView{v.p + i * v.rs + j * v.cs, v.rs, v.cs, v.conj};
}

// Split-K scratch of the driver running on this thread (set by each
// z*_run entry from its work array; one handle serves one thread at a time).
constexpr int64_t ZPART_TILES = 1024;  // 64 x 64 partial blocks (64 MB)
constexpr int ZCUS = 256;
thread_local double2* z_part = nullptr;

hipError_t zgemm(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const ZView& A, int ta, int64_t mda,
                 const ZView& B, int tb, int64_t mdb, double beta, const ZView& C, int64_t mdc, const int* gate)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    ZGemm g{M, N, K, A, B, C, ta, tb, mda, mdb, mdc, alpha, beta, gate, 0, 1, nullptr};
    // few tiles and a long K: split K so that about two workgroups per CU run
    const int64_t nt = (int64_t)tiles(M) * tiles(N);
    if (z_part && nt < ZCUS && K >= 512) {
        int64_t sp = std::min<int64_t>((2 * ZCUS + nt - 1) / nt, K / 256);
        sp = std::min<int64_t>(sp, ZPART_TILES / nt);
        if (sp >= 2) {
            g.kchunk = ((K + sp - 1) / sp + ZK - 1) / ZK * ZK;
            g.nsplit = (int)((K + g.kchunk - 1) / g.kchunk);
            g.part = z_part;
            hipLaunchKernelGGL(zgemm_kernel, dim3(tiles(M), tiles(N), (unsigned)g.nsplit), dim3(256), 0, s, g);
            hipLaunchKernelGGL(zsplit_reduce_kernel, dim3(tiles(M), tiles(N)), dim3(256), 0, s, g);
            return hipGetLastError();
        }
    }
    if (K <= 0) {  // C = beta C
        if (beta == 1.0) return hipSuccess;
        ZAxpby c{M, N, C, C, mdc, beta, 0.0, gate};
        hipLaunchKernelGGL(zaxpby_kernel, dim3(tiles(M), tiles(N)), dim3(256), 0, s, c);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(zgemm_kernel, dim3(tiles(M), tiles(N)), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t zaxpby(hipStream_t s, int64_t M, int64_t N, double alpha, const ZView& A, double beta, const ZView& C,
                  int64_t mdc, const int* gate)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    ZAxpby c{M, N, A, C, mdc, alpha, beta, gate};
    hipLaunchKernelGGL(zaxpby_kernel, dim3(tiles(M), tiles(N)), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t zleaf(hipStream_t s, const ZView& A, int64_t m, int64_t first, int64_t count, int mode, double2* w,
                 int* info, int64_t info_off, const int* gate)
{
    if (count <= 0) return hipSuccess;
    // blocks first .. first + count - 1: shift the view so that block 0 is `first`
    const ZView a = zview_sub(A, first * ZT, first * ZT);
    hipLaunchKernelGGL(zleaf_kernel, dim3((unsigned)count), dim3(256), 0, s, a, m - first * ZT, mode, w, info,
                       info_off + first * ZT, gate);
    return hipGetLastError();
}

hipError_t zconvert(hipStream_t s, const ZRfpViews& v, bool upper, double2* a, int64_t lda, bool to_rfp)
{
    struct Blk {
        ZView v;
        int64_t rows, cols, ro, co;
        bool diag;
    } blks[3] = {{v.t1, v.m1, v.m1, 0, 0, true}, {v.s, v.m2, v.m1, v.m1, 0, false}, {v.t2, v.m2, v.m2, v.m1, v.m1, true}};
    for (const Blk& b : blks) {
        const int64_t cnt = b.rows * b.cols;
        if (cnt <= 0) continue;
        hipLaunchKernelGGL(zconvert_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, b.v, b.rows, b.cols,
                           b.diag, b.ro, b.co, upper, a, lda, to_rfp);
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------- drivers

#define ZCK(x)                                  \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// Block width of the products that are not tied to a leaf (trailing
// updates, triangular products by whole block columns or rows).
constexpr int64_t ZB = 256;

int64_t zleaves(int64_t m) { return (m + ZT - 1) / ZT; }

// Work array of the drivers: leaf inverses of both diagonal blocks, the
// split-K partial blocks, ZB x max(n, nrhs) temporaries, and for the
// inversion an m1 x m2 block (the out-of-place products).
size_t zwork_elems(int64_t n, int64_t nrhs, bool inverse)
{
    const int64_t m1 = (n + 1) / 2, m2 = n / 2;  // the block orders of every layout
    const int64_t leaves = 2 * zleaves(m1);
    return (size_t)(leaves * ZT * ZT) + (size_t)(ZPART_TILES * ZT * ZT) +
           (size_t)ZB * (size_t)std::max<int64_t>(std::max<int64_t>(n, nrhs), 1) +
           (inverse ? (size_t)m1 * (size_t)m2 : 0);
}

struct ZWork {
    double2 *w1, *w2, *tmp, *big;
};
static ZWork zwork_split(const ZRfpViews& v, double2* work)
{
    ZWork z;
    z.w1 = work;
    z.w2 = z.w1 + zleaves(v.m1) * ZT * ZT;
    z_part = z.w2 + zleaves(v.m2) * ZT * ZT;
    z.tmp = z_part + ZPART_TILES * ZT * ZT;
    z.big = z.tmp + ZB * std::max<int64_t>(v.m1 + v.m2, 1);
    return z;
}

// Cholesky of the m x m lower view A in place, right-looking in panels of ZB
// columns, each factored in 64-column steps: leaf (factor and W_kk = L_kk^{-1}
// into w[k]), P = A_{>k,k} W_kk^H (through tmp, up to m x 64), the panel's
// remaining columns -= P P^H; after the panel, the trailing matrix -= the
// panel times its conjugate transpose (K = ZB).
static hipError_t zpotrf_view(hipStream_t s, const ZView& A, int64_t m, double2* w, double2* tmp, int* info,
                              int64_t info_off)
{
    for (int64_t p0 = 0; p0 < m; p0 += ZB) {
        const int64_t pe = std::min<int64_t>(m, p0 + ZB);
        for (int64_t k0 = p0; k0 < pe; k0 += ZT) {
            const int64_t nb = std::min<int64_t>(ZT, pe - k0), r = m - k0 - nb, cols = pe - k0 - nb;
            const int64_t kb = k0 / ZT;
            ZCK(zleaf(s, A, m, kb, 1, ZLEAF_FACTOR, w + kb * ZT * ZT, info, info_off, info));
            if (r <= 0) break;
            const ZView P = zview_sub(A, k0 + nb, k0);
            const ZView W{w + kb * ZT * ZT, 1, ZT, 0};
            const ZView T{tmp, 1, r, 0};
            ZCK(zgemm(s, r, nb, nb, 1.0, P, 0, ZMASK_NONE, W, 1, ZMASK_NONE, 0.0, T, ZMASK_NONE, info));
            ZCK(zaxpby(s, r, nb, 1.0, T, 0.0, P, ZMASK_NONE, info));
            if (cols > 0)
                ZCK(zgemm(s, r, cols, nb, -1.0, P, 0, ZMASK_NONE, P, 1, ZMASK_NONE, 1.0,
                          zview_sub(A, k0 + nb, k0 + nb), 0, info));
        }
        if (pe < m)
            ZCK(zgemm(s, m - pe, m - pe, pe - p0, -1.0, zview_sub(A, pe, p0), 0, ZMASK_NONE, zview_sub(A, pe, p0), 1,
                      ZMASK_NONE, 1.0, zview_sub(A, pe, pe), 0, info));
    }
    return hipSuccess;
}

hipError_t zpftrf_run(hipStream_t s, const ZRfpViews& v, double2* work, int* info)
{
    const ZWork z = zwork_split(v, work);
    // step 1: POTRF on T1
    ZCK(zpotrf_view(s, v.t1, v.m1, z.w1, z.tmp, info, 0));
    if (v.m2 == 0) return hipSuccess;
    // step 2: TRSM, S <- S L11^{-H}: panels of ZB columns, 64-column steps
    // inside a panel (X_j = S_j W_jj^H, then the panel's later columns), then
    // the columns after the panel at once
    for (int64_t p0 = 0; p0 < v.m1; p0 += ZB) {
        const int64_t pe = std::min<int64_t>(v.m1, p0 + ZB);
        for (int64_t j0 = p0; j0 < pe; j0 += ZT) {
            const int64_t nb = std::min<int64_t>(ZT, pe - j0), cols = pe - j0 - nb;
            const ZView Sj = zview_sub(v.s, 0, j0);
            const ZView W{z.w1 + (j0 / ZT) * ZT * ZT, 1, ZT, 0};
            const ZView T{z.tmp, 1, v.m2, 0};
            ZCK(zgemm(s, v.m2, nb, nb, 1.0, Sj, 0, ZMASK_NONE, W, 1, ZMASK_NONE, 0.0, T, ZMASK_NONE, info));
            ZCK(zaxpby(s, v.m2, nb, 1.0, T, 0.0, Sj, ZMASK_NONE, info));
            if (cols > 0)
                ZCK(zgemm(s, v.m2, cols, nb, -1.0, Sj, 0, ZMASK_NONE, zview_sub(v.t1, j0 + nb, j0), 1, ZMASK_NONE, 1.0,
                          zview_sub(v.s, 0, j0 + nb), ZMASK_NONE, info));
        }
        if (pe < v.m1)
            ZCK(zgemm(s, v.m2, v.m1 - pe, pe - p0, -1.0, zview_sub(v.s, 0, p0), 0, ZMASK_NONE,
                      zview_sub(v.t1, pe, p0), 1, ZMASK_NONE, 1.0, zview_sub(v.s, 0, pe), ZMASK_NONE, info));
    }
    // step 3: HERK, T2 <- T2 - S S^H (lower triangle)
    ZCK(zgemm(s, v.m2, v.m2, v.m1, -1.0, v.s, 0, ZMASK_NONE, v.s, 1, ZMASK_NONE, 1.0, v.t2, 0, info));
    // step 4: POTRF on T2, INFO counted from the start of A
    return zpotrf_view(s, v.t2, v.m2, z.w2, z.tmp, info, v.m1);
}

hipError_t zpftrs_run(hipStream_t s, const ZRfpViews& v, double2* b, int64_t ldb, int64_t nrhs, double2* work,
                      int* info)
{
    (void)info;  // a zero on the factor's diagonal yields infinities, as in LAPACK
    const ZWork z = zwork_split(v, work);
    const int64_t l1 = zleaves(v.m1), l2 = zleaves(v.m2);
    ZCK(zleaf(s, v.t1, v.m1, 0, l1, ZLEAF_INV, z.w1, nullptr, 0, nullptr));
    ZCK(zleaf(s, v.t2, v.m2, 0, l2, ZLEAF_INV, z.w2, nullptr, v.m1, nullptr));
    const ZView B{b, 1, ldb, 0};
    const ZView T{z.tmp, 1, ZT, 0};
    struct Part {
        ZView L;
        int64_t m, row0;
        double2* w;
    } parts[2] = {{v.t1, v.m1, 0, z.w1}, {v.t2, v.m2, v.m1, z.w2}};
    // forward, L Y = B: T1's rows, then B2 -= S Y1, then T2's rows; inside a
    // part, ZB-row panels of 64-row steps (the panel's later rows updated per
    // step, the rows after the panel once per panel)
    for (int p = 0; p < 2; p++) {
        const Part& q = parts[p];
        if (p == 1 && v.m2 > 0)
            ZCK(zgemm(s, v.m2, nrhs, v.m1, -1.0, v.s, 0, ZMASK_NONE, B, 0, ZMASK_NONE, 1.0, zview_sub(B, v.m1, 0),
                      ZMASK_NONE, nullptr));
        for (int64_t p0 = 0; p0 < q.m; p0 += ZB) {
            const int64_t pe = std::min<int64_t>(q.m, p0 + ZB);
            for (int64_t k0 = p0; k0 < pe; k0 += ZT) {
                const int64_t nb = std::min<int64_t>(ZT, pe - k0), rest = pe - k0 - nb;
                const ZView Bk = zview_sub(B, q.row0 + k0, 0);
                const ZView W{q.w + (k0 / ZT) * ZT * ZT, 1, ZT, 0};
                ZCK(zgemm(s, nb, nrhs, nb, 1.0, W, 0, ZMASK_NONE, Bk, 0, ZMASK_NONE, 0.0, T, ZMASK_NONE, nullptr));
                ZCK(zaxpby(s, nb, nrhs, 1.0, T, 0.0, Bk, ZMASK_NONE, nullptr));
                if (rest > 0)
                    ZCK(zgemm(s, rest, nrhs, nb, -1.0, zview_sub(q.L, k0 + nb, k0), 0, ZMASK_NONE, Bk, 0, ZMASK_NONE,
                              1.0, zview_sub(B, q.row0 + k0 + nb, 0), ZMASK_NONE, nullptr));
            }
            if (pe < q.m)
                ZCK(zgemm(s, q.m - pe, nrhs, pe - p0, -1.0, zview_sub(q.L, pe, p0), 0, ZMASK_NONE,
                          zview_sub(B, q.row0 + p0, 0), 0, ZMASK_NONE, 1.0, zview_sub(B, q.row0 + pe, 0), ZMASK_NONE,
                          nullptr));
        }
    }
    // backward, L^H X = Y: T2's rows from the last, then B1 -= S^H X2, then
    // T1's; ZB-row panels from the last, 64-row steps from the panel's last
    for (int p = 1; p >= 0; p--) {
        const Part& q = parts[p];
        if (p == 0 && v.m2 > 0)
            ZCK(zgemm(s, v.m1, nrhs, v.m2, -1.0, v.s, 1, ZMASK_NONE, zview_sub(B, v.m1, 0), 0, ZMASK_NONE, 1.0, B,
                      ZMASK_NONE, nullptr));
        for (int64_t p0 = (q.m - 1) / ZB * ZB; q.m > 0 && p0 >= 0; p0 -= ZB) {
            const int64_t pe = std::min<int64_t>(q.m, p0 + ZB);
            for (int64_t k0 = (pe - 1) / ZT * ZT; k0 >= p0; k0 -= ZT) {
                const int64_t nb = std::min<int64_t>(ZT, pe - k0);
                const ZView Bk = zview_sub(B, q.row0 + k0, 0);
                const ZView W{q.w + (k0 / ZT) * ZT * ZT, 1, ZT, 0};
                ZCK(zgemm(s, nb, nrhs, nb, 1.0, W, 1, ZMASK_NONE, Bk, 0, ZMASK_NONE, 0.0, T, ZMASK_NONE, nullptr));
                ZCK(zaxpby(s, nb, nrhs, 1.0, T, 0.0, Bk, ZMASK_NONE, nullptr));
                if (k0 > p0)  // the panel's rows above: B(p0:k0) -= L(k, p0:k0)^H X_k
                    ZCK(zgemm(s, k0 - p0, nrhs, nb, -1.0, zview_sub(q.L, k0, p0), 1, ZMASK_NONE, Bk, 0, ZMASK_NONE,
                              1.0, zview_sub(B, q.row0 + p0, 0), ZMASK_NONE, nullptr));
            }
            if (p0 > 0)  // rows before the panel: B(0:p0) -= L(p0:pe, 0:p0)^H X_panel
                ZCK(zgemm(s, p0, nrhs, pe - p0, -1.0, zview_sub(q.L, p0, 0), 1, ZMASK_NONE,
                          zview_sub(B, q.row0 + p0, 0), 0, ZMASK_NONE, 1.0, zview_sub(B, q.row0, 0), ZMASK_NONE,
                          nullptr));
        }
    }
    return hipSuccess;
}

// W = L^{-1} in place on the m x m lower view whose 64-row diagonal blocks
// already hold their inverses: the 2 x 2 partition at splits that are
// multiples of 64 from the view's start, both diagonal inverses first, then
// W21 = -W22 (L21 W11) through the scratch X (at least n2 x n1 elements).
static hipError_t ztrtri_rec(hipStream_t s, const ZView& A, int64_t m, double2* X, int* info)
{
    if (m <= ZT) return hipSuccess;
    const int64_t n1 = rec_split(m, ZT), n2 = m - n1;
    ZCK(ztrtri_rec(s, A, n1, X, info));
    ZCK(ztrtri_rec(s, zview_sub(A, n1, n1), n2, X, info));
    const ZView Xv{X, 1, n2, false};
    ZCK(zgemm(s, n2, n1, n1, 1.0, zview_sub(A, n1, 0), 0, ZMASK_NONE, A, 0, 0, 0.0, Xv, ZMASK_NONE, info));
    ZCK(zgemm(s, n2, n1, n2, -1.0, zview_sub(A, n1, n1), 0, 0, Xv, 0, ZMASK_NONE, 0.0, zview_sub(A, n1, 0),
              ZMASK_NONE, info));
    return hipSuccess;
}

// W^H W in place on the m x m lower view holding W: the 2 x 2 partition,
// C11 = LAUUM(W11) + W21^H W21, C21 = W22^H W21 (through the scratch X,
// copied back), C22 = LAUUM(W22); blocks of at most ZB rows by row blocks
// (C(I, 0:i0+nb) = W(i0:m, I)^H W(i0:m, 0:i0+nb) into tmp, then copied).
static hipError_t zlauum_rec(hipStream_t s, const ZView& A, int64_t m, double2* tmp, double2* X, const int* gate)
{
    if (m <= 0) return hipSuccess;
    if (m <= ZB) {
        for (int64_t i0 = 0; i0 < m; i0 += ZT) {
            const int64_t nb = std::min<int64_t>(ZT, m - i0);
            const ZView T{tmp, 1, ZT, 0};
            ZCK(zgemm(s, nb, i0 + nb, m - i0, 1.0, zview_sub(A, i0, i0), 1, 0, zview_sub(A, i0, 0), 0, -i0, 0.0, T,
                      ZMASK_NONE, gate));
            ZCK(zaxpby(s, nb, i0 + nb, 1.0, T, 0.0, zview_sub(A, i0, 0), -i0, gate));
        }
        return hipSuccess;
    }
    const int64_t n1 = rec_split(m, ZT), n2 = m - n1;
    const ZView A21 = zview_sub(A, n1, 0), A22 = zview_sub(A, n1, n1);
    ZCK(zlauum_rec(s, A, n1, tmp, X, gate));
    ZCK(zgemm(s, n1, n1, n2, 1.0, A21, 1, ZMASK_NONE, A21, 0, ZMASK_NONE, 1.0, A, 0, gate));
    const ZView Xv{X, 1, n2, false};
    ZCK(zgemm(s, n2, n1, n2, 1.0, A22, 1, 0, A21, 0, ZMASK_NONE, 0.0, Xv, ZMASK_NONE, gate));
    ZCK(zaxpby(s, n2, n1, 1.0, Xv, 0.0, A21, ZMASK_NONE, gate));
    return zlauum_rec(s, A22, n2, tmp, X, gate);
}

hipError_t zpftri_run(hipStream_t s, const ZRfpViews& v, double2* work, int* info)
{
    const ZWork z = zwork_split(v, work);
    // stage A: W = L^{-1} on the three blocks.  Every 64-row diagonal block
    // of both triangles is inverted in place at once, then the recursion
    // fills the off-diagonal blocks; S <- -W22 S W11 through the scratch.
    ZCK(zleaf(s, v.t1, v.m1, 0, zleaves(v.m1), ZLEAF_INV_INPLACE, z.w1, info, 0, info));
    ZCK(zleaf(s, v.t2, v.m2, 0, zleaves(v.m2), ZLEAF_INV_INPLACE, z.w2, info, v.m1, info));
    ZCK(ztrtri_rec(s, v.t1, v.m1, z.big, info));
    ZCK(ztrtri_rec(s, v.t2, v.m2, z.big, info));
    if (v.m2 > 0) {
        const ZView Xv{z.big, 1, v.m2, false};
        ZCK(zgemm(s, v.m2, v.m1, v.m1, 1.0, v.s, 0, ZMASK_NONE, v.t1, 0, 0, 0.0, Xv, ZMASK_NONE, info));
        ZCK(zgemm(s, v.m2, v.m1, v.m2, -1.0, v.t2, 0, 0, Xv, 0, ZMASK_NONE, 0.0, v.s, ZMASK_NONE, info));
    }
    // stage B: A^{-1} = W^H W: T1 <- LAUUM(W11) + W21^H W21, S <- W22^H W21
    // (through the scratch, copied back), T2 <- LAUUM(W22)
    ZCK(zlauum_rec(s, v.t1, v.m1, z.tmp, z.big, info));
    if (v.m2 > 0) {
        ZCK(zgemm(s, v.m1, v.m1, v.m2, 1.0, v.s, 1, ZMASK_NONE, v.s, 0, ZMASK_NONE, 1.0, v.t1, 0, info));
        const ZView Xv{z.big, 1, v.m2, false};
        ZCK(zgemm(s, v.m2, v.m1, v.m2, 1.0, v.t2, 1, 0, v.s, 0, ZMASK_NONE, 0.0, Xv, ZMASK_NONE, info));
        ZCK(zaxpby(s, v.m2, v.m1, 1.0, Xv, 0.0, v.s, ZMASK_NONE, info));
        ZCK(zlauum_rec(s, v.t2, v.m2, z.tmp, z.big, info));
    }
    return hipSuccess;
}

bool zrfp_views(char transr, char uplo, int64_t n, double2* arf, ZRfpViews* v)
{
    const int t = (transr >= 'a' && transr <= 'z') ? transr - 'a' + 'A' : transr;
    const int u = (uplo >= 'a' && uplo <= 'z') ? uplo - 'a' + 'A' : uplo;
    if ((t != 'N' && t != 'C') || (u != 'L' && u != 'U')) return false;
    RfpBlocks b;
    if (!rfp_blocks(t == 'N' ? 'N' : 'T', (char)u, n, &b)) return false;
    // the blocks the real format keeps transposed hold conjugates: for 'L'
    // L22, for 'U' L21 and L22 (the canonical lower view reads the stored
    // upper triangle); TRANSR = 'C' conjugates the whole rectangle
    const bool c = t == 'C';
    const bool x11 = false, x21 = u == 'U', x22 = true;
    v->n = n;
    v->m1 = b.m1;
    v->m2 = b.m2;
    v->t1 = ZView{arf + b.off11, b.rs11, b.cs11, x11 != c};
    v->s = ZView{arf + b.off21, b.rs21, b.cs21, x21 != c};
    v->t2 = ZView{arf + b.off22, b.rs22, b.cs22, x22 != c};
    return true;
}

}  // namespace rfp
