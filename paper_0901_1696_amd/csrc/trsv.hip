// Fused blocked triangular solves for PFTRS (Section 4): L Y = B and
// L^T X = Y over the whole lower factor held in RFP, one launch each.
//
// The factor is cut into 64-row block rows: those of T1 (L11) first, then
// those of T2 (L22).  A block (k, j) below the diagonal lies in T1, in S (L21)
// or in T2, and never straddles two of them.  One workgroup owns block row k
// and one slice of right-hand-side columns.  Forward, it accumulates
// B_k - sum_{j<k} L_kj Y_j on MFMA, taking each Y_j as soon as block row j
// has published it (one ready flag per block row and slice), then forms
// Y_k = W_k (B_k - ...) with W_k the inverse of the diagonal block, stores Y_k
// over B_k and raises its flag.  Backward runs the block rows from the bottom
// with the blocks of L^T and W_k^T.
//
// Workgroups are numbered in dependency order and only ever wait for lower
// numbers.  Dispatch is in order on every XCD, so the lowest unfinished
// workgroup is always resident with all its inputs published: every wait
// ends.  The waits are bounded spins all the same; a workgroup whose wait
// runs out writes NaN into its block of the solution, sets bit 0 of the
// handle's device status word (the caller reads it with rfp_solve_status),
// and still raises its flag, so that no other workgroup is held.
//
// Flags hold an epoch number, so the flag array is never cleared between
// calls.  The epoch lives in device memory: a one-thread kernel advances it
// before every launch and the launch reads it, so a solve captured in a HIP
// graph takes a fresh epoch on every replay.  Solved rows travel between
// workgroups (and XCDs) through device-scope atomic stores and loads ordered
// by the flags' release / acquire, never through plain cached accesses.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "rfp_common.h"

namespace rfp {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct MT;
template <>
struct MT<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc op(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct MT<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc op(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// One zero of each type in device memory: a masked-off element is loaded
// from here instead of being skipped, so that every load of a block is
// issued unconditionally (no branch around it) and the compiler can count
// the loads still in flight (a wait for one ring slot then leaves the later
// slots' loads outstanding).  Never written.
__device__ double g_zero_d = 0.0;
__device__ float g_zero_f = 0.0f;
template <typename T>
__device__ __forceinline__ const T* zero_ptr()
{
    if constexpr (sizeof(T) == 8) return (const T*)&g_zero_d;
    else return (const T*)&g_zero_f;
}

constexpr int BS = NB;     // rows per block row
constexpr int P = BS + 4;  // LDS row pitch

}  // namespace

template <typename T>
struct SolveArgs {
    Mat<const T> t1, s, t2;  // L11, L21, L22
    int64_t m1, m2;
    int nb1, nb2;            // block rows in T1 and T2
    const T* w;              // diagonal-block inverses, nb1 + nb2 blocks of BS x BS row-major
    T* b;                    // right-hand sides, column-major
    int64_t ldb, nrhs;
    int nslices;             // slices of 16 * NCB columns
    int* flags;              // [block row][slice]
    const int* epoch;        // device: this launch's epoch
    const int* gate;         // device, or null: the launch does nothing while *gate != 0
    int* status;             // device, or null: bit 0 set when a wait gives up
    int spin_limit;          // polls of an unpublished dependency before giving up
};

namespace {

template <typename T>
__device__ __forceinline__ void block_rows(const SolveArgs<T>& a, int k, int64_t* r0, int* cnt)
{
    const int64_t o = k < a.nb1 ? (int64_t)k * BS : (int64_t)(k - a.nb1) * BS;
    const int64_t len = k < a.nb1 ? a.m1 : a.m2;
    *r0 = k < a.nb1 ? o : a.m1 + o;
    *cnt = (int)(len - o < BS ? len - o : BS);
}

// Element (i, kk) of the block that block row k applies for dependency j:
// L(r0 + i, rj + kk) forward, L(rj + kk, r0 + i) backward.  Returns its
// address and the strides along i and kk.
template <typename T, bool FWD>
__device__ __forceinline__ const T* dep_block(const SolveArgs<T>& a, int k, int64_t r0, int j, int64_t rj,
                                              int64_t* si, int64_t* sk)
{
    const int rowb = FWD ? k : j, colb = FWD ? j : k;      // block (row, col) of L
    const int64_t gr = FWD ? r0 : rj, gc = FWD ? rj : r0;  // its first element in L
    Mat<const T> M;
    int64_t rr, cc;
    if (rowb < a.nb1) {
        M = a.t1; rr = gr; cc = gc;
    } else if (colb < a.nb1) {
        M = a.s; rr = gr - a.m1; cc = gc;
    } else {
        M = a.t2; rr = gr - a.m1; cc = gc - a.m1;
    }
    *si = FWD ? M.rs : M.cs;
    *sk = FWD ? M.cs : M.rs;
    return M.p + rr * M.rs + cc * M.cs;
}

}  // namespace

// Workgroup b -> (position q in dependency order, slice s).  The slices of
// one block row share an XCD (consecutive workgroups go to consecutive XCDs),
// so its factor block is fetched from HBM once per XCD; for a fixed slice the
// numbering still rises with q, which keeps every wait on an earlier
// workgroup.  The grid is padded to whole groups of XCD_COUNT block rows.
constexpr int XCD_COUNT = 8;

// R consecutive block rows per workgroup (R = 1 or 2): the workgroup
// accumulates the products of every earlier block row for all R of them,
// then solves them one after the other inside the workgroup (the second
// also subtracts the product with the first through LDS), publishing each as
// soon as it is solved.  With R = 2 half as many results cross between
// workgroups on the dependency chain, whose per-step latency (flag, device-
// scope loads and stores) is what bounds the solve for few right-hand sides.
template <typename T, int NCB, bool FWD, int R>
__global__ __launch_bounds__(256) void block_solve_kernel(SolveArgs<T> a)
{
    constexpr int CS = 16 * NCB;
    constexpr int LPT = BS * BS / 256;  // factor-block elements per thread
    constexpr int YPT = CS * BS / 256;  // solution-block elements per thread
    __shared__ __attribute__((aligned(16))) T Ls[BS][P];  // L block (or W, R = 1), Ls[i][kk]
    __shared__ __attribute__((aligned(16))) T Ys[CS][P];  // rows of a dependency or own rows, Ys[column][row]
    // R = 2: both diagonal inverses and the coupling block, staged once
    constexpr int RB = R == 2 ? BS : 1;
    __shared__ __attribute__((aligned(16))) T Wd[R][RB][R == 2 ? P : 1];
    __shared__ __attribute__((aligned(16))) T Cd[RB][R == 2 ? P : 1];

    if (a.gate && *a.gate) return;
    const int epoch = *a.epoch;
    const int nblk = a.nb1 + a.nb2;
    const int nsup = (nblk + R - 1) / R;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int grp = blockIdx.x / (XCD_COUNT * a.nslices), rem = blockIdx.x % (XCD_COUNT * a.nslices);
    const int slice = rem / XCD_COUNT;
    const int sq = grp * XCD_COUNT + rem % XCD_COUNT;
    if (sq >= nsup) return;  // padding of the last group: nobody waits for it
    const int q = sq * R;    // position of the first own block row in dependency order
    const int64_t c0 = (int64_t)slice * CS;
    // own block rows: position q + x in dependency order (present when < nblk)
    int kx[R], cntx[R];
    int64_t r0x[R];
#pragma unroll
    for (int x = 0; x < R; x++) {
        const int qx = q + x < nblk ? q + x : q;
        kx[x] = FWD ? qx : nblk - 1 - qx;
        block_rows(a, kx[x], &r0x[x], &cntx[x]);
    }
    const bool has2 = R == 2 && q + 1 < nblk;

    // the diagonal block's inverse, needed last (R = 1: fetched into
    // registers now; R = 2: both inverses and the block coupling the two rows
    // staged in LDS before the dependency loop)
    T wreg[R == 1 ? LPT : 1];
    auto fetch_w = [&](int x, T (&dst)[LPT]) {
        const T* wk = a.w + (int64_t)kx[x] * BS * BS;
        const int cnt = cntx[x];
#pragma unroll
        for (int e = 0; e < LPT; e++) {
            const int idx = t + 256 * e, i = idx / BS, kk = idx % BS;
            dst[e] = *((i < cnt && kk < cnt) ? wk + (FWD ? i * BS + kk : kk * BS + i) : zero_ptr<T>());
        }
    };
    if constexpr (R == 1) {
        fetch_w(0, wreg);
    } else {
        T tmp[LPT];
#pragma unroll
        for (int x = 0; x < R; x++) {
            fetch_w(x, tmp);
#pragma unroll
            for (int e = 0; e < LPT; e++) {
                const int idx = t + 256 * e;
                Wd[x][idx / BS][idx % BS] = tmp[e];
            }
        }
        if (has2) {
            int64_t si, sk;
            const T* lp = dep_block<T, FWD>(a, kx[1], r0x[1], kx[0], r0x[0], &si, &sk);
#pragma unroll
            for (int e = 0; e < LPT; e++) {
                const int idx = t + 256 * e, i = idx / BS, kk = idx % BS;  // L(i, kk) of the coupling block
                Cd[i][kk] = (i < cntx[1] && kk < cntx[0]) ? lp[i * si + kk * sk] : T(0);
            }
        }
        __syncthreads();
    }

    typedef typename MT<T>::acc acc_t;
    acc_t acc[R][NCB];
    // B_k in the MFMA result layout: wave w holds rows 16w .. 16w + 15
#pragma unroll
    for (int x = 0; x < R; x++)
#pragma unroll
        for (int cb = 0; cb < NCB; cb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = 16 * w + MT<T>::row(lane, e);
                const int64_t c = c0 + cb * 16 + r;
                const bool in = x == 0 || has2;
                acc[x][cb][e] = (in && i < cntx[x] && c < a.nrhs) ? a.b[(r0x[x] + i) + c * a.ldb] : T(0);
            }

    // Factor blocks stream through a ring of PD register buffers, PD - 1
    // blocks ahead of the products: a workgroup behind the front of published
    // rows is otherwise bound by one memory latency per block.  Step s applies
    // dependency s / R to own row s % R.  The thread's element e of a block is
    // (i, kk) = (idx % BS, idx / BS) when i runs along the unit stride, else
    // (idx / BS, idx % BS), idx = t + 256 e.
    constexpr int PD = NCB == 1 ? 4 : 2;
    static_assert(PD % R == 0, "ring slots map to fixed own rows");
    const int nsteps = q * R;
    T lreg[PD][LPT];
    bool ifast[PD];
    auto fetch_s = [&](int st, T (&dst)[LPT], bool& i_fast) {
        const int d = st / R, x = st % R;
        const int j = FWD ? d : nblk - 1 - d;
        int64_t rj, si, sk;
        int cntj;
        block_rows(a, j, &rj, &cntj);
        const T* lp = dep_block<T, FWD>(a, kx[x], r0x[x], j, rj, &si, &sk);
        i_fast = si == 1;
        const int cnt = (x == 0 || has2) ? cntx[x] : 0;
#pragma unroll
        for (int e = 0; e < LPT; e++) {
            const int idx = t + 256 * e;
            const int i = i_fast ? idx % BS : idx / BS, kk = i_fast ? idx / BS : idx % BS;
            dst[e] = *((i < cnt && kk < cntj) ? lp + i * si + kk * sk : zero_ptr<T>());
        }
    };
#pragma unroll
    for (int p = 0; p < PD - 1; p++)
        if (p < nsteps) fetch_s(p, lreg[p], ifast[p]);

    // Readiness is learnt in batches: wave 0 reads the flags of up to 64
    // upcoming dependencies at once and one acquire covers every dependency
    // found published, so a workgroup far behind the front pays one fence
    // per batch rather than one per block.
    bool ok = true;
    int ready = 0;  // dependencies 0 .. ready-1 are known to be published
    __shared__ int ready_sh;
    auto wait_ready = [&](int d) {  // workgroup-uniform; false when a wait gave up
        if (w == 0) {
            const int dd = d + lane;
            const int jj = FWD ? dd : nblk - 1 - dd;
            const int* f = a.flags + (int64_t)jj * a.nslices + slice;
            int spins = 0, avail = 0;
            for (;;) {
                const bool rdy =
                    dd < q && __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
                const uint64_t m = __ballot(rdy);
                avail = ~m ? __builtin_ctzll(~m) : 64;  // published run starting at d
                if (avail > 0 || spins >= a.spin_limit) break;
                spins++;
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane == 0) ready_sh = avail > 0 ? d + avail : -1;
        }
        __syncthreads();
        ready = ready_sh;
        return ready >= 0;
    };
    // Rows solved by other workgroups are read with device-scope loads:
    // when block rows share cache lines (an unaligned m1 or ldb), this
    // workgroup's own first read of B_k may have cached a neighbour's
    // unsolved rows, and a plain load could be served that stale copy.
    // The rows of dependencies already known to be published go through a
    // ring of YD register buffers, up to YD - 1 dependencies ahead.
    constexpr int YD = PD / R;
    T yreg[YD][YPT];
    int yfetched = 0;  // dependencies whose rows have been loaded into the ring
    auto fetch_y = [&](int d, T (&dst)[YPT]) {
        const int j = FWD ? d : nblk - 1 - d;
        int64_t rj;
        int cntj;
        block_rows(a, j, &rj, &cntj);
#pragma unroll
        for (int e = 0; e < YPT; e++) {
            const int idx = t + 256 * e, kk = idx % BS, c = idx / BS;
            const T* src = (kk < cntj && c0 + c < a.nrhs) ? &a.b[(rj + kk) + (c0 + c) * a.ldb] : zero_ptr<T>();
            dst[e] = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    // ac -= M Ys (M: Ls, or the coupling block)
    auto product = [&](acc_t (&ac)[NCB], T (&M)[BS][P]) {
#pragma unroll 4
        for (int kk = 0; kk < BS; kk += 4) {
            const T av = -M[16 * w + r][kk + g];
#pragma unroll
            for (int cb = 0; cb < NCB; cb++) ac[cb] = MT<T>::op(av, Ys[cb * 16 + r][kk + g], ac[cb]);
        }
    };
    for (int s0 = 0; s0 < nsteps && ok; s0 += PD) {
#pragma unroll
        for (int p = 0; p < PD; p++) {
            const int st = s0 + p, x = p % R, d = st / R, ys = (p / R) % YD;  // d % YD == ys
            if (st < nsteps && ok) {
#pragma unroll
                for (int e = 0; e < LPT; e++) {
                    const int idx = t + 256 * e;
                    const int i = ifast[p] ? idx % BS : idx / BS, kk = ifast[p] ? idx / BS : idx % BS;
                    Ls[i][kk] = lreg[p][e];
                }
                if (x == 0) {
                    if (yfetched <= d) {
                        if (d >= ready && !wait_ready(d)) ok = false;
                        if (ok) fetch_y(d, yreg[ys]);
                        yfetched = d + 1;
                    }
#pragma unroll
                    for (int e = 0; e < YPT; e++) {
                        const int idx = t + 256 * e;
                        Ys[idx / BS][idx % BS] = yreg[ys][e];
                    }
                }
                if (ok) {
                    __syncthreads();
                    const int sn = st + PD - 1;  // the ring slot just freed
                    if (sn < nsteps) fetch_s(sn, lreg[(p + PD - 1) % PD], ifast[(p + PD - 1) % PD]);
                    if (x == R - 1) {
#pragma unroll
                        for (int u = 1; u < YD; u++) {
                            const int dd = d + u;
                            if (dd >= yfetched && dd < q && dd < ready) {
                                fetch_y(dd, yreg[(ys + u) % YD]);
                                yfetched = dd + 1;
                            }
                        }
                    }
                    product(acc[x], Ls);
                    __syncthreads();
                }
            }
        }
    }

    // Own row x: X_k = W_k acc (forward) or W_k^T acc (backward), stored and
    // published; for a pair, the second row first subtracts the coupling
    // block times the first row's solution (through LDS).
    const T nan = T(__builtin_nan(""));
    auto solve_own = [&](int x) {
        if constexpr (R == 1) {
#pragma unroll
            for (int e = 0; e < LPT; e++) {
                const int idx = t + 256 * e;
                Ls[idx / BS][idx % BS] = wreg[e];
            }
        }
        T(&Wm)[BS][P] = R == 1 ? Ls : reinterpret_cast<T(&)[BS][P]>(Wd[x]);
#pragma unroll
        for (int cb = 0; cb < NCB; cb++)
#pragma unroll
            for (int e = 0; e < 4; e++) Ys[cb * 16 + r][16 * w + MT<T>::row(lane, e)] = acc[x][cb][e];
        __syncthreads();
        acc_t out[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; cb++) out[cb] = acc_t{0, 0, 0, 0};
#pragma unroll 4
        for (int kk = 0; kk < BS; kk += 4) {
            const T av = Wm[16 * w + r][kk + g];
#pragma unroll
            for (int cb = 0; cb < NCB; cb++) out[cb] = MT<T>::op(av, Ys[cb * 16 + r][kk + g], out[cb]);
        }
        __syncthreads();  // every wave is done with Ys
#pragma unroll
        for (int cb = 0; cb < NCB; cb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = 16 * w + MT<T>::row(lane, e);
                const int64_t c = c0 + cb * 16 + r;
                const T v = ok ? out[cb][e] : nan;
                Ys[cb * 16 + r][i] = v;  // the solved rows, for the second row of a pair
                if (i < cntx[x] && c < a.nrhs)
                    __hip_atomic_store(&a.b[(r0x[x] + i) + c * a.ldb], v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        if (!ok && t == 0 && a.status) atomicOr(a.status, 1);
        // publish: every wavefront waits for its device-scope stores to
        // complete, then one thread raises the flag with a release store
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (t == 0)
            __hip_atomic_store(a.flags + (int64_t)kx[x] * a.nslices + slice, epoch, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    };
    solve_own(0);
    if constexpr (R == 2) {
        if (has2) {
            // acc_1 -= L(k1, k0) X_k0, with X_k0 in Ys
            __syncthreads();
            product(acc[1], reinterpret_cast<T(&)[BS][P]>(Cd));
            __syncthreads();
            solve_own(1);
        }
    }
}

// Epoch of the next fused solve on a flag array: epoch + 1, wrapping to 1
// once it reaches EPOCH_WRAP (the flags are then cleared first, by the grid
// of the clear kernel, which reads the epoch but does not write it).
constexpr int EPOCH_WRAP = 1 << 30;
__global__ void epoch_clear_kernel(int* flags, int64_t n, const int* epoch)
{
    if (*epoch + 1 < EPOCH_WRAP) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) flags[i] = 0;
}
__global__ void epoch_bump_kernel(int* epoch)
{
    if (threadIdx.x == 0) *epoch = *epoch + 1 < EPOCH_WRAP ? *epoch + 1 : 1;
}

hipError_t epoch_bump(hipStream_t s, int* flags, int64_t nflags, int* epoch)
{
    if (nflags > 0)
        hipLaunchKernelGGL(epoch_clear_kernel, dim3((unsigned)std::min<int64_t>((nflags + 255) / 256, 64)), dim3(256),
                           0, s, flags, nflags, (const int*)epoch);
    hipLaunchKernelGGL(epoch_bump_kernel, dim3(1), dim3(64), 0, s, epoch);
    return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int64_t n, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int64_t block_solve_flags(int64_t m1, int64_t m2, int64_t nrhs)
{
    const int64_t nblk = (m1 + BS - 1) / BS + (m2 + BS - 1) / BS;
    return nblk * ((nrhs + 15) / 16);  // slices are at least 16 columns wide
}

hipError_t fill_int(hipStream_t s, int* p, int64_t n, int v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Block rows per workgroup for 16-column slices: 2, or 1 with RFP_SOLVE_PAIR=0.
static int solve_rows_per_group()
{
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("RFP_SOLVE_PAIR");
        v = (e && e[0] == '0') ? 1 : 2;
    }
    return v;
}

template <typename T, int NCB, int R>
static hipError_t launch_solve_r(const Exec& ex, bool forward, const SolveArgs<T>& a, int nblk)
{
    static char names[2][2][112];
    const int ti = sizeof(T) == 8 ? 0 : 1, di = forward ? 0 : 1;
    char* nm = names[ti][di];
    if (!nm[0]) {
        const char* tn = ti ? "float" : "double";
        snprintf(nm, sizeof names[ti][di], "rfp::block_solve_kernel<%s, %d, %s, %d>(rfp::SolveArgs<%s>)", tn, NCB,
                 forward ? "true" : "false", R, tn);
    }
    const double mtot = (double)(a.m1 + a.m2);
    ProfScope ps(ex, nm, mtot * mtot * (double)a.nrhs,
                 sizeof(T) * (mtot * mtot / 2 * a.nslices + 2.0 * mtot * (double)a.nrhs));
    const int nsup = (nblk + R - 1) / R;
    const int groups = (nsup + XCD_COUNT - 1) / XCD_COUNT;
    const dim3 grid((unsigned)(groups * XCD_COUNT * a.nslices));
    if (forward) hipLaunchKernelGGL((block_solve_kernel<T, NCB, true, R>), grid, dim3(256), 0, ex.stream, a);
    else hipLaunchKernelGGL((block_solve_kernel<T, NCB, false, R>), grid, dim3(256), 0, ex.stream, a);
    return hipGetLastError();
}

template <typename T, int NCB>
static hipError_t launch_solve(const Exec& ex, bool forward, const SolveArgs<T>& a, int nblk)
{
    // pairs (and the deeper ring) for 16-column slices, where a workgroup
    // streams the most factor blocks per right-hand side; wider slices keep
    // one block row per workgroup and a ring of two (more resident
    // workgroups measured faster there: n = 20000, 128 right-hand sides)
    if constexpr (NCB == 1)
        if (solve_rows_per_group() == 2) return launch_solve_r<T, NCB, 2>(ex, forward, a, nblk);
    return launch_solve_r<T, NCB, 1>(ex, forward, a, nblk);
}

// Slice width in 16-column blocks: narrow slices shorten each block row's
// chain of dependent steps, wide ones read the factor fewer times.
// RFP_SOLVE_COLS (16, 32, 64 or 128) overrides the choice.
int block_solve_width(int64_t nrhs)
{
    static int forced = -1;
    if (forced < 0) {
        const char* e = getenv("RFP_SOLVE_COLS");
        const int v = e ? atoi(e) : 0;
        forced = (v == 16 || v == 32 || v == 64 || v == 128) ? v / 16 : 0;
    }
    if (forced) return forced;
    // measured at n = 20000: 16-column slices up to 64 right-hand sides,
    // 32-column slices beyond (the factor is then re-read nrhs / 32 times)
    return nrhs <= 64 ? 1 : 2;
}

template <typename T>
hipError_t block_solve(const Exec& ex, bool forward, Mat<const T> t1, Mat<const T> s, Mat<const T> t2, int64_t m1,
                       int64_t m2, const T* winv, T* b, int64_t ldb, int64_t nrhs, int* flags, const int* epoch,
                       int* status, int spin_limit)
{
    SolveArgs<T> a;
    a.t1 = t1;
    a.s = s;
    a.t2 = t2;
    a.m1 = m1;
    a.m2 = m2;
    a.nb1 = (int)((m1 + BS - 1) / BS);
    a.nb2 = (int)((m2 + BS - 1) / BS);
    a.w = winv;
    a.b = b;
    a.ldb = ldb;
    a.nrhs = nrhs;
    a.flags = flags;
    a.epoch = epoch;
    a.gate = ex.gate;
    a.status = status;
    a.spin_limit = spin_limit;
    const int nblk = a.nb1 + a.nb2;
    if (nblk == 0 || nrhs <= 0) return hipSuccess;
    int ncb = block_solve_width(nrhs);
    if (ex.tune && !getenv("RFP_SOLVE_COLS")) {
        auto it = ex.tune->solve.find(tune_solve_key(sizeof(T) == 8 ? 0 : 1, m1 + m2, nrhs));
        if (it != ex.tune->solve.end() && (it->second == 1 || it->second == 2 || it->second == 4 || it->second == 8))
            ncb = it->second;
    }
    a.nslices = (int)((nrhs + 16 * ncb - 1) / (16 * ncb));
    switch (ncb) {
        case 1: return launch_solve<T, 1>(ex, forward, a, nblk);
        case 2: return launch_solve<T, 2>(ex, forward, a, nblk);
        case 4: return launch_solve<T, 4>(ex, forward, a, nblk);
        default: return launch_solve<T, 8>(ex, forward, a, nblk);
    }
}

template hipError_t block_solve<double>(const Exec&, bool, Mat<const double>, Mat<const double>, Mat<const double>,
                                        int64_t, int64_t, const double*, double*, int64_t, int64_t, int*,
                                        const int*, int*, int);
template hipError_t block_solve<float>(const Exec&, bool, Mat<const float>, Mat<const float>, Mat<const float>,
                                       int64_t, int64_t, const float*, float*, int64_t, int64_t, int*, const int*,
                                       int*, int);

}  // namespace rfp
