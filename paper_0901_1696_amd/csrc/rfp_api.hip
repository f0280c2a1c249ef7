// Drivers and C ABI of the MI355X RFP Cholesky library.
//
// The paper's simple related partition algorithm (Figure 3) splits the RFP
// array into T1 (A11), S (A21) and T2 (A22) and runs four full-format steps.
// Here the same 2 x 2 partition is applied recursively: the top level is the
// RFP split itself, and every step on T1 or T2 (POTRF, TRSM, TRTRI, TRMM,
// LAUUM) splits its triangle again at a multiple of the leaf order until the
// diagonal blocks fit one fused workgroup (factorization, 128) or one
// wavefront (solve and inversion, 64).  All off-diagonal work therefore lands in large
// GEMM-shaped products on the matrix cores, with the operands read in place
// from the RFP rectangle through strided views.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "rfp.h"
#include <cstdio>
#include <cstdlib>

#include "rfp_common.h"

namespace rfp {

// Per-launch event timing.  Event pairs come from a pool; when the pool is
// used up the finished pairs are folded into per-kernel totals (this waits
// for the last recorded launch).
struct Profiler {
    struct Rec {
        std::string name;
        int ev;
        double flops, bytes;
    };
    struct Agg {
        int64_t launches = 0;
        double ms = 0, flops = 0, bytes = 0;
    };
    static constexpr int POOL_PAIRS = 32768;
    std::vector<hipEvent_t> pool;
    std::vector<Rec> pending;
    std::map<std::string, Agg> agg;
    int used = 0;
    hipError_t err = hipSuccess;

    // create the whole pool at once (called when profiling is enabled)
    hipError_t reserve()
    {
        while ((int)pool.size() < 2 * POOL_PAIRS) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            pool.push_back(e);
        }
        return hipSuccess;
    }
    int begin(const char* name, double flops, double bytes, hipStream_t s)
    {
        if (used == POOL_PAIRS) fold();
        if ((int)pool.size() < 2 * (used + 1)) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
                err = hipErrorOutOfMemory;
                return -1;
            }
            pool.push_back(a);
            pool.push_back(b);
        }
        const int ev = 2 * used++;
        pending.push_back(Rec{name, ev, flops, bytes});
        (void)hipEventRecord(pool[ev], s);
        return ev;
    }
    void end(int ev, hipStream_t s)
    {
        if (ev >= 0) (void)hipEventRecord(pool[ev + 1], s);
    }
    void fold()
    {
        for (const Rec& r : pending) {
            float ms = 0;
            if (hipEventSynchronize(pool[r.ev + 1]) != hipSuccess ||
                hipEventElapsedTime(&ms, pool[r.ev], pool[r.ev + 1]) != hipSuccess)
                err = hipErrorUnknown;
            Agg& a = agg[r.name];
            a.launches++;
            a.ms += ms;
            a.flops += r.flops;
            a.bytes += r.bytes;
        }
        pending.clear();
        used = 0;
    }
    ~Profiler()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

ProfScope::ProfScope(const Exec& ex, const char* name, double flops, double bytes)
    : p(ex.prof), slot(-1), stream(ex.stream)
{
    if (p) slot = p->begin(name, flops, bytes, stream);
}

ProfScope::~ProfScope()
{
    if (p) p->end(slot, stream);
}

}  // namespace rfp

struct rfp_context {
    int device;
    void* splitk;         // split-K partial sums of the caller's stream
    size_t splitk_bytes;
    void* splitk2;        // ... and of the auxiliary stream (the two may run at once)
    size_t splitk2_bytes;
    void* inv;
    size_t inv_bytes;
    rfp::Profiler* prof;
    hipStream_t aux;      // second stream for the lookahead factorization (default priority)
    hipStream_t aux2;     // third stream: the off-diagonal solve overlapped with the first factor
    hipEvent_t ev[64];    // ring of ordering events between the streams
    hipEvent_t join;      // end of the third stream's work (waited much later than recorded)
    int nev, evi;
    int* flags;           // ready flags of the fused triangular solves
    size_t flags_bytes;
    int* ctl;             // device words: [0] epoch of the flags, [1] solve status (bit 0: a wait gave up)
    int spin_limit;       // polls of an unpublished block row before a fused-solve wait gives up
    double lowp_shift[3]; // diagonal shift of a FP32, FP16, BF16 factor, in units of its unit roundoff
    void* ir;             // mixed-precision solve workspace
    size_t ir_bytes;
    void* bat;            // batched-solver scratch (work counter + per-workgroup scratch)
    size_t bat_bytes;
    void* zwork;          // complex path: leaf inverses and block temporaries
    size_t zwork_bytes;
    int cus;              // compute units of the device
    rfp::TuneTable* tune; // autotuned kernel configurations (null: built-in rules)
    rfp_schedule_t sched; // factorization schedule knobs
    int sched_user;       // 1: set by rfp_set_schedule (tuned schedules are then not used)
};

namespace rfp {

static int upc(char c) { return (c >= 'a' && c <= 'z') ? c - 'a' + 'A' : c; }

static inline int64_t nleaves(int64_t n, int nb) { return (n + nb - 1) / nb; }

// Plan recording: when a Run has a recorder, the drivers append one record
// per primitive (GEMM or leaf kernel) instead of launching it.  Pointers are
// then symbolic: each buffer gets a fixed fake base, and a record stores
// (buffer, element offset, strides).
static constexpr uint64_t PLAN_BASE_SHIFT = 44;
struct PlanRec {
    rfp_plan_op* ops;
    int64_t cap, count;
    size_t esize;
};
static void plan_view(const void* p, int64_t rs, int64_t cs, size_t esize, int64_t* out)
{
    const uint64_t a = (uint64_t)(uintptr_t)p;
    const uint64_t buf = a >> PLAN_BASE_SHIFT;
    out[0] = (int64_t)buf - 1;
    out[1] = (int64_t)((a - (buf << PLAN_BASE_SHIFT)) / esize);
    out[2] = rs;
    out[3] = cs;
}

template <typename T>
struct Run {
    Exec ex;             // the caller's stream: the critical path
    Exec ex2;            // auxiliary stream (bulk trailing updates), when available
    Exec ex3;            // second auxiliary stream (no split-K), when available
    hipEvent_t* evs = nullptr;
    int nev = 0, *evi = nullptr;
    hipEvent_t joinev = nullptr;
    int on = 0;  // stream of the next GEMMs: 0 ex, 1 ex2, 2 ex3
    hipError_t err = hipSuccess;
    PlanRec* rec = nullptr;
    int nb = NB;  // leaf order of this call's recursion
    T* tri_scratch = nullptr;    // the 128-row inverse leaf's scratch: NB2 x NB2 per stream (index `on`)
    // Scratch of the out-of-place triangular multiplies, one per stream: an
    // r x c product fits when r <= rows and c <= cols (column-major with
    // leading dimension ld), or, with ld == 0, when r * c <= elems (leading
    // dimension r).  Without one (or when it is too small) the multiplies
    // recurse in place.
    struct Scratch {
        T* p = nullptr;
        int64_t ld = 0, rows = 0, cols = 0, elems = 0;
    };
    Scratch tsc[3];
    bool scratch_for(int64_t r, int64_t c, Mat<T>* X) const
    {
        const Scratch& q = tsc[on];
        if (!q.p || r <= 0 || c <= 0) return false;
        if (q.ld) {
            if (r > q.rows || c > q.cols) return false;
            *X = Mat<T>{q.p, 1, q.ld};
            return true;
        }
        if (r * c > q.elems) return false;
        *X = Mat<T>{q.p, 1, r};
        return true;
    }
    void chk(hipError_t e)
    {
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    rfp_plan_op* next(int kind)
    {
        if (rec->count >= rec->cap) {
            rec->count++;
            return nullptr;
        }
        rfp_plan_op* o = &rec->ops[rec->count++];
        std::memset(o, 0, sizeof(*o));
        o->kind = kind;
        o->a[0] = o->b[0] = o->c[0] = o->d[0] = o->w[0] = -1;
        return o;
    }
    void mm(int64_t m, int64_t n, int64_t k, T alpha, Mat<const T> A, int ta, Mat<const T> B, int tb, T beta,
            Mat<T> C, bool lower = false, bool inplace = false)
    {
        if (rec) {
            chk(gemm_validate(m, n, A.rs, A.cs, B.rs, B.cs, C.rs, C.cs, lower, inplace));
            if (rfp_plan_op* o = next(RFP_PLAN_GEMM)) {
                o->m = m; o->n = n; o->k = k;
                o->inplace = inplace ? 1 : 0;
                o->stream = on;
                o->alpha = (double)alpha; o->beta = (double)beta;
                o->tri_a = ta; o->tri_b = tb; o->c_lower = lower ? 1 : 0;
                plan_view(A.p, A.rs, A.cs, sizeof(T), o->a);
                plan_view(B.p, B.rs, B.cs, sizeof(T), o->b);
                plan_view(C.p, C.rs, C.cs, sizeof(T), o->c);
            }
            return;
        }
        chk(gemm<T>(on == 1 ? ex2 : on == 2 ? ex3 : ex, m, n, k, alpha, A, ta, B, tb, beta, C, lower, inplace));
    }
    // Stream ordering.  Stream 0 is the caller's, streams 1 and 2 the
    // auxiliary ones.  While recording a plan the streams are virtual and
    // every record and wait is logged, so the host replay can check the
    // schedule for races.  Ring events are waited right after they are
    // recorded; `join` (record_join) is the one event waited much later.
    int plan_events = 0;
    bool two_streams() const { return rec || (evs && ex2.stream != nullptr); }
    bool three_streams() const { return rec || (evs && ex2.stream && ex3.stream && joinev); }
    hipStream_t stream_of(int stream) const { return stream == 1 ? ex2.stream : stream == 2 ? ex3.stream : ex.stream; }
    hipEvent_t plan_record(int stream)
    {
        if (rfp_plan_op* o = next(RFP_PLAN_RECORD)) {
            o->stream = stream;
            o->m = plan_events;
        }
        return (hipEvent_t)(uintptr_t)(++plan_events);
    }
    hipEvent_t record(int stream)
    {
        if (rec) return plan_record(stream);
        if (!two_streams()) return nullptr;
        hipEvent_t ev = evs[(*evi)++ % nev];
        chk(hipEventRecord(ev, stream_of(stream)));
        return ev;
    }
    hipEvent_t record_join(int stream)
    {
        if (rec) return plan_record(stream);
        chk(hipEventRecord(joinev, stream_of(stream)));
        return joinev;
    }
    void wait(int stream, hipEvent_t ev)
    {
        if (!ev) return;
        if (rec) {
            if (rfp_plan_op* o = next(RFP_PLAN_WAIT)) {
                o->stream = stream;
                o->m = (int64_t)(uintptr_t)ev - 1;
            }
            return;
        }
        chk(hipStreamWaitEvent(stream_of(stream), ev, 0));
    }
    // Fused triangular solve with the whole factor (see block_solve).
    int* flags = nullptr;
    int64_t nflags = 0;
    int* ctl = nullptr;
    int spin_limit = DEFAULT_SPIN_LIMIT;
    void solve(bool forward, const RfpView<const T>& v, const T* winv, Mat<T> B, int64_t nrhs)
    {
        if (rec) {
            if (rfp_plan_op* o = next(RFP_PLAN_BLOCK_SOLVE)) {
                o->tri_a = forward ? 0 : 1;
                o->m = v.m1; o->n = nrhs; o->k = v.m2;
                plan_view(v.t1.p, v.t1.rs, v.t1.cs, sizeof(T), o->a);
                plan_view(v.s.p, v.s.rs, v.s.cs, sizeof(T), o->b);
                plan_view(v.t2.p, v.t2.rs, v.t2.cs, sizeof(T), o->c);
                plan_view(B.p, B.rs, B.cs, sizeof(T), o->d);
                plan_view(winv, NB, 1, sizeof(T), o->w);
            }
            return;
        }
        chk(epoch_bump(ex.stream, flags, nflags, ctl));
        chk(block_solve<T>(ex, forward, v.t1, v.s, v.t2, v.m1, v.m2, winv, B.p, B.cs, nrhs, flags, ctl, ctl + 1,
                           spin_limit));
    }
    void leaf_potrf(int64_t order, Mat<T> A, int64_t goff, T* winv)
    {
        if (rec) leaf(RFP_PLAN_POTRF_LEAF, A, order, winv, goff);
        else if (nb == NB2) chk(potrf128_leaf<T>(ex, A, (int)order, winv, goff));
        else chk(potrf_leaf<T>(ex, A, (int)order, winv, goff));
    }

    // Cholesky of a diagonal block of order n <= panel width: the 2 x 2
    // partition of Section 3 down to nb-row leaves, each leaf leaving the
    // inverse of its factor in winv (consecutive nb x nb blocks).
    void potrf_rec(int64_t n, Mat<T> A, int64_t goff, T* winv)
    {
        if (n <= 0) return;
        if (n <= nb) {
            leaf_potrf(n, A, goff, winv);
            return;
        }
        const int64_t n1 = rec_split(n, nb), n2 = n - n1;
        potrf_rec(n1, A, goff, winv);
        trsm_rlt(n2, n1, A.sub(n1, 0), A, winv);
        mm(n2, n2, n1, T(-1), A.sub(n1, 0), TRI_NONE, A.sub(n1, 0), TRI_NONE, T(1), A.sub(n1, n1), true);
        potrf_rec(n2, A.sub(n1, n1), goff + n1, winv + nleaves(n1, nb) * nb * nb);
    }

    // Right-looking blocked Cholesky of the lower triangle of A (order n) with
    // one step of lookahead: after the panel of step k, the critical stream
    // updates only panel column k + 1 and factors its diagonal block while
    // the auxiliary stream applies step k's update to the rest of the
    // trailing matrix.  Step k + 1's update of panel column k + 2 waits for
    // that bulk update (both write it).  Panels are 2 nb wide while the
    // trailing matrix is large (the bulk update, at k = 2 nb, then runs faster
    // than at k = nb and hides the diagonal chain) and nb wide once it is
    // small (the chain per column is then shorter: fewer small products per
    // leaf, and nothing large enough is left to hide it).
    //
    // fork: after the panel solve of every step, fork(o1, ev) is called with
    // the event that marks columns [0, o1) (and their leaf inverses) final on
    // stream 0.
    // trailing order above which panels are 2 nb wide, and trailing order up
    // to which the bulk update waits for the lookahead (the schedule knobs)
    int64_t wide_panels_above = DEFAULT_WIDE_PANELS_ABOVE;
    int64_t wide_panel_cols = DEFAULT_WIDE_PANEL_COLS;
    int64_t lookahead_wait_below = DEFAULT_LOOKAHEAD_WAIT_BELOW;
    template <typename F = void (*)(int64_t, hipEvent_t)>
    void potrf_la(int64_t n, Mat<T> A, int64_t goff, T* winv, F* fork = nullptr)
    {
        if (n <= 0) return;
        auto winv_at = [&](int64_t o) { return winv + (o / nb) * nb * nb; };
        auto width = [&](int64_t o) {
            return std::min<int64_t>(n - o > wide_panels_above ? wide_panel_cols : nb, n - o);
        };
        int64_t o = 0, w = width(0);
        potrf_rec(w, A, goff, winv);
        hipEvent_t bulk_prev = nullptr;
        while (o + w < n) {
            const int64_t o1 = o + w, w1 = width(o1), o2 = o1 + w1;
            // panel: L(o1:, panel) = A(o1:, panel) L_kk^{-T}
            trsm_rlt(n - o1, w, A.sub(o1, o), A.sub(o, o), winv_at(o));
            hipEvent_t panel_done = record(0);
            if (fork) (*fork)(o1, panel_done);
            // lookahead: the next panel column (lower part of its diagonal block), then that block
            wait(0, bulk_prev);
            mm(n - o1, w1, w, T(-1), A.sub(o1, o), TRI_NONE, A.sub(o1, o), TRI_NONE, T(1), A.sub(o1, o1), true);
            // The bulk update also waits for the lookahead, so that it overlaps
            // the leaf chain (one workgroup at a time) instead of taking the
            // compute units the lookahead (on the critical path) needs.
            const hipEvent_t la_done = n - o1 <= lookahead_wait_below && o2 < n ? record(0) : nullptr;
            potrf_rec(w1, A.sub(o1, o1), goff + o1, winv_at(o1));
            // bulk: columns beyond the next panel
            bulk_prev = nullptr;
            if (o2 < n) {
                wait(1, panel_done);
                wait(1, la_done);
                on = two_streams() ? 1 : 0;
                mm(n - o2, n - o2, w, T(-1), A.sub(o2, o), TRI_NONE, A.sub(o2, o), TRI_NONE, T(1), A.sub(o2, o2), true);
                on = 0;
                bulk_prev = record(1);
            }
            o = o1;
            w = w1;
        }
        wait(0, bulk_prev);
    }
    // the stream the next GEMMs and leaves go to
    const Exec& cur() const { return on == 1 ? ex2 : on == 2 ? ex3 : ex; }
    void leaf(int kind, Mat<const T> A, int64_t order, const T* w, int64_t info_base)
    {
        if (rfp_plan_op* o = next(kind)) {
            o->stream = on;
            o->m = order;
            o->info_base = info_base;
            plan_view(A.p, A.rs, A.cs, sizeof(T), o->a);
            if (w) plan_view(w, nb, 1, sizeof(T), o->b);
        }
    }

    // ---------------------------------------------------------- factorization
    // B (m x n) <- B L^{-T}; L lower of order n whose leaf inverses are in winv.
    void trsm_rlt(int64_t m, int64_t n, Mat<T> B, Mat<const T> L, const T* winv)
    {
        if (m <= 0 || n <= 0) return;
        if (n <= nb) {
            mm(m, n, n, T(1), B, TRI_NONE, Mat<const T>{winv, nb, 1}, TRI_LOWER, T(0), B, false, true);
            return;
        }
        const int64_t n1 = rec_split(n, nb), n2 = n - n1;
        trsm_rlt(m, n1, B, L, winv);
        mm(m, n2, n1, T(-1), B, TRI_NONE, L.sub(n1, 0), TRI_NONE, T(1), B.sub(0, n1));
        trsm_rlt(m, n2, B.sub(0, n1), L.sub(n1, n1), winv + nleaves(n1, nb) * nb * nb);
    }


    // C (m x n) += alpha A (lower triangles only when lower)
    void axpy(int64_t m, int64_t n, T alpha, Mat<const T> A, Mat<T> C, bool lower)
    {
        if (m <= 0 || n <= 0) return;
        if (rec) {
            if (rfp_plan_op* o = next(RFP_PLAN_AXPY)) {
                o->stream = on;
                o->m = m;
                o->n = n;
                o->alpha = (double)alpha;
                o->c_lower = lower ? 1 : 0;
                plan_view(A.p, A.rs, A.cs, sizeof(T), o->a);
                plan_view(C.p, C.rs, C.cs, sizeof(T), o->c);
            }
            return;
        }
        chk(axpy2d<T>(cur().stream, C, A, m, n, alpha, lower));
    }

    // B (m x n) <- B L^{-1}; L lower of order n whose leaf inverses are in winv.
    void trsm_rln(int64_t m, int64_t n, Mat<T> B, Mat<const T> L, const T* winv)
    {
        if (m <= 0 || n <= 0) return;
        if (n <= nb) {
            // B W with W = L^{-1} lower: the operand B(j, kk) = W(kk, j) is upper
            mm(m, n, n, T(1), B, TRI_NONE, Mat<const T>{winv, 1, nb}, TRI_UPPER, T(0), B, false, true);
            return;
        }
        const int64_t n1 = rec_split(n, nb), n2 = n - n1;
        trsm_rln(m, n2, B.sub(0, n1), L.sub(n1, n1), winv + nleaves(n1, nb) * nb * nb);
        mm(m, n1, n2, T(-1), B.sub(0, n1), TRI_NONE, L.sub(n1, 0).tr(), TRI_NONE, T(1), B);
        trsm_rln(m, n1, B, L, winv);
    }

    // ---------------------------------------------------------------- solve
    void leaves_inv(Mat<const T> A, int64_t n, T* winv)
    {
        if (rec) leaf(RFP_PLAN_TRTRI_LEAVES, A, n, winv, 0);
        else chk(trtri_leaves<T>(ex, A, n, winv));
    }
    void setinfo(int* p)
    {
        if (!rec) chk(set_int(ex.stream, p, 0));
    }

    // ------------------------------------------------------------ inversion
    // C (m x n) <- A
    void copy(int64_t m, int64_t n, Mat<const T> A, Mat<T> C)
    {
        if (m <= 0 || n <= 0) return;
        if (rec) {
            if (rfp_plan_op* o = next(RFP_PLAN_COPY)) {
                o->stream = on;
                o->m = m;
                o->n = n;
                plan_view(A.p, A.rs, A.cs, sizeof(T), o->a);
                plan_view(C.p, C.rs, C.cs, sizeof(T), o->c);
            }
            return;
        }
        chk(copy2d<T, T>(cur().stream, C, A, m, n, false));
    }

    // Leaf order of the inversion recursion: the 128-row inverse and LAUUM
    // leaves, and in-place base products of the triangular multiplies 128
    // wide (one tile across the aliased side).
    static constexpr int64_t tb() { return NB2; }
    // B (m x n) <- alpha B W, W lower of order n
    void trmm_rl(int64_t m, int64_t n, Mat<T> B, Mat<const T> W, T alpha)
    {
        if (m <= 0 || n <= 0) return;
        if (n <= tb()) {
            mm(m, n, n, alpha, B, TRI_NONE, W.tr(), TRI_UPPER, T(0), B, false, true);
            return;
        }
        Mat<T> X;
        if (scratch_for(m, n, &X)) {  // one product into the scratch, copied back
            mm(m, n, n, alpha, B, TRI_NONE, W.tr(), TRI_UPPER, T(0), X);
            copy(m, n, X, B);
            return;
        }
        const int64_t n1 = rec_split(n, tb()), n2 = n - n1;
        trmm_rl(m, n1, B, W, alpha);
        mm(m, n1, n2, alpha, B.sub(0, n1), TRI_NONE, W.sub(n1, 0).tr(), TRI_NONE, T(1), B);
        trmm_rl(m, n2, B.sub(0, n1), W.sub(n1, n1), alpha);
    }
    // B (m x n) <- W B, W lower of order m
    void trmm_ll(int64_t m, int64_t n, Mat<const T> W, Mat<T> B)
    {
        if (m <= 0 || n <= 0) return;
        if (m <= tb()) {
            mm(m, n, m, T(1), W, TRI_LOWER, B.tr(), TRI_NONE, T(0), B, false, true);
            return;
        }
        Mat<T> X;
        if (scratch_for(m, n, &X)) {
            mm(m, n, m, T(1), W, TRI_LOWER, B.tr(), TRI_NONE, T(0), X);
            copy(m, n, X, B);
            return;
        }
        const int64_t m1 = rec_split(m, tb()), m2 = m - m1;
        trmm_ll(m2, n, W.sub(m1, m1), B.sub(m1, 0));
        mm(m2, n, m1, T(1), W.sub(m1, 0), TRI_NONE, B.tr(), TRI_NONE, T(1), B.sub(m1, 0));
        trmm_ll(m1, n, W, B);
    }
    // B (m x n) <- W^T B, W lower of order m
    void trmm_llt(int64_t m, int64_t n, Mat<const T> W, Mat<T> B)
    {
        if (m <= 0 || n <= 0) return;
        if (m <= tb()) {
            mm(m, n, m, T(1), W.tr(), TRI_UPPER, B.tr(), TRI_NONE, T(0), B, false, true);
            return;
        }
        Mat<T> X;
        if (scratch_for(m, n, &X)) {
            mm(m, n, m, T(1), W.tr(), TRI_UPPER, B.tr(), TRI_NONE, T(0), X);
            copy(m, n, X, B);
            return;
        }
        const int64_t m1 = rec_split(m, tb()), m2 = m - m1;
        trmm_llt(m1, n, W, B);
        mm(m1, n, m2, T(1), W.sub(m1, 0).tr(), TRI_NONE, B.sub(m1, 0).tr(), TRI_NONE, T(1), B);
        trmm_llt(m2, n, W.sub(m1, m1), B.sub(m1, 0));
    }
    // B (m x n) <- alpha W2 B W1 (W1 lower of order n, W2 lower of order m):
    // with scratch, B W1 goes there and W2 times it straight back into B;
    // stream `on` waits for ev (W2 ready) before the second product.
    void trmm_both(int64_t m, int64_t n, Mat<T> B, Mat<const T> W1, Mat<const T> W2, T alpha, hipEvent_t ev)
    {
        Mat<T> X;
        if (m > 0 && n > 0 && scratch_for(m, n, &X)) {
            mm(m, n, n, alpha, B, TRI_NONE, W1.tr(), TRI_UPPER, T(0), X);
            wait(on, ev);
            mm(m, n, m, T(1), W2, TRI_LOWER, X.tr(), TRI_NONE, T(0), B);
            return;
        }
        trmm_rl(m, n, B, W1, alpha);
        wait(on, ev);
        trmm_ll(m, n, W2, B);
    }
    // in-place inverse of the lower triangle of A (order n)
    void trtri_rec(int64_t n, Mat<T> A, int64_t goff)
    {
        if (n <= 0) return;
        // one workgroup's MFMA leaf (a scratch block per stream)
        if (n <= tb()) {
            if (rec) leaf(RFP_PLAN_TRTRI_LEAF, A, n, nullptr, goff);
            else chk(trtri128_leaf<T>(cur(), A, (int)n, tri_scratch + (int64_t)on * NB2 * NB2, goff));
            return;
        }
        const int64_t n1 = rec_split(n, tb()), n2 = n - n1;
        // both diagonal inverses first, so that the scratch is free for the
        // off-diagonal block W21 = -W22 A21 W11
        trtri_rec(n1, A, goff);
        trtri_rec(n2, A.sub(n1, n1), goff + n1);
        trmm_both(n2, n1, A.sub(n1, 0), A, A.sub(n1, n1), T(-1), nullptr);
    }
    // lower triangle of W^T W in place (order n)
    void lauum_rec(int64_t n, Mat<T> W)
    {
        if (n <= 0) return;
        if (n <= tb()) {
            if (rec) leaf(RFP_PLAN_LAUUM_LEAF, W, n, nullptr, 0);
            else chk(lauum128_leaf<T>(cur(), W, (int)n));
            return;
        }
        const int64_t n1 = rec_split(n, tb()), n2 = n - n1;
        lauum_rec(n1, W);
        mm(n1, n1, n2, T(1), W.sub(n1, 0).tr(), TRI_NONE, W.sub(n1, 0).tr(), TRI_NONE, T(1), W, true);
        trmm_llt(n2, n1, W.sub(n1, n1), W.sub(n1, 0));
        lauum_rec(n2, W.sub(n1, n1));
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (dev < 0) return;  // plan recording: no device involved
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

static hipError_t ensure(void** p, size_t* have, size_t need)
{
    if (need <= *have) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    need = (need + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
    e = hipMalloc(p, need);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    *have = need;
    return hipSuccess;
}

static constexpr size_t SPLITK_BYTES = size_t(128) << 20;

static hipError_t prepare(rfp_context* h, size_t inv_need)
{
    hipError_t e = ensure(&h->splitk, &h->splitk_bytes, SPLITK_BYTES);
    if (e == hipSuccess) e = ensure(&h->splitk2, &h->splitk2_bytes, SPLITK_BYTES);
    if (e != hipSuccess) return e;
    if (!h->aux) {
        e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        for (int i = 0; i < 64; i++) {
            e = hipEventCreateWithFlags(&h->ev[i], hipEventDisableTiming);
            if (e != hipSuccess) return e;
            h->nev = i + 1;
        }
    }
    if (!h->aux2) {
        e = hipStreamCreateWithFlags(&h->aux2, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&h->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(h->aux2);
            h->aux2 = nullptr;
            return e;
        }
    }
    return ensure(&h->inv, &h->inv_bytes, inv_need);
}

// Ready flags for the fused solves: grown on demand and cleared once when
// allocated; launches then tell stale flags apart by their epoch, a device
// word (ctl[0]) that a one-thread kernel advances before every launch.  The
// control words are allocated and cleared once, with the first flags.
static hipError_t prepare_flags(rfp_context* h, int64_t count)
{
    hipError_t e = hipSuccess;
    if (!h->ctl) {
        e = hipMalloc((void**)&h->ctl, 256);
        if (e == hipSuccess) e = hipMemset(h->ctl, 0, 256);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
    }
    const size_t need = size_t(std::max<int64_t>(count, 1)) * sizeof(int);
    if (need <= h->flags_bytes) return hipSuccess;
    e = ensure((void**)&h->flags, &h->flags_bytes, need);
    if (e == hipSuccess) e = hipMemset(h->flags, 0, h->flags_bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}

// Both fused solves (forward, backward) over a factor whose 64-row diagonal
// blocks' inverses are in w (those of T1, then of T2).
template <typename T>
static hipError_t solve_with_leaves(rfp_context* h, const Exec& ex, const RfpView<const T>& v, const T* w, T* b,
                                    int64_t ldb, int64_t nrhs)
{
    const int64_t nf = (int64_t)(h->flags_bytes / sizeof(int));
    for (int fwd = 1; fwd >= 0; fwd--) {
        hipError_t e = epoch_bump(ex.stream, h->flags, nf, h->ctl);
        if (e == hipSuccess)
            e = block_solve<T>(ex, fwd == 1, v.t1, v.s, v.t2, v.m1, v.m2, w, b, ldb, nrhs, h->flags, h->ctl,
                               h->ctl + 1, h->spin_limit);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static rfp_schedule_t default_schedule()
{
    rfp_schedule_t sc;
    sc.wide_panels_above = DEFAULT_WIDE_PANELS_ABOVE;
    sc.chunk_max = DEFAULT_CHUNK_MAX;
    sc.lookahead_wait_below = DEFAULT_LOOKAHEAD_WAIT_BELOW;
    sc.leaf_lds_pad = DEFAULT_LEAF_LDS_PAD;
    sc.wide_panel_cols = DEFAULT_WIDE_PANEL_COLS;
    return sc;
}

static bool bad_schedule(const rfp_schedule_t& sc)
{
    return sc.wide_panels_above < 0 || sc.chunk_max < 0 || sc.lookahead_wait_below < 0 || sc.leaf_lds_pad < 0 ||
           sc.leaf_lds_pad > MAX_LEAF_LDS_PAD || sc.wide_panel_cols < NB2 || sc.wide_panel_cols % NB2 != 0;
}

// The schedule of a factorization of order n: the caller's, else a tuned one
// for n's size class, else the defaults.
static rfp_schedule_t schedule_for(const rfp_context* h, int64_t n)
{
    if (!h->sched_user && h->tune) {
        auto it = h->tune->sched.find(size_bucket(n));
        if (it != h->tune->sched.end()) return it->second;
    }
    return h->sched;
}

template <typename T>
static Run<T> make_run(rfp_context* h, hipStream_t s, int* info, int lowp = 0, const rfp_schedule_t* sc = nullptr)
{
    const rfp_schedule_t sched = sc ? *sc : h->sched;
    Run<T> r;
    r.ex.stream = s;
    r.ex.info = info;
    r.ex.splitk_ws = h->splitk;
    r.ex.splitk_bytes = h->splitk_bytes;
    r.ex.prof = h->prof;
    r.ex2 = r.ex;
    r.ex2.stream = h->aux;
    r.ex2.splitk_ws = h->splitk2;
    r.ex2.splitk_bytes = h->splitk2_bytes;
    r.evs = h->nev ? h->ev : nullptr;
    r.nev = h->nev;
    r.evi = &h->evi;
    r.ex.tune = r.ex2.tune = h->tune;
    // low-precision operands for every non-in-place product of all three streams
    r.ex.lowp = r.ex2.lowp = lowp;
    r.ex.leaf_pad = r.ex2.leaf_pad = (int)sched.leaf_lds_pad;
    r.wide_panels_above = sched.wide_panels_above;
    r.wide_panel_cols = sched.wide_panel_cols;
    r.lookahead_wait_below = sched.lookahead_wait_below;
    r.ex3 = r.ex;
    r.ex3.stream = h->aux2;
    r.ex3.splitk_ws = nullptr;  // its GEMMs never split K: no workspace shared with the other streams
    r.ex3.splitk_bytes = 0;
    // the caller's stream carries the critical path (panels and lookahead);
    // the auxiliary streams' bulk work yields issue slots to it
    r.ex.prio = 1;
    r.joinev = h->aux2 ? h->join : nullptr;
    return r;
}

static inline bool bad_tr(char c) { return upc(c) != 'N' && upc(c) != 'T'; }
static inline bool bad_ul(char c) { return upc(c) != 'L' && upc(c) != 'U'; }

template <typename T>
static int trttf_impl(rfp_context* h, char transr, char uplo, int64_t n, const T* a, int64_t lda, T* arf,
                      hipStream_t s, bool to_rfp)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n == 0) return 0;
    // argument positions differ: TRTTF (.., A=4, LDA=5, ARF=6); TFTTR (.., ARF=4, A=5, LDA=6)
    if (to_rfp) {
        if (!a) return -4;
        if (lda < std::max<int64_t>(1, n)) return -5;
        if (!arf) return -6;
    } else {
        if (!arf) return -4;
        if (!a) return -5;
        if (lda < std::max<int64_t>(1, n)) return -6;
    }
    DeviceGuard g(h->device);
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    RfpView<T> v = rfp_view(b, arf);
    // canonical lower view of the full matrix: the UPLO triangle read as lower
    Mat<T> F = (upc(uplo) == 'L') ? Mat<T>{(T*)a, 1, lda} : Mat<T>{(T*)a, lda, 1};
    hipError_t e;
    if (to_rfp) {
        e = copy2d<T, T>(s, v.t1, F, b.m1, b.m1, true);
        if (e == hipSuccess) e = copy2d<T, T>(s, v.s, F.sub(b.m1, 0), b.m2, b.m1, false);
        if (e == hipSuccess) e = copy2d<T, T>(s, v.t2, F.sub(b.m1, b.m1), b.m2, b.m2, true);
    } else {
        e = copy2d<T, T>(s, F, v.t1, b.m1, b.m1, true);
        if (e == hipSuccess) e = copy2d<T, T>(s, F.sub(b.m1, 0), v.s, b.m2, b.m1, false);
        if (e == hipSuccess) e = copy2d<T, T>(s, F.sub(b.m1, b.m1), v.t2, b.m2, b.m2, true);
    }
    return e == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

// Fake buffer bases used while recording a plan (buffer id + 1 in the high bits).
template <typename T>
static T* plan_base(int buf)
{
    return (T*)(uintptr_t)((uint64_t)(buf + 1) << PLAN_BASE_SHIFT);
}

template <typename T>
static int pftrf_impl(rfp_context* h, char transr, char uplo, int64_t n, T* arf, int* info, hipStream_t s,
                      PlanRec* rec = nullptr, int lowp = 0, const rfp_schedule_t* plan_sched = nullptr,
                      bool gated = false)
{
    // gated: *info is not reset; the factorization runs only if the caller
    // leaves it at 0 (every kernel of the factorization exits while it is not)
    if (!h && !rec) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !arf) return -4;
    if (!info) return -5;
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    const int64_t lv = std::max(nleaves(b.m1, NB2), nleaves(b.m2, NB2));
    Run<T> r;
    T* winv;
    DeviceGuard g(rec ? -1 : h->device);
    rfp_schedule_t sc;
    if (rec) {
        sc = plan_sched ? *plan_sched : default_schedule();
        if (bad_schedule(sc)) return -8;
        r.rec = rec;
        r.wide_panels_above = sc.wide_panels_above;
        r.wide_panel_cols = sc.wide_panel_cols;
        r.lookahead_wait_below = sc.lookahead_wait_below;
        winv = plan_base<T>(RFP_PLAN_BUF_WORK);
    } else {
        if (n == 0) return set_int(s, info, 0) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
        if (prepare(h, size_t(lv) * NB2 * NB2 * sizeof(T)) != hipSuccess) return RFP_ERR_RUNTIME;
        sc = schedule_for(h, n);
        const bool tuned = h->tune && h->tune->sched.count(size_bucket(n));
        if ((lowp == RFP_PREC_FP16 || lowp == RFP_PREC_BF16) && !h->sched_user && !tuned)
            sc.wide_panel_cols = DEFAULT_LOWP_WIDE_PANEL_COLS;
        r = make_run<T>(h, s, info, lowp, &sc);
        winv = (T*)h->inv;
    }
    r.nb = NB2;
    RfpView<T> v = rfp_view(b, arf);
    if (!gated) r.setinfo(info);
    // step 1: L11 = chol(A11)              (Figure 4, factorization step 1)
    // step 2: L21 = A21 L11^{-T}           (step 2, TRSM)
    // Step 2 runs right-looking by chunks of at least SCHUNK columns of L11,
    // each on the second auxiliary stream as soon as the factorization of
    // step 1 has passed it, alongside its remaining (latency-bound) panels:
    //   L21(:, c0:c1) = A21(:, c0:c1) L11(c0:c1, c0:c1)^{-T}
    //   A21(:, c1:)  -= L21(:, c0:c1) L11(c1:, c0:c1)^T
    //   A22          -= L21(:, c0:c1) L21(:, c0:c1)^T   (step 3's share of the chunk)
    // The columns after the last chunk are solved, and their share of step 3
    // applied, on stream 0 after step 1.
    // chunk: at most chunk_max columns (1536 by default), at least 4 leaves,
    // at most half of T1 so that smaller triangles still get two chunks;
    // chunk_max = 0: no overlap (steps 2 and 3 follow step 1)
    const int64_t SCHUNK = std::max<int64_t>(
        4 * r.nb, std::min<int64_t>(sc.chunk_max, std::max<int64_t>(4 * r.nb, b.m1 / 2 / r.nb * r.nb)));
    int64_t done = 0;
    hipEvent_t joined = nullptr;
    auto fork = [&](int64_t o1, hipEvent_t ev) {
        if (o1 - done < SCHUNK || o1 >= b.m1) return;
        r.wait(2, ev);
        r.on = 2;
        r.trsm_rlt(b.m2, o1 - done, v.s.sub(0, done), v.t1.sub(done, done),
                   winv + nleaves(done, r.nb) * r.nb * r.nb);
        r.mm(b.m2, b.m1 - o1, o1 - done, T(-1), v.s.sub(0, done), TRI_NONE, v.t1.sub(o1, done), TRI_NONE, T(1),
             v.s.sub(0, o1));
        r.mm(b.m2, b.m2, o1 - done, T(-1), v.s.sub(0, done), TRI_NONE, v.s.sub(0, done), TRI_NONE, T(1), v.t2, true);
        r.on = 0;
        joined = r.record_join(2);
        done = o1;
    };
    if (sc.chunk_max > 0 && b.m2 > 0 && b.m1 > SCHUNK && r.three_streams()) r.potrf_la(b.m1, v.t1, 0, winv, &fork);
    else r.potrf_la(b.m1, v.t1, 0, winv);
    r.wait(0, joined);
    r.trsm_rlt(b.m2, b.m1 - done, v.s.sub(0, done), v.t1.sub(done, done), winv + nleaves(done, r.nb) * r.nb * r.nb);
    // step 3: A22 <- A22 - L21 L21^T       (step 3, SYRK on T2's triangle; the
    // chunks' shares are already applied)
    r.mm(b.m2, b.m2, b.m1 - done, T(-1), v.s.sub(0, done), TRI_NONE, v.s.sub(0, done), TRI_NONE, T(1), v.t2, true);
    // step 4: L22 = chol(A22), INFO offset by m1
    r.potrf_la(b.m2, v.t2, b.m1, winv);
    return r.err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

template <typename T>
static int pftrs_impl(rfp_context* h, char transr, char uplo, int64_t n, int64_t nrhs, const T* arf, T* bp,
                      int64_t ldb, hipStream_t s, PlanRec* rec = nullptr)
{
    if (!h && !rec) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && !arf) return -5;
    if (n > 0 && nrhs > 0 && !bp) return -6;
    if (ldb < std::max<int64_t>(1, n)) return -7;
    if (n == 0 || nrhs == 0) return 0;
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    const int64_t l1 = nleaves(b.m1, NB), l2 = nleaves(b.m2, NB);
    Run<T> r;
    T* w1;
    DeviceGuard g(rec ? -1 : h->device);
    if (rec) {
        r.rec = rec;
        w1 = plan_base<T>(RFP_PLAN_BUF_WORK);
    } else {
        if (prepare(h, size_t(l1 + l2) * NB * NB * sizeof(T)) != hipSuccess) return RFP_ERR_RUNTIME;
        if (prepare_flags(h, block_solve_flags(b.m1, b.m2, nrhs)) != hipSuccess) return RFP_ERR_RUNTIME;
        r = make_run<T>(h, s, nullptr);
        r.flags = h->flags;
        r.nflags = (int64_t)(h->flags_bytes / sizeof(int));
        r.ctl = h->ctl;
        r.spin_limit = h->spin_limit;
        w1 = (T*)h->inv;
    }
    T* w2 = w1 + l1 * NB * NB;
    RfpView<const T> v = rfp_view(b, arf);
    // inverses of the 64-row diagonal blocks of L11 and L22, consecutive
    r.leaves_inv(v.t1, b.m1, w1);
    r.leaves_inv(v.t2, b.m2, w2);
    Mat<T> B{bp, 1, ldb};
    // L Y = B, then L^T X = Y (Figure 4, solution): the 2 x 2 block steps
    // (Y1 = L11^{-1} B1, B2 -= L21 Y1, Y2 = L22^{-1} B2 and back) run as one
    // blocked substitution per direction over all diagonal blocks of L11 and L22
    r.solve(true, v, w1, B, nrhs);
    r.solve(false, v, w1, B, nrhs);
    return r.err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

// PFTRI's workspace (elements): the m1 x m1 square, the 128-row leaf's
// scratch at `tri`, the second stream's multiply scratch at `side`
// (side_elems: the off-diagonal block of T2's top split).
struct PftriWork {
    int64_t tri, side, side_elems, total, q;
};
static PftriWork pftri_work(int64_t m1, int64_t m2)
{
    auto up = [](int64_t x) { return (x + 31) / 32 * 32; };  // 256-byte pieces
    PftriWork w;
    w.tri = up(m1 * m1);
    w.side = up(w.tri + 3 * (int64_t)NB2 * NB2);
    const int64_t s2 = m2 > NB2 ? rec_split(m2, NB2) : m2;
    w.side_elems = s2 * (m2 - s2);
    w.total = w.side + w.side_elems;
    w.q = m1 > NB2 ? m1 - rec_split(m1, NB2) : 0;
    return w;
}

template <typename T>
static int pftri_impl(rfp_context* h, char transr, char uplo, int64_t n, T* arf, int* info, hipStream_t s,
                      PlanRec* rec = nullptr)
{
    if (!h && !rec) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !arf) return -4;
    if (!info) return -5;
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    Run<T> r;
    // Workspace: tmp, m1 x m1 column-major (the multiplies' scratch of the
    // first stream in stage 2, then W21^T W21 of stage 3, formed before S
    // changes); the 128-row leaf's scratch; the second stream's multiply
    // scratch, one off-diagonal block of T2's recursion.
    const PftriWork pw = pftri_work(b.m1, b.m2);
    T* tmp;
    DeviceGuard g(rec ? -1 : h->device);
    if (rec) {
        r.rec = rec;
        tmp = plan_base<T>(RFP_PLAN_BUF_WORK);
    } else {
        if (n == 0) return set_int(s, info, 0) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
        if (prepare(h, sizeof(T) * (size_t)pw.total) != hipSuccess) return RFP_ERR_RUNTIME;
        r = make_run<T>(h, s, info);
        tmp = (T*)h->inv;
    }
    r.tri_scratch = tmp + pw.tri;
    r.tsc[0].p = tmp;
    r.tsc[0].elems = (int64_t)b.m1 * b.m1;
    r.tsc[2].p = tmp + pw.side;
    r.tsc[2].elems = pw.side_elems;
    RfpView<T> v = rfp_view(b, arf);
    Mat<T> Tmp{tmp, 1, b.m1};
    r.setinfo(info);
    const bool two = r.three_streams();
    const int side = two ? 2 : 0;  // the stream of the T2 side
    // stage 2 (TFTRI): W11 = L11^{-1}; S <- -S W11; W22 = L22^{-1}; S <- W22 S.
    // W22 comes on the second stream while the first inverts L11 and scales S.
    hipEvent_t start = two ? r.record(0) : nullptr;
    r.wait(side, start);
    r.on = side;
    r.trtri_rec(b.m2, v.t2, b.m1);
    r.on = 0;
    hipEvent_t w22 = two ? r.record_join(side) : nullptr;
    r.trtri_rec(b.m1, v.t1, 0);
    r.trmm_both(b.m2, b.m1, v.s, v.t1, v.t2, T(-1), w22);
    // stage 3: T1 <- W11^T W11 + W21^T W21; S <- W22^T W21; T2 <- W22^T W22.
    // W21^T W21 goes to a scratch triangle first, so that S can change on the
    // second stream (S <- W22^T S, then LAUUM of T2) while the first stream
    // forms W11^T W11 in T1 and adds the scratch triangle to it.
    r.mm(b.m1, b.m1, b.m2, T(1), v.s.tr(), TRI_NONE, v.s.tr(), TRI_NONE, T(0), Tmp, true);
    // from here the first stream's multiply scratch is the block of tmp
    // strictly above its diagonal: rows [0, q), columns [q, m1), q the order
    // of the second diagonal block of T1's top split
    if (pw.q > 0) {
        r.tsc[0].p = tmp + (size_t)pw.q * b.m1;
        r.tsc[0].ld = b.m1;
        r.tsc[0].rows = pw.q;
        r.tsc[0].cols = b.m1 - pw.q;
    } else {
        r.tsc[0] = typename Run<T>::Scratch{};
    }
    hipEvent_t syrk = two ? r.record(0) : nullptr;
    r.wait(side, syrk);
    r.on = side;
    r.trmm_llt(b.m2, b.m1, v.t2, v.s);
    r.lauum_rec(b.m2, v.t2);
    r.on = 0;
    hipEvent_t t2done = two ? r.record_join(side) : nullptr;
    r.lauum_rec(b.m1, v.t1);
    r.axpy(b.m1, b.m1, T(1), Tmp, v.t1, true);
    r.wait(0, t2done);
    return r.err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

// ------------------------------------------------ mixed precision + IR
// Workspace carve-up of the refinement driver (256-byte aligned pieces).
struct IrSpace {
    float* a32;            // scaled FP32 copy of the matrix, same RFP layout
    double* a64;           // FP64 copy of the matrix for the fall-back factor
    float* w32;            // inverses of the 64-row diagonal blocks of the FP32 factor
    double* s;             // diagonal scaling D^{-1/2}
    double* r;             // residual, n x nrhs, leading dimension n
    float* r32;            // scaled residual / correction in FP32
    double *bmax, *rmax, *xmax, *anorm, *normwork;
    double *cr, *cz, *cp, *cq;  // conjugate-gradient vectors, n x nrhs each
    double *rz0, *rz1, *pq;     // their per-column scalars
    double* symm;               // partial products of A X
    IrCtl* ctl;                 // device-side decisions and gates
    size_t bytes;
};
static IrSpace ir_space(void* base, int64_t n, int64_t nrhs, int64_t nleaf64)
{
    IrSpace w;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return (char*)base + o;
    };
    const size_t nt = (size_t)(n * (n + 1) / 2);
    w.a32 = (float*)take(sizeof(float) * nt);
    w.a64 = (double*)take(sizeof(double) * nt);
    w.w32 = (float*)take(sizeof(float) * (size_t)nleaf64 * NB * NB);
    w.s = (double*)take(sizeof(double) * (size_t)n);
    w.r = (double*)take(sizeof(double) * (size_t)(n * nrhs));
    w.r32 = (float*)take(sizeof(float) * (size_t)(n * nrhs));
    w.bmax = (double*)take(sizeof(double) * (size_t)nrhs);
    w.rmax = (double*)take(sizeof(double) * (size_t)nrhs);
    w.xmax = (double*)take(sizeof(double) * (size_t)nrhs);
    w.anorm = (double*)take(sizeof(double));
    w.normwork = (double*)take(sizeof(double) * (size_t)(n + 3));
    w.cr = (double*)take(sizeof(double) * (size_t)(n * nrhs));
    w.cz = (double*)take(sizeof(double) * (size_t)(n * nrhs));
    w.cp = (double*)take(sizeof(double) * (size_t)(n * nrhs));
    w.cq = (double*)take(sizeof(double) * (size_t)(n * nrhs));
    w.rz0 = (double*)take(sizeof(double) * (size_t)nrhs);
    w.rz1 = (double*)take(sizeof(double) * (size_t)nrhs);
    w.pq = (double*)take(sizeof(double) * (size_t)nrhs);
    w.symm = (double*)take(symm_thin_workspace((n + 1) / 2, n / 2));
    w.ctl = (IrCtl*)take(sizeof(IrCtl));
    w.bytes = off;
    return w;
}

// RFP_IR_TRACE=1 makes the refinement synchronise after every sweep and print
// its backward error to stderr (a debugging aid; the call is then no longer
// free of host synchronisation).
static bool ir_trace()
{
    static int on = -1;
    if (on < 0) {
        const char* e = getenv("RFP_IR_TRACE");
        on = (e && e[0] == '1') ? 1 : 0;
    }
    return on == 1;
}

// Scaling of the low-precision copy: the unit-diagonal matrix D^{-1/2} A
// D^{-1/2} has entries in [-1, 1] and so has its Cholesky factor, whose
// entries are the only values rounded to the operand precision (the trailing
// matrix stays FP32).  For FP16 the whole copy is multiplied by
// mu = 2^25, so that the factor's entries (at most sqrt(mu) = 5793 in
// magnitude) reach up to a tenth of the largest FP16 value (65504) and
// small entries keep their precision instead of underflowing (the scaling
// rule of Higham and Pranesh for squeezing a matrix into half precision,
// applied to the factor); a power of two keeps the scaling exact.  BF16 and
// FP32 have FP32's exponent range and take mu = 1.
static double ir_mu(int fprec) { return fprec == RFP_PREC_FP16 ? 33554432.0 : 1.0; }
// c u of the handle's setting for fprec (FP32, FP16 or BF16)
static double lowp_shift(const rfp_context* h, int fprec)
{
    const int k = fprec == RFP_PREC_FP32 ? 0 : fprec == RFP_PREC_FP16 ? 1 : 2;
    return h->lowp_shift[k] * unit_roundoff(fprec);
}

static int pfsv_ir_impl(rfp_context* h, int fprec, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf,
                        const double* b, int64_t ldb, double* x, int64_t ldx, double tol, int max_iter, int* iter,
                        int* info, hipStream_t st)
{
    if (!h) return RFP_ERR_HANDLE;
    if (fprec != RFP_PREC_FP32 && fprec != RFP_PREC_FP16 && fprec != RFP_PREC_BF16) return -1;
    if (bad_tr(transr)) return -2;
    if (bad_ul(uplo)) return -3;
    if (n < 0) return -4;
    if (nrhs < 0) return -5;
    if (n > 0 && !arf) return -6;
    if (n > 0 && nrhs > 0 && !b) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    if (n > 0 && nrhs > 0 && !x) return -9;
    if (ldx < std::max<int64_t>(1, n)) return -10;
    if (!(tol > 0.0)) return -11;
    if (max_iter < 1) return -12;
    if (!iter) return -13;
    if (!info) return -14;
    DeviceGuard g(h->device);
    if (n == 0 || nrhs == 0) {
        const bool ok0 = set_int(st, iter, 0) == hipSuccess && set_int(st, info, 0) == hipSuccess;
        return ok0 ? 0 : RFP_ERR_RUNTIME;
    }
    RfpBlocks blk;
    rfp_blocks(transr, uplo, n, &blk);
    const int64_t l1 = nleaves(blk.m1, NB), l2 = nleaves(blk.m2, NB);
    const int64_t lv = std::max(nleaves(blk.m1, NB2), nleaves(blk.m2, NB2));
    // Every workspace is sized before anything is enqueued, so that a call on
    // sizes seen before allocates nothing and can be captured in a HIP graph.
    if (prepare(h, std::max<size_t>(size_t(lv) * NB2 * NB2, size_t(l1 + l2) * NB * NB) * sizeof(double)) !=
        hipSuccess)
        return RFP_ERR_RUNTIME;
    if (prepare_flags(h, block_solve_flags(blk.m1, blk.m2, nrhs)) != hipSuccess) return RFP_ERR_RUNTIME;
    const IrSpace probe = ir_space(nullptr, n, nrhs, l1 + l2);
    if (ensure(&h->ir, &h->ir_bytes, probe.bytes) != hipSuccess) return RFP_ERR_RUNTIME;
    IrSpace w = ir_space(h->ir, n, nrhs, l1 + l2);
    RfpView<const double> v = rfp_view(blk, arf);
    RfpView<float> v32 = rfp_view(blk, w.a32);
    RfpView<const float> v32c = rfp_view(blk, (const float*)w.a32);
    IrCtl* c = w.ctl;
    Exec ex{};
    ex.stream = st;
    ex.prof = h->prof;
    ex.tune = h->tune;
    ex.splitk_ws = h->splitk;
    ex.splitk_bytes = h->splitk_bytes;
    Exec ex_run = ex, ex_ir = ex, ex_pcg = ex;
    ex_run.gate = &c->g_run;
    ex_ir.gate = &c->g_ir;
    ex_pcg.gate = &c->g_pcg;
    const double mu = ir_mu(fprec);
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t q) {
        if (q != hipSuccess && e == hipSuccess) e = q;
        return e == hipSuccess;
    };
    // scaled low-precision copy, its factor, and the norms that stay fixed
    ok(ir_start(st, c));
    ok(pf_cast_scale(st, v, v32, 1, mu, lowp_shift(h, fprec), w.s, &c->nonfinite));
    ok(pf_norm(st, v, 1, w.normwork, w.anorm));
    ok(col_max(st, b, ldb, n, nrhs, w.bmax));
    if (!ok(hipGetLastError())) return RFP_ERR_RUNTIME;
    int rc = pftrf_impl<float>(h, transr, uplo, n, w.a32, &c->lp_info, st, nullptr, fprec);
    if (rc != 0) return rc;
    ok(ir_setup_decide(st, c));  // -4 non-finite scaled copy, -3 factor not positive definite
    // inverses of the low-precision factor's 64-row diagonal blocks, once
    ok(trtri_leaves<float>(ex_run, v32c.t1, blk.m1, w.w32));
    ok(trtri_leaves<float>(ex_run, v32c.t2, blk.m2, w.w32 + l1 * NB * NB));
    // M^{-1} = mu D^{-1/2} (Ls Ls^T)^{-1} D^{-1/2}: the low-precision
    // preconditioner, applied as a scaled cast, the two FP32 fused solves and
    // an FP64 rescale into z (or added to z)
    auto prec = [&](const Exec& eg, const double* v_in, double* z, int64_t ldz, bool accumulate) {
        ok(ir_scale_cast(st, v_in, n, w.s, w.r32, n, n, nrhs, eg.gate));
        ok(solve_with_leaves<float>(h, eg, v32c, w.w32, w.r32, n, nrhs));
        ok(ir_update(st, z, ldz, w.s, mu, w.r32, n, n, nrhs, accumulate, eg.gate));
    };
    // The conjugate-gradient steps apply M^{-1} in FP64 arithmetic, with an
    // FP64 copy of the low-precision factor and FP64 inverses of its leaves:
    // the operator is then symmetric to FP64 rounding, where an FP32 solve's
    // rounding (about u_32 / shift relative) would swamp the small eigenvalues
    // of the preconditioned matrix of an ill-conditioned system.  The copy is
    // made once, when the sweeps switch to conjugate gradients, in the
    // fall-back's buffers (not used before the refinement has ended).
    const int64_t nt = n * (n + 1) / 2;
    double* w64 = (double*)h->inv;
    RfpView<const double> v64 = rfp_view(blk, (const double*)w.a64);
    Exec ex_cvt = ex;
    ex_cvt.gate = &c->g_cvt;
    auto widen = [&]() {
        ok(widen_copy(st, w.a64, w.a32, nt, ex_cvt.gate));
        ok(trtri_leaves<double>(ex_cvt, v64.t1, blk.m1, w64));
        ok(trtri_leaves<double>(ex_cvt, v64.t2, blk.m2, w64 + l1 * NB * NB));
    };
    auto prec64 = [&](const Exec& eg, const double* v_in, double* z) {
        ok(row_scale(st, z, n, v_in, n, w.s, 1.0, n, nrhs, eg.gate));
        ok(solve_with_leaves<double>(h, eg, v64, w64, z, n, nrhs));
        ok(row_scale(st, z, n, z, n, w.s, mu, n, nrhs, eg.gate));
    };
    // k steps of preconditioned conjugate gradients on A x = b (FP64
    // throughout), from the true residual r of the current x: the first
    // conjugate-gradient sweep starts the recurrence (p = z), later ones
    // continue it (p = z + beta p, the true residual replacing the recursive
    // one).  rz / rzn name the buffers of r.z across sweeps (every sweep
    // enqueues the same number of swaps, so the names stay consistent).
    double *rz = w.rz0, *rzn = w.rz1;
    auto pcg = [&](int k) {
        const int* gp = ex_pcg.gate;
        ok(ir_copy(st, w.cr, n, w.r, n, n, nrhs, gp));
        prec64(ex_pcg, w.cr, w.cz);
        ok(col_dot(st, w.cr, w.cz, n, n, nrhs, rzn, gp));
        ok(ir_copy(st, w.cp, n, w.cz, n, n, nrhs, &c->g_cvt));
        ok(pcg_dir(st, w.cp, w.cz, rzn, rz, n, n, nrhs, &c->g_cont));
        std::swap(rz, rzn);
        for (int i = 0; i < k; i++) {
            ok(symm_thin(ex_pcg, v, w.cp, n, 1.0, 0.0, w.cq, n, nrhs, w.symm));
            ok(col_dot(st, w.cp, w.cq, n, n, nrhs, w.pq, gp));
            ok(pcg_step(st, x, ldx, w.cr, w.cp, w.cq, rz, w.pq, n, n, nrhs, gp));
            if (i + 1 == k) break;
            prec64(ex_pcg, w.cr, w.cz);
            ok(col_dot(st, w.cr, w.cz, n, n, nrhs, rzn, gp));
            ok(pcg_dir(st, w.cp, w.cz, rzn, rz, n, n, nrhs, gp));
            std::swap(rz, rzn);
        }
    };
    // x = 0, r = b; each sweep corrects x from r, then r = b - A x in FP64
    // and the backward error goes to the decision kernel.  A sweep first
    // applies M^{-1} once (classical refinement); once that stops cutting the
    // backward error by 4x per sweep, sweeps run PCG_STEPS preconditioned
    // conjugate-gradient steps instead.  Both kinds are enqueued for every
    // sweep; the gates let exactly one of them run, and none after the
    // refinement has ended.
    constexpr int PCG_STEPS = 8;
    ok(ir_copy(st, w.r, n, b, ldb, n, nrhs, ex_run.gate));
    ok(ir_copy(st, x, ldx, nullptr, 0, n, nrhs, ex_run.gate));
    for (int it = 1; it <= max_iter && e == hipSuccess; it++) {
        prec(ex_ir, w.r, x, ldx, true);
        widen();
        pcg(PCG_STEPS);
        ok(ir_copy(st, w.r, n, b, ldb, n, nrhs, ex_run.gate));
        ok(symm_thin(ex_run, v, x, ldx, -1.0, 1.0, w.r, n, nrhs, w.symm));
        ok(col_max(st, w.r, n, n, nrhs, w.rmax, ex_run.gate));
        ok(col_max(st, x, ldx, n, nrhs, w.xmax, ex_run.gate));
        ok(backward_error(st, w.rmax, w.xmax, w.bmax, w.anorm, nrhs, &c->eta, ex_run.gate));
        ok(ir_decide(st, c, it, max_iter, tol));
        if (ir_trace()) {
            IrCtl hc;
            if (hipMemcpyAsync(&hc, c, sizeof hc, hipMemcpyDeviceToHost, st) == hipSuccess &&
                hipStreamSynchronize(st) == hipSuccess)
                fprintf(stderr, "rfp_dpfsv_ir: sweep %d backward error %.3e phase %d code %d\n", it, hc.eta, hc.phase,
                        hc.code);
        }
    }
    if (e != hipSuccess) return RFP_ERR_RUNTIME;
    // fall-back, gated on the decision: FP64 factor of a copy of A (its INFO
    // word is the gate, so a failing factor also skips the solve), then the
    // FP64 solve
    ok(gated_copy(st, w.a64, arf, nt, &c->g_fb));
    rc = pftrf_impl<double>(h, transr, uplo, n, w.a64, &c->fb_info, st, nullptr, 0, nullptr, true);
    if (rc != 0) return rc;
    Exec ex_fb = ex;
    ex_fb.gate = &c->fb_info;
    ok(ir_copy(st, x, ldx, b, ldb, n, nrhs, ex_fb.gate));
    ok(trtri_leaves<double>(ex_fb, v64.t1, blk.m1, w64));
    ok(trtri_leaves<double>(ex_fb, v64.t2, blk.m2, w64 + l1 * NB * NB));
    ok(solve_with_leaves<double>(h, ex_fb, v64, w64, x, ldx, nrhs));
    ok(ir_finish(st, c, iter, info));
    return e == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}


// ------------------------------------------ the rest of the routine table
// TFTRI (triangular inversion in RFP): the inverse of the lower view L
// (UPLO='L': the matrix itself; 'U': the stored upper U = L^T, whose inverse
// is the transpose of L's, in the same places) by the inversion stage of
// PFTRI: W11 = L11^{-1}, S <- -S W11, W22 = L22^{-1}, S <- W22 S.
// DIAG='U': the stored diagonal is saved, set to one for the inversion and
// restored.
template <typename T>
static int tftri_impl(rfp_context* h, char transr, char uplo, char diag, int64_t n, T* arf, int* info, hipStream_t s)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (upc(diag) != 'N' && upc(diag) != 'U') return -3;
    if (n < 0) return -4;
    if (n > 0 && !arf) return -5;
    if (!info) return -6;
    DeviceGuard g(h->device);
    if (n == 0) return set_int(s, info, 0) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
    const bool unit = upc(diag) == 'U';
    const size_t dn = unit ? (size_t)n : 0, tri = (size_t)3 * NB2 * NB2;
    if (prepare(h, sizeof(T) * (dn + tri)) != hipSuccess) return RFP_ERR_RUNTIME;
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    RfpView<T> v = rfp_view(b, arf);
    Run<T> r = make_run<T>(h, s, info);
    r.setinfo(info);
    T* dbuf = (T*)h->inv;
    r.tri_scratch = dbuf + dn;
    if (unit) r.chk(unit_diag<T>(s, v, dbuf, false));
    r.trtri_rec(b.m1, v.t1, 0);
    r.trmm_rl(b.m2, b.m1, v.s, v.t1, T(-1));
    r.trtri_rec(b.m2, v.t2, b.m1);
    r.trmm_ll(b.m2, b.m1, v.t2, v.s);
    if (unit) r.chk(unit_diag<T>(s, v, dbuf, true));
    return r.err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

// TFSM (triangular solve with a triangular matrix in RFP).  Every case is a
// solve from the right with the lower view L = [L11 0; L21 L22] (T1, S, T2)
// on a strided view Bv of the right-hand sides:
//   op(A) = L (UPLO='L', TRANS='N' or UPLO='U', TRANS='T') or L^T;
//   SIDE='L': X = op(A)^{-1} B, i.e. Bv = B^T and Bv <- Bv op(A)^{-T};
//   SIDE='R': X = B op(A)^{-1}, Bv = B and Bv <- Bv op(A)^{-1}.
// Bv L^{-T}: X1 = B1 L11^{-T}, X2 = (B2 - X1 L21^T) L22^{-T};
// Bv L^{-1}: X2 = B2 L22^{-1}, X1 = (B1 - X2 L21) L11^{-1};
// each triangle's solve is the 2 x 2 partition down to 64-row leaves, whose
// inverses (unit-diagonal ones for DIAG='U') turn the leaf solves into
// products.  alpha scales B first (alpha = 0: B = 0, A not read).
template <typename T>
static int tfsm_impl(rfp_context* h, char transr, char side, char uplo, char trans, char diag, int64_t m, int64_t n,
                     T alpha, const T* arf, T* bp, int64_t ldb, hipStream_t s)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (upc(side) != 'L' && upc(side) != 'R') return -2;
    if (bad_ul(uplo)) return -3;
    if (bad_tr(trans)) return -4;
    if (upc(diag) != 'N' && upc(diag) != 'U') return -5;
    if (m < 0) return -6;
    if (n < 0) return -7;
    const bool left = upc(side) == 'L';
    const int64_t k = left ? m : n;
    if (k > 0 && alpha != T(0) && !arf) return -9;
    if (m > 0 && n > 0 && !bp) return -10;
    if (ldb < std::max<int64_t>(1, m)) return -11;
    if (m == 0 || n == 0) return 0;
    DeviceGuard g(h->device);
    Mat<T> B{bp, 1, ldb};
    if (alpha == T(0)) return scale2d<T>(s, B, m, n, T(0), false) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
    RfpBlocks b;
    rfp_blocks(transr, uplo, k, &b);
    const int64_t l1 = nleaves(b.m1, NB), l2 = nleaves(b.m2, NB);
    if (prepare(h, size_t(l1 + l2) * NB * NB * sizeof(T)) != hipSuccess) return RFP_ERR_RUNTIME;
    Run<T> r = make_run<T>(h, s, nullptr);
    r.nb = NB;
    RfpView<const T> v = rfp_view(b, arf);
    T* w1 = (T*)h->inv;
    T* w2 = w1 + l1 * NB * NB;
    const bool unit = upc(diag) == 'U';
    if (alpha != T(1)) r.chk(scale2d<T>(s, B, m, n, alpha, false));
    r.chk(trtri_leaves<T>(r.ex, v.t1, b.m1, w1, unit));
    r.chk(trtri_leaves<T>(r.ex, v.t2, b.m2, w2, unit));
    const bool op_lower = (upc(uplo) == 'L') == (upc(trans) == 'N');
    // right-solve with L^{-T} when (left and op(A) = L) or (right and op(A) = L^T)
    const bool with_lt = left == op_lower;
    Mat<T> Bv = left ? B.tr() : B;  // nsys x k
    const int64_t ns = left ? n : m;
    Mat<T> B1 = Bv, B2 = Bv.sub(0, b.m1);
    const Mat<const T> T1 = v.t1, S = v.s, T2 = v.t2;
    if (with_lt) {
        r.trsm_rlt(ns, b.m1, B1, T1, w1);
        r.mm(ns, b.m2, b.m1, T(-1), B1, TRI_NONE, S, TRI_NONE, T(1), B2);
        r.trsm_rlt(ns, b.m2, B2, T2, w2);
    } else {
        r.trsm_rln(ns, b.m2, B2, T2, w2);
        r.mm(ns, b.m1, b.m2, T(-1), B2, TRI_NONE, S.tr(), TRI_NONE, T(1), B1);
        r.trsm_rln(ns, b.m1, B1, T1, w1);
    }
    return r.err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

// SFRK (symmetric rank-k update in RFP): C = alpha op(A) op(A)^T + beta C on
// the three blocks of the lower view, op(A) split into rows [0, m1) and
// [m1, n): T1 <- alpha A1 A1^T + beta T1 and T2 <- alpha A2 A2^T + beta T2
// (lower triangles only), S <- alpha A2 A1^T + beta S.  alpha = 0 or k = 0
// only scales C (A not read); beta = 0 does not read C.
template <typename T>
static int sfrk_impl(rfp_context* h, char transr, char uplo, char trans, int64_t n, int64_t k, T alpha, const T* a,
                     int64_t lda, T beta, T* c, hipStream_t s)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (bad_tr(trans)) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const bool notr = upc(trans) == 'N';
    if (n > 0 && k > 0 && alpha != T(0) && !a) return -7;
    if (lda < std::max<int64_t>(1, notr ? n : k)) return -8;
    if (n > 0 && !c) return -10;
    if (n == 0) return 0;
    DeviceGuard g(h->device);
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    RfpView<T> v = rfp_view(b, c);
    if (k == 0 || alpha == T(0)) {
        if (beta == T(1)) return 0;
        hipError_t e = scale2d<T>(s, v.t1, b.m1, b.m1, beta, true);
        if (e == hipSuccess) e = scale2d<T>(s, v.s, b.m2, b.m1, beta, false);
        if (e == hipSuccess) e = scale2d<T>(s, v.t2, b.m2, b.m2, beta, true);
        return e == hipSuccess ? 0 : RFP_ERR_RUNTIME;
    }
    if (prepare(h, 0) != hipSuccess) return RFP_ERR_RUNTIME;
    Run<T> r = make_run<T>(h, s, nullptr);
    Mat<const T> A = notr ? Mat<const T>{a, 1, lda} : Mat<const T>{a, lda, 1};  // op(A), n x k
    Mat<const T> A1 = A, A2 = A.sub(b.m1, 0);
    r.mm(b.m1, b.m1, k, alpha, A1, TRI_NONE, A1, TRI_NONE, beta, v.t1, true);
    r.mm(b.m2, b.m1, k, alpha, A2, TRI_NONE, A1, TRI_NONE, beta, v.s);
    r.mm(b.m2, b.m2, k, alpha, A2, TRI_NONE, A2, TRI_NONE, beta, v.t2, true);
    return r.err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

// TPTTF / TFTTP (packed <-> RFP).
template <typename T>
static int tpttf_impl(rfp_context* h, char transr, char uplo, int64_t n, const T* ap, T* arf, hipStream_t s,
                      bool to_rfp)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !(to_rfp ? (const void*)ap : (const void*)arf)) return -4;
    if (n > 0 && !(to_rfp ? (const void*)arf : (const void*)ap)) return -5;
    if (n == 0) return 0;
    DeviceGuard g(h->device);
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    return packed_copy<T>(s, rfp_view(b, arf), (T*)ap, upc(uplo) == 'U', to_rfp) == hipSuccess ? 0
                                                                                              : RFP_ERR_RUNTIME;
}

// ------------------------------------------------------------- autotuner
// Candidate configurations of one GEMM shape class are timed on scratch
// operands of the class's largest recorded shape (same orientation, masks
// and precision); the fastest is kept.  Every candidate computes the same
// product, so any choice is correct; only speed differs.
struct TuneShape {
    int dt, lp, sel, clower, tri_a, tri_b;
    int64_t m, n, k;
};

template <typename T>
static float time_gemm(const Exec& ex0, const TuneShape& sh, int tile, int split, T* A, T* B, T* C)
{
    Exec ex = ex0;
    TuneTable one;
    one.force_tile = tile;
    one.force_split = split;
    ex.tune = &one;
    const bool amc = sh.sel & 4, bnc = sh.sel & 2, cmc = sh.sel & 1;
    Mat<const T> Am = amc ? Mat<const T>{A, 1, sh.m} : Mat<const T>{A, sh.k, 1};
    Mat<const T> Bm = bnc ? Mat<const T>{B, 1, sh.n} : Mat<const T>{B, sh.k, 1};
    Mat<T> Cm = cmc ? Mat<T>{C, 1, sh.m} : Mat<T>{C, sh.n, 1};
    auto run = [&]() {
        return gemm<T>(ex, sh.m, sh.n, sh.k, T(-1), Am, sh.tri_a, Bm, sh.tri_b, T(1), Cm, sh.clower != 0, false);
    };
    if (run() != hipSuccess) return -1.f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    constexpr int REPS = 3;
    (void)hipEventRecord(e0, ex.stream);
    for (int i = 0; i < REPS; i++) (void)run();
    (void)hipEventRecord(e1, ex.stream);
    float ms = -1.f;
    if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms < 0 ? -1.f : ms * 1000.f / REPS;
}

static int tune_gemms(rfp_context* h, const std::vector<TuneShape>& shapes, hipStream_t st)
{
    // representative (largest) shape of every class
    std::map<uint64_t, TuneShape> rep;
    for (const TuneShape& sh : shapes) {
        const uint64_t key = tune_gemm_key(sh.dt, sh.lp, sh.sel, sh.clower, sh.m, sh.n, sh.k);
        auto it = rep.find(key);
        if (it == rep.end() || (double)sh.m * sh.n * sh.k > (double)it->second.m * it->second.n * it->second.k)
            rep[key] = sh;
    }
    size_t need = 0;
    for (auto& kv : rep) {
        const TuneShape& sh = kv.second;
        const size_t es = sh.dt ? 4 : 8;
        need = std::max(need, es * (size_t)(sh.m * sh.k + sh.n * sh.k + sh.m * sh.n) + 3 * 256);
    }
    void* buf = nullptr;
    if (need && hipMalloc(&buf, need) != hipSuccess) return RFP_ERR_RUNTIME;
    if (prepare(h, 0) != hipSuccess) {
        (void)hipFree(buf);
        return RFP_ERR_RUNTIME;
    }
    Exec ex{};
    ex.stream = st;
    ex.splitk_ws = h->splitk;
    ex.splitk_bytes = h->splitk_bytes;
    for (auto& kv : rep) {
        const TuneShape& sh = kv.second;
        ex.lowp = sh.lp;
        const size_t es = sh.dt ? 4 : 8;
        char* p = (char*)buf;
        void* A = p;
        void* B = p + ((es * (size_t)(sh.m * sh.k) + 255) & ~(size_t)255);
        void* C = (char*)B + ((es * (size_t)(sh.n * sh.k) + 255) & ~(size_t)255);
        // small finite operands (for FP32 two copies of 2^-7 per 8-byte word);
        // the values do not change the work
        const size_t total = need / 8;
        const uint64_t two_f32 = ((uint64_t)0x3C000000u << 32) | 0x3C000000u;
        double fillv = 1e-3;
        if (sh.dt) std::memcpy(&fillv, &two_f32, sizeof fillv);
        (void)fill_double(st, (double*)buf, (int64_t)total, fillv);
        TuneGemm best{-1, 0, 0.f};
        for (int tile = 0; tile < 4; tile++) {
            for (int split : {0, 1, 2, 4, 8, 16}) {
                if (split > 1 && (sh.k / split < 256 || (size_t)(split * sh.m * sh.n) * es > h->splitk_bytes))
                    continue;
                const float us = sh.dt ? time_gemm<float>(ex, sh, tile, split, (float*)A, (float*)B, (float*)C)
                                       : time_gemm<double>(ex, sh, tile, split, (double*)A, (double*)B, (double*)C);
                if (us > 0 && (best.tile < 0 || us < best.us)) best = TuneGemm{tile, split, us};
            }
        }
        if (best.tile >= 0) h->tune->gemm[kv.first] = best;
    }
    (void)hipStreamSynchronize(st);
    if (buf) (void)hipFree(buf);
    return 0;
}

__global__ void tune_diag_kernel(Mat<double> t1, int64_t m1, Mat<double> t2, int64_t m2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m1) t1.at(i, i) = 1.0;
    else if (i < m1 + m2) t2.at(i - m1, i - m1) = 1.0;
}

static int tune_solve(rfp_context* h, int64_t n, int64_t nrhs, hipStream_t st)
{
    // timing matrix: the identity in RFP (any data does the same work)
    const size_t nt = (size_t)(n * (n + 1) / 2);
    double *arf = nullptr, *b = nullptr;
    if (hipMalloc(&arf, nt * 8) != hipSuccess) return RFP_ERR_RUNTIME;
    if (hipMalloc(&b, (size_t)(n * nrhs) * 8) != hipSuccess) {
        (void)hipFree(arf);
        return RFP_ERR_RUNTIME;
    }
    (void)fill_double(st, arf, (int64_t)nt, 0.0);
    (void)fill_double(st, b, n * nrhs, 1.0);
    RfpBlocks blk;
    rfp_blocks('N', 'L', n, &blk);
    RfpView<double> v = rfp_view(blk, arf);
    hipLaunchKernelGGL(tune_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v.t1, v.m1, v.t2, v.m2);
    int best = 0;
    float best_us = 0.f;
    for (int ncb : {1, 2, 4, 8}) {
        if (ncb > 1 && 16 * (ncb / 2) >= nrhs) break;  // wider than the right-hand sides
        h->tune->solve[tune_solve_key(0, n, nrhs)] = ncb;
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)pftrs_impl<double>(h, 'N', 'L', n, nrhs, arf, b, n, st);
        (void)hipEventRecord(e0, st);
        (void)pftrs_impl<double>(h, 'N', 'L', n, nrhs, arf, b, n, st);
        (void)hipEventRecord(e1, st);
        float ms = -1.f;
        if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (ms > 0 && (best == 0 || ms * 1000.f < best_us)) {
            best = ncb;
            best_us = ms * 1000.f;
        }
    }
    if (best) h->tune->solve[tune_solve_key(0, n, nrhs)] = best;
    else h->tune->solve.erase(tune_solve_key(0, n, nrhs));
    (void)hipStreamSynchronize(st);
    (void)hipFree(arf);
    (void)hipFree(b);
    return 0;
}

// Factorization schedule for order n: the FP64 PFTRF of the identity (the
// same work as any matrix: no kernel depends on the values, and the factor of
// the identity is the identity, so repeated calls need no restore) timed
// under each candidate; the fastest is kept for n's size class.
static int tune_schedule(rfp_context* h, int64_t n, hipStream_t st)
{
    const size_t nt = (size_t)(n * (n + 1) / 2);
    double* arf = nullptr;
    int* info = nullptr;
    if (hipMalloc(&arf, nt * 8) != hipSuccess) return RFP_ERR_RUNTIME;
    if (hipMalloc(&info, sizeof(int)) != hipSuccess) {
        (void)hipFree(arf);
        return RFP_ERR_RUNTIME;
    }
    (void)fill_double(st, arf, (int64_t)nt, 0.0);
    RfpBlocks blk;
    rfp_blocks('N', 'L', n, &blk);
    RfpView<double> v = rfp_view(blk, arf);
    hipLaunchKernelGGL(tune_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v.t1, v.m1, v.t2, v.m2);
    const rfp_schedule_t saved = h->sched;
    const int saved_user = h->sched_user;
    h->sched_user = 1;  // time exactly the candidate
    rfp_schedule_t best = default_schedule();
    float best_ms = -1.f;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (int64_t wide : {int64_t(3072), int64_t(6144), int64_t(12288), INT64_MAX})
        for (int64_t chunk : {int64_t(1024), int64_t(1536), int64_t(2048)})
            for (int64_t pad : {int64_t(0), DEFAULT_LEAF_LDS_PAD}) {
                rfp_schedule_t sc = default_schedule();
                sc.wide_panels_above = wide;
                sc.chunk_max = chunk;
                sc.leaf_lds_pad = pad;
                h->sched = sc;
                (void)pftrf_impl<double>(h, 'N', 'L', n, arf, info, st);
                (void)hipEventRecord(e0, st);
                (void)pftrf_impl<double>(h, 'N', 'L', n, arf, info, st);
                (void)pftrf_impl<double>(h, 'N', 'L', n, arf, info, st);
                (void)hipEventRecord(e1, st);
                float ms = -1.f;
                if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms > 0 && (best_ms < 0 || ms < best_ms)) {
                    best_ms = ms;
                    best = sc;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->sched = saved;
    h->sched_user = saved_user;
    if (best_ms > 0) h->tune->sched[size_bucket(n)] = best;
    (void)hipStreamSynchronize(st);
    (void)hipFree(arf);
    (void)hipFree(info);
    return 0;
}

// GEMM shapes recorded from the drivers' plans (non-in-place products).
static void plan_shapes(char routine, int64_t n, std::vector<TuneShape>& out, int dt, int lp)
{
    for (const char* lay : {"NL", "TU", "NU", "TL"}) {
        int64_t cnt = 0;
        std::vector<rfp_plan_op> ops;
        PlanRec rec{nullptr, 0, 0, sizeof(double)};
        double* arf = plan_base<double>(RFP_PLAN_BUF_ARF);
        int* info = (int*)plan_base<int>(RFP_PLAN_BUF_INFO);
        for (int pass = 0; pass < 2; pass++) {
            rec.ops = pass ? ops.data() : nullptr;
            rec.cap = pass ? cnt : 0;
            rec.count = 0;
            if (routine == 'F') (void)pftrf_impl<double>(nullptr, lay[0], lay[1], n, arf, info, nullptr, &rec);
            else (void)pftri_impl<double>(nullptr, lay[0], lay[1], n, arf, info, nullptr, &rec);
            cnt = rec.count;
            if (!pass) ops.resize((size_t)cnt);
        }
        for (const rfp_plan_op& o : ops) {
            if (o.kind != RFP_PLAN_GEMM || o.inplace || o.m <= 0 || o.n <= 0) continue;
            TuneShape sh;
            sh.dt = dt;
            sh.lp = lp;
            sh.sel = (o.a[2] == 1 ? 4 : 0) | (o.b[2] == 1 ? 2 : 0) | (o.c[2] == 1 ? 1 : 0);
            sh.clower = o.c_lower;
            sh.tri_a = o.tri_a;
            sh.tri_b = o.tri_b;
            sh.m = o.m;
            sh.n = o.n;
            sh.k = o.k;
            out.push_back(sh);
        }
    }
}

}  // namespace rfp

using namespace rfp;

extern "C" {

int rfp_create(rfp_handle_t* h, int device)
{
    if (!h) return -1;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -2;
    rfp_context* c = (rfp_context*)std::calloc(1, sizeof(rfp_context));
    if (!c) return RFP_ERR_RUNTIME;
    c->device = device;
    c->sched = default_schedule();
    c->spin_limit = DEFAULT_SPIN_LIMIT;
    c->lowp_shift[0] = DEFAULT_LOWP_SHIFT_FP32;
    c->lowp_shift[1] = DEFAULT_LOWP_SHIFT_HALF;
    c->lowp_shift[2] = DEFAULT_LOWP_SHIFT_HALF;
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->cus <= 0)
        c->cus = 256;
    *h = c;
    return 0;
}

int rfp_destroy(rfp_handle_t h)
{
    if (!h) return RFP_ERR_HANDLE;
    {
        DeviceGuard g(h->device);
        (void)hipDeviceSynchronize();
        if (h->splitk) (void)hipFree(h->splitk);
        if (h->splitk2) (void)hipFree(h->splitk2);
        if (h->inv) (void)hipFree(h->inv);
        if (h->flags) (void)hipFree(h->flags);
        if (h->ctl) (void)hipFree(h->ctl);
        if (h->ir) (void)hipFree(h->ir);
        if (h->zwork) (void)hipFree(h->zwork);
        if (h->bat) (void)hipFree(h->bat);
        delete h->tune;
        for (int i = 0; i < h->nev; i++) (void)hipEventDestroy(h->ev[i]);
        if (h->aux) (void)hipStreamDestroy(h->aux);
        if (h->join) (void)hipEventDestroy(h->join);
        if (h->aux2) (void)hipStreamDestroy(h->aux2);
        delete h->prof;
    }
    std::free(h);
    return 0;
}

int rfp_profile_enable(rfp_handle_t h, int on)
{
    if (!h) return RFP_ERR_HANDLE;
    DeviceGuard g(h->device);
    if (on && !h->prof) {
        h->prof = new Profiler();
        if (h->prof->reserve() != hipSuccess) return RFP_ERR_RUNTIME;
    }
    if (!on && h->prof) {
        (void)hipDeviceSynchronize();
        delete h->prof;
        h->prof = nullptr;
    }
    return 0;
}

int rfp_profile_read(rfp_handle_t h, rfp_profile_entry* out, int cap, int* count)
{
    if (!h) return RFP_ERR_HANDLE;
    if (!count || cap < 0 || (cap > 0 && !out)) return -4;
    *count = 0;
    if (!h->prof) return 0;
    DeviceGuard g(h->device);
    Profiler* p = h->prof;
    p->fold();
    int i = 0;
    for (const auto& kv : p->agg) {
        if (i < cap) {
            rfp_profile_entry* e = &out[i];
            std::memset(e, 0, sizeof(*e));
            std::strncpy(e->name, kv.first.c_str(), sizeof(e->name) - 1);
            e->launches = kv.second.launches;
            e->total_ms = kv.second.ms;
            e->flops = kv.second.flops;
            e->bytes = kv.second.bytes;
        }
        i++;
    }
    *count = i;
    const hipError_t err = p->err;
    if (i <= cap) {  // everything delivered: start new totals
        p->agg.clear();
        p->err = hipSuccess;
    }
    return err == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

int rfp_dtrttf(rfp_handle_t h, char transr, char uplo, int64_t n, const double* a, int64_t lda, double* arf,
               hipStream_t stream)
{
    return trttf_impl<double>(h, transr, uplo, n, a, lda, arf, stream, true);
}

int rfp_dtfttr(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, double* a, int64_t lda,
               hipStream_t stream)
{
    return trttf_impl<double>(h, transr, uplo, n, a, lda, (double*)arf, stream, false);
}

int rfp_dpftrf(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream)
{
    return pftrf_impl<double>(h, transr, uplo, n, arf, info, stream);
}

int rfp_dpftrs(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf, double* b,
               int64_t ldb, hipStream_t stream)
{
    return pftrs_impl<double>(h, transr, uplo, n, nrhs, arf, b, ldb, stream);
}

int rfp_dpftri(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream)
{
    return pftri_impl<double>(h, transr, uplo, n, arf, info, stream);
}

// ------------------------------------------------- complex Hermitian path
static bool zbad_tr(char c) { return upc(c) != 'N' && upc(c) != 'C'; }

static int zconvert_impl(rfp_context* h, char transr, char uplo, int64_t n, double* a, int64_t lda, double* arf,
                         hipStream_t s, bool to_rfp)
{
    if (!h) return RFP_ERR_HANDLE;
    if (zbad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n == 0) return 0;
    // TRTTF (.., A=4, LDA=5, ARF=6); TFTTR (.., ARF=4, A=5, LDA=6)
    if (to_rfp) {
        if (!a) return -4;
        if (lda < std::max<int64_t>(1, n)) return -5;
        if (!arf) return -6;
    } else {
        if (!arf) return -4;
        if (!a) return -5;
        if (lda < std::max<int64_t>(1, n)) return -6;
    }
    DeviceGuard g(h->device);
    ZRfpViews v;
    zrfp_views(transr, uplo, n, (double2*)arf, &v);
    return zconvert(s, v, upc(uplo) == 'U', (double2*)a, lda, to_rfp) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

static hipError_t zensure(rfp_context* h, int64_t n, int64_t nrhs, bool inverse = false)
{
    return ensure(&h->zwork, &h->zwork_bytes, zwork_elems(n, nrhs, inverse) * sizeof(double2));
}

int rfp_ztrttf(rfp_handle_t h, char transr, char uplo, int64_t n, const double* a, int64_t lda, double* arf,
               hipStream_t stream)
{
    return zconvert_impl(h, transr, uplo, n, (double*)a, lda, arf, stream, true);
}

int rfp_ztfttr(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, double* a, int64_t lda,
               hipStream_t stream)
{
    return zconvert_impl(h, transr, uplo, n, a, lda, (double*)arf, stream, false);
}

int rfp_zpftrf(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (zbad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !arf) return -4;
    if (!info) return -5;
    DeviceGuard g(h->device);
    if (set_int(stream, info, 0) != hipSuccess) return RFP_ERR_RUNTIME;
    if (n == 0) return 0;
    if (zensure(h, n, 0) != hipSuccess) return RFP_ERR_RUNTIME;
    ZRfpViews v;
    zrfp_views(transr, uplo, n, (double2*)arf, &v);
    return zpftrf_run(stream, v, (double2*)h->zwork, info) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

int rfp_zpftrs(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf, double* b,
               int64_t ldb, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (zbad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && !arf) return -5;
    if (n > 0 && nrhs > 0 && !b) return -6;
    if (ldb < std::max<int64_t>(1, n)) return -7;
    if (n == 0 || nrhs == 0) return 0;
    DeviceGuard g(h->device);
    if (zensure(h, n, nrhs) != hipSuccess) return RFP_ERR_RUNTIME;
    ZRfpViews v;
    zrfp_views(transr, uplo, n, (double2*)arf, &v);
    return zpftrs_run(stream, v, (double2*)b, ldb, nrhs, (double2*)h->zwork, nullptr) == hipSuccess ? 0
                                                                                                  : RFP_ERR_RUNTIME;
}

int rfp_zpftri(rfp_handle_t h, char transr, char uplo, int64_t n, double* arf, int* info, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (zbad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !arf) return -4;
    if (!info) return -5;
    DeviceGuard g(h->device);
    if (set_int(stream, info, 0) != hipSuccess) return RFP_ERR_RUNTIME;
    if (n == 0) return 0;
    if (zensure(h, n, 0, true) != hipSuccess) return RFP_ERR_RUNTIME;
    ZRfpViews v;
    zrfp_views(transr, uplo, n, (double2*)arf, &v);
    return zpftri_run(stream, v, (double2*)h->zwork, info) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

int rfp_dtftri(rfp_handle_t h, char transr, char uplo, char diag, int64_t n, double* arf, int* info,
               hipStream_t stream)
{
    return tftri_impl<double>(h, transr, uplo, diag, n, arf, info, stream);
}

int rfp_dtfsm(rfp_handle_t h, char transr, char side, char uplo, char trans, char diag, int64_t m, int64_t n,
              double alpha, const double* arf, double* b, int64_t ldb, hipStream_t stream)
{
    return tfsm_impl<double>(h, transr, side, uplo, trans, diag, m, n, alpha, arf, b, ldb, stream);
}

int rfp_dsfrk(rfp_handle_t h, char transr, char uplo, char trans, int64_t n, int64_t k, double alpha,
              const double* a, int64_t lda, double beta, double* c, hipStream_t stream)
{
    return sfrk_impl<double>(h, transr, uplo, trans, n, k, alpha, a, lda, beta, c, stream);
}

int rfp_dtpttf(rfp_handle_t h, char transr, char uplo, int64_t n, const double* ap, double* arf, hipStream_t stream)
{
    return tpttf_impl<double>(h, transr, uplo, n, ap, arf, stream, true);
}

int rfp_dtfttp(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, double* ap, hipStream_t stream)
{
    return tpttf_impl<double>(h, transr, uplo, n, ap, (double*)arf, stream, false);
}

int rfp_strttf(rfp_handle_t h, char transr, char uplo, int64_t n, const float* a, int64_t lda, float* arf,
               hipStream_t stream)
{
    return trttf_impl<float>(h, transr, uplo, n, a, lda, arf, stream, true);
}

int rfp_stfttr(rfp_handle_t h, char transr, char uplo, int64_t n, const float* arf, float* a, int64_t lda,
               hipStream_t stream)
{
    return trttf_impl<float>(h, transr, uplo, n, a, lda, (float*)arf, stream, false);
}

int rfp_spftrf(rfp_handle_t h, char transr, char uplo, int64_t n, float* arf, int* info, hipStream_t stream)
{
    return pftrf_impl<float>(h, transr, uplo, n, arf, info, stream);
}

int rfp_spftrs(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, const float* arf, float* b,
               int64_t ldb, hipStream_t stream)
{
    return pftrs_impl<float>(h, transr, uplo, n, nrhs, arf, b, ldb, stream);
}

int rfp_spftri(rfp_handle_t h, char transr, char uplo, int64_t n, float* arf, int* info, hipStream_t stream)
{
    return pftri_impl<float>(h, transr, uplo, n, arf, info, stream);
}

int rfp_plan(char routine, char transr, char uplo, int64_t n, int64_t nrhs, int64_t ldb,
             const rfp_schedule_t* sched, rfp_plan_op* ops, int64_t cap, int64_t* count)
{
    if (!count || cap < 0 || (cap > 0 && !ops)) return -8;
    if (sched && bad_schedule(*sched)) return -7;
    PlanRec rec{ops, cap, 0, sizeof(double)};
    double* arf = plan_base<double>(RFP_PLAN_BUF_ARF);
    double* b = plan_base<double>(RFP_PLAN_BUF_B);
    int* info = (int*)plan_base<int>(RFP_PLAN_BUF_INFO);
    int rc;
    switch (upc(routine)) {
        case 'F': rc = pftrf_impl<double>(nullptr, transr, uplo, n, arf, info, nullptr, &rec, 0, sched); break;
        case 'S': rc = pftrs_impl<double>(nullptr, transr, uplo, n, nrhs, arf, b, ldb, nullptr, &rec); break;
        case 'I': rc = pftri_impl<double>(nullptr, transr, uplo, n, arf, info, nullptr, &rec); break;
        default: return -1;
    }
    *count = rec.count;
    return rc;
}

int rfp_dpfcast_s(rfp_handle_t h, char transr, char uplo, int64_t n, const double* arf, int scale, double mu,
                  double shift, double* s, float* arf32, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (n > 0 && !arf) return -4;
    if (!(mu > 0.0) || mu > 1e300) return -6;
    if (!(shift >= 0.0) || shift > 1e300) return -7;
    if (n > 0 && !s) return -8;
    if (n > 0 && !arf32) return -9;
    if (n == 0) return 0;
    DeviceGuard g(h->device);
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    return pf_cast_scale(stream, rfp_view(b, arf), rfp_view(b, arf32), scale, mu, shift, s) == hipSuccess ? 0
                                                                                                 : RFP_ERR_RUNTIME;
}

int rfp_dlansf(rfp_handle_t h, char norm, char transr, char uplo, int64_t n, const double* arf, double* out,
               hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    const int c = upc(norm);
    const int which = c == 'M' ? 0 : (c == '1' || c == 'O' || c == 'I') ? 1 : (c == 'F' || c == 'E') ? 2 : -1;
    if (which < 0) return -1;
    if (bad_tr(transr)) return -2;
    if (bad_ul(uplo)) return -3;
    if (n < 0) return -4;
    if (n > 0 && !arf) return -5;
    if (!out) return -6;
    DeviceGuard g(h->device);
    if (n == 0) return fill_double(stream, out, 1, 0.0) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
    // the norm's scratch lives in the refinement workspace
    const size_t need = sizeof(double) * (size_t)(n + 3);
    if (ensure(&h->ir, &h->ir_bytes, need) != hipSuccess) return RFP_ERR_RUNTIME;
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    return pf_norm(stream, rfp_view(b, arf), which, (double*)h->ir, out) == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

int rfp_dsfmv(rfp_handle_t h, char transr, char uplo, int64_t n, int64_t nrhs, double alpha, const double* arf,
              const double* x, int64_t ldx, double beta, double* y, int64_t ldy, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (bad_tr(transr)) return -1;
    if (bad_ul(uplo)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && nrhs > 0 && !arf) return -6;
    if (n > 0 && nrhs > 0 && !x) return -7;
    if (ldx < std::max<int64_t>(1, n)) return -8;
    if (n > 0 && nrhs > 0 && !y) return -10;
    if (ldy < std::max<int64_t>(1, n)) return -11;
    if (n == 0 || nrhs == 0) return 0;
    DeviceGuard g(h->device);
    RfpBlocks b;
    rfp_blocks(transr, uplo, n, &b);
    // the product's partial sums live in the refinement workspace
    if (ensure(&h->ir, &h->ir_bytes, symm_thin_workspace(b.m1, b.m2)) != hipSuccess) return RFP_ERR_RUNTIME;
    Exec ex{};
    ex.stream = stream;
    ex.prof = h->prof;
    return symm_thin(ex, rfp_view(b, arf), x, ldx, alpha, beta, y, ldy, nrhs, (double*)h->ir) == hipSuccess
               ? 0
               : RFP_ERR_RUNTIME;
}

int rfp_spftrf_mp(rfp_handle_t h, int fprec, char transr, char uplo, int64_t n, float* arf, int* info,
                  hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (fprec != RFP_PREC_FP32 && fprec != RFP_PREC_FP16 && fprec != RFP_PREC_BF16) return -1;
    const int rc = pftrf_impl<float>(h, transr, uplo, n, arf, info, stream, nullptr, fprec);
    return rc < 0 && rc > -100 ? rc - 1 : rc;  // argument positions shift by the leading FPREC
}

int rfp_dpfsv_ir(rfp_handle_t h, int fprec, char transr, char uplo, int64_t n, int64_t nrhs, const double* arf,
                 const double* b, int64_t ldb, double* x, int64_t ldx, double tol, int max_iter, int* iter, int* info,
                 hipStream_t stream)
{
    return pfsv_ir_impl(h, fprec, transr, uplo, n, nrhs, arf, b, ldb, x, ldx, tol, max_iter, iter, info, stream);
}

int rfp_pfsv_vbatched(rfp_handle_t h, int fprec, int64_t batch, const rfp_sys_t* sys, const rfp_sys_t* sys_host,
                      double* arf_pool, double* b_pool, int do_pftri, double tol, int max_iter, int* info, int* iter,
                      hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    int mode;
    switch (fprec) {
        case RFP_PREC_FP64: mode = 0; break;
        case RFP_PREC_FP32: mode = 1; break;
        case RFP_PREC_FP16: mode = 2; break;
        case RFP_PREC_BF16: mode = 3; break;
        default: return -1;
    }
    if (batch < 0) return -2;
    if (batch == 0) return 0;
    if (!sys) return -3;
    if (!arf_pool) return -5;
    if (!b_pool) return -6;
    if (mode != 0 && !(tol > 0.0)) return -8;
    if (mode != 0 && max_iter < 1) return -9;
    if (!info) return -10;
    if (!iter) return -11;
    DeviceGuard g(h->device);
    const int pftri = do_pftri ? 1 : 0;
    const int mi = mode ? max_iter : 1;
    // Sizes: the per-system scratch and the task count of the systems with
    // n > 256 come from the host copy of the table (without it such systems
    // are refused); the per-workgroup scratch is always sized for two
    // workgroups per compute unit, the most that run at once, so it does not
    // change with the batch's make-up.  A batch of one-task systems only
    // (n <= 256) runs two workgroups per compute unit; one with larger
    // systems runs one, whose tile tasks need the full register budget.
    int64_t tasks = batch, sysbytes = 0;
    bool all_small = true;
    if (sys_host) {
        sysbytes = batched_plan_host(sys_host, batch, mode, pftri, mi, &tasks);
        for (int64_t i = 0; i < batch && all_small; i++) all_small = sys_host[i].n <= 256;
    }
    const int occ = all_small ? 2 : 1;
    const int wgs = occ * h->cus;
    const size_t a_ctl = 256, a_st = batched_state_bytes(batch);
    const size_t a_q = (sizeof(unsigned long long) * (size_t)(tasks + 1) + 255) & ~(size_t)255;
    const size_t a_wg = (size_t)(2 * h->cus) * batched_wg_scratch_bytes();
    const size_t need = a_ctl + a_st + a_q + a_wg + (size_t)sysbytes;
    if (ensure(&h->bat, &h->bat_bytes, need) != hipSuccess) return RFP_ERR_RUNTIME;
    char* base = (char*)h->bat;
    Exec ex{};
    ex.stream = stream;
    ex.prof = h->prof;
    const double shift = mode ? lowp_shift(h, fprec) : 0.0;
    const hipError_t e = batched_solve(ex, sys, batch, arf_pool, b_pool, mode, pftri, tol, shift, mi, info, iter,
                                       base + a_ctl + a_st + a_q, wgs, occ, base + a_ctl + a_st + a_q + a_wg,
                                       sys_host ? (int64_t)(h->bat_bytes - (a_ctl + a_st + a_q + a_wg)) : 0,
                                       base + a_ctl,
                                       (unsigned long long*)(base + a_ctl + a_st), tasks + 1,
                                       (unsigned long long*)base);
    return e == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

int rfp_autotune(rfp_handle_t h, int64_t n, int64_t nrhs, int precs, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (n < 1) return -1;
    if (nrhs < 0) return -2;
    if (precs <= 0 || precs > 31) return -3;
    DeviceGuard g(h->device);
    if (!h->tune) h->tune = new TuneTable();
    std::vector<TuneShape> shapes;
    if (precs & RFP_TUNE_FP64) {
        plan_shapes('F', n, shapes, 0, 0);
        plan_shapes('I', n, shapes, 0, 0);
    }
    if (precs & RFP_TUNE_FP32) plan_shapes('F', n, shapes, 1, 0);
    if (precs & RFP_TUNE_FP16) plan_shapes('F', n, shapes, 1, 1);
    if (precs & RFP_TUNE_BF16) plan_shapes('F', n, shapes, 1, 2);
    int rc = tune_gemms(h, shapes, stream);
    if (rc == 0 && nrhs > 0 && (precs & RFP_TUNE_FP64)) rc = tune_solve(h, n, nrhs, stream);
    if (rc == 0 && (precs & RFP_TUNE_SCHEDULE)) rc = tune_schedule(h, n, stream);
    return rc;
}

int rfp_set_schedule(rfp_handle_t h, const rfp_schedule_t* sched)
{
    if (!h) return RFP_ERR_HANDLE;
    const rfp_schedule_t sc = sched ? *sched : default_schedule();
    if (bad_schedule(sc)) return -2;
    h->sched = sc;
    h->sched_user = sched ? 1 : 0;
    return 0;
}

int rfp_get_schedule(rfp_handle_t h, rfp_schedule_t* sched)
{
    if (!h) return RFP_ERR_HANDLE;
    if (!sched) return -2;
    *sched = h->sched;
    return 0;
}

__global__ void take_status_kernel(int* word, int* out)
{
    if (threadIdx.x == 0) {
        *out = *word;
        *word = 0;
    }
}

int rfp_solve_status(rfp_handle_t h, int* status, hipStream_t stream)
{
    if (!h) return RFP_ERR_HANDLE;
    if (!status) return -2;
    DeviceGuard g(h->device);
    if (!h->ctl && prepare_flags(h, 1) != hipSuccess) return RFP_ERR_RUNTIME;
    hipLaunchKernelGGL(take_status_kernel, dim3(1), dim3(64), 0, stream, h->ctl + 1, status);
    return hipGetLastError() == hipSuccess ? 0 : RFP_ERR_RUNTIME;
}

static int shift_slot(int fprec)
{
    return fprec == RFP_PREC_FP32 ? 0 : fprec == RFP_PREC_FP16 ? 1 : fprec == RFP_PREC_BF16 ? 2 : -1;
}

int rfp_set_lowp_shift(rfp_handle_t h, int fprec, double c)
{
    if (!h) return RFP_ERR_HANDLE;
    const int k = shift_slot(fprec);
    if (k < 0) return -2;
    if (!(c >= 0.0) || c > 1e6) return -3;
    h->lowp_shift[k] = c;
    return 0;
}

int rfp_get_lowp_shift(rfp_handle_t h, int fprec, double* c)
{
    if (!h) return RFP_ERR_HANDLE;
    const int k = shift_slot(fprec);
    if (k < 0) return -2;
    if (!c) return -3;
    *c = h->lowp_shift[k];
    return 0;
}

int rfp_set_solve_wait_limit(rfp_handle_t h, int64_t polls)
{
    if (!h) return RFP_ERR_HANDLE;
    h->spin_limit = polls < 0 ? DEFAULT_SPIN_LIMIT : (int)std::min<int64_t>(polls, INT32_MAX);
    return 0;
}

int rfp_tune_count(rfp_handle_t h)
{
    if (!h) return RFP_ERR_HANDLE;
    return h->tune ? (int)(h->tune->gemm.size() + h->tune->solve.size() + h->tune->sched.size()) : 0;
}

int rfp_tune_clear(rfp_handle_t h)
{
    if (!h) return RFP_ERR_HANDLE;
    delete h->tune;
    h->tune = nullptr;
    return 0;
}

int rfp_tune_force(rfp_handle_t h, int tile, int split)
{
    if (!h) return RFP_ERR_HANDLE;
    if (tile < -1 || tile > 3) return -1;
    if (split < 0 || split > 32) return -2;
    if (!h->tune) h->tune = new TuneTable();
    h->tune->force_tile = tile;
    h->tune->force_split = split;
    return 0;
}

int rfp_tune_save(rfp_handle_t h, const char* path)
{
    if (!h) return RFP_ERR_HANDLE;
    if (!path) return -1;
    FILE* f = fopen(path, "w");
    if (!f) return -1;
    fprintf(f, "{\"rfp_tune\": 1,\n \"gemm\": [\n");
    size_t i = 0;
    if (h->tune)
        for (auto& kv : h->tune->gemm) {
            const uint64_t k = kv.first;
            fprintf(f, "  {\"key\": %llu, \"dt\": %d, \"lp\": %d, \"sel\": %d, \"clower\": %d, \"mb\": %d, \"nb\": %d, "
                       "\"kb\": %d, \"tile\": %d, \"split\": %d, \"us\": %.3f}%s\n",
                    (unsigned long long)k, (int)(k >> 40), (int)((k >> 36) & 15), (int)((k >> 32) & 15),
                    (int)((k >> 30) & 1), (int)((k >> 20) & 1023), (int)((k >> 10) & 1023), (int)(k & 1023),
                    kv.second.tile, kv.second.split, kv.second.us, ++i < h->tune->gemm.size() ? "," : "");
        }
    fprintf(f, " ],\n \"solve\": [\n");
    i = 0;
    if (h->tune)
        for (auto& kv : h->tune->solve)
            fprintf(f, "  {\"key\": %llu, \"ncb\": %d}%s\n", (unsigned long long)kv.first, kv.second,
                    ++i < h->tune->solve.size() ? "," : "");
    fprintf(f, " ],\n \"sched\": [\n");
    i = 0;
    if (h->tune)
        for (auto& kv : h->tune->sched)
            fprintf(f, "  {\"bucket\": %d, \"wide_panels_above\": %lld, \"chunk_max\": %lld, "
                       "\"lookahead_wait_below\": %lld, \"leaf_lds_pad\": %lld, \"wide_panel_cols\": %lld}%s\n",
                    kv.first, (long long)kv.second.wide_panels_above, (long long)kv.second.chunk_max,
                    (long long)kv.second.lookahead_wait_below, (long long)kv.second.leaf_lds_pad,
                    (long long)kv.second.wide_panel_cols, ++i < h->tune->sched.size() ? "," : "");
    fprintf(f, " ]\n}\n");
    return fclose(f) == 0 ? 0 : -1;
}

int rfp_tune_load(rfp_handle_t h, const char* path)
{
    if (!h) return RFP_ERR_HANDLE;
    if (!path) return -1;
    FILE* f = fopen(path, "r");
    if (!f) return -1;
    TuneTable* t = new TuneTable();
    char line[512];
    bool ok = true, in_solve = false;
    while (fgets(line, sizeof line, f)) {
        if (strstr(line, "\"solve\"")) in_solve = true;
        if (const char* qs = strstr(line, "{\"bucket\":")) {
            int bucket;
            long long w, c, l, p, pc;
            rfp_schedule_t sc;
            if (sscanf(qs, "{\"bucket\": %d, \"wide_panels_above\": %lld, \"chunk_max\": %lld, "
                           "\"lookahead_wait_below\": %lld, \"leaf_lds_pad\": %lld, \"wide_panel_cols\": %lld}",
                       &bucket, &w, &c, &l, &p, &pc) != 6) {
                ok = false;
                break;
            }
            sc.wide_panels_above = w;
            sc.chunk_max = c;
            sc.lookahead_wait_below = l;
            sc.leaf_lds_pad = p;
            sc.wide_panel_cols = pc;
            if (bad_schedule(sc)) {
                ok = false;
                break;
            }
            t->sched[bucket] = sc;
            continue;
        }
        const char* q = strstr(line, "{\"key\":");
        if (!q) continue;
        unsigned long long key;
        if (!in_solve) {
            int dt, lp, sel, cl, mb, nb, kb, tile, split;
            float us;
            if (sscanf(q, "{\"key\": %llu, \"dt\": %d, \"lp\": %d, \"sel\": %d, \"clower\": %d, \"mb\": %d, \"nb\": %d, "
                          "\"kb\": %d, \"tile\": %d, \"split\": %d, \"us\": %f}",
                       &key, &dt, &lp, &sel, &cl, &mb, &nb, &kb, &tile, &split, &us) != 11 ||
                tile < 0 || tile > 3 || split < 0 || split > 32) {
                ok = false;
                break;
            }
            t->gemm[(uint64_t)key] = TuneGemm{tile, split, us};
        } else {
            int ncb;
            if (sscanf(q, "{\"key\": %llu, \"ncb\": %d}", &key, &ncb) != 2 ||
                !(ncb == 1 || ncb == 2 || ncb == 4 || ncb == 8)) {
                ok = false;
                break;
            }
            t->solve[(uint64_t)key] = ncb;
        }
    }
    fclose(f);
    if (!ok) {
        delete t;
        return -2;
    }
    delete h->tune;
    h->tune = t;
    return 0;
}

}  // extern "C"
