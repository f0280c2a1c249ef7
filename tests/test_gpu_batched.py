"""GPU parity of the batched solver against the oracle, per system, through
the C ABI: one-task systems (n <= 256) and tiled systems (n > 256, their
factorization, refinement and inversion spread over many workgroups), FP64
and the low-precision modes; and replay of the call captured in a HIP graph."""
import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import host

pytestmark = pytest.mark.gpu

LAYOUTS = oracle.LAYOUTS


@pytest.fixture(scope="module")
def h():
    return rfp.Handle(0)


def make_batch(ns, lays, nrs, seed, kappa=None, bad=()):
    """Pools and per-system data: A_i = M M^T / n_i + I (or cond ~ kappa)."""
    systems, arfs, Bs, As = [], [], [], []
    ao = bo = 0
    for idx, (n, li, nr) in enumerate(zip(ns, lays, nrs)):
        t, u = LAYOUTS[li]
        n, nr = int(n), int(nr)
        if kappa is None:
            A, B = synth.spd(n, nrhs=nr, seed=seed + idx) if n > 0 else (np.zeros((0, 0)), np.zeros((0, nr)))
        else:
            k = max(1, n // 2)
            A, B = synth.spd(n, k=k, alpha=synth.cond_alpha(n, k, kappa), nrhs=nr, seed=seed + idx)
        if idx in bad and n > 2:
            A = A.copy()
            A[n // 2, n // 2] = -1.0
        arf = oracle.trttf(t, u, A) if n > 0 else np.zeros(0)
        ldb = max(1, n) + (idx % 3)
        Bp = np.zeros((ldb, nr))
        Bp[:n] = B
        systems.append((n, ao, bo, ldb, nr, t, u))
        arfs.append(arf)
        Bs.append(Bp)
        As.append(A)
        ao += arf.size + 7  # gaps between systems stay untouched
        bo += ldb * nr + 5
    arf_pool = np.full(ao + 1, 123.0)
    b_pool = np.full(bo + 1, 321.0)
    for (n, a0, b0, ldb, nr, t, u), arf, Bp in zip(systems, arfs, Bs):
        arf_pool[a0:a0 + arf.size] = arf
        b_pool[b0:b0 + ldb * nr] = Bp.ravel(order="F")
    return systems, arfs, As, arf_pool, b_pool


def run_batch(h, mode, systems, arf_pool, b_pool, pftri=False, tol=1e-14, host_table=True, max_iter=20):
    raw = rfp.sys_table(systems)
    table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()
    ap = torch.from_numpy(arf_pool.copy()).cuda()
    bp = torch.from_numpy(b_pool.copy()).cuda()
    info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    it = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    rfp.rfp_pfsv_vbatched(h, mode, len(systems), table, ap, bp, info, it, sys_host=raw if host_table else None,
                          do_pftri=pftri, tol=tol, max_iter=max_iter)
    return host(ap), host(bp), host(info), host(it)


def _sys_b(bp, sysd):
    n, a0, b0, ldb, nr, t, u = sysd
    return bp[b0:b0 + ldb * nr].reshape(nr, ldb).T


@pytest.mark.parametrize("pftri", [False, True])
def test_batched_fp64_matches_oracle(h, pftri):
    ns, lays, nrs = synth.batch_sizes(60, 1, 256, 1, 20, seed=41)
    ns = np.concatenate([ns, [0, 1, 2, 128, 129, 255, 256]])
    lays = np.concatenate([lays, [0, 1, 2, 3, 0, 1, 2]])
    nrs = np.concatenate([nrs, [3, 1, 2, 17, 16, 5, 33]])
    systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=100)
    ap, bp, info, it = run_batch(h, rfp.PREC_FP64, systems, arf_pool, b_pool, pftri=pftri)
    assert np.all(info == 0) and np.all(it == 0)
    for sysd, arf in zip(systems, arfs):
        n, a0, b0, ldb, nr, t, u = sysd
        if n == 0:
            continue
        f, _ = oracle.pftrf(t, u, n, arf.copy())
        B = b_pool[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
        want = oracle.pftrs(t, u, n, f, np.asfortranarray(B))
        got = _sys_b(bp, sysd)
        assert oracle.rel_fro(got[:n], want) <= 1e-12 * n, (n, t, u)
        assert np.all(got[n:] == 0.0)  # rows beyond n untouched (they were zero)
        ref = oracle.pftri(t, u, n, f)[0] if pftri else f
        assert oracle.rel_fro(ap[a0:a0 + arf.size], ref) <= 1e-12 * n, (n, t, u)
    # nothing outside the systems was written
    used_a = np.zeros(arf_pool.size, bool)
    used_b = np.zeros(b_pool.size, bool)
    for (n, a0, b0, ldb, nr, t, u), arf in zip(systems, arfs):
        used_a[a0:a0 + arf.size] = True
        used_b[b0:b0 + ldb * nr] = True
    assert np.all(ap[~used_a] == 123.0) and np.all(bp[~used_b] == 321.0)


def test_batched_fp32_refinement(h):
    ns, lays, nrs = synth.batch_sizes(40, 16, 256, 1, 8, seed=4)
    systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=200, kappa=1e3)
    ap, bp, info, it = run_batch(h, rfp.PREC_FP32, systems, arf_pool, b_pool)
    assert np.all(info == 0)
    assert np.all(it > 0), it
    for sysd, arf in zip(systems, arfs):
        n, a0, b0, ldb, nr, t, u = sysd
        B = b_pool[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
        X = _sys_b(bp, sysd)[:n]
        assert oracle.backward_error(t, u, n, arf, B, X) <= 1e-14
        assert np.array_equal(ap[a0:a0 + arf.size], arf)  # the FP64 matrix is untouched


def test_batched_not_positive_definite(h):
    """A[n/2, n/2] = -1 in a one-task system (n = 100) and a tiled one
    (n = 700): INFO = n/2 + 1 in both; in the low-precision modes the scaled
    copy is not finite (-4) and the FP64 fall-back reports the same INFO.
    Without the host table the tiled systems are refused and left alone."""
    ns, lays, nrs = [40, 100, 200, 300, 700], [0, 3, 1, 2, 1], [2, 1, 3, 1, 2]
    for mode in [rfp.PREC_FP64, rfp.PREC_FP32, rfp.PREC_FP16]:
        systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=300, bad=(1, 4))
        ap, bp, info, it = run_batch(h, mode, systems, arf_pool, b_pool)
        assert info[0] == 0 and info[2] == 0 and info[3] == 0
        assert info[1] == 51 and info[4] == 351
        if mode != rfp.PREC_FP64:
            assert it[1] == -4 and it[4] == -4 and it[0] > 0 and it[2] > 0 and it[3] > 0
    systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=300)
    ap, bp, info, it = run_batch(h, rfp.PREC_FP64, systems, arf_pool, b_pool, host_table=False)
    assert list(info) == [0, 0, 0, -1, -1]
    for q in (3, 4):
        a0, size = systems[q][1], arfs[q].size
        assert np.array_equal(ap[a0:a0 + size], arfs[q])


def test_batched_graph_replay(h):
    """The call captured in a HIP graph and replayed: every replay, with its
    inputs restored eagerly in between, equals the eager result."""
    ns, lays, nrs = synth.batch_sizes(50, 16, 256, 1, 8, seed=9)
    ns = np.concatenate([ns, [300, 600]])
    lays = np.concatenate([lays, [1, 2]])
    nrs = np.concatenate([nrs, [3, 2]])
    systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=400)
    raw = rfp.sys_table(systems)
    table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()
    a0 = torch.from_numpy(arf_pool).cuda()
    b0 = torch.from_numpy(b_pool).cuda()
    ap, bp = a0.clone(), b0.clone()
    info = torch.zeros(len(systems), dtype=torch.int32, device="cuda")
    it = torch.zeros_like(info)
    rfp.rfp_pfsv_vbatched(h, rfp.PREC_FP32, len(systems), table, ap, bp, info, it, sys_host=raw)  # sizes
    torch.cuda.synchronize()
    want_b, want_it = bp.clone(), it.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    ap.copy_(a0)
    bp.copy_(b0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        rfp.rfp_pfsv_vbatched(h, rfp.PREC_FP32, len(systems), table, ap, bp, info, it, sys_host=raw)
    for rep in range(3):
        ap.copy_(a0)
        bp.copy_(b0)
        it.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bp, want_b), rep
        assert torch.equal(it, want_it), rep


TILED_NS = [257, 300, 385, 513, 700, 1001]


@pytest.mark.parametrize("pftri", [False, True])
def test_batched_tiled_fp64_matches_oracle(h, pftri):
    """Tiled systems (n > 256: 3 to 8 block rows, ragged last tiles, all
    layouts) mixed with one-task ones in one launch: factor, solve and
    inverse of every system against the oracle."""
    ns = TILED_NS + [16, 255, 1, 256]
    lays = [i % 4 for i in range(len(ns))]
    nrs = [3, 1, 17, 2, 5, 8, 2, 1, 4, 3]
    systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=500)
    ap, bp, info, it = run_batch(h, rfp.PREC_FP64, systems, arf_pool, b_pool, pftri=pftri)
    assert np.all(info == 0) and np.all(it == 0), (info, it)
    for sysd, arf in zip(systems, arfs):
        n, a0, b0, ldb, nr, t, u = sysd
        f, _ = oracle.pftrf(t, u, n, arf.copy())
        B = b_pool[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
        want = oracle.pftrs(t, u, n, f, np.asfortranarray(B))
        got = _sys_b(bp, sysd)
        assert oracle.rel_fro(got[:n], want) <= 1e-12 * n, (n, t, u)
        assert np.all(got[n:] == 0.0)
        ref = oracle.pftri(t, u, n, f)[0] if pftri else f
        assert oracle.rel_fro(ap[a0:a0 + arf.size], ref) <= 1e-12 * n, (n, t, u, pftri)
    used_a = np.zeros(arf_pool.size, bool)
    used_b = np.zeros(b_pool.size, bool)
    for (n, a0, b0, ldb, nr, t, u), arf in zip(systems, arfs):
        used_a[a0:a0 + arf.size] = True
        used_b[b0:b0 + ldb * nr] = True
    assert np.all(ap[~used_a] == 123.0) and np.all(bp[~used_b] == 321.0)


def test_batched_tiled_min_matrix_exact(h):
    """The min matrix factors into all ones and inverts to tridiag(-1, 2, -1)
    exactly, in any order of operations: bit-exact through the tiles."""
    for n, (t, u) in zip([300, 513], [("N", "L"), ("T", "U")]):
        A = synth.min_matrix(n)
        arf = oracle.trttf(t, u, A)
        X = synth.rng(n).integers(-3, 4, size=(n, 2)).astype(np.float64)
        B = A @ X
        systems = [(n, 0, 0, n, 2, t, u)]
        ap, bp, info, it = run_batch(h, rfp.PREC_FP64, systems, arf, B.ravel(order="F"), pftri=True)
        assert info[0] == 0
        assert np.array_equal(bp.reshape(2, n).T, X)
        inv = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        inv[n - 1, n - 1] = 1.0
        assert np.array_equal(ap, oracle.trttf(t, u, inv))


@pytest.mark.parametrize("mode", [rfp.PREC_FP32, rfp.PREC_FP16, rfp.PREC_BF16])
@pytest.mark.parametrize("pftri", [False, True])
def test_batched_tiled_low_precision(h, mode, pftri):
    """Low-precision factor + FP64 refinement on tiled and one-task systems
    with condition numbers 1e2 .. 1e6: every solution reaches the backward
    error bound (refinement converged, or the FP64 fall-back, whose factor is
    then left in the array), and with PFTRI the array holds the inverse of the
    FP64 matrix.  With the diagonal shift and the conjugate-gradient sweeps,
    every factor precision refines every one of these systems."""
    ns = [300, 513, 700, 1001, 100, 256]
    lays = [0, 1, 2, 3, 1, 2]
    nrs = [2, 1, 3, 2, 1, 4]
    kappas = [1e2, 1e4, 1e6, 1e3, 1e5, 1e2]
    systems, arfs, As, arf_pool, b_pool = [], [], [], None, None
    sys_all = []
    for q, (n, li, nr, kap) in enumerate(zip(ns, lays, nrs, kappas)):
        sys_q, arf_q, A_q, ap_q, bp_q = make_batch([n], [li], [nr], seed=600 + q, kappa=kap)
        sys_all.append((sys_q[0], arf_q[0], ap_q, bp_q))
    # concatenate the pools
    ao = bo = 0
    apool, bpool = [], []
    for (n, a0, b0, ldb, nr, t, u), arf, ap_q, bp_q in sys_all:
        systems.append((n, ao, bo, ldb, nr, t, u))
        arfs.append(arf)
        apool.append(ap_q)
        bpool.append(bp_q)
        ao += ap_q.size
        bo += bp_q.size
    arf_pool, b_pool = np.concatenate(apool), np.concatenate(bpool)
    ap, bp, info, it = run_batch(h, mode, systems, arf_pool, b_pool, pftri=pftri, max_iter=30)
    assert np.all(info == 0), info
    for (n, a0, b0, ldb, nr, t, u), arf, q in zip(systems, arfs, range(len(systems))):
        B = b_pool[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
        X = bp[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
        assert it[q] > 0, (n, it[q])
        assert oracle.backward_error(t, u, n, arf, B, X) <= 1e-14, (n, t, u, it[q])
        if pftri:
            f, _ = oracle.pftrf(t, u, n, arf.copy())
            inv, _ = oracle.pftri(t, u, n, f)
            assert oracle.rel_fro(ap[a0:a0 + arf.size], inv) <= 1e-12 * n * kappas[q]
        elif it[q] > 0:
            assert np.array_equal(ap[a0:a0 + arf.size], arf)  # refined: the FP64 matrix is untouched
        else:
            f, _ = oracle.pftrf(t, u, n, arf.copy())  # fell back: the FP64 factor is in place
            assert oracle.rel_fro(ap[a0:a0 + arf.size], f) <= 1e-12 * n


@pytest.mark.parametrize("mode", [rfp.PREC_FP16, rfp.PREC_BF16, rfp.PREC_FP32])
def test_batched_ill_conditioned_refines_without_fallback(h, mode):
    """Condition numbers 1e7 and 1e8 (kappa u_low >> 1 for FP16 and BF16):
    the shifted low-precision factor stays positive definite, and the
    conjugate-gradient sweeps bring every system (tiled and one-task) to the
    FP64 backward error without the FP64 fall-back; with the shift switched
    off, the FP16 and BF16 factors (and the FP32 factors at 1e8) are not
    positive definite (-3) and the FP64 fall-back answers."""
    ns, lays, nrs = [700, 1300, 256, 400], [0, 3, 1, 2], [2, 3, 1, 4]
    res = {}
    c_default = rfp.rfp_get_lowp_shift(h, mode)
    for c in (c_default, 0.0):
        systems, arfs, As, arf_pool, b_pool = [], [], [], [], []
        ao = bo = 0
        for q, (n, li, nr) in enumerate(zip(ns, lays, nrs)):
            s_q, a_q, _, ap_q, bp_q = make_batch([n], [li], [nr], seed=900 + q, kappa=1e7 if q % 2 else 1e8)
            n_, _, _, ldb, nr_, t, u = s_q[0]
            systems.append((n_, ao, bo, ldb, nr_, t, u))
            arfs.append(a_q[0])
            arf_pool.append(ap_q)
            b_pool.append(bp_q)
            ao += ap_q.size
            bo += bp_q.size
        arf_pool, b_pool = np.concatenate(arf_pool), np.concatenate(b_pool)
        rfp.rfp_set_lowp_shift(h, mode, c)
        try:
            ap, bp, info, it = run_batch(h, mode, systems, arf_pool, b_pool, max_iter=30)
        finally:
            rfp.rfp_set_lowp_shift(h, mode, c_default)
        assert np.all(info == 0), info
        for (n, a0, b0, ldb, nr, t, u), arf in zip(systems, arfs):
            B = b_pool[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
            X = bp[b0:b0 + ldb * nr].reshape(nr, ldb).T[:n]
            assert oracle.backward_error(t, u, n, arf, B, X) <= 1e-14, (c, n, t, u)
        res[c] = it
    assert np.all(res[c_default] > 0), res[c_default]
    # unshifted: FP16 / BF16 fail on every system, FP32 on the kappa = 1e8 ones
    lost = res[0.0] if mode != rfp.PREC_FP32 else res[0.0][0::2]
    assert np.all(lost == -3), res[0.0]


def test_batched_two_workgroups_per_cu_build(h):
    """A batch of one-task systems only (n <= 256) runs the two-per-CU build
    of the persistent loop; one tiled system (n = 257) added to the same
    batch switches the launch to the one-per-CU build.  The one-task systems
    come out bit for bit the same from both builds (one workgroup does all of
    a system's arithmetic, in the same order), and match the oracle."""
    ns = [1, 17, 64, 128, 200, 255, 256]
    lays = [i % 4 for i in range(len(ns))]
    nrs = [1, 2, 3, 4, 5, 6, 7]
    runs = {}
    for name, extra in (("small", []), ("with_tiled", [257])):
        systems, arfs, As, arf_pool, b_pool = make_batch(ns + extra, lays + [1] * len(extra),
                                                         nrs + [2] * len(extra), seed=700)
        torch.cuda.synchronize()
        rfp.rfp_profile_enable(h, True)
        try:
            ap, bp, info, it = run_batch(h, rfp.PREC_FP64, systems, arf_pool, b_pool)
            prof = rfp.rfp_profile_read(h)
        finally:
            rfp.rfp_profile_enable(h, False)
        assert np.all(info == 0) and np.all(it == 0), (name, info, it)
        runs[name] = (systems, arfs, b_pool, ap, bp, {k for k in prof if k.startswith("rfp::batched_kernel")})
    assert runs["small"][5] == {"rfp::batched_kernel_x2(rfp::BatchArgs)"}
    assert runs["with_tiled"][5] == {"rfp::batched_kernel(rfp::BatchArgs)"}
    systems, arfs, b_pool, ap, bp, _ = runs["small"]
    ap2, bp2 = runs["with_tiled"][3], runs["with_tiled"][4]
    for sysd, arf in zip(systems, arfs):
        n, a0, b0, ldb, nr, t, u = sysd
        assert np.array_equal(ap[a0:a0 + arf.size], ap2[a0:a0 + arf.size]), (n, t, u)
        assert np.array_equal(_sys_b(bp, sysd), _sys_b(bp2, sysd)), (n, t, u)
        f, _ = oracle.pftrf(t, u, n, arf.copy())
        want = oracle.pftrs(t, u, n, f, np.asfortranarray(_sys_b(b_pool, sysd)[:n]))
        assert oracle.rel_fro(ap[a0:a0 + arf.size], f) <= 1e-12 * n, (n, t, u)
        assert oracle.rel_fro(_sys_b(bp, sysd)[:n], want) <= 1e-12 * n, (n, t, u)
