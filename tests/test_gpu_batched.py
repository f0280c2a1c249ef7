"""GPU parity of the batched small-system solver against the oracle, per
system, through the C ABI; and replay of the same call captured in a HIP
graph."""
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


def run_batch(h, mode, systems, arf_pool, b_pool, pftri=False, tol=1e-14):
    table = torch.frombuffer(bytearray(rfp.sys_table(systems)), dtype=torch.uint8).cuda()
    ap = torch.from_numpy(arf_pool.copy()).cuda()
    bp = torch.from_numpy(b_pool.copy()).cuda()
    info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    it = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    rfp.rfp_dpfsv_batched(h, mode, len(systems), table, ap, bp, info, it, do_pftri=pftri, tol=tol)
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
    ns, lays, nrs = [40, 100, 200, 300], [0, 3, 1, 2], [2, 1, 3, 1]
    for mode in [rfp.PREC_FP64, rfp.PREC_FP32]:
        systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=300, bad=(1,))
        ap, bp, info, it = run_batch(h, mode, systems, arf_pool, b_pool)
        assert info[0] == 0 and info[2] == 0
        assert info[1] == 51  # A[50, 50] = -1: leading minor of order 51
        assert info[3] == -1  # n > 256 is refused and left alone
        a0, size = systems[3][1], arfs[3].size
        assert np.array_equal(ap[a0:a0 + size], arfs[3])
        if mode == rfp.PREC_FP32:
            assert it[1] == -3 and it[0] > 0 and it[2] > 0


def test_batched_graph_replay(h):
    """The call captured in a HIP graph and replayed: every replay, with its
    inputs restored eagerly in between, equals the eager result."""
    ns, lays, nrs = synth.batch_sizes(50, 16, 256, 1, 8, seed=9)
    systems, arfs, As, arf_pool, b_pool = make_batch(ns, lays, nrs, seed=400)
    table = torch.frombuffer(bytearray(rfp.sys_table(systems)), dtype=torch.uint8).cuda()
    a0 = torch.from_numpy(arf_pool).cuda()
    b0 = torch.from_numpy(b_pool).cuda()
    ap, bp = a0.clone(), b0.clone()
    info = torch.zeros(len(systems), dtype=torch.int32, device="cuda")
    it = torch.zeros_like(info)
    rfp.rfp_dpfsv_batched(h, rfp.PREC_FP32, len(systems), table, ap, bp, info, it)  # sizes the workspace
    torch.cuda.synchronize()
    want_b, want_it = bp.clone(), it.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    ap.copy_(a0)
    bp.copy_(b0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        rfp.rfp_dpfsv_batched(h, rfp.PREC_FP32, len(systems), table, ap, bp, info, it)
    for rep in range(3):
        ap.copy_(a0)
        bp.copy_(b0)
        it.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bp, want_b), rep
        assert torch.equal(it, want_it), rep
