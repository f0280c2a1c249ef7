"""CPU checks of the GPU library's host logic: the recorded plans of PFTRF,
PFTRS and PFTRI for all eight layouts, replayed primitive by primitive in
NumPy (with bounds, mask and aliasing checks), must reproduce the oracle."""
import numpy as np
import pytest

import oracle
import paper_0901_1696_amd as rfp
import synth
from plan_replay import Replayer, work_size

SIZES = [1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 130, 192, 200, 255, 256, 257, 300, 513]
LAYOUTS = oracle.LAYOUTS


def _bufs(routine, uplo, n, arf, b=None):
    bufs = {0: arf, 2: np.full(work_size(routine, uplo, n), np.nan)}
    if b is not None:
        bufs[1] = b
    return bufs


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_pftrf_plan(transr, uplo, n):
    A, _ = synth.spd(n, seed=n)
    arf = oracle.trttf(transr, uplo, A)
    want, info = oracle.pftrf(transr, uplo, n, arf)
    assert info == 0
    got = arf.copy()
    Replayer(_bufs("F", uplo, n, got)).run(rfp.rfp_plan("F", transr, uplo, n))
    assert oracle.rel_fro(got, want) <= 1e-13 * max(n, 1)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_pftrs_plan(transr, uplo, n):
    nrhs = 3
    A, B = synth.spd(n, nrhs=nrhs, seed=n + 1)
    f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    want = oracle.pftrs(transr, uplo, n, f, B)
    ldb = n + 5
    bflat = np.full(ldb * nrhs, np.nan)
    for c in range(nrhs):
        bflat[c * ldb:c * ldb + n] = B[:, c]
    Replayer(_bufs("S", uplo, n, f.copy(), bflat)).run(rfp.rfp_plan("S", transr, uplo, n, nrhs, ldb))
    got = np.stack([bflat[c * ldb:c * ldb + n] for c in range(nrhs)], axis=1)
    assert oracle.rel_fro(got, want) <= 1e-13 * max(n, 1)
    # rows beyond n in each column are never touched
    for c in range(nrhs):
        assert np.all(np.isnan(bflat[c * ldb + n:(c + 1) * ldb]))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_pftri_plan(transr, uplo, n):
    A, _ = synth.spd(n, seed=n + 2)
    f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    want, info = oracle.pftri(transr, uplo, n, f)
    assert info == 0
    got = f.copy()
    Replayer(_bufs("I", uplo, n, got)).run(rfp.rfp_plan("I", transr, uplo, n))
    assert oracle.rel_fro(got, want) <= 1e-13 * max(n, 1)


def test_two_stream_schedule_is_checked():
    """The factorization uses the auxiliary stream; the replay's race check is
    active (a schedule without the bulk-update wait is flagged)."""
    n = 2001
    ops = rfp.rfp_plan("F", "N", "L", n)
    assert any(o.stream == 1 for o in ops)
    assert any(o.kind == rfp.PLAN_WAIT for o in ops)
    A, _ = synth.spd(n, seed=9)
    arf = oracle.trttf("N", "L", A)
    # drop the waits of the critical stream: the next block column's update
    # then races with the previous step's bulk update
    broken = [o for o in ops if not (o.kind == rfp.PLAN_WAIT and o.stream == 0)]
    with pytest.raises(AssertionError):
        Replayer(_bufs("F", "L", n, arf.copy())).run(broken)


def test_plan_argument_errors():
    with pytest.raises(rfp.RfpError):
        rfp.rfp_plan("F", "X", "L", 5)
    with pytest.raises(rfp.RfpError):
        rfp.rfp_plan("S", "N", "L", 5, nrhs=1, ldb=3)
    with pytest.raises(rfp.RfpError):
        rfp.rfp_plan("Q", "N", "L", 5)


def test_plan_leaf_counts():
    """The factorization recursion reaches diagonal blocks of at most 128 rows
    (the solve and inversion ones 64), aligned from the start of T1 and T2,
    one leaf per block."""
    for n in [100, 1001, 4097]:
        for t, u in LAYOUTS:
            m1 = (n + 1) // 2 if u == "L" else n // 2
            m2 = n - m1
            ops = rfp.rfp_plan("F", t, u, n)
            leaves = [o for o in ops if o.kind == rfp.PLAN_POTRF_LEAF]
            assert len(leaves) == -(-m1 // 128) + -(-m2 // 128)
            assert all(o.m <= 128 for o in leaves)
            ops = rfp.rfp_plan("I", t, u, n)
            leaves = [o for o in ops if o.kind == rfp.PLAN_TRTRI_LEAF]
            assert len(leaves) == -(-m1 // 64) + -(-m2 // 64)


def test_pftrs_plan_is_two_fused_solves():
    """PFTRS is the diagonal-block inverses of L11 and L22 followed by one
    blocked substitution per direction over the whole factor."""
    for t, u in LAYOUTS:
        ops = rfp.rfp_plan("S", t, u, 1001, 7, 1003)
        assert [o.kind for o in ops] == [rfp.PLAN_TRTRI_LEAVES] * 2 + [rfp.PLAN_BLOCK_SOLVE] * 2
        assert [o.tri_a for o in ops[2:]] == [0, 1]
        assert all(o.stream == 0 for o in ops)
        assert tuple(ops[2].d) == (rfp.PLAN_BUF_B, 0, 1, 1003)


@pytest.mark.parametrize("transr,uplo", [("N", "L"), ("T", "U"), ("N", "U")])
@pytest.mark.parametrize("n", [1100, 1537])
def test_pftrf_plan_with_bulk_updates(transr, uplo, n):
    """Sizes where the diagonal triangles have three or more 256-column panels,
    so the auxiliary stream's bulk updates and the lookahead overlap: the
    replay (race check included) matches the oracle."""
    A, _ = synth.spd(n, seed=n + 3)
    arf = oracle.trttf(transr, uplo, A)
    want, _ = oracle.pftrf(transr, uplo, n, arf.copy())
    ops = rfp.rfp_plan("F", transr, uplo, n)
    assert any(o.stream == 1 for o in ops)
    got = arf.copy()
    Replayer(_bufs("F", uplo, n, got)).run(ops)
    assert oracle.rel_fro(got, want) <= 1e-13 * n


def _drop_waits_on(ops, waiter, recorder):
    """The plan without stream `waiter`'s waits for events recorded on stream `recorder`."""
    evs = {o.m for o in ops if o.kind == rfp.PLAN_RECORD and o.stream == recorder}
    return [o for o in ops if not (o.kind == rfp.PLAN_WAIT and o.stream == waiter and o.m in evs)]


@pytest.mark.parametrize("transr,uplo", [("N", "L"), ("T", "U")])
def test_pftrf_plan_three_streams(transr, uplo):
    """When the first diagonal triangle spans four or more panels, the first
    part of the off-diagonal solve runs on the second auxiliary stream while
    the factorization finishes: the replay matches the oracle, and dropping
    either side of that fork (its start after the panel solve, or the join
    before the rest of the solve) is flagged as a race."""
    n = 2300
    A, _ = synth.spd(n, seed=n + 4)
    arf = oracle.trttf(transr, uplo, A)
    want, _ = oracle.pftrf(transr, uplo, n, arf.copy())
    ops = rfp.rfp_plan("F", transr, uplo, n)
    assert any(o.stream == 2 and o.kind == rfp.PLAN_GEMM for o in ops)
    got = arf.copy()
    Replayer(_bufs("F", uplo, n, got)).run(ops)
    assert oracle.rel_fro(got, want) <= 1e-13 * n
    for waiter, recorder in ((0, 2), (2, 0)):
        broken = _drop_waits_on(ops, waiter, recorder)
        assert len(broken) < len(ops)
        with pytest.raises(AssertionError):
            Replayer(_bufs("F", uplo, n, arf.copy())).run(broken)
