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
@pytest.mark.parametrize("n", SIZES + [800, 1100])  # 800, 1100: copied-back products in the LAUUM recursion
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
    """The factorization recursion reaches diagonal blocks of at most 128 rows,
    aligned from the start of T1 and T2, one leaf per block; the inversion's
    recursion stops at blocks of at most 128 rows that tile both triangles."""
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
            assert all(o.m <= 128 for o in leaves)
            assert sum(o.m for o in leaves) == m1 + m2
            assert len(leaves) >= -(-m1 // 128) + -(-m2 // 128)


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
    """Default schedule at sizes where the diagonal triangles have five or more
    128-column panels (the trailing orders stay below the 6144 at which panels
    widen to 256), so the auxiliary stream's bulk updates and the lookahead
    overlap, and the off-diagonal chunks run on the third stream: the replay
    (race check included) matches the oracle."""
    A, _ = synth.spd(n, seed=n + 3)
    arf = oracle.trttf(transr, uplo, A)
    want, _ = oracle.pftrf(transr, uplo, n, arf.copy())
    ops = rfp.rfp_plan("F", transr, uplo, n)
    assert any(o.stream == 1 for o in ops)
    assert _panel_widths(ops) == {128}
    got = arf.copy()
    Replayer(_bufs("F", uplo, n, got)).run(ops)
    assert oracle.rel_fro(got, want) <= 1e-13 * n


def _panel_widths(ops):
    """Widths of the diagonal-triangle panels: a 256-column panel is factored
    as two 128-row leaves with the in-panel solve and update between them, so
    it shows as two consecutive POTRF leaves whose INFO bases differ by 128 and
    whose first is a full 128 rows, separated only by GEMMs."""
    leaves = [(i, o) for i, o in enumerate(ops) if o.kind == rfp.PLAN_POTRF_LEAF]
    widths = set()
    k = 0
    while k < len(leaves):
        i, o = leaves[k]
        if k + 1 < len(leaves):
            j, p = leaves[k + 1]
            between = ops[i + 1:j]
            if (o.m == 128 and p.info_base == o.info_base + 128 and between
                    and all(q.kind == rfp.PLAN_GEMM and q.stream == 0 for q in between)
                    and any(q.inplace for q in between) and not any(q.kind == rfp.PLAN_RECORD for q in between)):
                widths.add(256)
                k += 2
                continue
        widths.add(128)
        k += 1
    return widths


# Schedules that force every branch the full-size factorization takes:
# 256-column panels (with the recursive in-panel solve and update and the
# second leaf's INFO offset), the off-diagonal chunks on the third stream,
# no chunk overlap, and the bulk update never waiting for the lookahead.
FORCED = {
    "wide": dict(wide_panels_above=0),
    "wide+chunks": dict(wide_panels_above=0, chunk_max=512),
    "chunks": dict(chunk_max=512),
    "no-overlap": dict(chunk_max=0),
    "no-lookahead-wait": dict(wide_panels_above=0, lookahead_wait_below=0),
}


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("sched", sorted(FORCED))
def test_pftrf_plan_forced_schedules(transr, uplo, sched):
    """Every schedule branch on all eight layouts at n = 1100 / 1101: the
    replay (bounds, masks, aliasing, three-stream race check) matches the
    oracle, element by element."""
    sc = FORCED[sched]
    for n in (1100, 1101):
        A, _ = synth.spd(n, seed=n + 11)
        arf = oracle.trttf(transr, uplo, A)
        want, _ = oracle.pftrf(transr, uplo, n, arf.copy())
        ops = rfp.rfp_plan("F", transr, uplo, n, sched=sc)
        widths = _panel_widths(ops)
        assert (256 in widths) == (sc.get("wide_panels_above", 6144) == 0)
        assert any(o.stream == 2 for o in ops) == (sc.get("chunk_max", 1536) > 0)
        got = arf.copy()
        Replayer(_bufs("F", uplo, n, got)).run(ops)
        assert oracle.rel_fro(got, want) <= 1e-13 * n
        assert np.abs(got - want).max() <= 8 * n * 2.0 ** -53 * np.abs(want).max()


def _view_range(view, rows, cols, tri):
    """[lo, hi] of the element offsets a masked strided view touches (strides
    are positive, so the extremes sit at the mask's corners)."""
    _, off, rs, cs = view
    if rows <= 0 or cols <= 0:
        return None
    r1, c1 = rows - 1, cols - 1
    if tri == 0:
        return off, off + r1 * rs + c1 * cs
    if tri in (1, 3):  # i >= j (+1 if strict): rows below the diagonal
        d = 1 if tri == 3 else 0
        if r1 < d:
            return None
        return off + d * rs, off + r1 * rs + min(c1, r1 - d) * cs
    d = 1 if tri == 4 else 0  # i <= j (-1 if strict)
    if c1 < d:
        return None
    return off + d * cs, off + min(r1, c1 - d) * rs + c1 * cs


@pytest.mark.parametrize("transr,uplo,n", [("N", "L", 12801), ("T", "U", 12800), ("T", "L", 20001),
                                           ("N", "U", 20000)])
def test_full_size_default_plan_structure(transr, uplo, n):
    """At full size (too large for the element-set replay) the default plan
    takes every forced branch above: 256-column panels while the trailing
    order exceeds 6144, 128-column ones after, third-stream chunks; and every
    view of every primitive stays inside its buffer (interval check)."""
    ops = rfp.rfp_plan("F", transr, uplo, n)
    assert _panel_widths(ops) == {128, 256}
    assert any(o.stream == 2 and o.kind == rfp.PLAN_GEMM for o in ops)
    sizes = {0: n * (n + 1) // 2, 2: work_size("F", uplo, n)}
    for o in ops:
        views = []
        if o.kind == rfp.PLAN_GEMM:
            views = [(o.a, o.m, o.k, o.tri_a), (o.b, o.n, o.k, o.tri_b), (o.c, o.m, o.n, 1 if o.c_lower else 0)]
        elif o.kind == rfp.PLAN_POTRF_LEAF:
            views = [(o.a, o.m, o.m, 1), (o.b, o.b[2], o.b[2], 0)]
        for v, r, c, t in views:
            rng_ = _view_range(tuple(v), r, c, t)
            if rng_ is not None:
                assert 0 <= rng_[0] and rng_[1] < sizes[v[0]], (o.kind, list(v), r, c, t)


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
