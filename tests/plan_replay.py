"""Host-side replay of the GPU library's recorded plans (test support).

``rfp_plan`` lists the primitives (masked strided GEMMs and diagonal-block
leaf operations) the drivers would launch.  This module executes each one in
NumPy with the documented semantics and checks, for every access, that

  * the view stays inside its buffer (no out-of-bounds address on the GPU);
  * reads of a masked operand touch only its triangle;
  * an output that overlaps an input is one of the two in-place forms the
    GEMM kernel supports (C and A the same view with all columns in one
    128-wide tile, or B the transpose view of C with all rows in one tile),
    and overlaps nothing else;
  * the multi-stream schedule is race-free: ops on different streams that the
    recorded events do not order (vector clocks) touch disjoint data, or only
    read the same data.

The replay gives the same result as the GPU up to rounding; the tests compare
it with the oracle, which checks the block algebra of all eight layouts.
"""
import numpy as np

import paper_0901_1696_amd as rfp

NB = 64
TILE = 128


class PlanError(AssertionError):
    pass


def _idx(view, rows, cols):
    buf, off, rs, cs = view
    i = np.arange(rows)[:, None]
    j = np.arange(cols)[None, :]
    return buf, off + i * rs + j * cs


def _mask(tri, rows, cols):
    i = np.arange(rows)[:, None]
    j = np.arange(cols)[None, :]
    return {0: np.ones((rows, cols), bool), 1: i >= j, 2: i <= j, 3: i > j, 4: i < j}[tri]


class Replayer:
    def __init__(self, bufs):
        self.bufs = bufs  # {buffer id: 1-D float64 array}
        self.nops = 0
        self.vc = {q: [0, 0, 0] for q in range(3)}  # vector clock of each stream
        self.events = {}
        self.log = []  # (stream, clock, reads, writes) per compute op
        self._r, self._w = [], []

    def _check(self, buf, idx, mask, what):
        if buf not in self.bufs:
            raise PlanError(f"{what}: unknown buffer {buf}")
        sel = idx[mask]
        if sel.size and (sel.min() < 0 or sel.max() >= self.bufs[buf].size):
            raise PlanError(f"{what}: index range [{sel.min()}, {sel.max()}] outside buffer {buf} "
                            f"of size {self.bufs[buf].size}")

    def read(self, view, rows, cols, tri, what):
        buf, idx = _idx(view, rows, cols)
        mask = _mask(tri, rows, cols)
        self._check(buf, idx, mask, what)
        out = np.zeros((rows, cols))
        out[mask] = self.bufs[buf][idx[mask]]
        sel = set(idx[mask].ravel().tolist())
        self._r.append((buf, sel))
        return out, (buf, sel)

    def write(self, view, val, mask, what):
        rows, cols = val.shape
        buf, idx = _idx(view, rows, cols)
        self._check(buf, idx, mask, what)
        self.bufs[buf][idx[mask]] = val[mask]
        sel = set(idx[mask].ravel().tolist())
        self._w.append((buf, sel))
        return buf, sel

    def gemm(self, op):
        m, n, k = op.m, op.n, op.k
        A, ra = self.read(tuple(op.a), m, k, op.tri_a, "gemm A")
        B, rb = self.read(tuple(op.b), n, k, op.tri_b, "gemm B")
        cmask = _mask(1 if op.c_lower else 0, m, n)
        cbuf, cidx = _idx(tuple(op.c), m, n)
        self._check(cbuf, cidx, cmask, "gemm C")
        wset = set(cidx[cmask].ravel().tolist())
        # aliasing rules of the kernel: an overlap must be declared in-place and
        # be one of the two supported forms
        if ra[0] == cbuf and ra[1] & wset:
            if not (op.inplace and tuple(op.a) == tuple(op.c) and n <= TILE and op.beta == 0):
                raise PlanError(f"gemm: C overlaps A outside the supported in-place form {list(op.a)} {list(op.c)}")
        if rb[0] == cbuf and rb[1] & wset:
            cb, co, crs, ccs = tuple(op.c)
            if not (op.inplace and tuple(op.b) == (cb, co, ccs, crs) and m <= TILE and op.beta == 0):
                raise PlanError(f"gemm: C overlaps B outside the supported in-place form {list(op.b)} {list(op.c)}")
        C = np.zeros((m, n))
        if op.beta != 0:
            C[cmask] = self.bufs[cbuf][cidx[cmask]]
        R = op.alpha * (A @ B.T) + (op.beta * C if op.beta != 0 else 0.0)
        self.write(tuple(op.c), R, cmask, "gemm C")

    def axpy(self, op):
        m, n = op.m, op.n
        mask = _mask(1 if op.c_lower else 0, m, n)
        A, ra = self.read(tuple(op.a), m, n, 1 if op.c_lower else 0, "axpy A")
        C, rc = self.read(tuple(op.c), m, n, 1 if op.c_lower else 0, "axpy C")
        if ra[0] == rc[0] and ra[1] & rc[1]:
            raise PlanError("axpy: A and C overlap")
        self.write(tuple(op.c), C + op.alpha * A, mask, "axpy C")

    def copy(self, op):
        m, n = op.m, op.n
        A, ra = self.read(tuple(op.a), m, n, 0, "copy A")
        cbuf, cidx = _idx(tuple(op.c), m, n)
        if ra[0] == cbuf and ra[1] & set(cidx.ravel().tolist()):
            raise PlanError("copy: A and C overlap")
        self.write(tuple(op.c), A, np.ones((m, n), bool), "copy C")

    def leaf(self, op):
        nb = op.m
        low = _mask(1, nb, nb)
        X, _ = self.read(tuple(op.a), nb, nb, 1, "leaf A")
        if op.kind == rfp.PLAN_POTRF_LEAF:
            L = np.linalg.cholesky(X + np.tril(X, -1).T)
            self.write(tuple(op.a), L, low, "potrf leaf")
            bs = op.b[2]  # block order of the inverse (its row stride)
            W = np.eye(bs)
            W[:nb, :nb] = np.linalg.inv(L)
            self.write(tuple(op.b), W, np.ones((bs, bs), bool), "potrf leaf winv")
        elif op.kind == rfp.PLAN_TRTRI_LEAF:
            self.write(tuple(op.a), np.tril(np.linalg.inv(X)), low, "trtri leaf")
        elif op.kind == rfp.PLAN_LAUUM_LEAF:
            W = np.tril(X)
            self.write(tuple(op.a), W.T @ W, low, "lauum leaf")
        else:
            raise PlanError(f"unknown leaf kind {op.kind}")

    def leaves(self, op):
        n = op.m
        A, _ = self.read(tuple(op.a), n, n, 1, "trtri leaves A")
        wb, woff, _, _ = tuple(op.b)
        for b in range((n + NB - 1) // NB):
            o = b * NB
            nb = min(NB, n - o)
            W = np.eye(NB)
            W[:nb, :nb] = np.linalg.inv(np.tril(A[o:o + nb, o:o + nb]))
            self.write((wb, woff + b * NB * NB, NB, 1), W, np.ones((NB, NB), bool), "trtri leaves out")

    def block_solve(self, op):
        """Blocked substitution with the whole factor, block row by block row
        in the kernel's dependency order, through the stored block inverses."""
        m1, m2, r = op.m, op.k, op.n
        n = m1 + m2
        L = np.zeros((n, n))
        L[:m1, :m1], _ = self.read(tuple(op.a), m1, m1, 1, "solve L11")
        L[m1:, :m1], _ = self.read(tuple(op.b), m2, m1, 0, "solve L21")
        L[m1:, m1:], _ = self.read(tuple(op.c), m2, m2, 1, "solve L22")
        X, _ = self.read(tuple(op.d), n, r, 0, "solve B")
        blocks = [(o, min(NB, m1 - o)) for o in range(0, m1, NB)] + \
                 [(m1 + o, min(NB, m2 - o)) for o in range(0, m2, NB)]
        wb, woff, _, _ = tuple(op.w)
        forward = op.tri_a == 0
        order = range(len(blocks)) if forward else range(len(blocks) - 1, -1, -1)
        done = []
        for kb in order:
            o, c = blocks[kb]
            W, _ = self.read((wb, woff + kb * NB * NB, NB, 1), NB, NB, 0, "solve W")
            W = W[:c, :c] if forward else W[:c, :c].T
            acc = X[o:o + c].copy()
            for jb in done:
                oj, cj = blocks[jb]
                blk = L[o:o + c, oj:oj + cj] if forward else L[oj:oj + cj, o:o + c].T
                acc -= blk @ X[oj:oj + cj]
            X[o:o + c] = W @ acc
            done.append(kb)
        self.write(tuple(op.d), X, np.ones((n, r), bool), "solve X")

    def run(self, ops):
        for op in ops:
            self.nops += 1
            if op.kind == rfp.PLAN_RECORD:
                self.events[op.m] = list(self.vc[op.stream])
                continue
            if op.kind == rfp.PLAN_WAIT:
                ev = self.events[op.m]
                self.vc[op.stream] = [max(a, b) for a, b in zip(self.vc[op.stream], ev)]
                continue
            self._r, self._w = [], []
            if op.kind == rfp.PLAN_GEMM:
                self.gemm(op)
            elif op.kind == rfp.PLAN_TRTRI_LEAVES:
                self.leaves(op)
            elif op.kind == rfp.PLAN_BLOCK_SOLVE:
                self.block_solve(op)
            elif op.kind == rfp.PLAN_AXPY:
                self.axpy(op)
            elif op.kind == rfp.PLAN_COPY:
                self.copy(op)
            else:
                self.leaf(op)
            s = op.stream
            self.vc[s][s] += 1
            self.log.append((s, list(self.vc[s]), self._r, self._w))
        self.check_races()

    def check_races(self):
        def merge(lst):
            out = {}
            for buf, sel in lst:
                out.setdefault(buf, set()).update(sel)
            return out
        ops = [(s, vc, merge(r), merge(w)) for s, vc, r, w in self.log]
        by_stream = {q: [o for o in ops if o[0] == q] for q in range(3)}
        for qa, qb in ((0, 1), (0, 2), (1, 2)):
            for sa, va, ra, wa in by_stream[qa]:
                for sb, vb, rb, wb in by_stream[qb]:
                    if va[qa] <= vb[qa] or vb[qb] <= va[qb]:
                        continue  # ordered by the events
                    for buf in set(wa) | set(wb):
                        if (wa.get(buf, set()) & (rb.get(buf, set()) | wb.get(buf, set()))) or \
                           (wb.get(buf, set()) & ra.get(buf, set())):
                            raise PlanError(f"race between unordered ops on streams {qa} and {qb} "
                                            f"(buffer {buf})")


NB2 = 128


def work_size(routine, uplo, n):
    """Scratch the library allocates for each routine: PFTRF reuses one set of
    128-block leaf inverses sized for the larger diagonal block, PFTRS keeps
    the 64-block inverses of both T1 and T2, PFTRI one m1 x m1 square (the
    product W21^T W21 formed before S changes), the 128-row inverse leaf's
    scratch and the second stream's multiply scratch (one off-diagonal block
    of T2's top split), each piece starting at a multiple of 32 elements."""
    m1 = (n + 1) // 2 if uplo == "L" else n // 2
    m2 = n - m1
    nl = lambda m, b: (m + b - 1) // b
    if routine == "F":
        return max(nl(m1, NB2), nl(m2, NB2)) * NB2 * NB2
    if routine == "I":
        up = lambda x: (x + 31) // 32 * 32
        split = lambda m: (nl(m, NB2) + 1) // 2 * NB2
        s2 = split(m2) if m2 > NB2 else m2
        return up(up(m1 * m1) + 3 * NB2 * NB2) + s2 * (m2 - s2)
    return (nl(m1, NB) + nl(m2, NB)) * NB * NB
