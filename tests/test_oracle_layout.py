"""Pins of the oracle's index layer (CPU only).

The element maps are checked against what the paper prints (Figures 1, 2, 4,
5, 6, transcribed under tests/golden/), against invariants that hold for any
n (bijection onto [0, NT), TRANSR='T' is the transpose of TRANSR='N'), and
against LAPACK's own RFP conversion routines as an independent black box.
"""
import numpy as np
import pytest

import oracle
from golden_io import read_layout_grids, read_position_grids, read_printed_positions

LAYOUTS = oracle.LAYOUTS


def test_fig1_full_positions():
    grids = read_position_grids("fig1_full_positions_n7.txt")
    for uplo, grid in grids.items():
        for i in range(7):
            for j in range(7):
                p = grid[i][j]
                stored = (i >= j) if uplo == "L" else (i <= j)
                assert (p is not None) == stored
                if stored:
                    assert oracle.full_pos(7, i, j) + 1 == p


def test_fig2_packed_positions():
    grids = read_position_grids("fig2_packed_positions_n7.txt")
    for uplo, grid in grids.items():
        for i in range(7):
            for j in range(7):
                p = grid[i][j]
                if p is not None:
                    assert oracle.packed_pos(uplo, 7, i, j) + 1 == p


def _array_offset(transr, n, r, c):
    """Offset of printed cell (r, c): 'N' arrays are LDAR x n1 column-major,
    'T' arrays are n1 x LDAR with leading dimension n1."""
    ldar = n if n % 2 else n + 1
    n1 = (n + 1) // 2
    return r + c * (ldar if transr == "N" else n1)


def test_fig4_positions_and_cells():
    (t, u, n, grid), = read_layout_grids("fig4_rfp_NL_n7.txt")
    seen = set()
    for r, row in enumerate(grid):
        for c, (i, j, p) in enumerate(row):
            assert oracle.rfp_pos(t, u, n, i - 1, j - 1) + 1 == p
            assert _array_offset(t, n, r, c) + 1 == p
            seen.add(p)
    assert seen == set(range(1, 29))


def test_fig6_all_eight_layouts():
    blocks = read_layout_grids("fig6_rfp_layouts.txt")
    assert sorted((t, u, n) for t, u, n, _ in blocks) == sorted(
        (t, u, n) for t, u in LAYOUTS for n in (6, 7))
    for t, u, n, grid in blocks:
        ldar = n if n % 2 else n + 1
        n1 = (n + 1) // 2
        rows, cols = (ldar, n1) if t == "N" else (n1, ldar)
        assert len(grid) == rows and all(len(r) == cols for r in grid)
        for r, row in enumerate(grid):
            for c, (i, j, _) in enumerate(row):
                # the printed label names a stored element of the UPLO triangle
                assert (i >= j) if u == "L" else (i <= j)
                assert oracle.rfp_pos(t, u, n, i - 1, j - 1) == _array_offset(t, n, r, c)


def test_fig5_printed_positions():
    for t, u, n, i, j, p in read_printed_positions("fig5_printed_positions.txt"):
        assert oracle.rfp_pos(t, u, n, i - 1, j - 1) + 1 == p


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_bijection_and_transpose(transr, uplo):
    for n in list(range(0, 41)) + [100, 101, 200]:
        nt = n * (n + 1) // 2
        pos = set()
        ldar = n if n % 2 else n + 1
        n1 = (n + 1) // 2
        for j in range(n):
            for i in range(j, n):
                p = oracle.rfp_pos(transr, uplo, n, i, j)
                assert 0 <= p < nt
                pos.add(p)
                # symmetric element addressed either way round
                assert oracle.rfp_pos(transr, uplo, n, j, i) == p
                if transr == "T":
                    pn = oracle.rfp_pos("N", uplo, n, i, j)
                    r, c = pn % ldar, pn // ldar
                    assert p == c + r * n1
        assert len(pos) == nt


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_round_trips_bit_exact(transr, uplo):
    g = np.random.default_rng(7)
    for n in [1, 2, 3, 6, 7, 31, 32, 33, 64, 65]:
        a = np.asfortranarray(g.standard_normal((n + 3, n)))
        arf = oracle.trttf(transr, uplo, a)
        back = oracle.tfttr(transr, uplo, n, arf, lda=n + 3, fill=np.nan)
        tri = np.tril if uplo == "L" else np.triu
        mask = tri(np.ones((n, n), dtype=bool))
        assert np.array_equal(back[:n][mask], a[:n][mask])
        assert np.all(np.isnan(back[:n][~mask]))
        ap = oracle.tfttp(transr, uplo, n, arf)
        assert np.array_equal(oracle.tpttf(transr, uplo, n, ap), arf)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_against_lapack_conversions(transr, uplo):
    lapack = pytest.importorskip("scipy.linalg.lapack")
    g = np.random.default_rng(11)
    for n in list(range(1, 40)) + [100, 101]:
        a = np.asfortranarray(g.standard_normal((n, n)))
        ref, info = lapack.dtrttf(a, transr=transr, uplo=uplo)
        assert info == 0
        assert np.array_equal(oracle.trttf(transr, uplo, a), ref)
        ap, info = lapack.dtfttp(n, ref, transr=transr, uplo=uplo)
        assert info == 0
        assert np.array_equal(oracle.tfttp(transr, uplo, n, ref), ap)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_block_table_matches_element_map(transr, uplo):
    """The four-step path's block table (T1, S, T2 with strides) addresses the
    same storage as the element map, for every element of L11, L21, L22."""
    for n in range(1, 30):
        b = oracle.srpa_blocks(transr, uplo, n)
        m1, m2 = b["m1"], b["m2"]
        assert m1 + m2 == n
        off, rs, cs = b["t1"]
        for i in range(m1):
            for j in range(i + 1):
                assert off + i * rs + j * cs == oracle.rfp_pos(transr, uplo, n, i, j)
        off, rs, cs = b["s"]
        for i in range(m2):
            for j in range(m1):
                assert off + i * rs + j * cs == oracle.rfp_pos(transr, uplo, n, m1 + i, j)
        off, rs, cs = b["t2"]
        for i in range(m2):
            for j in range(i + 1):
                assert off + i * rs + j * cs == oracle.rfp_pos(transr, uplo, n, m1 + i, m1 + j)
