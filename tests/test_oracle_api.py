"""Pins of the oracle's TFTRI, TFSM and SFRK (the rest of the paper's table of
LAPACK 3.2 RFP routines): closed forms that are exact in binary64, LAPACK's
dtfsm / dsfrk through SciPy as black boxes, and brute force on the unpacked
matrix."""
import numpy as np
import pytest

import oracle
import synth

LAYOUTS = oracle.LAYOUTS
lapack = pytest.importorskip("scipy.linalg.lapack")


def _tri(n, uplo, seed, diag_boost=2.0):
    """A well-conditioned triangular matrix (dense, zero outside the triangle)."""
    g = synth.rng(seed)
    T = g.standard_normal((n, n)) / np.sqrt(n)
    T = np.tril(T) if uplo == "L" else np.triu(T)
    T[np.diag_indices(n)] = diag_boost + g.random(n)
    return T


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 64, 65, 300])
def test_tftri_all_ones_closed_form(transr, uplo, n):
    """The all-ones triangle's inverse is bidiagonal (1 on the diagonal, -1
    next to it): exact in any order.  DIAG='U' gives the same with any
    stored diagonal, which it leaves untouched."""
    ones = np.tril(np.ones((n, n))) if uplo == "L" else np.triu(np.ones((n, n)))
    inv = np.eye(n) - (np.eye(n, k=-1) if uplo == "L" else np.eye(n, k=1))
    got, info = oracle.tftri(transr, uplo, "N", n, oracle.trttf(transr, uplo, ones))
    assert info == 0 and np.array_equal(got, oracle.trttf(transr, uplo, inv))
    d = ones.copy()
    d[np.diag_indices(n)] = 7.5
    got, info = oracle.tftri(transr, uplo, "U", n, oracle.trttf(transr, uplo, d))
    want = inv.copy()
    want[np.diag_indices(n)] = 7.5
    assert info == 0 and np.array_equal(got, oracle.trttf(transr, uplo, want))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("diag", ["N", "U"])
def test_tftri_brute_force(transr, uplo, diag):
    n = 23
    T = _tri(n, uplo, seed=n)
    Tu = T.copy()
    if diag == "U":
        Tu[np.diag_indices(n)] = 1.0
    got, info = oracle.tftri(transr, uplo, diag, n, oracle.trttf(transr, uplo, T))
    want = np.linalg.inv(Tu)
    if diag == "U":
        want[np.diag_indices(n)] = T[np.diag_indices(n)]  # stored diagonal untouched
    assert info == 0
    assert np.allclose(oracle.tfttr(transr, uplo, n, got), np.tril(want) if uplo == "L" else np.triu(want),
                       rtol=1e-13, atol=1e-14)


def test_tftri_zero_diagonal():
    n = 9
    T = _tri(n, "L", seed=1)
    T[4, 4] = 0.0
    arf = oracle.trttf("N", "L", T)
    got, info = oracle.tftri("N", "L", "N", n, arf)
    assert info == 5 and np.array_equal(got, arf)
    assert oracle.tftri("N", "L", "U", n, arf)[1] == 0  # the diagonal is not read


SIDES = ["L", "R"]


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("side", SIDES)
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("diag", ["N", "U"])
def test_tfsm_against_lapack(transr, uplo, side, trans, diag):
    m, n = 13, 6
    k = m if side == "L" else n
    T = _tri(k, uplo, seed=k + 3)
    arf = oracle.trttf(transr, uplo, T)
    B = np.asfortranarray(synth.rng(5).standard_normal((m, n)))
    for alpha in (1.0, -0.75):
        want = lapack.dtfsm(alpha, arf.copy(), B.copy(order="F"), transr=transr, side=side, uplo=uplo, trans=trans,
                            diag=diag)
        got = oracle.tfsm(transr, side, uplo, trans, diag, m, n, alpha, arf, B)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("side", SIDES)
@pytest.mark.parametrize("trans", ["N", "T"])
def test_tfsm_all_ones_exact(transr, uplo, side, trans):
    """op(A) all-ones triangle, B = op(A) X (left) or X op(A) (right) with
    integer X: the solve is exact in binary64, also with DIAG='U' and any
    stored diagonal."""
    m, n = 40, 9
    k = m if side == "L" else n
    ones = np.tril(np.ones((k, k))) if uplo == "L" else np.triu(np.ones((k, k)))
    opA = ones if trans == "N" else ones.T
    X = synth.rng(k).integers(-5, 6, size=(m, n)).astype(np.float64)
    B = np.asfortranarray(opA @ X if side == "L" else X @ opA)
    got = oracle.tfsm(transr, side, uplo, trans, "N", m, n, 1.0, oracle.trttf(transr, uplo, ones), B)
    assert np.array_equal(got, X)
    d = ones.copy()
    d[np.diag_indices(k)] = 3.0
    got = oracle.tfsm(transr, side, uplo, trans, "U", m, n, 2.0, oracle.trttf(transr, uplo, d), B)
    assert np.array_equal(got, 2.0 * X)


def test_tfsm_alpha_zero_does_not_read_a():
    m, n = 5, 3
    arf = np.full(oracle.nt(m), np.nan)
    got = oracle.tfsm("N", "L", "L", "N", "N", m, n, 0.0, arf, np.ones((m, n), order="F"))
    assert np.array_equal(got, np.zeros((m, n)))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("n,k", [(1, 1), (7, 3), (12, 20)])
def test_sfrk_against_lapack(transr, uplo, trans, n, k):
    g = synth.rng(n * k)
    A = np.asfortranarray(g.standard_normal((n, k) if trans == "N" else (k, n)))
    C = oracle.trttf(transr, uplo, synth.spd(n, seed=k)[0])
    for alpha, beta in ((1.0, 0.0), (-0.5, 1.0), (2.0, -3.0)):
        want = lapack.dsfrk(n, k, alpha, A.copy(order="F"), beta, C.copy(), transr=transr, uplo=uplo, trans=trans)
        got = oracle.sfrk(transr, uplo, trans, n, k, alpha, A, beta, C)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_sfrk_closed_form(transr, uplo):
    """op(A) = all ones (n x k): op(A) op(A)^T = k everywhere, exact.  beta = 0
    never reads C (NaN there stays out); alpha = 0 never reads A."""
    n, k = 11, 6
    ones = np.ones((n, k), order="F")
    C = np.full(oracle.nt(n), np.nan)
    got = oracle.sfrk(transr, uplo, "N", n, k, 0.5, ones, 0.0, C)
    assert np.array_equal(got, np.full(oracle.nt(n), 3.0))
    C2 = oracle.trttf(transr, uplo, np.full((n, n), 2.0))
    got = oracle.sfrk(transr, uplo, "T", n, k, 0.0, np.full((k, n), np.nan, order="F"), -1.5, C2)
    assert np.array_equal(got, np.full(oracle.nt(n), -3.0))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 64, 65, 130])
def test_sfmv_against_numpy(transr, uplo, n):
    """The symmetric product against numpy's dense product of the unpacked
    matrix (alpha, beta, several right-hand sides)."""
    A, _ = synth.spd(n, seed=n + 70)
    arf = oracle.trttf(transr, uplo, A)
    g = synth.rng(n + 71)
    X = g.standard_normal((n, 5))
    Y = g.standard_normal((n, 5))
    got = oracle.sfmv(transr, uplo, n, -1.5, arf, X, 0.25, Y)
    want = -1.5 * (A @ X) + 0.25 * Y
    assert np.abs(got - want).max() <= 1e-14 * (np.abs(A) @ np.abs(X) + np.abs(Y)).max()


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_sfmv_min_matrix_exact(transr, uplo):
    """Integers throughout: the min matrix times integer columns is exact, and
    beta = 0 ignores a NaN-filled Y."""
    n = 33
    A = synth.min_matrix(n)
    arf = oracle.trttf(transr, uplo, A)
    X = synth.rng(3).integers(-4, 5, size=(n, 3)).astype(np.float64)
    got = oracle.sfmv(transr, uplo, n, 1.0, arf, X, 0.0, np.full((n, 3), np.nan))
    assert np.array_equal(got, A @ X)
