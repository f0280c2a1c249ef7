"""Pins of the oracle's factor, solve, inverse and metrics (CPU only).

What fixes the answer independently of the oracle's own code:
  * closed forms that are exact in binary64 for any summation order: the min
    matrix a_ij = min(i,j)+1 has the all-ones lower triangle as Cholesky
    factor and tridiag(-1,2,-1) (last diagonal 1) as inverse; D A D with
    D = diag(2^e) has factor D * ones; an integer right-hand side B = A X is
    solved exactly; A = diag(d) has factor diag(sqrt(d));
  * brute force through numpy.linalg on the unpacked matrix for small n;
  * LAPACK's own RFP routines (dpftrf / dpftrs / dpftri) as a black box;
  * the paper's statement that the RFP algorithm is the textbook one with a
    different summation order (Section 7), so the definition path and the
    four-step path must agree to rounding.
"""
import numpy as np
import pytest

import oracle
import synth

LAYOUTS = oracle.LAYOUTS
SIZES_EXACT = [1, 2, 3, 7, 8, 64, 65, 200]


def unpack_lower(t, u, n, arf):
    full = oracle.tfttr(t, u, n, arf)
    return np.tril(full) if u == "L" else np.triu(full).T


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES_EXACT)
def test_min_matrix_factor_exact(transr, uplo, n):
    A = synth.min_matrix(n)
    arf = oracle.trttf(transr, uplo, A)
    ones = np.tril(np.ones((n, n)))
    for fn in (oracle.pftrf, oracle.pftrf_srpa):
        f, info = fn(transr, uplo, n, arf)
        assert info == 0
        assert np.array_equal(unpack_lower(transr, uplo, n, f), ones)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 64, 65])
def test_scaled_min_matrix_factor_exact(transr, uplo, n):
    A, d = synth.scaled_min_matrix(n, seed=n)
    arf = oracle.trttf(transr, uplo, A)
    want = d[:, None] * np.tril(np.ones((n, n)))
    for fn in (oracle.pftrf, oracle.pftrf_srpa):
        f, info = fn(transr, uplo, n, arf)
        assert info == 0
        assert np.array_equal(unpack_lower(transr, uplo, n, f), want)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES_EXACT)
def test_min_matrix_inverse_exact(transr, uplo, n):
    A = synth.min_matrix(n)
    f, info = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    inv, info = oracle.pftri(transr, uplo, n, f)
    assert info == 0
    want = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    want[n - 1, n - 1] = 1.0
    got = oracle.tfttr(transr, uplo, n, inv)
    tri = np.tril if uplo == "L" else np.triu
    assert np.array_equal(tri(got), tri(want))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 64, 65])
def test_min_matrix_integer_solve_exact(transr, uplo, n):
    A = synth.min_matrix(n)
    X = np.asfortranarray(synth.rng(n).integers(-5, 6, size=(n, 3)).astype(np.float64))
    B = A @ X
    f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    assert np.array_equal(oracle.pftrs(transr, uplo, n, f, B), X)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_diagonal_and_identity(transr, uplo):
    for n in [1, 2, 5, 6]:
        d = np.arange(1, n + 1, dtype=np.float64) * 1.5
        f, info = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, np.diag(d)))
        assert info == 0
        assert np.array_equal(unpack_lower(transr, uplo, n, f), np.diag(np.sqrt(d)))
        f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, np.eye(n)))
        assert np.array_equal(unpack_lower(transr, uplo, n, f), np.eye(n))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_brute_force_numpy_small(transr, uplo):
    for n in range(1, 9):
        A, B = synth.spd(n, alpha=1.0, nrhs=3, seed=100 + n)
        arf = oracle.trttf(transr, uplo, A)
        f, info = oracle.pftrf(transr, uplo, n, arf)
        assert info == 0
        L = np.linalg.cholesky(A)
        assert np.allclose(unpack_lower(transr, uplo, n, f), L, rtol=0, atol=1e-14)
        X = oracle.pftrs(transr, uplo, n, f, B)
        assert np.allclose(X, np.linalg.solve(A, B), rtol=1e-13, atol=1e-14)
        inv, info = oracle.pftri(transr, uplo, n, f)
        assert info == 0
        assert np.allclose(oracle.tfttr(transr, uplo, n, inv) +
                           (np.triu(np.linalg.inv(A), 1) if uplo == "L" else np.tril(np.linalg.inv(A), -1)),
                           np.linalg.inv(A), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_definition_vs_four_step_path(transr, uplo):
    for n in [1, 2, 3, 10, 33, 64, 97, 128]:
        A, _ = synth.spd(n, seed=n)
        arf = oracle.trttf(transr, uplo, A)
        f1, i1 = oracle.pftrf(transr, uplo, n, arf)
        f2, i2 = oracle.pftrf_srpa(transr, uplo, n, arf)
        assert i1 == 0 and i2 == 0
        assert oracle.rel_fro(f2, f1) <= 1e-14 * max(n, 1)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_against_lapack_rfp(transr, uplo):
    lapack = pytest.importorskip("scipy.linalg.lapack")
    for n in list(range(1, 34)) + [64, 65, 129]:
        A, B = synth.spd(n, nrhs=4, seed=1000 + n)
        arf = oracle.trttf(transr, uplo, A)
        f, info = oracle.pftrf(transr, uplo, n, arf)
        assert info == 0
        ref, info = lapack.dpftrf(n, arf.copy(), transr=transr, uplo=uplo)
        assert info == 0
        assert oracle.rel_fro(f, ref) <= 1e-14 * n
        X = oracle.pftrs(transr, uplo, n, f, B)
        Xr, info = lapack.dpftrs(n, ref, B.copy(), transr=transr, uplo=uplo)
        assert oracle.rel_fro(X, Xr) <= 1e-13 * n
        inv, _ = oracle.pftri(transr, uplo, n, f)
        invr, info = lapack.dpftri(n, ref.copy(), transr=transr, uplo=uplo)
        assert info == 0
        assert oracle.rel_fro(inv, invr) <= 1e-13 * n


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_info_global_order(transr, uplo):
    """Break positive definiteness at leading minor p (in the first or the
    second diagonal block): INFO must be p for both oracle paths and match
    LAPACK's dpftrf."""
    lapack = pytest.importorskip("scipy.linalg.lapack")
    for n in [5, 6, 9, 10]:
        for p in range(1, n + 1):
            A = synth.min_matrix(n)
            # a_{p-1,p-1} = p makes the leading minor of order p exactly zero
            # (the factor's last diagonal entry there is sqrt(p - p) = 0);
            # subtracting 1 more makes it negative.
            A[p - 1, p - 1] -= 1.0
            arf = oracle.trttf(transr, uplo, A)
            _, i1 = oracle.pftrf(transr, uplo, n, arf)
            _, i2 = oracle.pftrf_srpa(transr, uplo, n, arf)
            _, i3 = lapack.dpftrf(n, arf.copy(), transr=transr, uplo=uplo)
            assert i1 == p and i2 == p and i3 == p


def test_metrics_detect_planted_errors():
    """The metrics are not blind: they are tiny on exact results and large
    when a single factor entry, solution entry or inverse entry is wrong."""
    n = 40
    A, B = synth.spd(n, nrhs=2, seed=5)
    for t, u in LAYOUTS:
        arf = oracle.trttf(t, u, A)
        f, _ = oracle.pftrf(t, u, n, arf)
        assert oracle.factor_residual(t, u, n, arf, f) < 1e-15
        bad = f.copy()
        bad[oracle.rfp_pos(t, u, n, 30, 3)] += 1e-6
        assert oracle.factor_residual(t, u, n, arf, bad) > 1e-8
        X = oracle.pftrs(t, u, n, f, B)
        assert oracle.backward_error(t, u, n, arf, B, X) < 1e-15
        Xb = X.copy()
        Xb[17, 1] *= 1.0 + 1e-8
        assert oracle.backward_error(t, u, n, arf, B, Xb) > 1e-10
        inv, _ = oracle.pftri(t, u, n, f)
        assert oracle.inverse_residual(t, u, n, arf, inv) < 1e-15
        ib = inv.copy()
        ib[oracle.rfp_pos(t, u, n, 20, 20)] += 1e-7
        assert oracle.inverse_residual(t, u, n, arf, ib) > 1e-10


def test_norm_inf_symmetric():
    n = 13
    A, _ = synth.spd(n, seed=3)
    for t, u in LAYOUTS:
        got = oracle.norm_inf(t, u, n, oracle.trttf(t, u, A))
        assert got == pytest.approx(np.abs(A).sum(axis=1).max(), rel=1e-15)


def test_quick_returns():
    for t, u in LAYOUTS:
        f, info = oracle.pftrf(t, u, 0, np.zeros(0))
        assert info == 0 and f.size == 0


# Closed-form pins of the metrics: small matrices whose backward error,
# factor residual, inverse residual and forward error are hand-computed
# rationals (or their square roots).  A dropped term of a denominator, a
# missing weight of the off-diagonal entries, a transposed product or a norm
# of the wrong kind each changes the value.

def test_backward_error_closed_form():
    """A = [[4, 1, -2], [1, 5, 0], [-2, 0, 6]] (||A||_inf = 8, the third row
    sum).  Column 1: x = (1, -1, 0), b = A x + (0, 0, 1) = (3, -4, -1):
    ||r|| = 1, ||x|| = 1, ||b|| = 4, eta = 1 / (8 + 4) = 1/12.  Column 2:
    x = (0, 0, 1), b = 0: r = -A x = (2, 0, -6), eta = 6 / (8 * 1 + 0) = 3/4.
    The metric is the max over columns; each column alone is checked too."""
    A = np.array([[4.0, 1, -2], [1, 5, 0], [-2, 0, 6]])
    assert np.all(np.linalg.eigvalsh(A) > 0)
    X = np.array([[1.0, 0], [-1, 0], [0, 1]], order="F")
    B = np.array([[3.0, 0], [-4, 0], [-1, 0]], order="F")
    for t, u in LAYOUTS:
        arf = oracle.trttf(t, u, A)
        assert oracle.backward_error(t, u, 3, arf, B[:, :1], X[:, :1]) == pytest.approx(1 / 12, rel=1e-15)
        assert oracle.backward_error(t, u, 3, arf, B[:, 1:], X[:, 1:]) == pytest.approx(3 / 4, rel=1e-15)
        assert oracle.backward_error(t, u, 3, arf, B, X) == pytest.approx(3 / 4, rel=1e-15)
    # leading dimensions beyond n are honoured
    Bp = np.full((5, 1), 99.0, order="F")
    Bp[:3, 0] = B[:, 0]
    Xp = np.full((5, 1), -99.0, order="F")
    Xp[:3, 0] = X[:, 0]
    lib = oracle.lib()
    arf = oracle.trttf("N", "L", A)
    got = lib.orc_backward_error(b"N", b"L", 3, 1, oracle._p(arf), oracle._p(Bp), 5, oracle._p(Xp), 5)
    assert got == pytest.approx(1 / 12, rel=1e-15)


def test_factor_residual_closed_form():
    """A = [[8, 4], [4, 5]] (||A||_F^2 = 64 + 2 * 16 + 25 = 121) and the
    candidate factor L = [[3, 0], [2, 1]]: L L^T = [[9, 6], [6, 5]], so
    L L^T - A = [[1, 2], [2, 0]] with squared norm 1 + 2 * 4 = 9: the residual
    is 3/11 (both triangles counted).  The exact factor gives 0 up to
    rounding; L^T L instead of L L^T would give sqrt(45) / 11."""
    A = np.array([[8.0, 4], [4, 5]])
    L = np.array([[3.0, 0], [2, 1]])
    for t, u in LAYOUTS:
        arf = oracle.trttf(t, u, A)
        f = oracle.trttf(t, u, L if u == "L" else L.T)
        assert oracle.factor_residual(t, u, 2, arf, f) == pytest.approx(3 / 11, rel=1e-15)
        Le = np.linalg.cholesky(A)
        fe = oracle.trttf(t, u, Le if u == "L" else Le.T)
        assert oracle.factor_residual(t, u, 2, arf, fe) < 1e-15


def test_inverse_residual_closed_form():
    """A = [[2, 1], [1, 2]] with the candidate inverse V = I:
    I - A V = -[[1, 1], [1, 1]], ||.||_F = 2; ||A||_F = sqrt(10),
    ||V||_F = sqrt(2): the residual is 2 / sqrt(20) = 1/sqrt(5).  With
    V = diag(1/2, 1/2): I - A/2 = [[0, -1/2], [-1/2, 0]], norm 1/sqrt(2),
    ||V||_F = 1/sqrt(2): residual 1/sqrt(10).  The exact inverse
    [[2, -1], [-1, 2]] / 3 gives 0 up to rounding."""
    A = np.array([[2.0, 1], [1, 2]])
    for t, u in LAYOUTS:
        arf = oracle.trttf(t, u, A)
        assert oracle.inverse_residual(t, u, 2, arf, oracle.trttf(t, u, np.eye(2))) == \
            pytest.approx(1 / np.sqrt(5), rel=1e-15)
        assert oracle.inverse_residual(t, u, 2, arf, oracle.trttf(t, u, 0.5 * np.eye(2))) == \
            pytest.approx(1 / np.sqrt(10), rel=1e-15)
        exact = np.array([[2.0, -1], [-1, 2]]) / 3
        assert oracle.inverse_residual(t, u, 2, arf, oracle.trttf(t, u, exact)) < 1e-15


def test_forward_error_closed_form():
    """Column 1: x = (1, 2, 3), x_ref = (1, 4, -2): ||x - x_ref|| = 5,
    ||x_ref|| = 4, error 5/4.  Column 2: x = x_ref = (0, 0, 8): 0.  Max 5/4;
    column 2 alone 0; a reference column of zeros gives ||x||."""
    X = np.array([[1.0, 0], [2, 0], [3, 8]], order="F")
    R = np.array([[1.0, 0], [4, 0], [-2, 8]], order="F")
    assert oracle.forward_error(X, R) == 5 / 4
    assert oracle.forward_error(X[:, 1:], R[:, 1:]) == 0.0
    assert oracle.forward_error(np.array([3.0, -7]), np.zeros(2)) == 7.0
