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
