"""Pins of the complex Hermitian oracle (zrfp_oracle.c) to things other than
itself: LAPACK's own complex RFP routines (scipy's ztrttf, zpftrf, zpftrs,
zpftri), dense NumPy (Cholesky, solve, inverse), exact Gaussian-integer
factors, and closed forms of the error metrics.  CPU only."""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import oracle as O

SIZES = [1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 20, 33]


def hpd(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return m @ m.conj().T / n + np.eye(n)


def gauss_int_factor(n):
    """L with 1 on the diagonal and 1+1j below: A = L L^H has Gaussian-integer
    entries and L is its Cholesky factor exactly (every step is exact)."""
    L = np.tril(np.full((n, n), 1 + 1j), -1) + np.eye(n)
    return L, L @ L.conj().T


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_ztrttf_matches_lapack(t, u, n):
    a = hpd(n, n)
    ref, info = lapack.ztrttf(np.asfortranarray(a), transr=t, uplo=u)
    assert info == 0
    assert np.array_equal(O.ztrttf(t, u, a), ref)


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n", [1, 4, 7, 12])
def test_ztfttr_round_trip_and_lapack(t, u, n):
    a = hpd(n, 100 + n)
    arf = O.ztrttf(t, u, a)
    full = O.ztfttr(t, u, n, arf)
    tri = np.tril(a) if u == "L" else np.triu(a)
    assert np.array_equal(full, tri)
    ref, info = lapack.ztfttr(n, arf, transr=t, uplo=u)
    assert info == 0
    assert np.array_equal(np.tril(ref) if u == "L" else np.triu(ref), tri)


def test_conjugated_parts_follow_the_real_transposed_parts():
    # n = 5, 'N', 'L': A22 (columns 3, 4) is stored transposed, so conjugated;
    # 'C' conjugates everything else instead.
    for (i, j) in [(3, 3), (4, 3), (4, 4)]:
        assert O.zrfp_pos("N", "L", 5, i, j)[1]
        assert not O.zrfp_pos("C", "L", 5, i, j)[1]
    for (i, j) in [(0, 0), (2, 1), (4, 2)]:
        assert not O.zrfp_pos("N", "L", 5, i, j)[1]
        assert O.zrfp_pos("C", "L", 5, i, j)[1]
    # positions are the real format's
    for t, tr in (("N", "N"), ("C", "T")):
        for u in "LU":
            for i in range(6):
                for j in range(6):
                    if (u == "L" and i >= j) or (u == "U" and i <= j):
                        assert O.zrfp_pos(t, u, 6, i, j)[0] == O.rfp_pos(tr, u, 6, i, j)


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_zpftrf_matches_lapack_and_dense(t, u, n):
    a = hpd(n, 7 * n)
    arf = O.ztrttf(t, u, a)
    f_def, i1 = O.zpftrf(t, u, n, arf)
    f_srpa, i2 = O.zpftrf_srpa(t, u, n, arf)
    ref, i3 = lapack.zpftrf(n, arf, transr=t, uplo=u)
    assert i1 == i2 == i3 == 0
    tol = 8 * n * 2.0 ** -53 * np.abs(ref).max()
    assert np.abs(f_def - ref).max() <= tol
    assert np.abs(f_srpa - ref).max() <= tol
    # the stored triangle is L (lower) or L^H (upper) of the dense factor
    L = np.linalg.cholesky(a)
    full = O.ztfttr(t, u, n, f_def)
    want = L if u == "L" else L.conj().T
    assert np.abs(full - want).max() <= tol
    assert O.zfactor_residual(t, u, n, arf, f_def) < 1e-15


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 9, 16, 31])
def test_zpftrf_gaussian_integer_exact(t, u, n):
    L, a = gauss_int_factor(n)
    arf = O.ztrttf(t, u, a)
    for fn in (O.zpftrf, O.zpftrf_srpa):
        f, info = fn(t, u, n, arf)
        assert info == 0
        want = O.ztrttf(t, u, L if u == "L" else L.conj().T)
        assert np.array_equal(f, want)


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n,k", [(6, 0), (6, 2), (7, 3), (7, 5), (8, 6)])
def test_zpftrf_info_matches_lapack(t, u, n, k):
    a = hpd(n, 3 * n + k)
    a[k, k] = -abs(a[k, k]) - 50.0  # the leading minor of order k+1 is not positive definite
    arf = O.ztrttf(t, u, a)
    _, ref = lapack.zpftrf(n, arf, transr=t, uplo=u)
    assert ref == k + 1
    assert O.zpftrf(t, u, n, arf)[1] == k + 1
    assert O.zpftrf_srpa(t, u, n, arf)[1] == k + 1


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n", [1, 3, 8, 13, 20])
def test_zpftrs_matches_lapack_and_dense(t, u, n):
    rng = np.random.default_rng(n)
    a = hpd(n, 11 * n)
    b = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    arf = O.ztrttf(t, u, a)
    f, _ = O.zpftrf(t, u, n, arf)
    x = O.zpftrs(t, u, n, f, b)
    ref, info = lapack.zpftrs(n, f, np.asfortranarray(b), transr=t, uplo=u)
    assert info == 0
    assert np.abs(x - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(x - np.linalg.solve(a, b)).max() <= 1e-12 * np.abs(ref).max()
    assert O.zbackward_error(t, u, n, arf, b, x) < 1e-15


@pytest.mark.parametrize("t,u", O.ZLAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 12, 20])
def test_zpftri_matches_lapack_and_dense(t, u, n):
    a = hpd(n, 13 * n)
    arf = O.ztrttf(t, u, a)
    f, _ = O.zpftrf(t, u, n, arf)
    inv, info = O.zpftri(t, u, n, f)
    ref, info2 = lapack.zpftri(n, f, transr=t, uplo=u)
    assert info == info2 == 0
    assert np.abs(inv - ref).max() <= 1e-12 * np.abs(ref).max()
    dense = np.linalg.inv(a)
    full = O.ztfttr(t, u, n, inv)
    tri = np.tril(dense) if u == "L" else np.triu(dense)
    assert np.abs(full - tri).max() <= 1e-12 * np.abs(dense).max()
    assert O.zinverse_residual(t, u, n, arf, inv) < 1e-15


def test_zpftri_gaussian_integer_inverse():
    # L = unit lower with 1+1j below: W = L^{-1} has Gaussian-integer entries,
    # so A^{-1} = W^H W is exact
    for n in (2, 5, 9):
        L, a = gauss_int_factor(n)
        W = np.linalg.inv(L)
        W = np.round(W.real) + 1j * np.round(W.imag)
        assert np.array_equal(W @ L, np.eye(n))
        want = W.conj().T @ W
        for t, u in O.ZLAYOUTS:
            f = O.ztrttf(t, u, L if u == "L" else L.conj().T)
            inv, info = O.zpftri(t, u, n, f)
            assert info == 0
            assert np.array_equal(inv, O.ztrttf(t, u, want))


def test_metric_closed_forms():
    # backward error: A = 2 I, b = 2 e0, x = 1.5 e0 -> r = -e0 and
    # eta = 1 / (||A|| ||x|| + ||b||) = 1 / (2 * 1.5 + 2) = 0.2
    n = 4
    a = 2 * np.eye(n, dtype=complex)
    b = np.zeros((n, 1), complex)
    b[0] = 2
    x = np.zeros((n, 1), complex)
    x[0] = 1.5
    for t, u in O.ZLAYOUTS:
        arf = O.ztrttf(t, u, a)
        assert O.zbackward_error(t, u, n, arf, b, x) == pytest.approx(0.2, rel=1e-15)
        # moduli of complex entries: x = 1.5j e0, b = 2j e0 -> same 0.2
        assert O.zbackward_error(t, u, n, arf, 1j * b, 1j * x) == pytest.approx(0.2, rel=1e-15)
    # factor residual: A = I (n = 2), "factor" [[1, 0], [1j, 1]]:
    # L L^H - A = [[0, -1j], [1j, 1]] -> sqrt((1 + 1 + 1) / 2) (both triangles)
    a = np.eye(2, dtype=complex)
    lf = np.array([[1, 0], [1j, 1]])
    for t, u in O.ZLAYOUTS:
        arf_a = O.ztrttf(t, u, a)
        arf_l = O.ztrttf(t, u, lf if u == "L" else lf.conj().T)
        assert O.zfactor_residual(t, u, 2, arf_a, arf_l) == pytest.approx(np.sqrt(1.5), rel=1e-15)
    # inverse residual: A = 2 I, inverse 0.25 I (n = 4): ||0.5 I|| / (||2 I|| ||0.25 I||) = 1 / sqrt(n)
    for t, u in O.ZLAYOUTS:
        arf_a = O.ztrttf(t, u, 2 * np.eye(4, dtype=complex))
        arf_v = O.ztrttf(t, u, 0.25 * np.eye(4, dtype=complex))
        assert O.zinverse_residual(t, u, 4, arf_a, arf_v) == pytest.approx(0.5, rel=1e-15)
