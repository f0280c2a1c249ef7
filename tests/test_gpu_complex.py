"""GPU parity of the complex Hermitian path (ZTRTTF/ZTFTTR, ZPFTRF, ZPFTRS,
ZPFTRI) against the complex oracle, through the C ABI, in all eight layouts
(TRANSR 'N'/'C' x UPLO 'L'/'U' x odd/even n).

Sizes span one to several 64-row leaves and 64 x 64 product tiles with
ragged tails.  Bars: conversions bit-exact; Gaussian-integer factors and
inverses bit-exact; factor, solve and inverse within a relative Frobenius
error of 1e-12 * n of the oracle (the matrices are M M^H / n + I, condition
number below 5), and the factor elementwise within 8 n u max|L|."""
import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import dev, dev_colmajor, host, host_colmajor, info_tensor, read_info

pytestmark = pytest.mark.gpu

LAYOUTS = oracle.ZLAYOUTS
SIZES = [1, 2, 3, 63, 64, 65, 127, 130, 200, 257, 301, 513]
U = 2.0 ** -53


@pytest.fixture(scope="module")
def h():
    return rfp.Handle(0)


def rel(x, ref):
    r = np.linalg.norm(ref.ravel())
    return np.linalg.norm((x - ref).ravel()) / (r if r > 0 else 1.0)


def gauss_int_factor(n):
    L = np.tril(np.full((n, n), 1 + 1j), -1) + np.eye(n)
    return L, L @ L.conj().T


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 3, 6, 7, 64, 65, 129, 200, 257])
def test_zconversions_bit_exact(h, transr, uplo, n):
    g = np.random.default_rng(n)
    lda = n + 3
    a = np.asfortranarray(g.standard_normal((lda, n)) + 1j * g.standard_normal((lda, n)))
    want = oracle.ztrttf(transr, uplo, a[:n, :n])
    arf = torch.zeros(oracle.nt(n), dtype=torch.complex128, device="cuda")
    rfp.rfp_ztrttf(h, transr, uplo, n, _with_ld(a, n), arf)
    assert np.array_equal(host(arf), want)
    # back: only the UPLO triangle is written, the rest keeps its sentinel
    out = np.full((lda, n), 7 - 3j, dtype=complex, order="F")
    t_out = dev_colmajor(out)
    rfp.rfp_ztfttr(h, transr, uplo, n, arf, _view_ld(t_out, n))
    got = host_colmajor(t_out)
    tri = np.tril if uplo == "L" else np.triu
    m = tri(np.ones((n, n), bool))
    assert np.array_equal(got[:n][m], a[:n, :n][m])
    assert np.all(got[:n][~m] == 7 - 3j)
    assert np.all(got[n:] == 7 - 3j)


def _with_ld(a, n):
    """(lda x n) column-major device tensor viewed as n x n with leading dimension lda."""
    return _view_ld(dev_colmajor(a), n)


def _view_ld(t, n):
    return t[:n, :n]


def _factor_case(h, transr, uplo, n, seed):
    a, _ = synth.hpd(n, seed=seed)
    arf = oracle.ztrttf(transr, uplo, a)
    t = dev(arf)
    info = info_tensor()
    rfp.rfp_zpftrf(h, transr, uplo, n, t, info)
    return arf, t, read_info(info)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_zpftrf_parity(h, transr, uplo, n):
    arf, t, info = _factor_case(h, transr, uplo, n, seed=n)
    assert info == 0
    ref, rinfo = oracle.zpftrf(transr, uplo, n, arf)
    assert rinfo == 0
    got = host(t)
    assert rel(got, ref) <= 1e-12 * n
    assert np.abs(got - ref).max() <= 8 * n * U * np.abs(ref).max()
    if n <= 301:
        assert oracle.zfactor_residual(transr, uplo, n, arf, got) < 1e-14


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 9, 64, 65, 130, 200])
def test_zpftrf_gaussian_integer_exact(h, transr, uplo, n):
    L, a = gauss_int_factor(n)
    arf = oracle.ztrttf(transr, uplo, a)
    t = dev(arf)
    info = info_tensor()
    rfp.rfp_zpftrf(h, transr, uplo, n, t, info)
    assert read_info(info) == 0
    want = oracle.ztrttf(transr, uplo, L if uplo == "L" else L.conj().T)
    assert np.array_equal(host(t), want)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n,k", [(7, 2), (130, 5), (130, 64), (130, 66), (200, 150), (257, 256)])
def test_zpftrf_info(h, transr, uplo, n, k):
    a, _ = synth.hpd(n, seed=n + k)
    a[k, k] = -abs(a[k, k]) - 50.0
    arf = oracle.ztrttf(transr, uplo, a)
    _, want = oracle.zpftrf(transr, uplo, n, arf)
    assert want == k + 1
    info = info_tensor()
    rfp.rfp_zpftrf(h, transr, uplo, n, dev(arf), info)
    assert read_info(info) == want


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n,nrhs", [(1, 1), (3, 2), (64, 5), (65, 16), (130, 3), (257, 33), (301, 70)])
def test_zpftrs_parity(h, transr, uplo, n, nrhs):
    a, b = synth.hpd(n, nrhs=nrhs, seed=3 * n + nrhs)
    arf = oracle.ztrttf(transr, uplo, a)
    f, _ = oracle.zpftrf(transr, uplo, n, arf)
    want = oracle.zpftrs(transr, uplo, n, f, b)
    tb = dev_colmajor(b)
    rfp.rfp_zpftrs(h, transr, uplo, n, dev(f), tb)
    got = host_colmajor(tb)
    assert rel(got, want) <= 1e-12 * n
    assert oracle.zbackward_error(transr, uplo, n, arf, b, got) < 1e-15


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_zpftrs_ldb_larger_than_n(h, transr, uplo):
    n, nrhs, ldb = 130, 4, 141
    a, b = synth.hpd(n, nrhs=nrhs, seed=5)
    arf = oracle.ztrttf(transr, uplo, a)
    f, _ = oracle.zpftrf(transr, uplo, n, arf)
    want = oracle.zpftrs(transr, uplo, n, f, b)
    big = np.full((ldb, nrhs), 5 + 5j, dtype=complex, order="F")
    big[:n] = b
    tb = dev_colmajor(big)
    rfp.rfp_zpftrs(h, transr, uplo, n, dev(f), tb[:n])
    got = host_colmajor(tb)
    assert rel(got[:n], want) <= 1e-12 * n
    assert np.all(got[n:] == 5 + 5j)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 63, 65, 130, 200, 257, 301])
def test_zpftri_parity(h, transr, uplo, n):
    a, _ = synth.hpd(n, seed=7 * n)
    arf = oracle.ztrttf(transr, uplo, a)
    f, _ = oracle.zpftrf(transr, uplo, n, arf)
    want, rinfo = oracle.zpftri(transr, uplo, n, f)
    t = dev(f)
    info = info_tensor()
    rfp.rfp_zpftri(h, transr, uplo, n, t, info)
    assert read_info(info) == rinfo == 0
    got = host(t)
    assert rel(got, want) <= 1e-12 * n
    assert oracle.zinverse_residual(transr, uplo, n, arf, got) < 1e-14


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [600, 1100])
def test_zpftri_parity_recursive(h, transr, uplo, n):
    """Triangles of 300 and 550 rows: the W^H W recursion splits blocks above
    256 rows (at 550 twice), the inverse recursion down to 64-row blocks."""
    a, _ = synth.hpd(n, seed=5 * n)
    arf = oracle.ztrttf(transr, uplo, a)
    f, _ = oracle.zpftrf(transr, uplo, n, arf)
    want, rinfo = oracle.zpftri(transr, uplo, n, f)
    t = dev(f)
    info = info_tensor()
    rfp.rfp_zpftri(h, transr, uplo, n, t, info)
    assert read_info(info) == rinfo == 0
    got = host(t)
    assert rel(got, want) <= 1e-12 * n
    assert np.abs(got - want).max() <= 1e-11 * n * np.abs(want).max()


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [2, 9, 65, 130])
def test_zpftri_gaussian_integer_exact(h, transr, uplo, n):
    L, _ = gauss_int_factor(n)
    W = np.linalg.inv(L)
    W = np.round(W.real) + 1j * np.round(W.imag)
    want = oracle.ztrttf(transr, uplo, W.conj().T @ W)
    t = dev(oracle.ztrttf(transr, uplo, L if uplo == "L" else L.conj().T))
    info = info_tensor()
    rfp.rfp_zpftri(h, transr, uplo, n, t, info)
    assert read_info(info) == 0
    assert np.array_equal(host(t), want)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_zpftri_zero_diagonal_info(h, transr, uplo):
    n = 130
    a, _ = synth.hpd(n, seed=11)
    arf = oracle.ztrttf(transr, uplo, a)
    f, _ = oracle.zpftrf(transr, uplo, n, arf)
    full = oracle.ztfttr(transr, uplo, n, f)
    full[100, 100] = 0
    f0 = oracle.ztrttf(transr, uplo, full)
    assert oracle.zpftri(transr, uplo, n, f0)[1] == 101
    info = info_tensor()
    rfp.rfp_zpftri(h, transr, uplo, n, dev(f0), info)
    assert read_info(info) == 101


def test_zpftrf_solve_end_to_end_n1001(h):
    n, nrhs = 1001, 16
    for transr, uplo in (("N", "L"), ("C", "U")):
        a, b = synth.hpd(n, nrhs=nrhs, seed=1001)
        arf = oracle.ztrttf(transr, uplo, a)
        t = dev(arf)
        info = info_tensor()
        rfp.rfp_zpftrf(h, transr, uplo, n, t, info)
        assert read_info(info) == 0
        tb = dev_colmajor(b)
        rfp.rfp_zpftrs(h, transr, uplo, n, t, tb)
        x = host_colmajor(tb)
        assert oracle.zbackward_error(transr, uplo, n, arf, b, x) < 1e-15
        # sampled entries of the factor against the definition at full size
        ref, _ = oracle.zpftrf(transr, uplo, n, arf)
        got = host(t)
        assert rel(got, ref) <= 1e-12 * n


def test_zargument_codes(h):
    t = torch.zeros(oracle.nt(4), dtype=torch.complex128, device="cuda")
    info = info_tensor()
    with pytest.raises(rfp.RfpError) as e:
        rfp.rfp_zpftrf(h, "T", "L", 4, t, info)  # complex TRANSR is 'N' or 'C'
    assert e.value.code == -1
    with pytest.raises(rfp.RfpError) as e:
        rfp.rfp_zpftrf(h, "N", "X", 4, t, info)
    assert e.value.code == -2
    with pytest.raises(rfp.RfpError) as e:
        rfp.rfp_zpftrf(h, "N", "L", -1, t, info)
    assert e.value.code == -3


@pytest.mark.parametrize("transr,uplo", [("N", "U"), ("C", "L")])
def test_zsplit_k_products_n1100(h, transr, uplo):
    """n = 1100: block products with K >= 512 and fewer than 256 tiles take the
    split-K form (partial sums added in a fixed order): the HERK of ZPFTRF,
    S Y1 and S^H X2 of ZPFTRS, and the triangular products of ZPFTRI."""
    n, nrhs = 1100, 8
    a, b = synth.hpd(n, nrhs=nrhs, seed=1100)
    arf = oracle.ztrttf(transr, uplo, a)
    t = dev(arf)
    info = info_tensor()
    rfp.rfp_zpftrf(h, transr, uplo, n, t, info)
    assert read_info(info) == 0
    ref, _ = oracle.zpftrf(transr, uplo, n, arf)
    got = host(t)
    assert rel(got, ref) <= 1e-12 * n
    assert np.abs(got - ref).max() <= 8 * n * U * np.abs(ref).max()
    tb = dev_colmajor(b)
    rfp.rfp_zpftrs(h, transr, uplo, n, t, tb)
    x = host_colmajor(tb)
    assert rel(x, oracle.zpftrs(transr, uplo, n, ref, b)) <= 1e-12 * n
    assert oracle.zbackward_error(transr, uplo, n, arf, b, x) < 1e-15
    rfp.rfp_zpftri(h, transr, uplo, n, t, info)
    assert read_info(info) == 0
    inv = oracle.ztfttr(transr, uplo, n, host(t))
    dense = np.linalg.inv(a)
    tri = np.tril if uplo == "L" else np.triu
    m = tri(np.ones((n, n), bool))
    assert rel(inv[m], dense[m]) <= 1e-12 * n
    # the same products again: identical bits (the split sums are ordered)
    t2 = dev(arf)
    rfp.rfp_zpftrf(h, transr, uplo, n, t2, info)
    assert np.array_equal(host(t2), got)
