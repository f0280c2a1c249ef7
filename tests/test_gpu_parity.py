"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Sizes run from 1 to 1001 so that every kernel sees several 64-row leaves,
several 128-wide GEMM tiles and ragged tails, in all eight RFP layouts.
Bars: layout conversions bit-exact; min-matrix closed forms bit-exact; FP64
factor, solve and inverse within a relative Frobenius error of 1e-12 * n of
the oracle (the matrices here have condition number below 5)."""
import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import dev, dev_colmajor, host, host_colmajor, info_tensor, read_info

pytestmark = pytest.mark.gpu

LAYOUTS = oracle.LAYOUTS
SIZES = [1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 300, 513, 1001]
EXACT_SIZES = [1, 2, 3, 64, 65, 128, 129, 257, 300, 513]


@pytest.fixture(scope="module")
def h():
    return rfp.Handle(0)


def tol(n):
    return 1e-12 * max(n, 1)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 3, 6, 7, 64, 65, 129, 200, 257])
def test_conversions_bit_exact(h, transr, uplo, n):
    g = np.random.default_rng(n)
    lda = n + 3
    a = np.asfortranarray(g.standard_normal((lda, n)))
    tri = np.tril if uplo == "L" else np.triu
    mask = tri(np.ones((n, n), bool))
    a_nan = a.copy()
    a_nan[:n][~mask] = np.nan            # the other triangle must never be read
    want = oracle.trttf(transr, uplo, a[:n])
    arf = torch.full((oracle.nt(n),), np.nan, dtype=torch.float64, device="cuda")
    rfp.rfp_dtrttf(h, transr, uplo, n, dev_colmajor(a_nan), arf)
    got = host(arf)
    assert np.array_equal(got, want)
    back = dev_colmajor(np.full((lda, n), -3.0))
    rfp.rfp_dtfttr(h, transr, uplo, n, arf, back)
    b = host_colmajor(back)
    assert np.array_equal(b[:n][mask], a[:n][mask])
    assert np.all(b[:n][~mask] == -3.0) and np.all(b[n:] == -3.0)


def _factor(h, transr, uplo, n, arf_np):
    arf = dev(arf_np)
    info = info_tensor()
    rfp.rfp_dpftrf(h, transr, uplo, n, arf, info)
    return host(arf), read_info(info)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", EXACT_SIZES)
def test_pftrf_min_matrix_exact(h, transr, uplo, n):
    arf = oracle.trttf(transr, uplo, synth.min_matrix(n))
    got, info = _factor(h, transr, uplo, n, arf)
    assert info == 0
    want = oracle.trttf(transr, uplo, np.tril(np.ones((n, n))) if uplo == "L" else np.triu(np.ones((n, n))))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_pftrf_random(h, transr, uplo, n):
    A, _ = synth.spd(n, seed=10 * n + 1)
    arf = oracle.trttf(transr, uplo, A)
    want, winfo = oracle.pftrf(transr, uplo, n, arf)
    got, info = _factor(h, transr, uplo, n, arf)
    assert info == winfo == 0
    assert oracle.rel_fro(got, want) <= tol(n)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_pftrs_random(h, transr, uplo, n):
    nrhs = 5
    A, B = synth.spd(n, nrhs=nrhs, seed=10 * n + 2)
    f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    want = oracle.pftrs(transr, uplo, n, f, B)
    ldb = n + 2
    Bp = np.full((ldb, nrhs), 7.0)
    Bp[:n] = B
    bd = dev_colmajor(Bp)
    rfp.rfp_dpftrs(h, transr, uplo, n, dev(f), bd)
    got = host_colmajor(bd)
    assert oracle.rel_fro(got[:n], want) <= tol(n)
    assert np.all(got[n:] == 7.0)


@pytest.mark.parametrize("transr,uplo", [("N", "L"), ("T", "U"), ("N", "U"), ("T", "L")])
@pytest.mark.parametrize("nrhs", [1, 16, 17, 33, 64, 65, 128, 130, 300])
def test_pftrs_slice_widths(h, transr, uplo, nrhs):
    """Right-hand-side slices of 16, 32, 64 and 128 columns, ragged last
    slices, over a factor with ragged 64-row blocks in both triangles."""
    n = 333
    A, B = synth.spd(n, nrhs=nrhs, seed=nrhs + 4)
    f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    want = oracle.pftrs(transr, uplo, n, f, B)
    ldb = n + 3
    Bp = np.full((ldb, nrhs), -3.0)
    Bp[:n] = B
    bd = dev_colmajor(Bp)
    rfp.rfp_dpftrs(h, transr, uplo, n, dev(f), bd)
    got = host_colmajor(bd)
    assert oracle.rel_fro(got[:n], want) <= tol(n)
    assert np.all(got[n:] == -3.0)


def test_pftrs_repeated_calls_reuse_flags(h):
    """Back-to-back solves on one handle with growing and shrinking shapes
    (the ready flags are reused across launches by epoch, never cleared)."""
    cases = [(700, 3, "N", "L"), (1001, 140, "T", "U"), (130, 1, "N", "U"), (1001, 140, "T", "U"),
             (65, 20, "T", "L")]
    outs = []
    for n, nrhs, t, u in cases:
        A, B = synth.spd(n, nrhs=nrhs, seed=n + nrhs)
        f, _ = oracle.pftrf(t, u, n, oracle.trttf(t, u, A))
        bd = dev_colmajor(B)
        rfp.rfp_dpftrs(h, t, u, n, dev(f), bd)
        outs.append((bd, oracle.pftrs(t, u, n, f, B), n))
    for bd, want, n in outs:
        assert oracle.rel_fro(host_colmajor(bd), want) <= tol(n)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 64, 65, 129, 300])
def test_pftrs_min_matrix_integer_exact(h, transr, uplo, n):
    A = synth.min_matrix(n)
    X = synth.rng(n).integers(-4, 5, size=(n, 3)).astype(np.float64)
    B = A @ X
    f = oracle.trttf(transr, uplo, np.tril(np.ones((n, n))) if uplo == "L" else np.triu(np.ones((n, n))))
    bd = dev_colmajor(B)
    rfp.rfp_dpftrs(h, transr, uplo, n, dev(f), bd)
    assert np.array_equal(host_colmajor(bd), X)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", SIZES)
def test_pftri_random(h, transr, uplo, n):
    A, _ = synth.spd(n, seed=10 * n + 3)
    f, _ = oracle.pftrf(transr, uplo, n, oracle.trttf(transr, uplo, A))
    want, _ = oracle.pftri(transr, uplo, n, f)
    arf = dev(f)
    info = info_tensor()
    rfp.rfp_dpftri(h, transr, uplo, n, arf, info)
    got = host(arf)
    assert read_info(info) == 0
    assert oracle.rel_fro(got, want) <= tol(n)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", EXACT_SIZES)
def test_pftri_min_matrix_exact(h, transr, uplo, n):
    f = oracle.trttf(transr, uplo, np.tril(np.ones((n, n))) if uplo == "L" else np.triu(np.ones((n, n))))
    arf = dev(f)
    info = info_tensor()
    rfp.rfp_dpftri(h, transr, uplo, n, arf, info)
    want = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    want[n - 1, n - 1] = 1.0
    assert read_info(info) == 0
    assert np.array_equal(host(arf), oracle.trttf(transr, uplo, want))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [9, 130, 301])
def test_pftrf_info_global_order(h, transr, uplo, n):
    """A leading minor p that is not positive definite, in either diagonal
    block: INFO = p, as the oracle says."""
    m1 = (n + 1) // 2 if uplo == "L" else n // 2
    for p in sorted({1, 2, m1 - 1, m1, m1 + 1, m1 + 70, n - 1, n} & set(range(1, n + 1))):
        A = synth.min_matrix(n)
        A[p - 1, p - 1] -= 1.0
        arf = oracle.trttf(transr, uplo, A)
        _, want = oracle.pftrf(transr, uplo, n, arf)
        _, info = _factor(h, transr, uplo, n, arf)
        assert info == want == p


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_guard_zones_untouched(h, transr, uplo):
    """Every routine writes only inside its RFP array and right-hand side."""
    n, guard, nrhs = 257, 4096, 3
    A, B = synth.spd(n, nrhs=nrhs, seed=5)
    arf = oracle.trttf(transr, uplo, A)
    buf = torch.full((oracle.nt(n) + 2 * guard,), 1234.5, dtype=torch.float64, device="cuda")
    buf[guard:guard + oracle.nt(n)] = dev(arf)
    view = buf[guard:guard + oracle.nt(n)]
    info = info_tensor()
    rfp.rfp_dpftrf(h, transr, uplo, n, view, info)
    bbuf = torch.full((n * nrhs + 2 * guard,), -99.0, dtype=torch.float64, device="cuda")
    bbuf[guard:guard + n * nrhs] = dev(np.asfortranarray(B).ravel(order="F"))
    bview = bbuf[guard:guard + n * nrhs].view(nrhs, n).t()
    rfp.rfp_dpftrs(h, transr, uplo, n, view, bview)
    rfp.rfp_dpftri(h, transr, uplo, n, view, info)
    hb = host(buf)
    assert read_info(info) == 0
    assert np.all(hb[:guard] == 1234.5) and np.all(hb[guard + oracle.nt(n):] == 1234.5)
    hbb = host(bbuf)
    assert np.all(hbb[:guard] == -99.0) and np.all(hbb[guard + n * nrhs:] == -99.0)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 64, 65, 257, 1001])
def test_single_precision_path(h, transr, uplo, n):
    """FP32 kernels (the low-precision factor of the mixed path) against the
    FP64 oracle, at FP32 accuracy."""
    A, B = synth.spd(n, nrhs=2, seed=n + 77)
    arf = oracle.trttf(transr, uplo, A)
    want, _ = oracle.pftrf(transr, uplo, n, arf)
    a32 = dev(arf.astype(np.float32))
    info = info_tensor()
    rfp.rfp_spftrf(h, transr, uplo, n, a32, info)
    assert read_info(info) == 0
    assert oracle.rel_fro(host(a32).astype(np.float64), want) <= 1e-5
    b32 = dev_colmajor(B.astype(np.float32))
    rfp.rfp_spftrs(h, transr, uplo, n, a32, b32)
    xw = oracle.pftrs(transr, uplo, n, want, B)
    assert oracle.rel_fro(host_colmajor(b32).astype(np.float64), xw) <= 1e-4


def test_cfg1_n1001_full_path(h):
    """The small benchmark configuration: n = 1001 (odd), TRANSR='N',
    UPLO='L', nrhs = 4, A = M M^T/n + I, seed 1001."""
    n, nrhs = 1001, 4
    A, B = synth.spd(n, nrhs=nrhs, seed=1001)
    arf = oracle.trttf("N", "L", A)
    f_or, _ = oracle.pftrf("N", "L", n, arf)
    x_or = oracle.pftrs("N", "L", n, f_or, B)
    inv_or, _ = oracle.pftri("N", "L", n, f_or)
    f, info = _factor(h, "N", "L", n, arf)
    assert info == 0
    assert oracle.rel_fro(f, f_or) <= tol(n)
    bd = dev_colmajor(B)
    rfp.rfp_dpftrs(h, "N", "L", n, dev(f), bd)
    x = host_colmajor(bd)
    assert oracle.rel_fro(x, x_or) <= tol(n)
    assert oracle.backward_error("N", "L", n, arf, B, x) <= 1e-15
    ad = dev(f)
    info = info_tensor()
    rfp.rfp_dpftri(h, "N", "L", n, ad, info)
    assert read_info(info) == 0
    assert oracle.rel_fro(host(ad), inv_or) <= tol(n)


@pytest.mark.parametrize("n", [8001, 8000])
def test_pftrs_large_backward_error_all_layouts(h, n):
    """Full-size behaviour of the fused solve, checked by a property that holds
    at any size: the normwise backward error of the PFTRF + PFTRS solution,
    from the dense FP64 matrix on the GPU.  Odd n puts block rows across
    cache-line boundaries of B, where solved rows written by one workgroup
    share lines with rows another workgroup read earlier; repeated calls."""
    A, B = synth.spd_device(n, nrhs=130, seed=n, device="cuda")
    anorm = A.abs().sum(dim=1).max()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t, u in LAYOUTS:
        arf = torch.empty(rfp.nt(n), dtype=torch.float64, device="cuda")
        rfp.rfp_dtrttf(h, t, u, n, A, arf)
        rfp.rfp_dpftrf(h, t, u, n, arf, info)
        assert read_info(info) == 0
        for nrhs in (1, 16, 33, 130):
            for _ in range(2):
                X = B[:, :nrhs].clone()  # column-major copy (B itself stays the right-hand side)
                assert X.stride(0) == 1 and X.data_ptr() != B.data_ptr()
                rfp.rfp_dpftrs(h, t, u, n, arf, X)
                R = B[:, :nrhs] - A @ X
                eta = (R.abs().amax(0) / (anorm * X.abs().amax(0) + B[:, :nrhs].abs().amax(0))).max().item()
                assert eta <= 1e-14, (t, u, nrhs, eta)
