"""GPU parity of the mixed-precision rows against the oracle, through the C ABI:
scaled cast (bit-exact), LANSF norms, and the refinement driver's end result
(the oracle's backward error and the FP64 oracle solution)."""
import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import dev, dev_colmajor, host, host_colmajor

pytestmark = pytest.mark.gpu

LAYOUTS = oracle.LAYOUTS


@pytest.fixture(scope="module")
def h():
    return rfp.Handle(0)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 3, 64, 65, 129, 300, 1001])
@pytest.mark.parametrize("scale,mu,shift", [(0, 1.0, 0.0), (1, 1.0, 0.0), (1, 4096.0, 0.0), (1, 2.0 ** 25, 4 * 2.0 ** -11),
                                            (1, 1.0, 3.3e-7)])
def test_cast_scale_bit_exact(h, transr, uplo, n, scale, mu, shift):
    A, _ = synth.spd(n, seed=n + 31)
    arf = oracle.trttf(transr, uplo, A)
    s_want, out_want = oracle.pfcast_s(transr, uplo, n, arf, scale=bool(scale), mu=mu, shift=shift)
    s = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    out = torch.full((rfp.nt(n),), -7.0, dtype=torch.float32, device="cuda")
    rfp.rfp_dpfcast_s(h, transr, uplo, n, dev(arf), scale, mu, s, out, shift=shift)
    assert np.array_equal(host(s), s_want)
    assert np.array_equal(host(out), out_want)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 65, 300, 1001])
def test_lansf(h, transr, uplo, n):
    A, _ = synth.spd(n, seed=n + 5)
    A[0, -1] = A[-1, 0] = -4.25
    arf = oracle.trttf(transr, uplo, A)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    d = dev(arf)
    rfp.rfp_dlansf(h, "M", transr, uplo, n, d, out[0:])
    rfp.rfp_dlansf(h, "I", transr, uplo, n, d, out[1:])
    rfp.rfp_dlansf(h, "F", transr, uplo, n, d, out[2:])
    got = host(out)
    assert got[0] == oracle.norm_max(transr, uplo, n, arf)
    assert abs(got[1] - oracle.norm_inf(transr, uplo, n, arf)) <= 1e-13 * got[1]
    assert abs(got[2] - oracle.norm_fro(transr, uplo, n, arf)) <= 1e-13 * got[2]


def _ir(h, fprec, transr, uplo, n, arf, b, x, **kw):
    """rfp_dpfsv_ir with device outputs; returns them as host ints."""
    out = torch.full((2,), -77, dtype=torch.int32, device="cuda")
    rfp.rfp_dpfsv_ir(h, fprec, transr, uplo, n, arf, b, x, out[0:1], out[1:2], **kw)
    it, info = (int(v) for v in host(out))
    return it, info


def _ir_case(n, kappa, nrhs, seed, transr="N", uplo="L"):
    k = max(1, n // 2)
    A, B = synth.spd(n, k=k, alpha=synth.cond_alpha(n, k, kappa), nrhs=nrhs, seed=seed)
    arf = oracle.trttf(transr, uplo, A)
    return A, B, arf


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n,kappa", [(65, 1e3), (300, 1e3), (300, 1e6), (1001, 1e6)])
def test_ir_fp32_converges_to_fp64_accuracy(h, transr, uplo, n, kappa):
    nrhs = 3
    A, B, arf = _ir_case(n, kappa, nrhs, seed=n + int(np.log10(kappa)), transr=transr, uplo=uplo)
    x = dev_colmajor(np.zeros((n, nrhs)))
    it, info = _ir(h, rfp.PREC_FP32, transr, uplo, n, dev(arf), dev_colmajor(B), x, tol=1e-14)
    X = host_colmajor(x)
    assert info == 0
    assert it > 0, f"refinement did not converge (code {it})"
    assert oracle.backward_error(transr, uplo, n, arf, B, X) <= 1e-14
    f, _ = oracle.pftrf(transr, uplo, n, arf.copy())
    X64 = oracle.pftrs(transr, uplo, n, f, B)
    assert oracle.rel_fro(X, X64) <= kappa * 1e-13


def test_ir_fallbacks(h):
    n, nrhs = 200, 2
    A, B, arf = _ir_case(n, 1e3, nrhs, seed=7)
    d, bd = dev(arf), dev_colmajor(B)
    # one sweep allowed, unreachable tolerance: max_iter fall-back, FP64 answer
    x = dev_colmajor(np.zeros((n, nrhs)))
    it, info = _ir(h, rfp.PREC_FP32, "N", "L", n, d, bd, x, tol=1e-300, max_iter=1)
    assert (it, info) == (-1, 0)
    assert oracle.backward_error("N", "L", n, arf, B, host_colmajor(x)) <= 1e-15
    # unreachable tolerance with room to iterate: the backward error stalls
    x = dev_colmajor(np.zeros((n, nrhs)))
    it, info = _ir(h, rfp.PREC_FP32, "N", "L", n, d, bd, x, tol=1e-300, max_iter=60)
    assert (it, info) == (-2, 0)
    assert oracle.backward_error("N", "L", n, arf, B, host_colmajor(x)) <= 1e-15
    # b is only read, arf untouched
    assert np.array_equal(host_colmajor(bd), B)
    assert np.array_equal(host(d), arf)


def test_ir_not_positive_definite(h):
    """Leading minor 100 negative with a positive diagonal: the FP32 factor
    fails (-3) and so does the FP64 fall-back (INFO = 100).  A negative
    diagonal entry makes the scaled copy non-finite (-4); the fall-back's INFO
    names that entry."""
    n = 130
    A = synth.min_matrix(n)
    A[99, 99] -= 2.0
    B = synth.rhs(n, 1, seed=3)
    arf = oracle.trttf("T", "U", A)
    assert oracle.pftrf("T", "U", n, arf)[1] == 100
    x = dev_colmajor(np.zeros((n, 1)))
    assert _ir(h, rfp.PREC_FP32, "T", "U", n, dev(arf), dev_colmajor(B), x) == (-3, 100)
    A2, B2, _ = _ir_case(n, 1e2, 1, seed=3)
    A2[100, 100] = -1.0
    arf2 = oracle.trttf("N", "U", A2)
    x = dev_colmajor(np.zeros((n, 1)))
    for fprec in (rfp.PREC_FP32, rfp.PREC_FP16):
        assert _ir(h, fprec, "N", "U", n, dev(arf2), dev_colmajor(B2), x) == (-4, 101)


def test_ir_argument_errors(h):
    n = 10
    d = torch.zeros(rfp.nt(n), dtype=torch.float64, device="cuda")
    b = torch.zeros((n, 1), dtype=torch.float64, device="cuda")
    x = torch.zeros((n, 1), dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    for kw, code in [(dict(fprec=9), -1), (dict(transr="X"), -2), (dict(tol=0.0), -11), (dict(max_iter=0), -12)]:
        args = dict(fprec=rfp.PREC_FP32, transr="N", tol=1e-14, max_iter=5)
        args.update(kw)
        with pytest.raises(rfp.RfpError) as e:
            rfp.rfp_dpfsv_ir(h, args["fprec"], args["transr"], "L", n, d, b, x, out[0:1], out[1:2], tol=args["tol"],
                             max_iter=args["max_iter"])
        assert e.value.code == code
    # n = 0 and nrhs = 0 return at once, with both outputs 0
    assert _ir(h, rfp.PREC_FP32, "N", "L", 0, d, b[:0], x[:0]) == (0, 0)


@pytest.mark.parametrize("fprec", [rfp.PREC_FP32, rfp.PREC_FP16, rfp.PREC_BF16])
@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 65, 300, 700])
def test_low_precision_factor_min_matrix_exact(h, fprec, transr, uplo, n):
    """Min matrix: the factor is all ones, so every operand rounded to FP16 or
    BF16 is exact and the low-precision factor is exact too."""
    A = synth.min_matrix(n)
    arf = torch.from_numpy(oracle.trttf(transr, uplo, A).astype(np.float32)).cuda()
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    rfp.rfp_spftrf_mp(h, fprec, transr, uplo, n, arf, info)
    ones = np.tril(np.ones((n, n))) if uplo == "L" else np.triu(np.ones((n, n)))
    assert int(host(info)[0]) == 0
    assert np.array_equal(host(arf), oracle.trttf(transr, uplo, ones).astype(np.float32))


@pytest.mark.parametrize("fprec,bound", [(rfp.PREC_FP32, 2e-6), (rfp.PREC_FP16, 2e-3), (rfp.PREC_BF16, 2e-2)])
@pytest.mark.parametrize("transr,uplo", [("N", "L"), ("T", "U")])
def test_low_precision_factor_residual(h, fprec, bound, transr, uplo):
    """||L L^T - A|| / ||A|| of the low-precision factor is of the order of the
    operand precision (parity unpinned beyond that: the factor is not unique
    at this precision)."""
    n = 700
    A, _ = synth.spd(n, seed=12)
    arf64 = oracle.trttf(transr, uplo, A)
    arf = torch.from_numpy(arf64.astype(np.float32)).cuda()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rfp.rfp_spftrf_mp(h, fprec, transr, uplo, n, arf, info)
    assert int(host(info)[0]) == 0
    res = oracle.factor_residual(transr, uplo, n, arf64, host(arf).astype(np.float64))
    assert res <= bound


@pytest.mark.parametrize("fprec", [rfp.PREC_FP16, rfp.PREC_BF16])
@pytest.mark.parametrize("n,kappa", [(300, 1e2), (1001, 1e3)])
def test_ir_half_precision_updates(h, fprec, n, kappa):
    nrhs = 2
    A, B, arf = _ir_case(n, kappa, nrhs, seed=n + 17)
    x = dev_colmajor(np.zeros((n, nrhs)))
    it, info = _ir(h, fprec, "N", "L", n, dev(arf), dev_colmajor(B), x, tol=1e-14, max_iter=60)
    assert info == 0 and it > 0, f"code {it}"
    assert oracle.backward_error("N", "L", n, arf, B, host_colmajor(x)) <= 1e-14


def test_ir_captured_in_graph_replays_like_eager(h):
    """The refinement takes every decision on the device: captured once in a
    HIP graph (after an eager call has sized the workspace), each replay with
    new right-hand sides gives the eager result bit for bit, with the same
    sweep count, and so does a replay whose right-hand sides hold a NaN,
    which makes the refinement stall and take the FP64 fall-back."""
    n, nrhs = 700, 3
    A, B0, arf = _ir_case(n, 1e3, nrhs, seed=41)
    d = dev(arf)
    b = dev_colmajor(B0)
    x = dev_colmajor(np.zeros((n, nrhs)))
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    kw = dict(tol=1e-14, max_iter=12)

    def eager(Bv):
        bb, xx = dev_colmajor(Bv), dev_colmajor(np.zeros((n, nrhs)))
        oo = torch.zeros(2, dtype=torch.int32, device="cuda")
        rfp.rfp_dpfsv_ir(h, rfp.PREC_FP16, "N", "L", n, d, bb, xx, oo[0:1], oo[1:2], **kw)
        return host_colmajor(xx), tuple(int(v) for v in host(oo))

    eager(B0)  # sizes every workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rfp.rfp_dpfsv_ir(h, rfp.PREC_FP16, "N", "L", n, d, b, x, out[0:1], out[1:2], **kw)
    torch.cuda.synchronize()
    cases = [B0, synth.rhs(n, nrhs, seed=5), 1e-3 * synth.rhs(n, nrhs, seed=6), B0]
    for Bv in cases:
        want_x, want_code = eager(Bv)
        b.copy_(dev_colmajor(Bv))
        x.fill_(123.0)
        out.fill_(-55)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = tuple(int(v) for v in host(out))
        assert got == want_code and got[0] > 0
        assert np.array_equal(host_colmajor(x), want_x)
        assert oracle.backward_error("N", "L", n, arf, Bv, want_x) <= 1e-14
        _ = torch.randn(1000, device="cuda").sum()  # other work between replays
    # a replay that falls back: NaN in the right-hand sides stalls the refinement
    Bn = B0.copy()
    Bn[3, 1] = np.nan
    want_x, want_code = eager(Bn)
    assert want_code[0] < 0
    b.copy_(dev_colmajor(Bn))
    g.replay()
    torch.cuda.synchronize()
    assert tuple(int(v) for v in host(out)) == want_code
    gx = host_colmajor(x)
    assert np.array_equal(np.isnan(gx), np.isnan(want_x))
    assert np.array_equal(gx[~np.isnan(gx)], want_x[~np.isnan(want_x)])


def test_solve_wait_give_up_is_reported(h):
    """With a wait limit of 0 polls, fused-solve workgroups whose dependencies
    are not yet published give up at once: their blocks of X become NaN, every
    kernel still ends, and the handle's status word reports it (then clears).
    With the default limit the same solve is exact and the status stays 0."""
    n, nrhs = 4000, 16
    f = oracle.trttf("N", "L", np.tril(np.ones((n, n))))
    X = synth.rng(1).integers(-3, 4, size=(n, nrhs)).astype(np.float64)
    B = synth.min_matrix(n) @ X
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    rfp.rfp_solve_status(h, st)  # clear
    rfp.rfp_set_solve_wait_limit(h, 0)
    try:
        bd = dev_colmajor(B)
        rfp.rfp_dpftrs(h, "N", "L", n, dev(f), bd)
        rfp.rfp_solve_status(h, st)
        assert int(host(st)[0]) == 1
        assert np.isnan(host_colmajor(bd)).any()
        rfp.rfp_solve_status(h, st)
        assert int(host(st)[0]) == 0  # cleared by the previous read
    finally:
        rfp.rfp_set_solve_wait_limit(h, -1)
    bd = dev_colmajor(B)
    rfp.rfp_dpftrs(h, "N", "L", n, dev(f), bd)
    rfp.rfp_solve_status(h, st)
    assert int(host(st)[0]) == 0
    assert np.array_equal(host_colmajor(bd), X)


def test_lowp_shift_setting(h):
    assert rfp.rfp_get_lowp_shift(h, rfp.PREC_FP32) == 64.0
    assert rfp.rfp_get_lowp_shift(h, rfp.PREC_FP16) == 4.0
    assert rfp.rfp_get_lowp_shift(h, rfp.PREC_BF16) == 4.0
    rfp.rfp_set_lowp_shift(h, rfp.PREC_BF16, 0.0)
    assert rfp.rfp_get_lowp_shift(h, rfp.PREC_BF16) == 0.0
    assert rfp.rfp_get_lowp_shift(h, rfp.PREC_FP16) == 4.0
    with pytest.raises(RuntimeError):
        rfp.rfp_set_lowp_shift(h, rfp.PREC_FP16, -1.0)
    with pytest.raises(RuntimeError):
        rfp.rfp_set_lowp_shift(h, rfp.PREC_FP64, 1.0)
    rfp.rfp_set_lowp_shift(h, rfp.PREC_BF16, 4.0)


@pytest.mark.parametrize("fprec", [rfp.PREC_FP16, rfp.PREC_BF16, rfp.PREC_FP32])
@pytest.mark.parametrize("kappa", [1e6, 1e8])
def test_ir_shifted_factor_refines_ill_conditioned(h, fprec, kappa):
    """kappa(A) u_low >> 1: the shifted low-precision factor stays positive
    definite and, as the preconditioner of the conjugate-gradient sweeps,
    brings the solution to the FP64 backward error.  Without the shift, the
    FP16 / BF16 factor of the kappa = 1e8 matrix is not positive definite."""
    n, nrhs = 1001, 2
    A, B, arf = _ir_case(n, kappa, nrhs, seed=n + int(np.log10(kappa)))
    x = dev_colmajor(np.zeros((n, nrhs)))
    it, info = _ir(h, fprec, "N", "L", n, dev(arf), dev_colmajor(B), x, tol=1e-14, max_iter=30)
    assert info == 0 and it > 0, f"code {it}"
    assert oracle.backward_error("N", "L", n, arf, B, host_colmajor(x)) <= 1e-14
    if fprec == rfp.PREC_FP32 or kappa < 1e8:
        return
    c0 = rfp.rfp_get_lowp_shift(h, fprec)
    rfp.rfp_set_lowp_shift(h, fprec, 0.0)
    try:
        x = dev_colmajor(np.zeros((n, nrhs)))
        it0, info0 = _ir(h, fprec, "N", "L", n, dev(arf), dev_colmajor(B), x, tol=1e-14, max_iter=30)
    finally:
        rfp.rfp_set_lowp_shift(h, fprec, c0)
    assert (it0, info0) == (-3, 0)
    assert oracle.backward_error("N", "L", n, arf, B, host_colmajor(x)) <= 1e-14
