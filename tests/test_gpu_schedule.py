"""GPU parity of every branch of the factorization schedule, through the C ABI.

The default schedule takes its 256-column panels (with the recursive in-panel
solve and update, and the second leaf's INFO offset) only while a diagonal
triangle's trailing order exceeds 6144, and its three-stream chunked
off-diagonal solve only when a triangle spans more than one chunk.  The
schedule knobs are runtime settings of the handle, so these branches are
forced here at sizes the oracle finishes in seconds (n = 1100 / 1101, all
eight layouts), and two full-size cases run at the default schedule
(n = 12801 'N','L' and n = 12800 'T','U', where both branches occur).
Bars: relative Frobenius error <= 1e-12 n against the oracle, and the
largest elementwise error <= 8 n u max|L| (u = 2^-53), so that an error
confined to a few entries (a seam, one tile) cannot hide in the norm."""
import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import dev, host, info_tensor, read_info

pytestmark = pytest.mark.gpu

LAYOUTS = oracle.LAYOUTS
U = 2.0 ** -53

FORCED = {
    "wide": dict(wide_panels_above=0),
    "wide+chunks": dict(wide_panels_above=0, chunk_max=512),
    "chunks": dict(chunk_max=512),
    "no-overlap": dict(chunk_max=0),
    "no-lookahead-wait": dict(wide_panels_above=0, lookahead_wait_below=0),
    "no-leaf-pad": dict(wide_panels_above=0, chunk_max=512, leaf_lds_pad=0),
}


@pytest.fixture(scope="module")
def h():
    hd = rfp.Handle(0)
    yield hd
    rfp.rfp_set_schedule(hd, None)


def _check_factor(got, want, n):
    assert oracle.rel_fro(got, want) <= 1e-12 * n
    err = np.abs(got - want).max()
    assert err <= 8 * n * U * np.abs(want).max(), err


def test_schedule_set_get_and_errors(h):
    rfp.rfp_set_schedule(h, None)
    assert rfp.rfp_get_schedule(h) == rfp.DEFAULT_SCHEDULE
    rfp.rfp_set_schedule(h, dict(wide_panels_above=0, chunk_max=512))
    got = rfp.rfp_get_schedule(h)
    assert got["wide_panels_above"] == 0 and got["chunk_max"] == 512
    for bad in (dict(chunk_max=-1), dict(leaf_lds_pad=65537), dict(wide_panels_above=-5)):
        with pytest.raises(rfp.RfpError) as e:
            rfp.rfp_set_schedule(h, bad)
        assert e.value.code == -2
    assert rfp.rfp_get_schedule(h)["chunk_max"] == 512  # unchanged by the rejected calls
    rfp.rfp_set_schedule(h, None)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("sched", sorted(FORCED))
def test_pftrf_forced_schedule(h, transr, uplo, sched):
    rfp.rfp_set_schedule(h, FORCED[sched])
    try:
        for n in (1100, 1101):
            A, _ = synth.spd(n, seed=n + 11)
            arf = oracle.trttf(transr, uplo, A)
            want, winfo = oracle.pftrf(transr, uplo, n, arf)
            a = dev(arf)
            info = info_tensor()
            rfp.rfp_dpftrf(h, transr, uplo, n, a, info)
            assert read_info(info) == winfo == 0
            _check_factor(host(a), want, n)
    finally:
        rfp.rfp_set_schedule(h, None)


@pytest.mark.parametrize("transr,uplo", [("N", "L"), ("T", "U"), ("N", "U"), ("T", "L")])
def test_pftrf_forced_wide_min_matrix_exact(h, transr, uplo):
    """The min matrix's all-ones factor is exact in any order: bit-exact
    through the 256-column panels and the chunks."""
    n = 1101
    rfp.rfp_set_schedule(h, FORCED["wide+chunks"])
    try:
        a = dev(oracle.trttf(transr, uplo, synth.min_matrix(n)))
        info = info_tensor()
        rfp.rfp_dpftrf(h, transr, uplo, n, a, info)
        assert read_info(info) == 0
        ones = np.tril(np.ones((n, n))) if uplo == "L" else np.triu(np.ones((n, n)))
        assert np.array_equal(host(a), oracle.trttf(transr, uplo, ones))
    finally:
        rfp.rfp_set_schedule(h, None)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
def test_pftrf_info_in_second_leaf_of_wide_panel(h, transr, uplo):
    """A leading minor that is not positive definite inside the second
    128-row leaf of a 256-column panel (INFO offset goff + 128), in either
    diagonal triangle, with the chunks on: INFO = p as the oracle says."""
    n = 1100
    m1 = (n + 1) // 2 if uplo == "L" else n // 2
    rfp.rfp_set_schedule(h, FORCED["wide+chunks"])
    try:
        for p in (130, 200, 256, 256 + 129, m1 + 129, m1 + 256):
            A = synth.min_matrix(n)
            A[p - 1, p - 1] -= 1.0
            arf = oracle.trttf(transr, uplo, A)
            _, want = oracle.pftrf(transr, uplo, n, arf)
            a = dev(arf)
            info = info_tensor()
            rfp.rfp_dpftrf(h, transr, uplo, n, a, info)
            assert read_info(info) == want == p
    finally:
        rfp.rfp_set_schedule(h, None)


@pytest.mark.parametrize("fprec", [rfp.PREC_FP16, rfp.PREC_BF16])
def test_low_precision_operands_on_every_stream(h, fprec):
    """In FP16 / BF16 mode every product that is not in place takes the
    low-precision operand kernel, including the chunked off-diagonal solve
    and its share of step 3 on the third stream: the profiled launches of the
    FP32 GEMM split exactly as the recorded plan's in-place and other products."""
    n = 2300
    rfp.rfp_set_schedule(h, FORCED["wide+chunks"])
    try:
        ops = [o for o in rfp.rfp_plan("F", "N", "L", n, sched=FORCED["wide+chunks"])
               if o.kind == rfp.PLAN_GEMM and o.m > 0 and o.n > 0]
        assert any(o.stream == 2 for o in ops)
        A, _ = synth.spd(n, seed=5)
        a = dev(oracle.trttf("N", "L", A).astype(np.float32))
        info = info_tensor()
        torch.cuda.synchronize()
        rfp.rfp_profile_enable(h, True)
        rfp.rfp_spftrf_mp(h, fprec, "N", "L", n, a, info)
        prof = rfp.rfp_profile_read(h)
        rfp.rfp_profile_enable(h, False)
        assert read_info(info) == 0
        lp = {0: 0, 1: 0, 2: 0}
        for name, e in prof.items():
            if name.startswith("rfp::gemm_kernel<float,"):
                lp[int(name.split("<")[1].split(",")[6])] += e["launches"]
        assert lp[0] == sum(o.inplace for o in ops)
        assert lp[fprec] == sum(not o.inplace for o in ops)
        assert lp[3 - fprec] == 0
    finally:
        rfp.rfp_set_schedule(h, None)


@pytest.mark.parametrize("transr,uplo,n", [("N", "L", 12801), ("T", "U", 12800)])
def test_pftrf_full_size_default_schedule(h, transr, uplo, n):
    """Default schedule at a size where it takes 256-column panels (trailing
    order above 6144), the 128-column tail and the third-stream chunks,
    against the oracle's factor of the same matrix."""
    rfp.rfp_set_schedule(h, None)
    ops = rfp.rfp_plan("F", transr, uplo, n)
    assert any(o.kind == rfp.PLAN_GEMM and o.stream == 2 for o in ops)
    Ad, _ = synth.spd_device(n, seed=n, device="cuda")
    A = np.asfortranarray(Ad.cpu().numpy())
    del Ad
    arf = oracle.trttf(transr, uplo, A)  # packed on the host by the oracle
    del A
    a = dev(arf)
    info = info_tensor()
    rfp.rfp_dpftrf(h, transr, uplo, n, a, info)
    assert read_info(info) == 0
    got = host(a)
    want, winfo = oracle.pftrf(transr, uplo, n, arf)
    assert winfo == 0
    _check_factor(got, want, n)
