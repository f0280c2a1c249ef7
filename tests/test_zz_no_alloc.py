"""The entry point that allocates nothing (rfp_dpftrs_noalloc), through the
C ABI, against the handle-based rfp_dpftrs on the same inputs: the same
kernels give the same bits.  Two calls in a row, the second smaller, then an
argument error and a problem beyond the fixed scratch."""
import numpy as np
import pytest
import torch

import oracle
import paper_0901_1696_amd as rfp
import synth
from gpu_util import dev, dev_colmajor, host_colmajor

pytestmark = pytest.mark.gpu


def _case(n, nrhs, t, u, seed):
    A, B = synth.spd(n, nrhs=nrhs, seed=seed)
    f, info = oracle.pftrf(t, u, n, oracle.trttf(t, u, A))
    assert info == 0
    return f, B


def test_noalloc_matches_handle_pftrs():
    h = rfp.Handle(0)
    for n, nrhs, t, u in [(1537, 40, "T", "U"), (301, 3, "N", "L")]:
        f, B = _case(n, nrhs, t, u, seed=n + nrhs)
        ref = dev_colmajor(B)
        rfp.rfp_dpftrs(h, t, u, n, dev(f), ref)
        got = dev_colmajor(B)
        rfp.rfp_dpftrs_noalloc(t, u, n, dev(f), got)
        want = host_colmajor(ref)
        assert np.array_equal(host_colmajor(got), want)
        assert oracle.rel_fro(want, oracle.pftrs(t, u, n, f, B)) <= 1e-12 * n
    h.close()


def test_noalloc_errors():
    b = torch.zeros((10, 1), dtype=torch.float64, device="cuda")
    a = torch.zeros(rfp.nt(10), dtype=torch.float64, device="cuda")
    with pytest.raises(rfp.RfpError) as e:
        rfp.rfp_dpftrs_noalloc("X", "L", 10, a, b)
    assert e.value.code == -1
    # 991 diagonal blocks fit; n = 64000 needs 1000
    big = torch.zeros((64000, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(rfp.RfpError) as e:
        rfp.rfp_dpftrs_noalloc("N", "L", 64000, a, big)
    assert e.value.code == rfp.RFP_ERR_SCRATCH
