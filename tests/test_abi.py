"""The C ABI library loads on a machine without a GPU and exports every
entry point that include/rfp.h declares; argument checking follows the
paper's argument order (checked through the host-only plan entry point,
which shares the validation code of the real calls)."""
import ctypes
import os
import re

import pytest

import paper_0901_1696_amd as rfp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "rfp.h")).read()
    return sorted(set(re.findall(r"^int\s+(rfp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_names():
    assert declared() == sorted(rfp.exported_symbols())


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rfp.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


def test_null_handle_is_rejected():
    L = rfp.lib()
    assert L.rfp_dpftrf(None, b"N", b"L", 3, None, None, None) == rfp.RFP_ERR_HANDLE
    assert L.rfp_dpftrs(None, b"N", b"L", 3, 1, None, None, 3, None) == rfp.RFP_ERR_HANDLE
    assert L.rfp_dpftri(None, b"N", b"L", 3, None, None, None) == rfp.RFP_ERR_HANDLE
    assert L.rfp_destroy(None) == rfp.RFP_ERR_HANDLE
    assert L.rfp_create(None, 0) == -1


@pytest.mark.parametrize("routine", ["F", "S", "I"])
def test_argument_codes(routine):
    def code(transr="N", uplo="L", n=4, nrhs=1, ldb=4):
        try:
            rfp.rfp_plan(routine, transr, uplo, n, nrhs, ldb)
            return 0
        except rfp.RfpError as e:
            return e.code
    assert code() == 0
    assert code(transr="n", uplo="u") == 0
    assert code(transr="X") == -1
    assert code(uplo="Q") == -2
    assert code(n=-1) == -3
    if routine == "S":
        assert code(nrhs=-1) == -4
        assert code(ldb=3) == -7
        assert code(n=0, ldb=1) == 0
