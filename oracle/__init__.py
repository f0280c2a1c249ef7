"""CPU FP64 oracle for RFP Cholesky factorization, solution and inversion.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  It shares no code with the GPU
library and never imports it.

Thin ctypes wrappers over ``rfp_oracle.c``.  Arrays are NumPy float64; full
matrices and right-hand sides are column-major (Fortran order).  The paper
passages each routine follows are cited in the C source.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load the oracle library, building it first only if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = ctypes.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


_i64 = ctypes.c_longlong
_chr = ctypes.c_char
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def _declare(L):
    L.orc_full_pos.restype = _i64
    L.orc_full_pos.argtypes = [_i64, _i64, _i64]
    L.orc_packed_pos.restype = _i64
    L.orc_packed_pos.argtypes = [_chr, _i64, _i64, _i64]
    L.orc_rfp_pos.restype = _i64
    L.orc_rfp_pos.argtypes = [_chr, _chr, _i64, _i64, _i64]
    for name in ("orc_trttf",):
        getattr(L, name).restype = None
        getattr(L, name).argtypes = [_chr, _chr, _i64, _dp, _i64, _dp]
    L.orc_tfttr.restype = None
    L.orc_tfttr.argtypes = [_chr, _chr, _i64, _dp, _dp, _i64]
    L.orc_tpttf.restype = None
    L.orc_tpttf.argtypes = [_chr, _chr, _i64, _dp, _dp]
    L.orc_tfttp.restype = None
    L.orc_tfttp.argtypes = [_chr, _chr, _i64, _dp, _dp]
    L.orc_pftrf.restype = ctypes.c_int
    L.orc_pftrf.argtypes = [_chr, _chr, _i64, _dp]
    L.orc_pftrf_srpa.restype = ctypes.c_int
    L.orc_pftrf_srpa.argtypes = [_chr, _chr, _i64, _dp]
    L.orc_srpa_blocks.restype = None
    L.orc_srpa_blocks.argtypes = [_chr, _chr, _i64, ctypes.POINTER(_i64)]
    L.orc_pftrs.restype = None
    L.orc_pftrs.argtypes = [_chr, _chr, _i64, _i64, _dp, _dp, _i64]
    L.orc_pftri.restype = ctypes.c_int
    L.orc_pftri.argtypes = [_chr, _chr, _i64, _dp]
    L.orc_norm_inf.restype = ctypes.c_double
    L.orc_norm_inf.argtypes = [_chr, _chr, _i64, _dp]
    L.orc_backward_error.restype = ctypes.c_double
    L.orc_norm_max.argtypes = [_chr, _chr, _i64, _dp]
    L.orc_norm_max.restype = ctypes.c_double
    L.orc_sfmv.argtypes = [_chr, _chr, _i64, _i64, ctypes.c_double, _dp, _dp, _i64, ctypes.c_double, _dp, _i64]
    L.orc_norm_fro.argtypes = [_chr, _chr, _i64, _dp]
    L.orc_norm_fro.restype = ctypes.c_double
    L.orc_pfcast_s.argtypes = [_chr, _chr, _i64, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _vp]
    L.orc_backward_error.argtypes = [_chr, _chr, _i64, _i64, _dp, _dp, _i64, _dp, _i64]
    L.orc_tftri.restype = ctypes.c_int
    L.orc_tftri.argtypes = [_chr, _chr, _chr, _i64, _dp]
    L.orc_tfsm.restype = None
    L.orc_tfsm.argtypes = [_chr, _chr, _chr, _chr, _chr, _i64, _i64, ctypes.c_double, _dp, _dp, _i64]
    L.orc_sfrk.restype = None
    L.orc_sfrk.argtypes = [_chr, _chr, _chr, _i64, _i64, ctypes.c_double, _dp, _i64, ctypes.c_double, _dp]
    L.orc_forward_error.restype = ctypes.c_double
    L.orc_forward_error.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
    L.orc_factor_residual.restype = ctypes.c_double
    L.orc_factor_residual.argtypes = [_chr, _chr, _i64, _dp, _dp]
    L.orc_inverse_residual.restype = ctypes.c_double
    L.orc_inverse_residual.argtypes = [_chr, _chr, _i64, _dp, _dp]
    # complex Hermitian (zrfp_oracle.c): complex arrays as interleaved doubles
    L.orc_zrfp_pos.restype = _i64
    L.orc_zrfp_pos.argtypes = [_chr, _chr, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_int)]
    L.orc_ztrttf.restype = None
    L.orc_ztrttf.argtypes = [_chr, _chr, _i64, _dp, _i64, _dp]
    L.orc_ztfttr.restype = None
    L.orc_ztfttr.argtypes = [_chr, _chr, _i64, _dp, _dp, _i64]
    for name in ("orc_zpftrf", "orc_zpftrf_srpa", "orc_zpftri"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [_chr, _chr, _i64, _dp]
    L.orc_zpftrs.restype = None
    L.orc_zpftrs.argtypes = [_chr, _chr, _i64, _i64, _dp, _dp, _i64]
    L.orc_zbackward_error.restype = ctypes.c_double
    L.orc_zbackward_error.argtypes = [_chr, _chr, _i64, _i64, _dp, _dp, _i64, _dp, _i64]
    L.orc_zfactor_residual.restype = ctypes.c_double
    L.orc_zfactor_residual.argtypes = [_chr, _chr, _i64, _dp, _dp]
    L.orc_zinverse_residual.restype = ctypes.c_double
    L.orc_zinverse_residual.argtypes = [_chr, _chr, _i64, _dp, _dp]


def _c(ch):
    return ch.encode() if isinstance(ch, str) else ch


def _p(a):
    assert a.dtype == np.float64
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.require(a, dtype=np.float64, requirements=["F", "A", "W"])


def nt(n):
    """Number of stored entries n(n+1)/2 (Section 2)."""
    return n * (n + 1) // 2


# ---------------------------------------------------------------- index layer
def rfp_pos(transr, uplo, n, i, j):
    return lib().orc_rfp_pos(_c(transr), _c(uplo), n, i, j)


def packed_pos(uplo, n, i, j):
    return lib().orc_packed_pos(_c(uplo), n, i, j)


def full_pos(lda, i, j):
    return lib().orc_full_pos(lda, i, j)


def trttf(transr, uplo, a):
    """Full (column-major, lda = a.shape[0]) -> RFP array of n(n+1)/2."""
    a = _f64(a)
    n = a.shape[1]
    arf = np.zeros(nt(n))
    lib().orc_trttf(_c(transr), _c(uplo), n, _p(a), a.shape[0], _p(arf))
    return arf


def tfttr(transr, uplo, n, arf, lda=None, fill=0.0):
    lda = n if lda is None else lda
    a = np.full((lda, n), fill, order="F")
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    lib().orc_tfttr(_c(transr), _c(uplo), n, _p(arf), _p(a), lda)
    return a


def tpttf(transr, uplo, n, ap):
    ap = np.ascontiguousarray(ap, dtype=np.float64)
    arf = np.zeros(nt(n))
    lib().orc_tpttf(_c(transr), _c(uplo), n, _p(ap), _p(arf))
    return arf


def tfttp(transr, uplo, n, arf):
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    ap = np.zeros(nt(n))
    lib().orc_tfttp(_c(transr), _c(uplo), n, _p(arf), _p(ap))
    return ap


def srpa_blocks(transr, uplo, n):
    out = (_i64 * 11)()
    lib().orc_srpa_blocks(_c(transr), _c(uplo), n, out)
    v = list(out)
    return {"m1": v[0], "m2": v[1], "t1": tuple(v[2:5]), "s": tuple(v[5:8]), "t2": tuple(v[8:11])}


# ----------------------------------------------------------------- numerics
def pftrf(transr, uplo, n, arf):
    """Definition-path factor.  Returns (factor RFP array, info)."""
    out = np.array(arf, dtype=np.float64, copy=True)
    info = lib().orc_pftrf(_c(transr), _c(uplo), n, _p(out))
    return out, info


def pftrf_srpa(transr, uplo, n, arf):
    """The paper's four-step path.  Returns (factor RFP array, info)."""
    out = np.array(arf, dtype=np.float64, copy=True)
    info = lib().orc_pftrf_srpa(_c(transr), _c(uplo), n, _p(out))
    return out, info


def pftrs(transr, uplo, n, arf_factor, b):
    """Solve with the factor; b is n x nrhs (any order).  Returns X (F order)."""
    x = np.array(b, dtype=np.float64, order="F", copy=True)
    if x.ndim == 1:
        x = x.reshape(-1, 1, order="F")
    arf_factor = np.ascontiguousarray(arf_factor, dtype=np.float64)
    lib().orc_pftrs(_c(transr), _c(uplo), n, x.shape[1], _p(arf_factor), _p(x), x.shape[0])
    return x


def pftri(transr, uplo, n, arf_factor):
    """Inverse from the factor.  Returns (RFP of A^{-1}, info)."""
    out = np.array(arf_factor, dtype=np.float64, copy=True)
    info = lib().orc_pftri(_c(transr), _c(uplo), n, _p(out))
    return out, info


# ------------------------------------------------------------------ metrics
def norm_inf(transr, uplo, n, arf):
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    return lib().orc_norm_inf(_c(transr), _c(uplo), n, _p(arf))


def norm_max(transr, uplo, n, arf):
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    return lib().orc_norm_max(_c(transr), _c(uplo), n, _p(arf))


def sfmv(transr, uplo, n, alpha, arf, x, beta, y):
    """alpha A X + beta Y for the symmetric A in RFP (x, y: n x nrhs)."""
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    x = np.asfortranarray(np.asarray(x, dtype=np.float64).reshape(n, -1))
    y = np.asfortranarray(np.array(y, dtype=np.float64).reshape(n, -1))
    nrhs = x.shape[1]
    lib().orc_sfmv(_c(transr), _c(uplo), n, nrhs, float(alpha), _p(arf), _p(x), max(1, n), float(beta), _p(y),
                   max(1, n))
    return y


def norm_fro(transr, uplo, n, arf):
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    return lib().orc_norm_fro(_c(transr), _c(uplo), n, _p(arf))


def pfcast_s(transr, uplo, n, arf, scale=True, mu=1.0, shift=0.0):
    """(s, arf32): diagonal scaling vector and the scaled (and diagonally
    shifted) FP32 RFP copy."""
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    s = np.empty(n)
    out = np.zeros(arf.size, dtype=np.float32)
    lib().orc_pfcast_s(_c(transr), _c(uplo), n, _p(arf), 1 if scale else 0, float(mu), float(shift), _p(s),
                       out.ctypes.data_as(_vp))
    return s, out


def backward_error(transr, uplo, n, arf_a, b, x):
    b = _f64(b if b.ndim == 2 else b.reshape(-1, 1))
    x = _f64(x if x.ndim == 2 else x.reshape(-1, 1))
    arf_a = np.ascontiguousarray(arf_a, dtype=np.float64)
    return lib().orc_backward_error(_c(transr), _c(uplo), n, b.shape[1], _p(arf_a),
                                    _p(b), b.shape[0], _p(x), x.shape[0])


def tftri(transr, uplo, diag, n, arf):
    """TFTRI: (inverse in RFP, info); the input array is not modified."""
    out = np.ascontiguousarray(arf, dtype=np.float64).copy()
    info = lib().orc_tftri(_c(transr), _c(uplo), _c(diag), n, _p(out))
    return out, info


def tfsm(transr, side, uplo, trans, diag, m, n, alpha, arf, b):
    """TFSM: returns X (m x n, Fortran order); b is not modified."""
    arf = np.ascontiguousarray(arf, dtype=np.float64)
    x = np.array(b, dtype=np.float64, order="F", copy=True)
    lib().orc_tfsm(_c(transr), _c(side), _c(uplo), _c(trans), _c(diag), m, n, float(alpha), _p(arf), _p(x),
                   max(1, x.shape[0]))
    return x


def sfrk(transr, uplo, trans, n, k, alpha, a, beta, c):
    """SFRK: returns the updated RFP array; c is not modified.  a is the
    n x k (TRANS='N') or k x n (TRANS='T') column-major matrix."""
    a = _f64(a)
    out = np.ascontiguousarray(c, dtype=np.float64).copy()
    lib().orc_sfrk(_c(transr), _c(uplo), _c(trans), n, k, float(alpha), _p(a), max(1, a.shape[0]), float(beta),
                   _p(out))
    return out


def forward_error(x, x_ref):
    """max over columns ||x - x_ref||_inf / ||x_ref||_inf."""
    x = _f64(x if x.ndim == 2 else x.reshape(-1, 1))
    x_ref = _f64(x_ref if x_ref.ndim == 2 else x_ref.reshape(-1, 1))
    assert x.shape == x_ref.shape
    return lib().orc_forward_error(x.shape[0], x.shape[1], _p(x), x.shape[0], _p(x_ref), x_ref.shape[0])


def factor_residual(transr, uplo, n, arf_a, arf_l):
    arf_a = np.ascontiguousarray(arf_a, dtype=np.float64)
    arf_l = np.ascontiguousarray(arf_l, dtype=np.float64)
    return lib().orc_factor_residual(_c(transr), _c(uplo), n, _p(arf_a), _p(arf_l))


def inverse_residual(transr, uplo, n, arf_a, arf_inv):
    arf_a = np.ascontiguousarray(arf_a, dtype=np.float64)
    arf_inv = np.ascontiguousarray(arf_inv, dtype=np.float64)
    return lib().orc_inverse_residual(_c(transr), _c(uplo), n, _p(arf_a), _p(arf_inv))


def rel_fro(x, ref):
    """Relative Frobenius difference ||x - ref||_F / ||ref||_F (plain NumPy)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm((x - ref).ravel())
    r = np.linalg.norm(ref.ravel())
    return d / r if r > 0 else d


LAYOUTS = [(t, u) for t in "NT" for u in "LU"]


# ------------------------------------------------- complex Hermitian (zrfp)
ZLAYOUTS = [(t, u) for t in "NC" for u in "LU"]


def _zp(a):
    assert a.dtype == np.complex128 and (a.flags["C_CONTIGUOUS"] or a.flags["F_CONTIGUOUS"])
    return a.ctypes.data_as(_dp)


def _z(a, order="F"):
    return np.array(a, dtype=np.complex128, order=order, copy=True)


def zrfp_pos(transr, uplo, n, i, j):
    """(offset, stored number is the conjugate) of stored-triangle element (i, j)."""
    c = ctypes.c_int(0)
    p = lib().orc_zrfp_pos(_c(transr), _c(uplo), n, i, j, ctypes.byref(c))
    return p, bool(c.value)


def ztrttf(transr, uplo, a):
    """Full complex (column-major) -> complex RFP array of n(n+1)/2."""
    a = _z(a)
    n = a.shape[1]
    arf = np.zeros(nt(n), dtype=np.complex128)
    lib().orc_ztrttf(_c(transr), _c(uplo), n, _zp(a), a.shape[0], _zp(arf))
    return arf


def ztfttr(transr, uplo, n, arf, fill=0.0):
    a = np.full((n, n), fill, dtype=np.complex128, order="F")
    arf = np.ascontiguousarray(arf, dtype=np.complex128)
    lib().orc_ztfttr(_c(transr), _c(uplo), n, _zp(arf), _zp(a), max(n, 1))
    return a


def zpftrf(transr, uplo, n, arf):
    """Definition-path complex factor.  Returns (factor array, info)."""
    out = np.array(arf, dtype=np.complex128, copy=True)
    return out, lib().orc_zpftrf(_c(transr), _c(uplo), n, _zp(out))


def zpftrf_srpa(transr, uplo, n, arf):
    """The paper's four steps, complex Hermitian.  Returns (factor array, info)."""
    out = np.array(arf, dtype=np.complex128, copy=True)
    return out, lib().orc_zpftrf_srpa(_c(transr), _c(uplo), n, _zp(out))


def zpftrs(transr, uplo, n, arf_factor, b):
    x = np.array(b, dtype=np.complex128, order="F", copy=True)
    if x.ndim == 1:
        x = x.reshape(-1, 1, order="F")
    arf_factor = np.ascontiguousarray(arf_factor, dtype=np.complex128)
    lib().orc_zpftrs(_c(transr), _c(uplo), n, x.shape[1], _zp(arf_factor), _zp(x), x.shape[0])
    return x


def zpftri(transr, uplo, n, arf_factor):
    out = np.array(arf_factor, dtype=np.complex128, copy=True)
    return out, lib().orc_zpftri(_c(transr), _c(uplo), n, _zp(out))


def zbackward_error(transr, uplo, n, arf_a, b, x):
    b = _z(b if b.ndim == 2 else b.reshape(-1, 1))
    x = _z(x if x.ndim == 2 else x.reshape(-1, 1))
    arf_a = np.ascontiguousarray(arf_a, dtype=np.complex128)
    return lib().orc_zbackward_error(_c(transr), _c(uplo), n, b.shape[1], _zp(arf_a), _zp(b), b.shape[0],
                                     _zp(x), x.shape[0])


def zfactor_residual(transr, uplo, n, arf_a, arf_l):
    arf_a = np.ascontiguousarray(arf_a, dtype=np.complex128)
    arf_l = np.ascontiguousarray(arf_l, dtype=np.complex128)
    return lib().orc_zfactor_residual(_c(transr), _c(uplo), n, _zp(arf_a), _zp(arf_l))


def zinverse_residual(transr, uplo, n, arf_a, arf_inv):
    arf_a = np.ascontiguousarray(arf_a, dtype=np.complex128)
    arf_inv = np.ascontiguousarray(arf_inv, dtype=np.complex128)
    return lib().orc_zinverse_residual(_c(transr), _c(uplo), n, _zp(arf_a), _zp(arf_inv))
