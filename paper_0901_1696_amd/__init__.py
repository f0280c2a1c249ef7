"""Python binding of the MI355X RFP Cholesky library (``librfp.so``).

Argument marshalling only: every routine forwards torch device tensors (their
data pointers) and the current HIP stream to the C ABI declared in
``include/rfp.h``; all arithmetic happens in the library's HIP kernels.  There
is no fallback path: if the library is not built, loading fails loudly.

Array conventions (as in the C ABI):
  * RFP arrays: 1-D contiguous tensors of at least n(n+1)/2 entries.
  * Full matrices and right-hand sides: column-major, i.e. a 2-D tensor with
    ``stride(0) == 1`` (e.g. ``x.t().contiguous().t()``), leading dimension
    ``stride(1)``; a contiguous 1-D tensor is one column.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfp.so")

RFP_ERR_HANDLE = -101
RFP_ERR_RUNTIME = -102
RFP_ERR_SCRATCH = -103
LAYOUTS = [(t, u) for t in "NT" for u in "LU"]
PREC_FP32, PREC_FP16, PREC_BF16, PREC_FP64 = 0, 1, 2, 3

_lib = None


class RfpError(RuntimeError):
    def __init__(self, routine, code):
        self.code = code
        what = {RFP_ERR_HANDLE: "bad handle", RFP_ERR_RUNTIME: "HIP runtime error",
                RFP_ERR_SCRATCH: "problem exceeds the fixed scratch"}.get(
            code, f"illegal argument {-code}" if code < 0 else f"status {code}")
        super().__init__(f"{routine}: {what} (return code {code})")


_i64 = ctypes.c_int64
_chr = ctypes.c_char
_vp = ctypes.c_void_p
_int = ctypes.c_int

_SIGS = {
    "rfp_create": [ctypes.POINTER(_vp), _int],
    "rfp_destroy": [_vp],
    "rfp_dtrttf": [_vp, _chr, _chr, _i64, _vp, _i64, _vp, _vp],
    "rfp_dtfttr": [_vp, _chr, _chr, _i64, _vp, _vp, _i64, _vp],
    "rfp_dpftrf": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_dpftrs": [_vp, _chr, _chr, _i64, _i64, _vp, _vp, _i64, _vp],
    "rfp_dpftrs_noalloc": [_chr, _chr, _i64, _i64, _vp, _vp, _i64, _vp],
    "rfp_dtftri": [_vp, _chr, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_dtfsm": [_vp, _chr, _chr, _chr, _chr, _chr, _i64, _i64, ctypes.c_double, _vp, _vp, _i64, _vp],
    "rfp_dsfrk": [_vp, _chr, _chr, _chr, _i64, _i64, ctypes.c_double, _vp, _i64, ctypes.c_double, _vp, _vp],
    "rfp_dtpttf": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_dtfttp": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_dpftri": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_strttf": [_vp, _chr, _chr, _i64, _vp, _i64, _vp, _vp],
    "rfp_stfttr": [_vp, _chr, _chr, _i64, _vp, _vp, _i64, _vp],
    "rfp_spftrf": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_spftrs": [_vp, _chr, _chr, _i64, _i64, _vp, _vp, _i64, _vp],
    "rfp_spftri": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_spftrf_mp": [_vp, _int, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_dpfcast_s": [_vp, _chr, _chr, _i64, _vp, _int, ctypes.c_double, ctypes.c_double, _vp, _vp, _vp],
    "rfp_set_lowp_shift": [_vp, _int, ctypes.c_double],
    "rfp_get_lowp_shift": [_vp, _int, _vp],
    "rfp_dlansf": [_vp, _chr, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_dsfmv": [_vp, _chr, _chr, _i64, _i64, ctypes.c_double, _vp, _vp, _i64, ctypes.c_double, _vp, _i64, _vp],
    "rfp_autotune": [_vp, _i64, _i64, _int, _vp],
    "rfp_tune_count": [_vp],
    "rfp_tune_clear": [_vp],
    "rfp_tune_force": [_vp, _int, _int],
    "rfp_tune_save": [_vp, ctypes.c_char_p],
    "rfp_tune_load": [_vp, ctypes.c_char_p],
    "rfp_pfsv_vbatched": [_vp, _int, _i64, _vp, _vp, _vp, _vp, _int, ctypes.c_double, _int, _vp, _vp, _vp],
    "rfp_dpfsv_ir": [_vp, _int, _chr, _chr, _i64, _i64, _vp, _vp, _i64, _vp, _i64, ctypes.c_double, _int,
                     _vp, _vp, _vp],
    "rfp_solve_status": [_vp, _vp, _vp],
    "rfp_set_solve_wait_limit": [_vp, _i64],
    "rfp_plan": [_chr, _chr, _chr, _i64, _i64, _i64, _vp, _vp, _i64, ctypes.POINTER(_i64)],
    "rfp_set_schedule": [_vp, _vp],
    "rfp_get_schedule": [_vp, _vp],
    "rfp_profile_enable": [_vp, _int],
    "rfp_profile_read": [_vp, _vp, _int, ctypes.POINTER(_int)],
    "rfp_ztrttf": [_vp, _chr, _chr, _i64, _vp, _i64, _vp, _vp],
    "rfp_ztfttr": [_vp, _chr, _chr, _i64, _vp, _vp, _i64, _vp],
    "rfp_zpftrf": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
    "rfp_zpftrs": [_vp, _chr, _chr, _i64, _i64, _vp, _vp, _i64, _vp],
    "rfp_zpftri": [_vp, _chr, _chr, _i64, _vp, _vp, _vp],
}


class ProfileEntry(ctypes.Structure):
    """Layout of ``rfp_profile_entry`` (include/rfp.h)."""
    _fields_ = [("name", ctypes.c_char * 160), ("launches", _i64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]

PLAN_GEMM, PLAN_POTRF_LEAF, PLAN_TRTRI_LEAF, PLAN_TRTRI_LEAVES, PLAN_LAUUM_LEAF = 1, 2, 3, 4, 5
PLAN_RECORD, PLAN_WAIT, PLAN_BLOCK_SOLVE, PLAN_AXPY, PLAN_COPY = 6, 7, 8, 9, 10
PLAN_BUF_ARF, PLAN_BUF_B, PLAN_BUF_WORK = 0, 1, 2


class PlanOp(ctypes.Structure):
    """One record of ``rfp_plan`` (layout of ``rfp_plan_op`` in include/rfp.h)."""
    _fields_ = [("kind", ctypes.c_int32), ("tri_a", ctypes.c_int32), ("tri_b", ctypes.c_int32),
                ("c_lower", ctypes.c_int32), ("inplace", ctypes.c_int32), ("stream", ctypes.c_int32),
                ("m", _i64), ("n", _i64), ("k", _i64),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("a", _i64 * 4), ("b", _i64 * 4), ("c", _i64 * 4), ("info_base", _i64),
                ("d", _i64 * 4), ("w", _i64 * 4)]


def exported_symbols():
    """Names the C ABI exports (the declarations of include/rfp.h)."""
    return list(_SIGS)


def lib():
    """Load ``librfp.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_0901_1696_amd.build` "
                               "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _int
        _lib = L
    return _lib


def nt(n):
    return n * (n + 1) // 2


def _c(ch):
    return ch.encode() if isinstance(ch, str) else ch


def _stream(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _colmajor(x, name):
    """(pointer, leading dimension, ncols) of a column-major tensor."""
    if x.dim() == 1:
        if not x.is_contiguous():
            raise ValueError(f"{name}: 1-D tensor must be contiguous")
        return x.data_ptr(), max(1, x.shape[0]), 1
    if x.dim() != 2 or (x.stride(0) != 1 and x.shape[0] > 1):
        raise ValueError(f"{name}: expected a column-major 2-D tensor (stride(0) == 1)")
    return x.data_ptr(), max(1, x.stride(1) if x.shape[1] > 1 else x.shape[0]), x.shape[1]


def _check(routine, code):
    if code != 0:
        raise RfpError(routine, code)


class Handle:
    """Owns an ``rfp_handle_t`` (scratch memory on one device)."""

    def __init__(self, device=0):
        h = _vp()
        _check("rfp_create", lib().rfp_create(ctypes.byref(h), int(device)))
        self._h = h
        self.device = device

    @property
    def value(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().rfp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rfp_profile_enable(h, on=True):
    _check("rfp_profile_enable", lib().rfp_profile_enable(h.value, 1 if on else 0))


def rfp_profile_read(h):
    """{kernel name: dict(launches, total_ms, flops, bytes)}; waits for the device and resets."""
    count = _int(0)
    _check("rfp_profile_read", lib().rfp_profile_read(h.value, None, 0, ctypes.byref(count)))
    buf = (ProfileEntry * max(1, count.value))()
    _check("rfp_profile_read", lib().rfp_profile_read(h.value, buf, count.value, ctypes.byref(count)))
    return {e.name.decode(): dict(launches=e.launches, total_ms=e.total_ms, flops=e.flops, bytes=e.bytes)
            for e in list(buf)[:count.value]}


class Schedule(ctypes.Structure):
    """Layout of ``rfp_schedule_t`` (include/rfp.h): the factorization schedule knobs."""
    _fields_ = [("wide_panels_above", _i64), ("chunk_max", _i64), ("lookahead_wait_below", _i64),
                ("leaf_lds_pad", _i64), ("wide_panel_cols", _i64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


INT64_MAX = 2 ** 63 - 1
DEFAULT_SCHEDULE = dict(wide_panels_above=6144, chunk_max=1536, lookahead_wait_below=INT64_MAX,
                        leaf_lds_pad=24576, wide_panel_cols=256)


def _schedule(sched):
    """A Schedule from None (the defaults), a Schedule, or a dict of fields
    (missing fields take their defaults)."""
    if sched is None or isinstance(sched, Schedule):
        return sched
    vals = dict(DEFAULT_SCHEDULE)
    vals.update(sched)
    return Schedule(**vals)


def rfp_set_schedule(h, sched=None):
    """Set the handle's factorization schedule (None restores the defaults)."""
    sc = _schedule(sched)
    _check("rfp_set_schedule", lib().rfp_set_schedule(h.value, None if sc is None else ctypes.byref(sc)))


def rfp_get_schedule(h):
    sc = Schedule()
    _check("rfp_get_schedule", lib().rfp_get_schedule(h.value, ctypes.byref(sc)))
    return sc.as_dict()


def rfp_plan(routine, transr, uplo, n, nrhs=0, ldb=None, sched=None):
    """Primitive sequence of PFTRF ('F'), PFTRS ('S') or PFTRI ('I'), recorded
    on the host without touching a device (see include/rfp.h); sched as for
    :func:`rfp_set_schedule`."""
    ldb = max(1, n) if ldb is None else ldb
    sc = _schedule(sched)
    psc = None if sc is None else ctypes.byref(sc)
    count = _i64(0)
    rc = lib().rfp_plan(_c(routine), _c(transr), _c(uplo), n, nrhs, ldb, psc, None, 0, ctypes.byref(count))
    if rc != 0:
        raise RfpError("rfp_plan", rc)
    ops = (PlanOp * max(1, count.value))()
    rc = lib().rfp_plan(_c(routine), _c(transr), _c(uplo), n, nrhs, ldb, psc, ops, count.value,
                        ctypes.byref(count))
    if rc != 0:
        raise RfpError("rfp_plan", rc)
    return list(ops)[:count.value]


def rfp_dtrttf(h, transr, uplo, n, a, arf, stream=None):
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_dtrttf", lib().rfp_dtrttf(h.value, _c(transr), _c(uplo), n, pa, lda, _ptr(arf), _stream(stream)))


def rfp_dtfttr(h, transr, uplo, n, arf, a, stream=None):
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_dtfttr", lib().rfp_dtfttr(h.value, _c(transr), _c(uplo), n, _ptr(arf), pa, lda, _stream(stream)))


def rfp_dpftrf(h, transr, uplo, n, arf, info, stream=None):
    _check("rfp_dpftrf", lib().rfp_dpftrf(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def rfp_dpftrs(h, transr, uplo, n, arf, b, stream=None):
    pb, ldb, nrhs = _colmajor(b, "b")
    _check("rfp_dpftrs", lib().rfp_dpftrs(h.value, _c(transr), _c(uplo), n, nrhs, _ptr(arf), pb, ldb,
                                          _stream(stream)))


def rfp_dpftrs_noalloc(transr, uplo, n, arf, b, stream=None):
    """PFTRS with the library's fixed scratch (no handle, no allocation)."""
    pb, ldb, nrhs = _colmajor(b, "b")
    _check("rfp_dpftrs_noalloc", lib().rfp_dpftrs_noalloc(_c(transr), _c(uplo), n, nrhs, _ptr(arf), pb, ldb,
                                                          _stream(stream)))


def rfp_dpftri(h, transr, uplo, n, arf, info, stream=None):
    _check("rfp_dpftri", lib().rfp_dpftri(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def _zcheck(t, name):
    import torch
    if t.dtype != torch.complex128:
        raise ValueError(f"{name}: expected a torch.complex128 tensor")


def rfp_ztrttf(h, transr, uplo, n, a, arf, stream=None):
    """Complex: full Hermitian (column-major complex128) -> complex RFP (TRANSR 'N' or 'C')."""
    _zcheck(a, "a")
    _zcheck(arf, "arf")
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_ztrttf", lib().rfp_ztrttf(h.value, _c(transr), _c(uplo), n, pa, lda, _ptr(arf), _stream(stream)))


def rfp_ztfttr(h, transr, uplo, n, arf, a, stream=None):
    _zcheck(a, "a")
    _zcheck(arf, "arf")
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_ztfttr", lib().rfp_ztfttr(h.value, _c(transr), _c(uplo), n, _ptr(arf), pa, lda, _stream(stream)))


def rfp_zpftrf(h, transr, uplo, n, arf, info, stream=None):
    _zcheck(arf, "arf")
    _check("rfp_zpftrf", lib().rfp_zpftrf(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def rfp_zpftrs(h, transr, uplo, n, arf, b, stream=None):
    _zcheck(arf, "arf")
    _zcheck(b, "b")
    pb, ldb, nrhs = _colmajor(b, "b")
    _check("rfp_zpftrs", lib().rfp_zpftrs(h.value, _c(transr), _c(uplo), n, nrhs, _ptr(arf), pb, ldb,
                                          _stream(stream)))


def rfp_zpftri(h, transr, uplo, n, arf, info, stream=None):
    _zcheck(arf, "arf")
    _check("rfp_zpftri", lib().rfp_zpftri(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def rfp_dtftri(h, transr, uplo, diag, n, arf, info, stream=None):
    _check("rfp_dtftri", lib().rfp_dtftri(h.value, _c(transr), _c(uplo), _c(diag), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def rfp_dtfsm(h, transr, side, uplo, trans, diag, alpha, arf, b, stream=None):
    """B (m x n, column-major tensor) <- X as in TFSM; m, n from b."""
    pb, ldb, n = _colmajor(b, "b")
    m = b.shape[0]
    _check("rfp_dtfsm", lib().rfp_dtfsm(h.value, _c(transr), _c(side), _c(uplo), _c(trans), _c(diag), m, n,
                                        float(alpha), _ptr(arf), pb, ldb, _stream(stream)))


def rfp_dsfrk(h, transr, uplo, trans, n, k, alpha, a, beta, c, stream=None):
    """C (RFP) <- alpha op(A) op(A)^T + beta C; a column-major (n x k or k x n)."""
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_dsfrk", lib().rfp_dsfrk(h.value, _c(transr), _c(uplo), _c(trans), n, k, float(alpha), pa, lda,
                                        float(beta), _ptr(c), _stream(stream)))


def rfp_dtpttf(h, transr, uplo, n, ap, arf, stream=None):
    _check("rfp_dtpttf", lib().rfp_dtpttf(h.value, _c(transr), _c(uplo), n, _ptr(ap), _ptr(arf), _stream(stream)))


def rfp_dtfttp(h, transr, uplo, n, arf, ap, stream=None):
    _check("rfp_dtfttp", lib().rfp_dtfttp(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(ap), _stream(stream)))


def rfp_strttf(h, transr, uplo, n, a, arf, stream=None):
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_strttf", lib().rfp_strttf(h.value, _c(transr), _c(uplo), n, pa, lda, _ptr(arf), _stream(stream)))


def rfp_stfttr(h, transr, uplo, n, arf, a, stream=None):
    pa, lda, _ = _colmajor(a, "a")
    _check("rfp_stfttr", lib().rfp_stfttr(h.value, _c(transr), _c(uplo), n, _ptr(arf), pa, lda, _stream(stream)))


def rfp_spftrf(h, transr, uplo, n, arf, info, stream=None):
    _check("rfp_spftrf", lib().rfp_spftrf(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def rfp_spftrs(h, transr, uplo, n, arf, b, stream=None):
    pb, ldb, nrhs = _colmajor(b, "b")
    _check("rfp_spftrs", lib().rfp_spftrs(h.value, _c(transr), _c(uplo), n, nrhs, _ptr(arf), pb, ldb,
                                          _stream(stream)))


def rfp_spftri(h, transr, uplo, n, arf, info, stream=None):
    _check("rfp_spftri", lib().rfp_spftri(h.value, _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                          _stream(stream)))


def rfp_spftrf_mp(h, fprec, transr, uplo, n, arf, info, stream=None):
    _check("rfp_spftrf_mp", lib().rfp_spftrf_mp(h.value, int(fprec), _c(transr), _c(uplo), n, _ptr(arf), _ptr(info),
                                                _stream(stream)))


def rfp_dpfcast_s(h, transr, uplo, n, arf, scale, mu, s, arf32, shift=0.0, stream=None):
    _check("rfp_dpfcast_s", lib().rfp_dpfcast_s(h.value, _c(transr), _c(uplo), n, _ptr(arf), int(scale), float(mu),
                                                float(shift), _ptr(s), _ptr(arf32), _stream(stream)))


def rfp_set_lowp_shift(h, fprec, c):
    """Diagonal shift of the fprec low-precision factors, in units of that
    precision's unit roundoff (0 switches it off)."""
    _check("rfp_set_lowp_shift", lib().rfp_set_lowp_shift(h.value, int(fprec), float(c)))


def rfp_get_lowp_shift(h, fprec):
    out = ctypes.c_double()
    _check("rfp_get_lowp_shift", lib().rfp_get_lowp_shift(h.value, int(fprec), ctypes.byref(out)))
    return out.value


def rfp_dsfmv(h, transr, uplo, n, alpha, arf, x, beta, y, stream=None):
    """Y = alpha A X + beta Y, A symmetric in RFP; x and y column-major
    (n x nrhs) device tensors."""
    px, ldx, nrhs = _colmajor(x, "x")
    py, ldy, ny = _colmajor(y, "y")
    if ny != nrhs:
        raise ValueError("x and y must have the same number of columns")
    _check("rfp_dsfmv", lib().rfp_dsfmv(h.value, _c(transr), _c(uplo), n, nrhs, float(alpha), _ptr(arf), px, ldx,
                                        float(beta), py, ldy, _stream(stream)))


def rfp_dlansf(h, norm, transr, uplo, n, arf, out, stream=None):
    _check("rfp_dlansf", lib().rfp_dlansf(h.value, _c(norm), _c(transr), _c(uplo), n, _ptr(arf), _ptr(out),
                                          _stream(stream)))


def rfp_dpfsv_ir(h, fprec, transr, uplo, n, arf, b, x, iter, info, tol=1e-14, max_iter=20, stream=None):
    """Mixed-precision solve with FP64 refinement.  iter and info are device
    int32 tensors (one element each) that receive the sweep count or fall-back
    reason and the fall-back's INFO; nothing synchronises."""
    pb, ldb, nrhs = _colmajor(b, "b")
    px, ldx, nx = _colmajor(x, "x")
    if nx != nrhs:
        raise ValueError("x and b must have the same number of columns")
    _check("rfp_dpfsv_ir", lib().rfp_dpfsv_ir(h.value, int(fprec), _c(transr), _c(uplo), n, nrhs, _ptr(arf), pb, ldb,
                                              px, ldx, float(tol), int(max_iter), _ptr(iter), _ptr(info),
                                              _stream(stream)))


def rfp_solve_status(h, status, stream=None):
    """Copy the handle's fused-solve status word into the device int32 tensor
    `status` and clear it (bit 0: a bounded wait gave up)."""
    _check("rfp_solve_status", lib().rfp_solve_status(h.value, _ptr(status), _stream(stream)))


def rfp_set_solve_wait_limit(h, polls):
    _check("rfp_set_solve_wait_limit", lib().rfp_set_solve_wait_limit(h.value, int(polls)))


class SysDesc(ctypes.Structure):
    """Layout of ``rfp_sys_t`` (include/rfp.h): one system of a batch."""
    _fields_ = [("n", _i64), ("arf_off", _i64), ("b_off", _i64), ("ldb", _i64), ("nrhs", _i64),
                ("transr", ctypes.c_char), ("uplo", ctypes.c_char), ("pad", ctypes.c_char * 6)]


def sys_table(systems):
    """Bytes of an ``rfp_sys_t`` array from (n, arf_off, b_off, ldb, nrhs, transr, uplo) tuples."""
    arr = (SysDesc * max(1, len(systems)))()
    for k, (n, ao, bo, ldb, nr, t, u) in enumerate(systems):
        arr[k] = SysDesc(n, ao, bo, ldb, nr, _c(t), _c(u), b"")
    return bytes(arr)[:ctypes.sizeof(SysDesc) * len(systems)]


def rfp_pfsv_vbatched(h, fprec, batch, sys, arf_pool, b_pool, info, iter, sys_host=None, do_pftri=False,
                      tol=1e-14, max_iter=20, stream=None):
    """sys: device tensor holding the ``rfp_sys_t`` table (e.g. a uint8 tensor
    from :func:`sys_table`); sys_host: the same table as bytes on the host
    (needed for systems with n > 256, which are refused without it)."""
    hbuf = None
    if sys_host is not None:
        hbuf = (ctypes.c_char * max(1, len(sys_host))).from_buffer_copy(bytes(sys_host) or b"\0")
    _check("rfp_pfsv_vbatched", lib().rfp_pfsv_vbatched(h.value, int(fprec), int(batch), _ptr(sys),
                                                        None if hbuf is None else ctypes.addressof(hbuf),
                                                        _ptr(arf_pool), _ptr(b_pool), 1 if do_pftri else 0,
                                                        float(tol), int(max_iter), _ptr(info), _ptr(iter),
                                                        _stream(stream)))


TUNE_FP64, TUNE_FP32, TUNE_FP16, TUNE_BF16, TUNE_SCHEDULE = 1, 2, 4, 8, 16


def rfp_autotune(h, n, nrhs=0, precs=TUNE_FP64, stream=None):
    _check("rfp_autotune", lib().rfp_autotune(h.value, int(n), int(nrhs), int(precs), _stream(stream)))


def rfp_tune_count(h):
    c = lib().rfp_tune_count(h.value)
    if c < 0:
        raise RfpError("rfp_tune_count", c)
    return c


def rfp_tune_clear(h):
    _check("rfp_tune_clear", lib().rfp_tune_clear(h.value))


def rfp_tune_force(h, tile, split=0):
    _check("rfp_tune_force", lib().rfp_tune_force(h.value, int(tile), int(split)))


def rfp_tune_save(h, path):
    _check("rfp_tune_save", lib().rfp_tune_save(h.value, os.fsencode(path)))


def rfp_tune_load(h, path):
    _check("rfp_tune_load", lib().rfp_tune_load(h.value, os.fsencode(path)))
