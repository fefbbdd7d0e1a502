"""Thin ctypes binding of libcfx.so (include/cfx.h).

Each function marshals PyTorch CUDA tensors (row-major, FP64) into the C ABI
call of the same name and raises on a non-zero status.  No computation
happens here; if libcfx.so is missing the call raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfx.so")

PREC = {"fp64": 0, "bf16": 1, "fp16": 2, "fp8": 3}
STATUS = {0: "CFX_OK", 1: "CFX_PENDING", -1001: "CFX_ENOMEM", -1002: "CFX_EHIP",
          -1003: "CFX_EBUSY", -1004: "CFX_ENOTSUP", -1005: "CFX_ESOLVE"}

_lib = None


class LuOpts(C.Structure):
    _fields_ = [("v", C.c_int32), ("leaves", C.c_int32), ("precision", C.c_int32),
                ("lookahead", C.c_int32), ("min_leaf_rows", C.c_int32)]


class IrOpts(C.Structure):
    _fields_ = [("lu", LuOpts), ("tol", C.c_double), ("max_outer", C.c_int32),
                ("gmres_restart", C.c_int32), ("gmres_tol", C.c_double)]


class IrReport(C.Structure):
    _fields_ = [("eta", C.c_double), ("eta_first", C.c_double), ("outer", C.c_int32),
                ("inner", C.c_int32), ("converged", C.c_int32), ("info", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServeCfg(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("ir", IrOpts), ("batch_max", C.c_int32), ("lowp_min_n", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("keep_resident", C.c_int32), ("factor_id", C.c_uint64),
                ("n", C.c_int64), ("nrhs", C.c_int64), ("A", C.c_void_p), ("lda", C.c_int64),
                ("B", C.c_void_p), ("ldb", C.c_int64), ("X", C.c_void_p), ("ldx", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("info", C.c_int32), ("factor_id", C.c_uint64),
                ("resident_hit", C.c_int32), ("batched", C.c_int32), ("outer", C.c_int32),
                ("inner", C.c_int32), ("eta", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("fallback", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("resident_hits", C.c_int64), ("resident_misses", C.c_int64),
                ("evictions", C.c_int64), ("batches", C.c_int64), ("batched_requests", C.c_int64),
                ("resident_factors", C.c_int64), ("bytes_in_use", C.c_size_t),
                ("bytes_peak", C.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Profile(C.Structure):
    _fields_ = [("tslu_ms", C.c_double), ("laswp_ms", C.c_double), ("trsm_ms", C.c_double),
                ("schur_ms", C.c_double), ("schur_flops", C.c_double),
                ("schur_launches", C.c_int64), ("panels", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class CfxError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        what = STATUS.get(code, f"invalid argument {-code}" if code < 0 else str(code))
        super().__init__(f"{fn} failed: {what} ({code})")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python -m paper_2010_05975_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        sz = C.c_size_t
        L.cfx_version.restype = C.c_char_p
        L.cfx_create.argtypes = [C.POINTER(vp)]
        L.cfx_destroy.argtypes = [vp]
        L.cfx_getrf_buffer_size.argtypes = [vp, i64, C.POINTER(LuOpts), C.POINTER(sz)]
        L.cfx_getrf.argtypes = [vp, i64, vp, i64, vp, vp, C.POINTER(LuOpts), vp, sz, vp]
        L.cfx_tslu.argtypes = [vp, i64, i64, vp, i64, i64, i32, vp, vp, sz, vp]
        L.cfx_getrs.argtypes = [vp, i64, i64, vp, i64, vp, vp, i64, vp]
        L.cfx_gesv_ir_buffer_size.argtypes = [vp, i64, i64, C.POINTER(IrOpts), C.POINTER(sz)]
        L.cfx_gesv_ir.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, i64, C.POINTER(IrOpts),
                                  C.POINTER(IrReport), vp, sz, vp]
        L.cfx_gesv_batched_buffer_size.argtypes = [vp, i32, C.POINTER(sz)]
        L.cfx_gesv_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, i32, vp]
        L.cfx_batched_tune.argtypes = [vp, vp]
        L.cfx_batched_tuning.argtypes = [vp, vp]
        L.cfx_batched_set_tuning.argtypes = [vp, vp]
        L.cfx_overlap_tuning.argtypes = [vp, vp, vp, vp]
        L.cfx_set_overlap_tuning.argtypes = [vp, i32, i32, i32]
        L.cfx_serve_create.argtypes = [C.POINTER(ServeCfg), C.POINTER(vp)]
        L.cfx_serve_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.cfx_serve_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result)]
        L.cfx_serve_release.argtypes = [vp, C.c_uint64]
        L.cfx_serve_stats_get.argtypes = [vp, C.POINTER(ServeStats)]
        L.cfx_serve_destroy.argtypes = [vp]
        L.cfx_profile_begin.argtypes = [vp]
        L.cfx_profile_end.argtypes = [vp, C.POINTER(Profile)]
        L.cfx_getrs_check.argtypes = [vp, vp]
        L.cfx_schur_delay.argtypes = [vp, vp]
        L.cfx_tournament_fusion.argtypes = [vp, vp]
        L.cfx_full_trsm_rows.argtypes = [vp, vp]
        L.cfx_set_full_trsm_rows.argtypes = [vp, i32]
        L.cfx_set_tournament_fusion.argtypes = [vp, i32]
        L.cfx_set_schur_delay.argtypes = [vp, i32]
        L.cfx_reserved_cus.argtypes = [vp, vp]
        L.cfx_set_reserved_cus.argtypes = [vp, i32]
        L.cfx_getrf_masked.argtypes = [vp, i64, vp, i64, vp, vp, vp, C.POINTER(LuOpts), vp, sz, vp]
        L.cfx_getrs_masked.argtypes = [vp, i64, i64, vp, i64, vp, vp, i64, vp]
        L.cfx_getrs_noalloc.argtypes = [vp, i64, i64, vp, i64, vp, vp, i64, vp]
        L.cfx_schur_update_buffer_size.argtypes = [vp, i32, i64, i64, i64, C.POINTER(sz)]
        L.cfx_schur_update.argtypes = [vp, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, vp, sz, vp]
        L.cfx_set_solve_spin_limit.argtypes = [vp, i32]
        for f in ("cfx_create", "cfx_destroy", "cfx_getrf_buffer_size", "cfx_getrf",
                  "cfx_tslu", "cfx_getrs", "cfx_getrs_check", "cfx_set_solve_spin_limit",
                  "cfx_getrf_masked", "cfx_getrs_masked", "cfx_schur_delay", "cfx_set_schur_delay",
                  "cfx_reserved_cus", "cfx_set_reserved_cus",
                  "cfx_tournament_fusion", "cfx_set_tournament_fusion",
                  "cfx_full_trsm_rows", "cfx_set_full_trsm_rows",
                  "cfx_getrs_noalloc",
                  "cfx_schur_update_buffer_size", "cfx_schur_update",
                  "cfx_gesv_ir_buffer_size", "cfx_gesv_ir",
                  "cfx_gesv_batched_buffer_size", "cfx_gesv_batched", "cfx_batched_tune",
                  "cfx_batched_tuning", "cfx_batched_set_tuning", "cfx_serve_create",
                  "cfx_serve_submit", "cfx_serve_poll", "cfx_serve_release", "cfx_serve_stats_get",
                  "cfx_serve_destroy",
                  "cfx_profile_begin", "cfx_profile_end"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(fn, rc):
    if rc != 0:
        raise CfxError(fn, rc)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _mat(A, name):
    if A.device.type != "cuda" or A.dtype != torch.float64 or A.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float64 CUDA tensor")
    if A.stride(1) != 1:
        raise TypeError(f"{name} must be row-major (unit column stride)")
    return max(A.stride(0), A.shape[1], 1)


class Handle:
    """Owns a cfx_handle (create/destroy) on the current device."""

    def __init__(self):
        h = C.c_void_p()
        _check("cfx_create", lib().cfx_create(C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().cfx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_handle() -> Handle:
    dev = torch.cuda.current_device()
    if dev not in _default:
        _default[dev] = Handle()
    return _default[dev]


def version() -> str:
    return lib().cfx_version().decode()


def getrf_buffer_size(n, v=256, leaves=64, precision="fp64", lookahead=0, handle=None, min_leaf_rows=0):
    h = handle or default_handle()
    o = LuOpts(v, leaves, PREC[precision], lookahead, min_leaf_rows)
    b = C.c_size_t()
    _check("cfx_getrf_buffer_size", lib().cfx_getrf_buffer_size(h.h, n, C.byref(o), C.byref(b)))
    return b.value


def workspace(n, v=256, leaves=64, precision="fp64", lookahead=0, device=None, handle=None, min_leaf_rows=0):
    nbytes = getrf_buffer_size(n, v, leaves, precision, lookahead, handle, min_leaf_rows)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def getrf(A, v=256, leaves=64, precision="fp64", lookahead=0, work=None, ipiv=None, info=None,
          stream=None, handle=None, min_leaf_rows=0):
    """cfx_getrf: factor A in place; returns (ipiv int32[n], info int32[1])."""
    h = handle or default_handle()
    lda = _mat(A, "A")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    if work is None:
        work = workspace(n, v, leaves, precision, lookahead, A.device, h, min_leaf_rows)
    o = LuOpts(v, leaves, PREC[precision], lookahead, min_leaf_rows)
    _check("cfx_getrf", lib().cfx_getrf(h.h, n, _ptr(A), lda, _ptr(ipiv), _ptr(info), C.byref(o),
                                        _ptr(work), work.numel(), _stream(stream)))
    return ipiv[:n], info


def getrf_masked(A, v=256, leaves=64, precision="fp64", lookahead=0, work=None, ipiv=None, rowmap=None,
                 info=None, stream=None, handle=None, min_leaf_rows=0):
    """cfx_getrf_masked: factor A in place without moving rows; returns
    (ipiv, rowmap, info) (int32 device tensors)."""
    h = handle or default_handle()
    lda = _mat(A, "A")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    if ipiv is None:
        ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    if rowmap is None:
        rowmap = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    if info is None:
        info = torch.empty(1, dtype=torch.int32, device=A.device)
    if work is None:
        work = workspace(n, v, leaves, precision, lookahead, A.device, h, min_leaf_rows)
    o = LuOpts(v, leaves, PREC[precision], lookahead, min_leaf_rows)
    _check("cfx_getrf_masked", lib().cfx_getrf_masked(h.h, n, _ptr(A), lda, _ptr(ipiv), _ptr(rowmap), _ptr(info),
                                                      C.byref(o), _ptr(work), work.numel(), _stream(stream)))
    return ipiv, rowmap, info


def getrs_masked(LU, rowmap, B, stream=None, handle=None):
    """cfx_getrs_masked: solve in place in B with the factors of getrf_masked."""
    h = handle or default_handle()
    lda = _mat(LU, "LU")
    Bm = B.view(-1, 1) if B.dim() == 1 else B
    ldb = _mat(Bm, "B")
    n, nrhs = Bm.shape
    _check("cfx_getrs_masked", lib().cfx_getrs_masked(h.h, n, nrhs, _ptr(LU), lda, _ptr(rowmap), _ptr(Bm), ldb,
                                                      _stream(stream)))
    return B


def tslu(W, vb, leaves, row0=0, work=None, stream=None, handle=None):
    """cfx_tslu: tournament pivots of the panel W[:, :vb]; returns int32[vb]."""
    h = handle or default_handle()
    ldw = _mat(W, "W")
    rows = W.shape[0]
    piv = torch.empty(vb, dtype=torch.int32, device=W.device)
    if work is None:
        work = workspace(rows, vb, leaves, "fp64", 0, W.device, h)
    _check("cfx_tslu", lib().cfx_tslu(h.h, rows, vb, _ptr(W), ldw, row0, leaves, _ptr(piv),
                                      _ptr(work), work.numel(), _stream(stream)))
    return piv


def getrs(LU, ipiv, B, stream=None, handle=None):
    """cfx_getrs: solve in place in B (n x nrhs, or n) with the factors of getrf."""
    h = handle or default_handle()
    lda = _mat(LU, "LU")
    vec = B.dim() == 1
    Bm = B.view(-1, 1) if vec else B
    ldb = _mat(Bm, "B")
    n, nrhs = Bm.shape
    _check("cfx_getrs", lib().cfx_getrs(h.h, n, nrhs, _ptr(LU), lda, _ptr(ipiv), _ptr(Bm), ldb,
                                        _stream(stream)))
    return B


def schur_update(L21, U12, Cm, precision="fp64", max_workgroups=0, work=None, stream=None, handle=None):
    """cfx_schur_update: Cm -= L21 U12 in place (Cm m x n, L21 m x K, U12 K x n,
    row-major float64 CUDA tensors with unit column stride)."""
    h = handle or default_handle()
    ldl, ldu, ldc = _mat(L21, "L21"), _mat(U12, "U12"), _mat(Cm, "C")
    m, K = L21.shape
    n = U12.shape[1]
    if U12.shape[0] != K or tuple(Cm.shape) != (m, n):
        raise ValueError("shapes of L21, U12 and C do not match")
    p = PREC[precision]
    if work is None:
        b = C.c_size_t()
        _check("cfx_schur_update_buffer_size",
               lib().cfx_schur_update_buffer_size(h.h, p, m, n, K, C.byref(b)))
        work = torch.empty(max(b.value, 256), dtype=torch.uint8, device=Cm.device) if b.value else None
    _check("cfx_schur_update", lib().cfx_schur_update(
        h.h, p, m, n, K, _ptr(L21), ldl, _ptr(U12), ldu, _ptr(Cm), ldc, int(max_workgroups),
        _ptr(work), 0 if work is None else work.numel(), _stream(stream)))
    return Cm


def getrs_noalloc(LU, ipiv, B, stream=None, handle=None):
    """cfx_getrs_noalloc: as getrs, with the fixed per-device scratch."""
    h = handle or default_handle()
    lda = _mat(LU, "LU")
    Bm = B.view(-1, 1) if B.dim() == 1 else B
    ldb = _mat(Bm, "B")
    n, nrhs = Bm.shape
    _check("cfx_getrs_noalloc", lib().cfx_getrs_noalloc(h.h, n, nrhs, _ptr(LU), lda, _ptr(ipiv), _ptr(Bm),
                                                        ldb, _stream(stream)))
    return B


def getrs_check(stream=None, handle=None):
    """cfx_getrs_check: synchronises the stream; returns the status code
    (0, or CFX_ESOLVE = -1005 when a one-launch solve gave up a wait)."""
    h = handle or default_handle()
    return int(lib().cfx_getrs_check(h.h, _stream(stream)))


def set_solve_spin_limit(polls, handle=None):
    """cfx_set_solve_spin_limit: polls before a solve's wait gives up."""
    h = handle or default_handle()
    _check("cfx_set_solve_spin_limit", lib().cfx_set_solve_spin_limit(h.h, int(polls)))


def ir_opts(precision="bf16", v=256, leaves=64, lookahead=0, tol=5e-15, max_outer=20,
            gmres_restart=30, gmres_tol=1e-6, min_leaf_rows=0):
    return IrOpts(LuOpts(v, leaves, PREC[precision], lookahead, min_leaf_rows), tol, max_outer, gmres_restart,
                  gmres_tol)


def gesv_ir_buffer_size(n, nrhs=1, handle=None, **kw):
    h = handle or default_handle()
    o = ir_opts(**kw)
    b = C.c_size_t()
    _check("cfx_gesv_ir_buffer_size",
           lib().cfx_gesv_ir_buffer_size(h.h, n, nrhs, C.byref(o), C.byref(b)))
    return b.value


def gesv_ir(A, B, X=None, work=None, stream=None, handle=None, **kw):
    """cfx_gesv_ir: X = A^{-1} B by (mixed-precision) LU + GMRES-IR.  A and B
    are not modified.  Returns (X, report dict).  Keyword options as ir_opts."""
    h = handle or default_handle()
    lda = _mat(A, "A")
    n = A.shape[0]
    vec = B.dim() == 1
    Bm = B.view(-1, 1) if vec else B
    ldb = _mat(Bm, "B")
    nrhs = Bm.shape[1]
    if X is None:
        X = torch.empty_like(Bm)
    Xm = X.view(-1, 1) if X.dim() == 1 else X
    ldx = _mat(Xm, "X")
    o = ir_opts(**kw)
    if work is None:
        nbytes = gesv_ir_buffer_size(n, nrhs, h, **kw)
        work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=A.device)
    rep = IrReport()
    _check("cfx_gesv_ir", lib().cfx_gesv_ir(h.h, n, nrhs, _ptr(A), lda, _ptr(Bm), ldb, _ptr(Xm), ldx,
                                            C.byref(o), C.byref(rep), _ptr(work), work.numel(),
                                            _stream(stream)))
    return (X.view(-1) if vec else X), rep.as_dict()


class Batch:
    """Device descriptor arrays of a batch of systems (kept alive with the
    tensors they point to).  As[i]: n_i x n_i, Bs[i]: n_i x nrhs_i (or n_i),
    float64 CUDA tensors, row-major (row stride may exceed the width)."""

    def __init__(self, As, Bs, device=None):
        if len(As) != len(Bs):
            raise ValueError("As and Bs differ in length")
        dev = device or (As[0].device if As else "cuda")
        self.As = list(As)
        self.Bs = [b.view(-1, 1) if b.dim() == 1 else b for b in Bs]
        self.count = len(As)
        n = [a.shape[0] for a in self.As]
        lda = [_mat(a, "A") for a in self.As]
        nrhs = [b.shape[1] for b in self.Bs]
        ldb = [_mat(b, "B") for b in self.Bs]
        self.ipiv = [torch.empty(max(k, 1), dtype=torch.int32, device=dev) for k in n]
        i32 = lambda v: torch.tensor(v, dtype=torch.int32, device=dev)
        i64 = lambda v: torch.tensor(v, dtype=torch.int64, device=dev)
        self.d_n, self.d_nrhs = i32(n), i32(nrhs)
        self.d_lda, self.d_ldb = i64(lda), i64(ldb)
        self.d_A = i64([a.data_ptr() for a in self.As])
        self.d_B = i64([b.data_ptr() for b in self.Bs])
        self.d_ipiv = i64([p.data_ptr() for p in self.ipiv])
        self.info = torch.zeros(max(self.count, 1), dtype=torch.int32, device=dev)
        self.work = torch.empty(max(gesv_batched_buffer_size(self.count), 256), dtype=torch.uint8,
                                device=dev)


def gesv_batched_buffer_size(count, handle=None):
    h = handle or default_handle()
    b = C.c_size_t()
    _check("cfx_gesv_batched_buffer_size", lib().cfx_gesv_batched_buffer_size(h.h, count, C.byref(b)))
    return b.value


def gesv_batched(batch: Batch, graph=True, stream=None, handle=None):
    """cfx_gesv_batched on a Batch: factors in place in batch.As, solutions
    in batch.Bs, pivots in batch.ipiv; returns batch.info (device int32)."""
    h = handle or default_handle()
    flags = 0 if graph else 1
    _check("cfx_gesv_batched", lib().cfx_gesv_batched(
        h.h, batch.count, _ptr(batch.d_n), _ptr(batch.d_nrhs), _ptr(batch.d_A), _ptr(batch.d_lda),
        _ptr(batch.d_B), _ptr(batch.d_ldb), _ptr(batch.d_ipiv), _ptr(batch.info), _ptr(batch.work),
        batch.work.numel(), flags, _stream(stream)))
    return batch.info[:batch.count]


def batched_tune(stream=None, handle=None):
    """cfx_batched_tune: time v in {8, 16, 32} per size class; returns the table."""
    h = handle or default_handle()
    _check("cfx_batched_tune", lib().cfx_batched_tune(h.h, _stream(stream)))
    return batched_tuning(h)


def batched_tuning(handle=None):
    h = handle or default_handle()
    t = (C.c_int32 * 5)()
    _check("cfx_batched_tuning", lib().cfx_batched_tuning(h.h, t))
    return list(t)


def batched_set_tuning(vb, handle=None):
    h = handle or default_handle()
    t = (C.c_int32 * 5)(*vb)
    _check("cfx_batched_set_tuning", lib().cfx_batched_set_tuning(h.h, t))


def full_trsm_rows(handle=None):
    """cfx_full_trsm_rows: trailing size from which all of U12 is solved first."""
    h = handle or default_handle()
    r = C.c_int32()
    _check("cfx_full_trsm_rows", lib().cfx_full_trsm_rows(h.h, C.byref(r)))
    return r.value


def set_full_trsm_rows(rows, handle=None):
    h = handle or default_handle()
    _check("cfx_set_full_trsm_rows", lib().cfx_set_full_trsm_rows(h.h, int(rows)))


def tournament_fusion(handle=None):
    """cfx_tournament_fusion: nodes of at most this many rows run as one launch."""
    h = handle or default_handle()
    r = C.c_int32()
    _check("cfx_tournament_fusion", lib().cfx_tournament_fusion(h.h, C.byref(r)))
    return r.value


def set_tournament_fusion(node_rows, handle=None):
    h = handle or default_handle()
    _check("cfx_set_tournament_fusion", lib().cfx_set_tournament_fusion(h.h, int(node_rows)))


def schur_delay(handle=None):
    """cfx_schur_delay: panels per trailing update (tile-stationary schedule)."""
    h = handle or default_handle()
    d = C.c_int32()
    _check("cfx_schur_delay", lib().cfx_schur_delay(h.h, C.byref(d)))
    return d.value


def set_schur_delay(delay, handle=None):
    h = handle or default_handle()
    _check("cfx_set_schur_delay", lib().cfx_set_schur_delay(h.h, int(delay)))


def reserved_cus(handle=None):
    """cfx_reserved_cus: compute units kept free of the overlapped updates."""
    h = handle or default_handle()
    c = C.c_int32()
    _check("cfx_reserved_cus", lib().cfx_reserved_cus(h.h, C.byref(c)))
    return c.value


def set_reserved_cus(cus, handle=None):
    h = handle or default_handle()
    _check("cfx_set_reserved_cus", lib().cfx_set_reserved_cus(h.h, int(cus)))


def overlap_tuning(handle=None):
    """(schur_workgroups, chunk_cols, one_stream) of cfx_getrf's lookahead overlap."""
    h = handle or default_handle()
    w, c, o = C.c_int32(), C.c_int32(), C.c_int32()
    _check("cfx_overlap_tuning", lib().cfx_overlap_tuning(h.h, C.byref(w), C.byref(c), C.byref(o)))
    return w.value, c.value, o.value


def set_overlap_tuning(schur_workgroups, chunk_cols, one_stream=0, handle=None):
    """cfx_set_overlap_tuning: schur_workgroups -1 (by precision, the default),
    0 (one workgroup per tile) or >= 8; chunk_cols >= 1; one_stream 0 or 1."""
    h = handle or default_handle()
    _check("cfx_set_overlap_tuning",
           lib().cfx_set_overlap_tuning(h.h, int(schur_workgroups), int(chunk_cols), int(one_stream)))


SOLVE, RESOLVE = 0, 1


class Server:
    """cfx_serve_*: a request loop on the current device.  The arena is a
    uint8 CUDA tensor owned here; A, B, X of a request are held until its
    result is polled (the library reads and writes them meanwhile)."""

    def __init__(self, arena_bytes, max_slots=4, batch_max=0, lowp_min_n=0, **ir_kw):
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        cfg = ServeCfg(C.c_void_p(self.arena.data_ptr()), arena_bytes, max_slots, ir_opts(**ir_kw),
                       batch_max, int(lowp_min_n))
        s = C.c_void_p()
        _check("cfx_serve_create", lib().cfx_serve_create(C.byref(cfg), C.byref(s)))
        self.s = s
        self.held = {}

    def submit(self, A, B, X, kind=SOLVE, factor_id=0, keep_resident=False):
        lda = _mat(A, "A")
        Bm = B.view(-1, 1) if B.dim() == 1 else B
        Xm = X.view(-1, 1) if X.dim() == 1 else X
        ldb, ldx = _mat(Bm, "B"), _mat(Xm, "X")
        r = Request(kind, int(bool(keep_resident)), factor_id, A.shape[0], Bm.shape[1], A.data_ptr(), lda,
                    Bm.data_ptr(), ldb, Xm.data_ptr(), ldx)
        # the server's streams do not wait for the caller's: finish the work
        # queued on the current stream (that may still be writing A, B or X)
        torch.cuda.current_stream().synchronize()
        t = C.c_uint64()
        _check("cfx_serve_submit", lib().cfx_serve_submit(self.s, C.byref(r), C.byref(t)))
        self.held[t.value] = (A, B, X)
        return t.value

    def poll(self, ticket):
        res = Result()
        rc = lib().cfx_serve_poll(self.s, ticket, C.byref(res))
        if rc == 1:
            return None
        _check("cfx_serve_poll", rc)
        self.held.pop(ticket, None)
        return res.as_dict()

    def wait(self, ticket, sleep=1e-4, timeout=120.0):
        import time as _t
        t0 = _t.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if _t.monotonic() - t0 > timeout:
                raise TimeoutError(f"request {ticket} not done after {timeout} s")
            _t.sleep(sleep)

    def release(self, factor_id):
        return lib().cfx_serve_release(self.s, factor_id)

    def stats(self):
        st = ServeStats()
        _check("cfx_serve_stats_get", lib().cfx_serve_stats_get(self.s, C.byref(st)))
        return st.as_dict()

    def close(self):
        if self.s:
            lib().cfx_serve_destroy(self.s)
            self.s = None
            self.held.clear()
            self.arena = None      # the server no longer touches it

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_begin(handle=None):
    """cfx_profile_begin: record per-phase events on subsequent getrf calls."""
    h = handle or default_handle()
    _check("cfx_profile_begin", lib().cfx_profile_begin(h.h))


def profile_end(handle=None) -> dict:
    """cfx_profile_end: wait for the recorded events; per-phase milliseconds."""
    h = handle or default_handle()
    p = Profile()
    _check("cfx_profile_end", lib().cfx_profile_end(h.h, C.byref(p)))
    return p.as_dict()
