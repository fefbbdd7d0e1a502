"""ctypes wrapper of the C oracle (libcfx_oracle.so) plus numpy helpers.

Test infrastructure only.  Matrices are row-major float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class _Counters(C.Structure):
    _fields_ = [("divisions", C.c_int64), ("multiply_subtracts", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("CFX_ORACLE_LIB")  # a planted-mistake build, in tests
        if path is None:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        L.oracle_tslu.argtypes = [C.c_int64, C.c_int64, dp, C.c_int64, C.c_int64,
                                  C.c_int64, i64p, dp]
        L.oracle_tslu.restype = C.c_int
        L.oracle_getrf.argtypes = [C.c_int64, dp, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                   i32p, i32p, dp, C.c_int64, C.POINTER(_Counters)]
        L.oracle_getrf.restype = C.c_int
        L.oracle_getrs.argtypes = [C.c_int64, C.c_int64, dp, C.c_int64, i32p, dp, C.c_int64]
        L.oracle_getrs.restype = C.c_int
        L.oracle_eta.argtypes = [C.c_int64, dp, C.c_int64, dp, C.c_int64, dp, C.c_int64]
        L.oracle_eta.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(a, dtype):
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise TypeError(f"expected C-contiguous {dtype} array")


def tslu(W: np.ndarray, vb: int, L: int, row0: int = 0):
    """Tournament pivots of one panel W (rows x >= vb): (piv int64[vb], margin)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    rows = W.shape[0]
    piv = np.zeros(vb, dtype=np.int64)
    mar = C.c_double(0.0)
    rc = lib().oracle_tslu(rows, vb, _dp(W), W.shape[1], row0, L,
                           piv.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(mar))
    if rc != 0:
        raise ValueError(f"oracle_tslu rejected argument {-rc}")
    return piv, mar.value


class Factorization:
    def __init__(self, LU, ipiv, info, margins, counters):
        self.LU = LU
        self.ipiv = ipiv
        self.info = info
        self.margins = margins
        self.counters = counters


def getrf(A: np.ndarray, v: int, L: int, npanels: int = 0, overwrite: bool = False, min_leaf_rows: int = 0):
    """TP(v, L) LU of a square row-major matrix.  Returns a Factorization.
    min_leaf_rows = R > 0: a panel with r rows has min(L, max(1, ceil(r/R)))
    leaves."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    if not overwrite:
        A = A.copy()
    n = A.shape[0]
    assert A.shape == (n, n)
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    info = C.c_int32(0)
    npan = (n + v - 1) // v if (n > 0 and v > 0) else 0
    margins = np.ones(max(npan, 1), dtype=np.float64)
    cnt = _Counters()
    rc = lib().oracle_getrf(n, _dp(A), max(n, 1), v, L, min_leaf_rows,
                            ipiv.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(info),
                            _dp(margins), npanels, C.byref(cnt))
    if rc != 0:
        raise ValueError(f"oracle_getrf rejected argument {-rc}")
    return Factorization(A, ipiv[:n], info.value, margins[:npan],
                         (cnt.divisions, cnt.multiply_subtracts))


def getrs(LU: np.ndarray, ipiv: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve with oracle factors; B is (n,) or (n, nrhs); returns X (new array)."""
    LU = np.ascontiguousarray(LU, dtype=np.float64)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    vec = B.ndim == 1
    X = np.array(B, dtype=np.float64, copy=True, order="C")
    if vec:
        X = X[:, None].copy()
    n, nrhs = X.shape
    rc = lib().oracle_getrs(n, nrhs, _dp(LU), max(n, 1),
                            ipiv.ctypes.data_as(C.POINTER(C.c_int32)), _dp(X), max(nrhs, 1))
    if rc != 0:
        raise ValueError(f"oracle_getrs rejected argument {-rc}")
    return X[:, 0] if vec else X


def eta(A: np.ndarray, x: np.ndarray, b: np.ndarray) -> float:
    """Normwise backward error max over columns of ||b-Ax||_inf/(||A|| ||x|| + ||b||)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    X = np.ascontiguousarray(x, dtype=np.float64)
    Bm = np.ascontiguousarray(b, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
        Bm = Bm[:, None]
    n, nrhs = X.shape
    worst = 0.0
    for c in range(nrhs):
        xc = np.ascontiguousarray(X[:, c])
        bc = np.ascontiguousarray(Bm[:, c])
        e = lib().oracle_eta(n, _dp(A), A.shape[1], _dp(xc), 1, _dp(bc), 1)
        if e != e:              # a non-finite column makes the whole result NaN
            return e
        worst = max(worst, e)
    return worst


# --------------------------------------------------------------------------
# Permutation helpers (plain definitions used by tests)
# --------------------------------------------------------------------------

def ipiv_to_perm(ipiv: np.ndarray) -> np.ndarray:
    """perm such that (P A)[i] = A[perm[i]] for the interchanges in ipiv."""
    n = len(ipiv)
    perm = np.arange(n)
    for i in range(n):
        r = int(ipiv[i])
        perm[i], perm[r] = perm[r], perm[i]
    return perm


def unpack(LU: np.ndarray):
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    return L, U


def lu_residual(A0: np.ndarray, LU: np.ndarray, ipiv: np.ndarray) -> float:
    """||P A - L U||_F / ||A||_F (numpy matmul)."""
    L, U = unpack(LU)
    PA = A0[ipiv_to_perm(ipiv)]
    return float(np.linalg.norm(PA - L @ U) / np.linalg.norm(A0))


def ipiv_sign(ipiv: np.ndarray) -> int:
    return -1 if int(np.sum(ipiv != np.arange(len(ipiv)))) % 2 else 1


# --------------------------------------------------------------------------
# Mixed-precision Schur update (FactorizeA11 of Alg. 1 with low-precision
# operands).  The paper fixes no low precision; the reading used here: each
# FP64 operand is rounded once, directly to BF16 or FP16 (round to nearest,
# ties to even; no intermediate FP32 rounding); products of two such values
# are exact in FP64, and the FP64 sum of the products is the reference for
# the FP32 accumulation of the matrix cores.
# --------------------------------------------------------------------------

# precision p (significand bits), emin, largest finite value, and whether
# the format has infinities (OCP FP8 E4M3 has none: an overflow, an infinite
# or a NaN input all give NaN)
_FORMATS = {"bf16": (8, -126, 3.3895313892515355e38, True),
            "fp16": (11, -14, 65504.0, True),
            "fp8": (4, -6, 448.0, False)}


def round_lowp(x, precision: str) -> np.ndarray:
    """Round FP64 values to BF16, FP16 or FP8 E4M3 (nearest, ties to even),
    returned as FP64.  Written from the format definition: a value with
    exponent e (2^e <= |x| < 2^(e+1), e clamped below at emin for
    subnormals) is rounded to a multiple of 2^(e - p + 1); beyond the largest
    finite value (after rounding) the result is infinite (BF16, FP16) or NaN
    (E4M3, which has no infinities; its infinite inputs give NaN too)."""
    if precision not in _FORMATS:
        raise ValueError(precision)
    p, emin, vmax, has_inf = _FORMATS[precision]
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, dtype=np.float64, copy=True)
    if not has_inf:
        out[np.isinf(x)] = np.nan
    fin = np.isfinite(x) & (x != 0)
    xf = x[fin]
    _, e2 = np.frexp(np.abs(xf))                 # |x| = m 2^e2, m in [0.5, 1)
    e = np.maximum(e2 - 1, emin)
    q = np.ldexp(1.0, e - p + 1)                 # quantum, a power of two
    r = np.rint(xf / q) * q                      # exact scaling; rint ties to even
    big = np.abs(r) > vmax
    r[big] = (np.inf * np.sign(r[big])) if has_inf else np.nan
    out[fin] = r
    return out


def fp8_scale_exponents(M: np.ndarray, axis: int) -> np.ndarray:
    """Power-of-two scale exponents of the FP8 operands: for each row
    (axis=1) or column (axis=0) with largest magnitude f 2^E (f in [0.5, 1)),
    s = 8 - E, so that the scaled largest magnitude lies in [128, 256), well
    inside the E4M3 range; s = 0 for an all-zero or non-finite vector."""
    mx = np.max(np.abs(M), axis=axis) if M.size else np.zeros(M.shape[1 - axis])
    _, E = np.frexp(mx)
    s = (8 - E).astype(np.int64)
    s[~(np.isfinite(mx) & (mx > 0))] = 0
    return s


def lowp_operands(L21: np.ndarray, U12: np.ndarray, precision: str):
    """The rounded operands of one low-precision Schur update, as FP64
    values: (Lr, Ur) with Lr Ur the product the update subtracts.  BF16 and
    FP16 round every entry once; FP8 scales row i of L21 by 2^sL_i and column
    j of U12 by 2^sU_j, rounds, and scales back (exact powers of two); a row
    (column) holding a non-finite value becomes all NaN, so its row (column)
    of the update is NaN."""
    if precision != "fp8":
        return round_lowp(L21, precision), round_lowp(U12, precision)
    sL = fp8_scale_exponents(L21, 1)
    sU = fp8_scale_exponents(U12, 0)
    with np.errstate(invalid="ignore", over="ignore"):
        Lr = np.ldexp(round_lowp(np.ldexp(L21, sL[:, None]), "fp8"), -sL[:, None])
        Ur = np.ldexp(round_lowp(np.ldexp(U12, sU[None, :]), "fp8"), -sU[None, :])
    Lr[~np.all(np.isfinite(L21), axis=1)] = np.nan
    Ur[:, ~np.all(np.isfinite(U12), axis=0)] = np.nan
    return Lr, Ur


def schur_lowp(C: np.ndarray, L21: np.ndarray, U12: np.ndarray, precision: str) -> np.ndarray:
    """FactorizeA11 with low-precision operands: C - Lr Ur, the rounded
    operands multiplied and summed in FP64 (each product is exact)."""
    Lr, Ur = lowp_operands(L21, U12, precision)
    with np.errstate(invalid="ignore"):
        return C - Lr @ Ur


def tail_after_lowp_update(A: np.ndarray, v: int, L: int, precision: str):
    """The first panel of TP(v, L) in FP64 (oracle getrf limited to one
    panel), then the trailing matrix S = A22 - lowp(L21) lowp(U12) with the
    rounded operands multiplied and summed in FP64.  Returns (first-panel
    Factorization, S)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    f = getrf(A, v, L, npanels=1)
    n = A.shape[0]
    vb = min(v, n)
    PA = A[ipiv_to_perm(np.concatenate([f.ipiv[:vb], np.arange(vb, n)]).astype(np.int32))]
    L21 = f.LU[vb:, :vb]
    U12 = f.LU[:vb, vb:]
    S = schur_lowp(PA[vb:, vb:], L21, U12, precision)
    return f, S
