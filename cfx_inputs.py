"""Seeded synthetic inputs for the blocked tournament-pivoted LU.

This module is shared by the CPU oracle side and the GPU side of every test
and of the benchmark.  It holds no LU arithmetic: it only draws random numbers
(numpy PCG64, ``default_rng(seed)``) and assembles the matrices, right-hand
sides and request streams of the workloads below.

Workloads (the paper gives only problem sizes for its dense LU experiments,
Sec. 8 "Problem sizes", never the matrix entries, so all entries are
synthetic):

* ``uniform``   -- A_ij ~ U(-1, 1) i.i.d., the small single-matrix case
                   (N = 512, panel width 32).
* ``normal``    -- A_ij ~ N(0, 1) i.i.d., the large FP64 cases
                   (N = 16384 and 32768, panel width 256).
* ``householder`` -- A = H1 diag(s) H2 with H1, H2 products of 8 seeded
                   Householder reflectors and s log-spaced from 1 to 1/cond,
                   so kappa_2(A) = cond exactly and x* = A^{-1} b has a closed
                   form (used by the mixed-precision and serving cases).
* ``batched``   -- many independent small systems, sizes uniform in [16, 512],
                   N(0,1) entries plus a 0 or 2 sqrt(n) diagonal shift.
* ``serving``   -- a Poisson request stream with log-uniform sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_matrix(n: int, seed: int) -> np.ndarray:
    """Row-major n x n FP64 matrix with i.i.d. U(-1, 1) entries."""
    return rng(seed).uniform(-1.0, 1.0, size=(n, n))


def normal_matrix(n: int, seed: int) -> np.ndarray:
    """Row-major n x n FP64 matrix with i.i.d. N(0, 1) entries."""
    return rng(seed).standard_normal(size=(n, n))


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Row-major n x nrhs FP64 right-hand sides with N(0, 1) entries."""
    return rng(seed).standard_normal(size=(n, nrhs))


# ---------------------------------------------------------------------------
# Householder construction A = H1 diag(s) H2
# ---------------------------------------------------------------------------

@dataclass
class HouseholderSpec:
    """Reflector vectors and singular values of A = H1 diag(s) H2.

    H1 = R(w1[0]) R(w1[1]) ... R(w1[7]),  H2 likewise with w2, where
    R(w) = I - 2 w w^T / (w^T w) is symmetric and orthogonal.
    """
    w1: np.ndarray  # (nrefl, n)
    w2: np.ndarray  # (nrefl, n)
    s: np.ndarray   # (n,) singular values, s_0 = 1 down to s_{n-1} = 1/cond


def ipiv_pattern(kind: str, n: int, seed: int) -> np.ndarray:
    """int32[n] LAPACK-style interchange vectors (row i with row ipiv[i]):
    "chain"   ipiv[i] = i + 1 (every interchange shares a row with the next);
    "near"    ipiv[i] in [i, i + 3);
    "uniform" ipiv[i] uniform in [i, n);
    "invalid" as "uniform", with every 7th entry replaced by one outside
              [i, n) (i - 1, n, -5 or 2^31 - 1 in turn)."""
    g = rng(seed)
    i = np.arange(n, dtype=np.int64)
    if kind == "chain":
        r = i + 1
    elif kind == "near":
        r = i + g.integers(0, 3, n)
    elif kind in ("uniform", "invalid"):
        r = i + np.floor(g.random(n) * (n - i)).astype(np.int64)
    else:
        raise ValueError(kind)
    r = np.minimum(r, n - 1)
    if kind == "invalid":
        bad = np.array([-1, n, -5, 2**31 - 1], dtype=np.int64)
        k = np.arange(0, n, 7)
        r[k] = np.where(bad[k % 4] == -1, k - 1, bad[k % 4])
    return r.astype(np.int32)


def householder_spec(n: int, cond: float, seed: int, nrefl: int = 8) -> HouseholderSpec:
    g = rng(seed)
    w1 = g.standard_normal(size=(nrefl, n))
    w2 = g.standard_normal(size=(nrefl, n))
    if n == 1:
        s = np.ones(1)
    else:
        s = cond ** (-np.arange(n, dtype=np.float64) / (n - 1))
    return HouseholderSpec(w1=w1, w2=w2, s=s)


def _reflect_rows(M, w):
    """M <- R(w) M  (works on numpy arrays and torch tensors)."""
    c = 2.0 / float((w * w).sum())
    t = w @ M                      # row vector w^T M
    M -= c * (w[:, None] * t[None, :])
    return M


def _reflect_cols(M, w):
    """M <- M R(w)."""
    c = 2.0 / float((w * w).sum())
    t = M @ w                      # column vector M w
    M -= c * (t[:, None] * w[None, :])
    return M


def householder_matrix(spec: HouseholderSpec, device: str | None = None):
    """Assemble A = H1 diag(s) H2.

    With ``device=None`` the result is a numpy array; otherwise a torch FP64
    tensor built on that device (the large N = 32768 case is assembled on the
    GPU because sixteen rank-one passes over 8.6 GB are slow on the host).
    """
    n = spec.s.shape[0]
    if device is None:
        A = np.diag(spec.s.copy())
        w1, w2 = spec.w1, spec.w2
    else:
        import torch
        A = torch.diag(torch.from_numpy(spec.s).to(device))
        w1 = torch.from_numpy(spec.w1).to(device)
        w2 = torch.from_numpy(spec.w2).to(device)
    # A = R1 R2 ... Rk D Q1 ... Qk : apply the left factors innermost-first.
    for i in reversed(range(spec.w1.shape[0])):
        _reflect_rows(A, w1[i])
    for i in range(spec.w2.shape[0]):
        _reflect_cols(A, w2[i])
    return A


def householder_solution(spec: HouseholderSpec, b: np.ndarray) -> np.ndarray:
    """Closed-form x* = H2^{-1} diag(1/s) H1^{-1} b (each R(w) is its own inverse)."""
    x = np.array(b, dtype=np.float64, copy=True)
    if x.ndim == 1:
        x = x[:, None]
    for i in range(spec.w1.shape[0]):   # H1^{-1} = R_k ... R_1: R_1 acts first
        _reflect_rows(x, spec.w1[i])
    x /= spec.s[:, None]
    for i in range(spec.w2.shape[0]):   # H2^{-1} = Q_k ... Q_1: Q_1 acts first
        _reflect_rows(x, spec.w2[i])
    return x


# ---------------------------------------------------------------------------
# Special matrices with known factors (pins for the oracle)
# ---------------------------------------------------------------------------

def wilkinson_growth_matrix(n: int) -> np.ndarray:
    """1 on the diagonal, -1 strictly below it, 1 in the last column."""
    A = np.tril(-np.ones((n, n)), -1) + np.eye(n)
    A[:, -1] = 1.0
    return A


def dyadic_dd_factors(n: int, seed: int):
    """Unit-lower L0 and upper U0 with small dyadic entries such that
    A = L0 U0 is strictly column diagonally dominant and every partial sum of
    the elimination is exactly representable in FP64.

    Off-diagonal entries of L0 and U0 are k/512 with |k| <= 2 and the diagonal
    of U0 is 64 + j/8 (0 <= j < 8).  For n <= 64 every product is a multiple
    of 2^-18 and every partial sum is below 2^7, so 25 bits suffice and the
    elimination is exact; the column sums off the diagonal stay below 17.
    """
    if n > 64:
        raise ValueError("exactness argument holds for n <= 64")
    g = rng(seed)
    L0 = np.tril(g.integers(-2, 3, size=(n, n)) / 512.0, -1) + np.eye(n)
    U0 = np.triu(g.integers(-2, 3, size=(n, n)) / 512.0, 1)
    U0 += np.diag(64.0 + g.integers(0, 8, size=n) / 8.0)
    return L0, U0


# ---------------------------------------------------------------------------
# Batched and serving workloads
# ---------------------------------------------------------------------------

@dataclass
class BatchedSpec:
    sizes: np.ndarray   # int32 (count,)
    nrhs: np.ndarray    # int32 (count,)
    shift: np.ndarray   # float64 (count,), 0 or 2 sqrt(n)
    seeds: np.ndarray   # int64 (count,), per-system seed


def batched_spec(count: int, seed: int, nmin: int = 16, nmax: int = 512,
                 rmin: int = 1, rmax: int = 8) -> BatchedSpec:
    g = rng(seed)
    sizes = g.integers(nmin, nmax + 1, size=count).astype(np.int32)
    nrhs = g.integers(rmin, rmax + 1, size=count).astype(np.int32)
    shifted = g.integers(0, 2, size=count).astype(bool)
    shift = np.where(shifted, 2.0 * np.sqrt(sizes.astype(np.float64)), 0.0)
    seeds = g.integers(0, 2**62, size=count, dtype=np.int64)
    return BatchedSpec(sizes=sizes, nrhs=nrhs, shift=shift, seeds=seeds)


def batched_system(spec: BatchedSpec, i: int):
    """(A, B) of system i: A ~ N(0,1) + shift I, B ~ N(0,1)."""
    n = int(spec.sizes[i])
    g = rng(int(spec.seeds[i]))
    A = g.standard_normal(size=(n, n))
    A[np.diag_indices(n)] += spec.shift[i]
    B = g.standard_normal(size=(n, int(spec.nrhs[i])))
    return A, B


@dataclass
class Request:
    t_arrival: float    # seconds from stream start
    n: int
    nrhs: int
    cond: float
    seed: int
    resolve_of: int     # index of an earlier request whose factor is reused, or -1


def serving_stream(rate: float, duration: float, seed: int, nmin: int = 64,
                   nmax: int = 8192, cmin: float = 1e2, cmax: float = 1e8,
                   rmax: int = 16, resolve_frac: float = 0.3) -> list[Request]:
    """Poisson arrivals (exponential gaps), log-uniform sizes and conditions."""
    g = rng(seed)
    out: list[Request] = []
    t = 0.0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        idx = len(out)
        if idx > 0 and g.uniform() < resolve_frac:
            j = int(g.integers(0, idx))
            base = out[j] if out[j].resolve_of < 0 else out[out[j].resolve_of]
            src = j if out[j].resolve_of < 0 else out[j].resolve_of
            out.append(Request(t, base.n, int(g.integers(1, rmax + 1)), base.cond,
                               int(g.integers(0, 2**62)), src))
            continue
        n = int(round(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
        cond = float(math.exp(g.uniform(math.log(cmin), math.log(cmax))))
        out.append(Request(t, n, int(g.integers(1, rmax + 1)), cond,
                           int(g.integers(0, 2**62)), -1))
    return out
