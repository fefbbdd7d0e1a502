"""Write the stored oracle results of the plain FP64 workload at full size.

For A ~ N(0, 1) (seed 0, the generator in cfx_inputs) of order N in
{16384, 32768}, the CPU oracle runs the whole TP(v = 256, L = 8)
factorisation with leaves of at least 4096 rows (min(8, ceil(r / 4096))
leaves for a panel of r rows) (Alg. 1 with tournament pivoting, Sec. 7.3 / Sec. 7.4 Step 1)
and this script stores, per N, in c2_n<N>_seed0.npz:
  ipiv      int32[N]   the oracle's LAPACK-style interchanges
  margins   float64[N/256]  minimum pivot margin of every panel
  info      int32      first exactly zero pivot (0: none)
  residual  float64    ||P A - L U||_F / ||A||_F of the oracle's factors
  digest    str        SHA-256 of rows 0, N/2 and N-1 of A (the GPU test
                       checks that it regenerates the same input)
  seconds   float64    wall time of the oracle factorisation alone
  threads   int32      OpenMP threads it ran with (OMP_NUM_THREADS, else
                       the CPU count)
Only oracle/ computes anything here (numpy's matmul forms L U for the
residual).  It runs on the CPU in about 5 minutes (N = 16384) and 30 minutes
(N = 32768) on 8 cores:

    python tests/golden/make_c2_golden.py 16384 32768
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import cfx_inputs as G  # noqa: E402
from oracle import oracle as O  # noqa: E402

V, LEAVES, SEED = 256, 8, 0
MIN_LEAF_ROWS = 4096      # leaves of at least 4096 rows: min(8, ceil(r / 4096)) per panel


def path(n: int) -> str:
    return os.path.join(HERE, f"c2_n{n}_seed{SEED}.npz")


def digest(A: np.ndarray) -> str:
    n = A.shape[0]
    h = hashlib.sha256()
    for r in (0, n // 2, n - 1):
        h.update(np.ascontiguousarray(A[r]).tobytes())
    return h.hexdigest()


def frob_residual(A: np.ndarray, LU: np.ndarray, ipiv: np.ndarray, block: int = 1024) -> float:
    """||P A - L U||_F / ||A||_F, L U formed block row by block row."""
    n = A.shape[0]
    perm = O.ipiv_to_perm(ipiv)
    U = np.triu(LU)
    num = 0.0
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        Lb = np.tril(LU[r0:r1, :r1], r0 - 1)      # strictly lower part of rows r0..r1
        Lb[np.arange(r1 - r0), np.arange(r0, r1)] = 1.0
        D = A[perm[r0:r1]] - Lb @ U[:r1]
        num += float(np.sum(D * D))
    return float(np.sqrt(num) / np.linalg.norm(A))


def make(n: int) -> None:
    A = G.normal_matrix(n, SEED)
    dg = digest(A)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    print(f"N={n}: oracle getrf (v={V}, L={LEAVES}, {threads} threads) ...", flush=True)
    t0 = time.time()
    f = O.getrf(A, V, LEAVES, min_leaf_rows=MIN_LEAF_ROWS)
    t1 = time.time()
    print(f"  {t1 - t0:.0f} s; min margin {f.margins.min():.3e}; info {f.info}", flush=True)
    res = frob_residual(A, f.LU, f.ipiv)
    print(f"  residual {res:.3e} ({time.time() - t1:.0f} s)", flush=True)
    np.savez_compressed(path(n), ipiv=f.ipiv.astype(np.int32), margins=f.margins.astype(np.float64),
                        info=np.int32(f.info), residual=np.float64(res), digest=np.str_(dg),
                        v=np.int32(V), leaves=np.int32(LEAVES), seed=np.int32(SEED),
                        min_leaf_rows=np.int32(MIN_LEAF_ROWS),
                        numpy_version=np.str_(np.__version__), seconds=np.float64(t1 - t0),
                        threads=np.int32(threads))


def load(n: int) -> dict:
    with np.load(path(n), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["16384", "32768"]:
        make(int(arg))
