"""Shared helpers of the GPU tests (no LU arithmetic)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def compare_panels(ipiv_gpu, ipiv_ref, margins, v, thresh=1e-10):
    """ipiv must agree bit for bit on every panel before the first panel whose
    oracle margin is <= thresh.  Returns the number of panels compared."""
    n = len(ipiv_ref)
    npan = len(margins)
    for p in range(npan):
        if margins[p] <= thresh:
            return p
        k0, k1 = p * v, min(n, (p + 1) * v)
        assert np.array_equal(ipiv_gpu[k0:k1], ipiv_ref[k0:k1]), f"panel {p} pivots differ"
    return npan
