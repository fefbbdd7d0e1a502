"""cfx_getrs_noalloc (the solve whose scratch is a fixed per-device array)
against cfx_getrs, through the C ABI: two calls in a row, the second with a
smaller input, each equal bit for bit to the allocating entry point's result
(same kernels, same order of operations), and the size limit."""
import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O
from tests.gpu_util import say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_05975_amd import cfx as m
    m.lib()
    return m


def factor(cfx, n, seed):
    A = G.normal_matrix(n, seed)
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=128, leaves=4)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    return A, dA, ipiv


@pytest.mark.parametrize("cases", [[(3000, 5), (1000, 2)], [(4096, 1), (777, 1)], [(2500, 64), (64, 3)]])
def test_noalloc_matches_getrs_twice(cfx, cases):
    for n, nrhs in cases:
        say(f"getrs_noalloc n={n} nrhs={nrhs}")
        A, dA, ipiv = factor(cfx, n, 90 + n)
        B = G.rhs(n, nrhs, 91 + n)
        want = to_dev(B)
        cfx.getrs(dA, ipiv, want)
        got = to_dev(B)
        cfx.getrs_noalloc(dA, ipiv, got)
        torch.cuda.synchronize()
        assert cfx.getrs_check() == 0
        w, g = want.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(g, w)
        assert O.eta(A, g, B) <= 5e-15


def test_noalloc_rejects_beyond_its_scratch(cfx):
    say("getrs_noalloc size limit")
    n = 4096
    LU = torch.eye(n, dtype=torch.float64, device="cuda")
    ipiv = torch.arange(n, dtype=torch.int32, device="cuda")
    B = torch.zeros((n, 1100), dtype=torch.float64, device="cuda")   # 36 MB of right-hand sides
    with pytest.raises(cfx.CfxError) as e:
        cfx.getrs_noalloc(LU, ipiv, B)
    assert e.value.code == -1004
    B = torch.ones((n, 1000), dtype=torch.float64, device="cuda")    # 32.8 MB: fits
    cfx.getrs_noalloc(LU, ipiv, B)
    torch.cuda.synchronize()
    assert torch.all(B == 1.0)
