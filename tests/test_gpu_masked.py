"""Row masking instead of row interchanges (cfx_getrf_masked /
cfx_getrs_masked; Sec. 7.3 "Row Swapping vs. Row Masking"), through the C
ABI.

The pins: the masked factorisation chooses the same pivots with the same
arithmetic, so its factors, read through the returned row map, equal the
interchanged factors of cfx_getrf bit for bit (every precision, with and
without lookahead); the row map is the permutation that ipiv composes to;
the factors match the oracle's (pivots bit for bit under the margin rule,
values to rounding); and the masked solve equals the ordinary one."""
import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O
from tests.gpu_util import compare_panels, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_05975_amd import cfx as m
    m.lib()
    return m


def both(cfx, A, v, L, prec="fp64", la=0):
    dS = to_dev(A)
    ipiv_s, info_s = cfx.getrf(dS, v=v, leaves=L, precision=prec, lookahead=la)
    dM = to_dev(A)
    ipiv_m, rowmap, info_m = cfx.getrf_masked(dM, v=v, leaves=L, precision=prec, lookahead=la)
    torch.cuda.synchronize()
    n = A.shape[0]
    return (dS.cpu().numpy(), ipiv_s.cpu().numpy()[:n], int(info_s.cpu()[0]),
            dM.cpu().numpy(), ipiv_m.cpu().numpy()[:n], rowmap.cpu().numpy()[:n], int(info_m.cpu()[0]))


@pytest.mark.parametrize("n,v,L,prec,la", [(512, 32, 4, "fp64", 0), (512, 32, 4, "fp64", 1),
                                           (1000, 64, 3, "fp64", 1), (3000, 128, 4, "fp64", 1),
                                           (2048, 256, 8, "fp64", 1), (777, 100, 5, "fp64", 0),
                                           (1500, 128, 4, "bf16", 1), (1500, 128, 4, "fp16", 0),
                                           (1300, 64, 4, "fp8", 1)])
def test_masked_equals_interchanged_bitwise(cfx, n, v, L, prec, la):
    say(f"masked vs interchanged n={n} v={v} L={L} {prec} la={la}")
    A = G.normal_matrix(n, 100 + n)
    S, ipiv_s, info_s, M, ipiv_m, rowmap, info_m = both(cfx, A, v, L, prec, la)
    assert info_s == info_m == 0
    assert np.array_equal(ipiv_s, ipiv_m)
    assert np.array_equal(rowmap, O.ipiv_to_perm(ipiv_s))
    assert np.array_equal(M[rowmap], S)
    # rows were really left in place: every stored row is the input row's
    # factor row, and the row map is not the identity
    assert not np.array_equal(rowmap, np.arange(n))


@pytest.mark.parametrize("n,v,L", [(600, 64, 4), (1025, 128, 3)])
def test_masked_matches_oracle(cfx, n, v, L):
    say(f"masked vs oracle n={n} v={v} L={L}")
    A = G.normal_matrix(n, 7 + n)
    ref = O.getrf(A, v, L)
    dM = to_dev(A)
    ipiv, rowmap, info = cfx.getrf_masked(dM, v=v, leaves=L, lookahead=1)
    torch.cuda.synchronize()
    rm = rowmap.cpu().numpy()[:n]
    LU = dM.cpu().numpy()[rm]
    piv = ipiv.cpu().numpy()[:n]
    assert int(info.cpu()[0]) == ref.info == 0
    npan = compare_panels(piv, ref.ipiv, ref.margins, v)
    assert npan == len(ref.margins)
    np.testing.assert_allclose(LU, ref.LU, rtol=0, atol=1e-9 * np.abs(ref.LU).max())
    assert O.lu_residual(A, LU, piv) <= 1e-12
    # (P A)[i] = A[rowmap[i]]: the stored rows are the input rows' factors
    L_, U_ = O.unpack(LU)
    assert np.abs(A[rm] - L_ @ U_).max() <= 1e-12 * np.abs(A).max() * n


@pytest.mark.parametrize("nrhs", [1, 5])
def test_masked_solve_equals_ordinary(cfx, nrhs):
    n, v, L = 2500, 128, 4
    say(f"getrs_masked nrhs={nrhs}")
    A = G.normal_matrix(n, 31)
    dS = to_dev(A)
    ipiv, info = cfx.getrf(dS, v=v, leaves=L)
    dM = to_dev(A)
    _, rowmap, _ = cfx.getrf_masked(dM, v=v, leaves=L)
    B = G.rhs(n, nrhs, 32)
    x1, x2 = to_dev(B), to_dev(B)
    cfx.getrs(dS, ipiv, x1)
    cfx.getrs_masked(dM, rowmap, x2)
    torch.cuda.synchronize()
    assert cfx.getrs_check() == 0
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert O.eta(A, x2.cpu().numpy(), B) <= 5e-15


def test_masked_singular_reports_info(cfx):
    say("masked singular")
    n = 300
    A = G.normal_matrix(n, 41)
    A[:, 77] = 0.0
    S, ipiv_s, info_s, M, ipiv_m, rowmap, info_m = both(cfx, A, 64, 3)
    assert info_s == info_m == 78
    assert np.array_equal(M[rowmap], S)
