"""The tile-stationary schedule (cfx_set_schur_delay: the trailing matrix
receives d panels' Schur updates at once, K = d v) against the CPU oracle,
through the C ABI.

Only the grouping of the sums changes (d panels' products accumulate
together), so the pins are those of the ordinary factorisation: pivots bit
for bit up to the first panel whose oracle margin is <= 1e-10, factors
within rounding of the oracle's, ||PA - LU||_F / ||A||_F <= 1e-12; for the
low-precision updates the backward error of the factors at the format's
precision and GMRES-IR to 5e-15."""
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


def run(cfx, A, v, L, d, prec="fp64", la=1):
    h = cfx.Handle()
    try:
        cfx.set_schur_delay(d, handle=h)
        assert cfx.schur_delay(handle=h) == d
        dA = to_dev(A)
        ipiv, info = cfx.getrf(dA, v=v, leaves=L, precision=prec, lookahead=la, handle=h)
        torch.cuda.synchronize()
    finally:
        h.close()
    n = A.shape[0]
    return dA.cpu().numpy(), ipiv.cpu().numpy()[:n], int(info.cpu()[0])


@pytest.mark.parametrize("n,v,L,d,la", [(1000, 64, 3, 2, 1), (1000, 64, 3, 2, 0), (2048, 128, 4, 4, 1),
                                        (777, 100, 5, 3, 1), (3000, 256, 8, 2, 1), (1500, 32, 4, 8, 0),
                                        (300, 64, 2, 4, 1)])
def test_delayed_matches_oracle(cfx, n, v, L, d, la):
    say(f"delayed schedule n={n} v={v} L={L} d={d} la={la}")
    A = G.normal_matrix(n, 500 + n + d)
    ref = O.getrf(A, v, L)
    LU, piv, info = run(cfx, A, v, L, d, la=la)
    assert info == ref.info == 0
    npan = compare_panels(piv, ref.ipiv, ref.margins, v)
    assert npan == len(ref.margins)
    np.testing.assert_allclose(LU, ref.LU, rtol=0, atol=1e-9 * np.abs(ref.LU).max())
    res = O.lu_residual(A, LU, piv)
    say(f"  ||PA-LU||/||A|| = {res:.3e}")
    assert res <= 1e-12


def test_delayed_is_deterministic_and_close_to_undelayed(cfx):
    n, v, L = 1600, 128, 4
    say("delayed schedule determinism")
    A = G.normal_matrix(n, 77)
    a = run(cfx, A, v, L, 3)
    b = run(cfx, A, v, L, 3)
    c = run(cfx, A, v, L, 1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[1], c[1])
    # FP64 matrix-core accumulators hold FP64: d panels accumulated in one
    # launch give the same operations, in the same order, as d launches
    assert np.array_equal(a[0], c[0])


@pytest.mark.parametrize("prec,hi", [("bf16", 0.3), ("fp16", 0.05), ("fp8", 3.0)])
def test_delayed_lowp_backward_error(cfx, prec, hi):
    n, v, L = 1024, 64, 4
    say(f"delayed lowp {prec}")
    A = G.normal_matrix(n, 3)
    LU, piv, info = run(cfx, A, v, L, 4, prec)
    assert info == 0
    r = O.lu_residual(A, LU, piv)
    say(f"  ||PA-LU||/||A|| = {r:.3e}")
    assert 1e-6 < r < hi
    ref = O.getrf(A, v, L)
    assert np.array_equal(piv[:v], ref.ipiv[:v])


def test_delayed_gesv_ir(cfx):
    n = 2048
    say("delayed gesv_ir bf16")
    spec = G.householder_spec(n, 1e2, 5)
    A = G.householder_matrix(spec)
    b = G.rhs(n, 1, 6)
    h = cfx.Handle()
    try:
        cfx.set_schur_delay(4, handle=h)
        X, rep = cfx.gesv_ir(to_dev(A), to_dev(b), handle=h, precision="bf16", v=128, leaves=4, lookahead=1)
    finally:
        h.close()
    eta = O.eta(A, X.cpu().numpy(), b)
    say(f"  {rep}; oracle eta {eta:.3e}")
    assert rep["converged"] == 1 and eta <= 5e-15


def test_delayed_singular_and_settings(cfx):
    say("delayed singular and settings")
    n = 400
    A = G.normal_matrix(n, 9)
    A[:, 150] = 0.0
    LU, piv, info = run(cfx, A, 64, 3, 3)
    assert info == 151
    h = cfx.Handle()
    try:
        for bad in (0, 9, -1):
            with pytest.raises(cfx.CfxError) as e:
                cfx.set_schur_delay(bad, handle=h)
            assert e.value.code == -2
        cfx.set_schur_delay(2, handle=h)
        with pytest.raises(cfx.CfxError) as e:
            cfx.getrf_masked(to_dev(G.normal_matrix(64, 1)), v=16, leaves=2, handle=h)
        assert e.value.code == -1004
    finally:
        h.close()
