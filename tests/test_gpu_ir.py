"""GPU tests of the mixed-precision factorisation (BF16/FP16 Schur updates)
and of GMRES-IR (cfx_gesv_ir), through the C ABI.

The low-precision factors are not unique to compare element by element over
many panels (rounding changes later pivots), so the pins are: exact factors
when every operand is representable; one low-precision update compared with
the oracle's rounded-operand update; the backward error of the factors at
the format's precision; and for the solve, the oracle's compensated eta of
the returned x (<= 5e-15) and the forward error against the closed-form
solution of the Householder systems."""
import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O
from tests.gpu_util import compare_panels, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["bf16", "fp16"]


@pytest.fixture(scope="module")
def cfx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_05975_amd import cfx as m
    m.lib()
    return m


def run_getrf(cfx, A, v, L, precision, lookahead=0):
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=v, leaves=L, precision=precision, lookahead=lookahead)
    torch.cuda.synchronize()
    return dA.cpu().numpy(), ipiv.cpu().numpy(), int(info.cpu()[0])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,v,L,la", [(64, 16, 3, 0), (64, 8, 4, 1), (50, 7, 5, 0), (64, 32, 1, 1)])
def test_lowp_getrf_exact_for_representable_factors(cfx, prec, n, v, L, la):
    say(f"lowp dd exact {prec} n={n} v={v} L={L} la={la}")
    L0, U0 = G.dyadic_dd_factors(n, 1)
    A = L0 @ U0
    LU, ipiv, info = run_getrf(cfx, A, v, L, prec, la)
    assert info == 0
    assert np.array_equal(ipiv, np.arange(n))
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)


@pytest.mark.parametrize("prec", PRECS + ["fp8"])
@pytest.mark.parametrize("n,v,L", [(300, 256, 4), (160, 128, 2), (100, 64, 3), (77, 40, 2),
                                   (256, 128, 2), (512, 256, 4)])
def test_lowp_single_update_matches_oracle(cfx, prec, n, v, L):
    """n = v + m with m <= v: one low-precision Schur update (K = v), then
    the last panel factors the m x m tail in FP64 (a single leaf)."""
    say(f"lowp one update {prec} n={n} v={v} L={L}")
    A = G.normal_matrix(n, 21)
    f, S = O.tail_after_lowp_update(A, v, L, prec)
    m = n - v
    tail = O.getrf(S, m, L)
    LU, ipiv, info = run_getrf(cfx, A, v, L, prec)
    assert info == 0
    assert f.margins[0] > 1e-10
    assert np.array_equal(ipiv[:v], f.ipiv[:v])
    # first panel (FP64 arithmetic): U00, U12 as the oracle's
    tol = 1e-9 * np.abs(f.LU).max()
    np.testing.assert_allclose(LU[:v, :], f.LU[:v, :], rtol=0, atol=tol)
    # the tail: the GPU's last panel factors its own low-precision Schur
    # complement S_gpu in FP64, so L22 U22 = P22 S_gpu up to FP64 rounding.
    # The rounding to the low format is a quantisation decided from FP64
    # values: the check rounds the GPU's own first-panel factors (equal to
    # the oracle's to 1e-9, but an ulp apart can round to different BF16
    # neighbours), multiplies and sums them exactly (FP64), and allows the
    # FP32 accumulation of the matrix cores: K terms, relative 2^-24 each.
    perm22 = O.ipiv_to_perm((ipiv[v:] - v).astype(np.int32))
    perm0 = O.ipiv_to_perm(np.concatenate([f.ipiv[:v], np.arange(v, n)]).astype(np.int32))
    PA22 = A[perm0][v:, v:][perm22]
    L22, U22 = O.unpack(LU[v:, v:])
    R = L22 @ U22
    Lr, Ur = O.lowp_operands(LU[v:, :v], LU[:v, v:], prec)
    Sg = PA22 - Lr @ Ur
    scale = (np.abs(Lr) @ np.abs(Ur)).max()
    d_lp = np.abs(R - Sg).max()
    d_64 = np.abs(R - (PA22 - LU[v:, :v] @ LU[:v, v:])).max()     # FP64 complement
    say(f"  |L22U22 - P S_lowp| = {d_lp:.3e}, vs FP64 complement {d_64:.3e}, scale {scale:.3e}")
    assert d_lp <= 2.0 ** -24 * v * scale + 1e-12 * np.abs(Sg).max()
    assert d_64 > 1e-6 * scale            # the operands really were rounded
    # L21 as the oracle's, its rows moved by the last panel's interchanges
    np.testing.assert_allclose(LU[v:, :v], f.LU[v:, :v][perm22], rtol=0, atol=tol)
    if tail.margins[0] > 1e-4:
        assert np.array_equal(ipiv[v:] - v, tail.ipiv)


@pytest.mark.parametrize("prec,hi", [("bf16", 0.3), ("fp16", 0.05), ("fp8", 3.0)])
@pytest.mark.parametrize("la", [0, 1])
def test_lowp_getrf_backward_error(cfx, prec, hi, la):
    say(f"lowp backward error {prec} la={la}")
    n, v, L = 1024, 64, 4
    A = G.normal_matrix(n, 3)
    LU, ipiv, info = run_getrf(cfx, A, v, L, prec, la)
    assert info == 0
    r = O.lu_residual(A, LU, ipiv)
    say(f"  ||PA-LU||/||A|| = {r:.3e}")
    assert 1e-6 < r < hi
    ref = O.getrf(A, v, L)
    assert np.array_equal(ipiv[:v], ref.ipiv[:v])


# ---------------------------------------------------------------------------
# GMRES-IR
# ---------------------------------------------------------------------------

def householder_case(n, cond, seed):
    spec = G.householder_spec(n, cond, seed)
    A = G.householder_matrix(spec)
    b = G.rhs(n, 1, seed + 1)
    xs = G.householder_solution(spec, b)
    return A, b, xs


@pytest.mark.parametrize("prec,n,wgs,chunk", [("bf16", 2100, 8, 64), ("fp16", 2100, 12, 300),
                                              ("bf16", 2048, 24, 4096), ("fp16", 2048, 8, 256)])
def test_lowp_bounded_schur_grid_bitwise_equal(cfx, prec, n, wgs, chunk):
    """A bounded, persistent grid for the low-precision Schur launches
    (few workgroups walking many tiles; ragged or whole tiles) changes
    scheduling only: the factors are bitwise those of the unbounded grid."""
    v, L = 128, 4
    say(f"lowp bounded schur grid {prec} wgs={wgs} chunk={chunk} n={n}")
    A = G.normal_matrix(n, 13)
    ref = run_getrf(cfx, A, v, L, prec, 1)
    h = cfx.Handle()
    try:
        cfx.set_overlap_tuning(wgs, chunk, 0, handle=h)
        dA = to_dev(A)
        ipiv, info = cfx.getrf(dA, v=v, leaves=L, precision=prec, lookahead=1, handle=h)
        torch.cuda.synchronize()
    finally:
        h.close()
    assert int(info.cpu()[0]) == ref[2]
    assert np.array_equal(ipiv.cpu().numpy(), ref[1])
    assert np.array_equal(dA.cpu().numpy(), ref[0])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("cond", [1e2, 1e6])
def test_gesv_ir_householder(cfx, prec, cond):
    n = 2048
    say(f"gesv_ir {prec} cond={cond:g} n={n}")
    A, b, xs = householder_case(n, cond, 5)
    dA, db = to_dev(A), to_dev(b)
    X, rep = cfx.gesv_ir(dA, db, precision=prec, v=128, leaves=4, tol=5e-15, max_outer=20,
                         gmres_restart=30, gmres_tol=1e-6)
    x = X.cpu().numpy()
    eta = O.eta(A, x, b)
    fwd = np.abs(x - xs).max() / np.abs(xs).max()
    say(f"  report {rep}; oracle eta {eta:.3e}; forward error {fwd:.3e}")
    assert rep["info"] == 0 and rep["converged"] == 1
    assert eta <= 5e-15
    # the library's own eta (compensated residual) agrees with the oracle's
    assert abs(rep["eta"] - eta) <= 0.05 * eta + 1e-19
    assert rep["eta_first"] > 1e-10          # the factors alone are far from the target
    assert fwd <= 100 * cond * 5e-15 + 1e-13
    # inputs untouched
    assert np.array_equal(dA.cpu().numpy(), A) and np.array_equal(db.cpu().numpy(), b)


@pytest.mark.parametrize("cond", [1e2, 1e6])
def test_gesv_ir_fp8_experiment(cfx, cond):
    """FP8 Schur updates (3 fraction bits) with FP64 GMRES-IR: whatever the
    outcome, the report is consistent with the oracle; a converged solve
    meets eta <= 5e-15 by the oracle's own measure."""
    n = 2048
    say(f"gesv_ir fp8 cond={cond:g} n={n}")
    A, b, xs = householder_case(n, cond, 5)
    X, rep = cfx.gesv_ir(to_dev(A), to_dev(b), precision="fp8", v=128, leaves=4, tol=5e-15, max_outer=20,
                         gmres_restart=30, gmres_tol=1e-6)
    x = X.cpu().numpy()
    eta = O.eta(A, x, b)
    say(f"  report {rep}; oracle eta {eta:.3e}")
    assert rep["info"] == 0
    assert np.isfinite(rep["eta"]) and abs(rep["eta"] - eta) <= 0.05 * eta + 1e-19
    if rep["converged"]:
        assert eta <= 5e-15
    else:
        assert eta > 5e-15


def test_gesv_ir_stagnation_stops_early(cfx):
    """BF16 factors of a cond-1e12 system: eta cannot reach the target; the
    refinement stops once eta fails to halve over two steps, long before
    max_outer, and reports no convergence."""
    n = 1024
    say("gesv_ir stagnation")
    A, b, xs = householder_case(n, 1e12, 9)
    X, rep = cfx.gesv_ir(to_dev(A), to_dev(b), precision="bf16", v=128, leaves=4, tol=5e-15, max_outer=50,
                         gmres_restart=20, gmres_tol=1e-6)
    say(f"  {rep}")
    assert rep["converged"] == 0
    assert 2 <= rep["outer"] < 50
    assert np.isfinite(rep["eta"]) and rep["eta"] > 5e-15


def test_gesv_ir_fp64_factors(cfx):
    n = 1000
    say("gesv_ir fp64 factors")
    A, b, xs = householder_case(n, 1e6, 7)
    X, rep = cfx.gesv_ir(to_dev(A), to_dev(b), precision="fp64", v=64, leaves=4)
    x = X.cpu().numpy()
    say(f"  {rep}")
    assert rep["converged"] == 1 and rep["outer"] <= 3
    assert O.eta(A, x, b) <= 5e-15


@pytest.mark.parametrize("prec", PRECS)
def test_gesv_ir_several_rhs_with_strides(cfx, prec):
    n, nrhs = 700, 3
    say(f"gesv_ir nrhs={nrhs} {prec}")
    A = G.normal_matrix(n, 11) + 2 * np.sqrt(n) * np.eye(n)
    Bw = G.rhs(n, nrhs + 2, 12)
    dBw = to_dev(Bw)
    dB = dBw[:, 1:1 + nrhs]                     # ldb = nrhs + 2
    dXw = torch.zeros((n, nrhs + 5), dtype=torch.float64, device="cuda")
    dX = dXw[:, 2:2 + nrhs]                     # ldx = nrhs + 5
    dA = to_dev(A)
    _, rep = cfx.gesv_ir(dA, dB, X=dX, precision=prec, v=64, leaves=3)
    X = dXw.cpu().numpy()
    say(f"  {rep}")
    assert rep["converged"] == 1
    for c in range(nrhs):
        assert O.eta(A, X[:, 2 + c], Bw[:, 1 + c]) <= 5e-15
    assert np.all(X[:, :2] == 0) and np.all(X[:, 2 + nrhs:] == 0)
    assert np.array_equal(dBw.cpu().numpy(), Bw) and np.array_equal(dA.cpu().numpy(), A)


def test_gesv_ir_singular_reports_info(cfx):
    n = 96
    say("gesv_ir singular")
    A = G.normal_matrix(n, 2)
    A[:, 40] = 0.0
    _, rep = cfx.gesv_ir(to_dev(A), to_dev(G.rhs(n, 1, 3)), precision="bf16", v=32, leaves=2,
                         max_outer=3)
    say(f"  {rep}")
    assert rep["info"] == 41
    assert rep["converged"] == 0


def test_gesv_ir_empty(cfx):
    say("gesv_ir empty")
    A = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    B = torch.zeros((0, 1), dtype=torch.float64, device="cuda")
    _, rep = cfx.gesv_ir(A, B, precision="bf16", v=32, leaves=2)
    assert rep["converged"] == 1 and rep["info"] == 0
