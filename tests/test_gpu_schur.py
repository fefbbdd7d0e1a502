"""The Schur-complement update alone (cfx_schur_update, FactorizeA11 of
Alg. 1) against the oracle, element by element, in every precision, on
whole-tile shapes (the vectorised kernel variants, C moved non-temporally)
and ragged ones (the guarded variants), through the C ABI.

Reference: FP64 C - L21 U12 for FP64; for BF16/FP16/FP8 the oracle's
rounded operands (oracle.lowp_operands: the same rounding from FP64, FP8
after the same power-of-two row/column scaling) multiplied and summed in
FP64.  Tolerance: the accumulation of K products, FP64 (2^-52 per term) or
FP32 (2^-23 per term, matrix cores), plus the final subtraction."""
import numpy as np
import pytest

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


def operands(m, n, K, seed, wide_range=False):
    rng = np.random.default_rng(seed)
    L21 = rng.standard_normal((m, K))
    U12 = rng.standard_normal((K, n))
    C = rng.standard_normal((m, n))
    if wide_range:      # rows / columns whose magnitudes span many binades
        L21 *= 2.0 ** rng.integers(-40, 40, size=(m, 1))
        U12 *= 2.0 ** rng.integers(-40, 40, size=(1, n))
        C = C * (np.abs(L21) @ np.abs(U12))
    return L21, U12, C


def check(cfx, prec, m, n, K, seed, wgs=0, wide=False):
    L21, U12, C = operands(m, n, K, seed, wide)
    dC = to_dev(C)
    cfx.schur_update(to_dev(L21), to_dev(U12), dC, precision=prec, max_workgroups=wgs)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    if prec == "fp64":
        ref = C - L21 @ U12
        bound = (K + 2) * 2.0 ** -52 * (np.abs(L21) @ np.abs(U12) + np.abs(C))
    else:
        Lr, Ur = O.lowp_operands(L21, U12, prec)
        ref = C - Lr @ Ur
        bound = K * 2.0 ** -23 * (np.abs(Lr) @ np.abs(Ur)) + 2.0 ** -51 * (np.abs(C) + np.abs(ref))
        # the operands really were rounded: the FP64 update is measurably different
        assert np.abs((C - L21 @ U12) - ref).max() > 1e-9 * (np.abs(L21) @ np.abs(U12)).max()
    err = np.abs(got - ref)
    say(f"  {prec} {m}x{n} K={K}: max err / bound = {(err / np.maximum(bound, 1e-300)).max():.3e}")
    assert np.all(err <= bound), (prec, m, n, K)


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp16", "fp8"])
@pytest.mark.parametrize("m,n,K", [(256, 384, 256), (512, 256, 128), (384, 128, 64), (256, 256, 80)])
def test_whole_tiles(cfx, prec, m, n, K):
    say(f"schur whole tiles {prec} {m}x{n} K={K}")
    check(cfx, prec, m, n, K, 11 + m + n + K)


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp16", "fp8"])
@pytest.mark.parametrize("m,n,K", [(300, 200, 100), (129, 1, 37), (1, 257, 256), (77, 130, 1)])
def test_ragged(cfx, prec, m, n, K):
    say(f"schur ragged {prec} {m}x{n} K={K}")
    check(cfx, prec, m, n, K, 21 + m + n + K)


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp8"])
def test_bounded_persistent_grid(cfx, prec):
    say(f"schur bounded grid {prec}")
    check(cfx, prec, 640, 512, 256, 31, wgs=24)


def test_fp8_scaling_spans_binades(cfx):
    """Rows of L21 and columns of U12 between 2^-40 and 2^40: unscaled E4M3
    would flush or overflow them; the power-of-two scaling keeps each at
    the format's relative precision."""
    say("schur fp8 wide range")
    check(cfx, "fp8", 256, 256, 96, 41, wide=True)
    check(cfx, "fp8", 200, 150, 96, 42, wide=True)


def test_empty_shapes_are_no_ops(cfx):
    C = torch.ones((4, 0), dtype=torch.float64, device="cuda")
    cfx.schur_update(torch.ones((4, 3), dtype=torch.float64, device="cuda"),
                     torch.ones((3, 0), dtype=torch.float64, device="cuda"), C)
    C2 = torch.ones((4, 5), dtype=torch.float64, device="cuda")
    cfx.schur_update(torch.ones((4, 0), dtype=torch.float64, device="cuda"),
                     torch.ones((0, 5), dtype=torch.float64, device="cuda"), C2, precision="bf16")
    torch.cuda.synchronize()
    assert torch.all(C2 == 1.0)


def test_fp8_subnormal_operands(cfx):
    """Scaled operands in the E4M3 subnormal range (below 2^-6) keep their
    value: columns 1.. of every L21 row hold 0.01 (E4M3 subnormal 5 2^-9
    after the row's scaling by 2^0), the rows of U12 that meet them are 1,
    and U12's first row is 0 there, so those columns of the update consist
    of subnormal products only."""
    say("schur fp8 subnormal operands")
    m, n, K = 128, 128, 64
    L21 = np.full((m, K), 0.01)
    L21[:, 0] = 200.0
    U12 = np.ones((K, n))
    U12[0, :] = 0.0
    C = np.zeros((m, n))
    dC = to_dev(C)
    cfx.schur_update(to_dev(L21), to_dev(U12), dC, precision="fp8")
    got = dC.cpu().numpy()
    Lr, Ur = O.lowp_operands(L21, U12, "fp8")
    assert Lr[0, 1] == 5 * 2.0 ** -9
    ref = C - Lr @ Ur
    assert np.all(np.abs(got - ref) <= K * 2.0 ** -23 * (np.abs(Lr) @ np.abs(Ur)))


def test_fp8_non_finite_rows_and_columns(cfx):
    say("schur fp8 non-finite operands")
    L21, U12, C = operands(256, 256, 64, 51)
    L21[7, 3] = np.nan
    L21[200, 0] = np.inf
    U12[5, 100] = -np.inf
    dC = to_dev(C)
    cfx.schur_update(to_dev(L21), to_dev(U12), dC, precision="fp8")
    got = dC.cpu().numpy()
    ref = O.schur_lowp(C, L21, U12, "fp8")
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    Lr, Ur = O.lowp_operands(L21, U12, "fp8")
    Lr, Ur = np.nan_to_num(Lr), np.nan_to_num(Ur)
    assert np.all(np.abs(got[ok] - ref[ok]) <= (64 * 2.0 ** -23 * (np.abs(Lr) @ np.abs(Ur)) + 1e-15)[ok])
