"""Pins of the oracle's low-precision pieces (round_lowp and the trailing
matrix after one low-precision Schur update) against values fixed by the
BF16 / FP16 formats themselves and by exactly representable inputs."""
import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O


def test_bf16_round_to_nearest_even():
    u = 2.0 ** -8   # half an ulp of BF16 at 1
    x = np.array([1.0, 1 + u, 1 + 3 * u, 1 + u + 2.0 ** -20, -(1 + u), -(1 + 3 * u), 3.0, 0.0, -0.0])
    want = np.array([1.0, 1.0, 1 + 4 * u, 1 + 2 * u, -1.0, -(1 + 4 * u), 3.0, 0.0, -0.0])
    got = O.round_lowp(x, "bf16")
    assert np.array_equal(got, want)
    assert np.array_equal(np.signbit(got), np.signbit(want))


def test_rounding_is_direct_from_fp64():
    # 1 + 2^-8 + 2^-30 lies above the BF16 midpoint 1 + 2^-8: the nearest BF16
    # value is 1 + 2^-7 (an FP32 intermediate would first land exactly on the
    # midpoint and then tie to 1).  Likewise for FP16 around 1 + 2^-11.
    assert O.round_lowp(np.array([1 + 2.0 ** -8 + 2.0 ** -30]), "bf16")[0] == 1 + 2.0 ** -7
    assert O.round_lowp(np.array([1 + 2.0 ** -11 + 2.0 ** -40]), "fp16")[0] == 1 + 2.0 ** -10
    assert O.round_lowp(np.array([-(1 + 2.0 ** -8 + 2.0 ** -30)]), "bf16")[0] == -(1 + 2.0 ** -7)


def test_bf16_special_values():
    x = np.array([np.inf, -np.inf, np.nan, 1e39, 3.3895313892515355e38, 2.0 ** -130, 3 * 2.0 ** -134,
                  2.0 ** -134])
    got = O.round_lowp(x, "bf16")
    assert got[0] == np.inf and got[1] == -np.inf and np.isnan(got[2])
    assert got[3] == np.inf                       # beyond the largest finite value
    assert got[4] == 3.3895313892515355e38        # largest finite BF16
    assert got[5] == 2.0 ** -130                  # subnormal, representable
    # subnormal quantum 2^-133: 1.5 quanta ties to the even 2 quanta, 0.5 to 0
    assert got[6] == 2.0 ** -132 and got[7] == 0.0


def test_matches_numpy_float16():
    """Special case that reduces to a library routine: numpy's FP16 cast
    rounds FP64 directly to nearest-even."""
    x = G.normal_matrix(128, 5).ravel() * np.logspace(-9, 4, 128 * 128)
    assert np.array_equal(O.round_lowp(x, "fp16"), x.astype(np.float16).astype(np.float64))


def test_bf16_error_bound_and_format():
    x = G.normal_matrix(64, 3).ravel() * 1e3
    r = O.round_lowp(x, "bf16")
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 2.0 ** -20))
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert np.array_equal(O.round_lowp(r, "bf16"), r)


def test_fp16_round_to_nearest_even():
    u = 2.0 ** -11
    x = np.array([1 + u, 1 + 3 * u, 65504.0, 65519.0, 65520.0, 2.0 ** -24, 2.0 ** -26])
    want = np.array([1.0, 1 + 4 * u, 65504.0, 65504.0, np.inf, 2.0 ** -24, 0.0])
    assert np.array_equal(O.round_lowp(x, "fp16"), want)


def test_tail_exact_for_representable_factors():
    """Dyadic factors with off-diagonal entries k/512 are exact in BF16 and
    FP16, so the low-precision trailing matrix equals the FP64 one."""
    n, v = 64, 16
    L0, U0 = G.dyadic_dd_factors(n, 1)
    A = L0 @ U0
    full = O.getrf(A, v, 1, npanels=1)
    for prec in ("bf16", "fp16"):
        f, S = O.tail_after_lowp_update(A, v, 1, prec)
        assert np.array_equal(S, full.LU[v:, v:])


@pytest.mark.parametrize("prec,lo,hi", [("bf16", 1e-4, 2e-2), ("fp16", 1e-5, 3e-3)])
def test_tail_differs_at_the_format_precision(prec, lo, hi):
    """For general inputs the low-precision tail differs from the FP64 one by
    the rounding of the operands: relative size between u_lp/40 and 4 u_lp."""
    n, v = 200, 64
    A = G.normal_matrix(n, 9)
    full = O.getrf(A, v, 2, npanels=1)
    f, S = O.tail_after_lowp_update(A, v, 2, prec)
    assert np.array_equal(f.ipiv[:v], full.ipiv[:v])
    d = np.abs(S - full.LU[v:, v:]).max()
    scale = (np.abs(f.LU[v:, :v]) @ np.abs(f.LU[:v, v:])).max()
    assert lo <= d / scale <= hi
