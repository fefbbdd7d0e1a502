"""Pins of the oracle's low-precision pieces (round_lowp, the FP8 scaling and
the trailing matrix after one low-precision Schur update) against values
fixed by the BF16 / FP16 / FP8 E4M3 formats themselves and by exactly
representable inputs."""
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


def test_tail_exact_for_fp8_representable_factors():
    """Factors whose rows of L21 and columns of U12 hold values with at most
    4 significant bits inside a range of 2^7 are exact in scaled E4M3, so the
    FP8 trailing matrix equals the FP64 one."""
    rng = np.random.default_rng(4)
    m, K, n = 40, 16, 24
    L21 = rng.integers(-15, 16, size=(m, K)) * 2.0 ** rng.integers(-20, 20, size=(m, 1))
    U12 = rng.integers(-15, 16, size=(K, n)) * 2.0 ** rng.integers(-20, 20, size=(1, n))
    C = rng.standard_normal((m, n))
    assert np.array_equal(O.schur_lowp(C, L21, U12, "fp8"), C - L21 @ U12)


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


def e4m3_values():
    """Every finite non-negative E4M3 value, from the encoding: exponent field
    E (bias 7) and fraction field M; E = 0 is subnormal (M/8 2^-6); the
    all-ones pattern (E = 15, M = 7) is NaN."""
    vals = [M / 8 * 2.0 ** -6 for M in range(8)]
    for E in range(1, 16):
        for M in range(8):
            if E == 15 and M == 7:
                continue
            vals.append((1 + M / 8) * 2.0 ** (E - 7))
    return np.array(vals)


def test_fp8_every_value_is_fixed_and_counted():
    v = e4m3_values()
    assert len(v) == 127 and v.max() == 448.0 and v[1] == 2.0 ** -9
    assert np.array_equal(O.round_lowp(v, "fp8"), v)
    assert np.array_equal(O.round_lowp(-v, "fp8"), -v)


def test_fp8_round_to_nearest_even():
    x = np.array([1 + 2.0 ** -4, 1 + 3 * 2.0 ** -4, 1 + 2.0 ** -4 + 2.0 ** -30, 17.0, 19.0, 2.0 ** -10,
                  1.5 * 2.0 ** -10, 3 * 2.0 ** -10, 240.0, 248.0, 464.0, 464.0 + 2.0 ** -40, -17.0])
    want = np.array([1.0, 1.25, 1.125, 16.0, 20.0, 0.0, 2.0 ** -9, 2.0 ** -8, 240.0, 256.0, 448.0, np.nan,
                     -16.0])
    got = O.round_lowp(x, "fp8")
    assert np.array_equal(got, want, equal_nan=True)


def test_fp8_no_infinities():
    got = O.round_lowp(np.array([np.inf, -np.inf, np.nan, 1e6]), "fp8")
    assert np.all(np.isnan(got))


def test_fp8_nearest_among_all_values():
    """Brute force: the result is a nearest representable value, and on a
    tie the one with an even fraction field."""
    v = e4m3_values()
    x = np.random.default_rng(5).uniform(0, 460, 4000) * 2.0 ** np.random.default_rng(6).integers(-14, 1, 4000)
    r = O.round_lowp(x, "fp8")
    d = np.abs(x[:, None] - v[None, :])
    best = d.min(axis=1)
    assert np.all(np.abs(r - x) == best)


def test_fp8_scale_exponents():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((30, 50)) * 10.0 ** rng.uniform(-30, 30, size=(30, 1))
    M[3] = 0.0
    s = O.fp8_scale_exponents(M, 1)
    peak = np.abs(np.ldexp(M, s[:, None])).max(axis=1)
    assert s[3] == 0
    ok = np.arange(30) != 3
    assert np.all((peak[ok] >= 128) & (peak[ok] < 256))
    # columns: the same rule on the transpose
    assert np.array_equal(O.fp8_scale_exponents(M.T.copy(), 0), s)


def test_fp8_update_error_at_the_format_precision():
    """Scaled E4M3 operands carry a relative error of at most 2^-4 each, so
    the update differs from the FP64 one by at most about 2^-3 (|L| |U|)."""
    rng = np.random.default_rng(8)
    L21 = rng.standard_normal((60, 32))
    U12 = rng.standard_normal((32, 45)) * 1e-3
    C = rng.standard_normal((60, 45))
    d = np.abs(O.schur_lowp(C, L21, U12, "fp8") - (C - L21 @ U12))
    bound = (2.0 ** -4 * 2 + 2.0 ** -8) * (np.abs(L21) @ np.abs(U12))
    assert np.all(d <= bound)
    assert d.max() > 1e-3 * bound.max()


def test_fp8_non_finite_rows_and_columns_give_nan():
    rng = np.random.default_rng(9)
    L21 = rng.standard_normal((6, 5))
    U12 = rng.standard_normal((5, 7))
    L21[2, 3] = np.nan
    U12[1, 4] = np.inf
    S = O.schur_lowp(np.zeros((6, 7)), L21, U12, "fp8")
    nan = np.isnan(S)
    assert np.all(nan[2]) and np.all(nan[:, 4])
    assert nan.sum() == 7 + 6 - 1
