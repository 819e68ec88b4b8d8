"""Pins of Eq. 8 dequantisation (Sec. 5.2) and of the exact-rounding helper."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_round import dequant_exact, dequant_table, round_fraction, to_bits


@pytest.mark.parametrize("m", [7, 14])
def test_oracle_dequant_matches_exact_rational(m):
    for b in range(256):
        exact = dequant_exact(b, m)
        got = oracle.dequant(b, float(m))
        # FP64: 2mb/255 rounds once (relative 2^-53), the subtraction of m once more
        assert abs(Fraction(got) - exact) <= Fraction(m, 2 ** 50)


def test_dequant_endpoints_and_symmetry():
    for m in (7, 14):
        assert oracle.dequant(0, m) == -m
        assert oracle.dequant(255, m) == m
        for b in range(256):
            # antisymmetric about the middle code: q(255 - b) = -q(b)
            assert dequant_exact(255 - b, m) == -dequant_exact(b, m)


def test_round_fraction_agrees_with_numpy_on_exact_cases():
    # dyadic values with few bits are exact in every format
    for v in [0.5, -1.75, 3.0, 1.0 / 1024, 255.0, -7.0]:
        for fmt in ("f32", "f16", "bf16"):
            assert round_fraction(Fraction(v), fmt) == v
    # numpy's float32/float16 rounding of a double that is not near a tie
    rng = np.random.default_rng(0)
    for x in rng.normal(size=200) * 10:
        assert round_fraction(Fraction(float(x)), "f32") == float(np.float32(x))
        assert round_fraction(Fraction(float(x)), "f16") == float(np.float16(x))


def test_round_fraction_ties_to_even():
    # 1 + 2^-24 is the f32 midpoint between 1 and 1 + 2^-23: ties to even -> 1
    assert round_fraction(Fraction(1) + Fraction(1, 2 ** 24), "f32") == 1.0
    assert round_fraction(Fraction(1) + Fraction(3, 2 ** 24), "f32") == 1.0 + 2.0 ** -22
    assert round_fraction(Fraction(1) + Fraction(1, 2 ** 11), "f16") == 1.0


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16"])
def test_tables_are_monotone_and_distinct_where_expected(fmt):
    for m in (7, 14):
        t = dequant_table(m, fmt)
        assert np.all(np.diff(t) >= 0)
        assert t[0] == -m and t[255] == m
        bits = to_bits(t, fmt)
        assert bits.shape == (256,)


@pytest.mark.parametrize("m", [7, 14])
def test_fp16_dequant_by_fp32_fma_is_exact(m):
    """The renderer's FP16 feature path computes RN16(RN32(b * RN32(2m/255) - m));
    for every code this equals the correctly rounded float16 of 2mb/255 - m."""
    a32 = Fraction(round_fraction(Fraction(2 * m, 255), "f32"))
    for b in range(256):
        fma32 = round_fraction(Fraction(b) * a32 - m, "f32")
        assert round_fraction(Fraction(fma32), "f16") == round_fraction(dequant_exact(b, m), "f16"), b
