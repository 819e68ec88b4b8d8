"""Correct rounding of exact rationals to binary floating-point formats.

Used to build the bit-exact reference values of Eq. 8 dequantisation
(2 m b / 255 - m) in f32, f16 and bf16.
"""
from fractions import Fraction

import numpy as np

FORMATS = {"f32": (24, -126), "f16": (11, -14), "bf16": (8, -126)}


def round_fraction(q: Fraction, fmt: str) -> float:
    """Round q to nearest, ties to even, in the given format; returns a float
    (every such value is exactly representable in double)."""
    p, emin = FORMATS[fmt]
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    scale = Fraction(2) ** (e - (p - 1))
    n = a / scale
    fl = n.numerator // n.denominator
    rem = n - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * float(fl * scale)


def dequant_exact(b: int, m: int) -> Fraction:
    """Eq. 8 value of byte b with range m, as an exact rational."""
    return Fraction(2 * m * b, 255) - m


def dequant_table(m: int, fmt: str) -> np.ndarray:
    return np.array([round_fraction(dequant_exact(b, m), fmt) for b in range(256)], np.float64)


def to_bits(values: np.ndarray, fmt: str) -> np.ndarray:
    if fmt == "f32":
        return np.asarray(values, np.float32).view(np.uint32).astype(np.uint32)
    if fmt == "f16":
        return np.asarray(values, np.float16).view(np.uint16).astype(np.uint32)
    if fmt == "bf16":
        return (np.asarray(values, np.float32).view(np.uint32) >> 16).astype(np.uint32)
    raise ValueError(fmt)
