"""The kernels form x / 3 and x / 6 (the SSPRK3 stage combination and the
interpolated barotropic forcing) as q = RN(x r), q + (x - q d) r with r =
RN(1/d) and fused multiply-adds, and rely on this giving the bits of x / d.
Checked here in exact rational arithmetic with round-to-nearest-even at 53
and 24 bits: |1 - d r| is 2^-(p+1), and the corrected quotient equals the
correctly rounded one for random x over a wide exponent range, x of every
size class near 1, and integers."""
from fractions import Fraction

import numpy as np
import pytest


def rn(v: Fraction, p: int) -> Fraction:
    """v rounded to p significant bits, ties to even (no exponent limits)."""
    if v == 0:
        return Fraction(0)
    sign = -1 if v < 0 else 1
    a = abs(v)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    scale = Fraction(2) ** (p - 1 - e)          # a * scale in [2^(p-1), 2^p)
    m = a * scale
    n, r = divmod(m.numerator, m.denominator)
    twice = 2 * r
    if twice > m.denominator or (twice == m.denominator and n % 2 == 1):
        n += 1
    return sign * Fraction(n) / scale


def corrected_quotient(x: Fraction, d: int, p: int) -> Fraction:
    r = rn(Fraction(1, d), p)
    q = rn(x * r, p)
    e = rn(x - q * d, p)                        # fused: one rounding
    return rn(q + e * r, p)                     # fused: one rounding


@pytest.mark.parametrize("p", [53, 24])
@pytest.mark.parametrize("d", [3, 6])
def test_reciprocal_error_is_half_an_ulp_or_less(d, p):
    r = rn(Fraction(1, d), p)
    assert abs(1 - d * r) == Fraction(1, 2 ** (p + 1))


@pytest.mark.parametrize("p", [53, 24])
@pytest.mark.parametrize("d", [3, 6])
def test_corrected_quotient_is_correctly_rounded(d, p):
    rng = np.random.default_rng(1000 * d + p)
    xs = []
    for _ in range(1500):
        m = int(rng.integers(2 ** (p - 1), 2 ** p))
        e = int(rng.integers(-60, 60))
        xs.append((-1) ** int(rng.integers(2)) * Fraction(m) * Fraction(2) ** (e - p + 1))
    xs += [Fraction(2 ** (p - 1) + k, 2 ** (p - 1)) for k in range(0, 2 ** (p - 1), 2 ** (p - 1) // 512)]
    xs += [Fraction(k) for k in range(-300, 301)]
    for x in xs:
        assert corrected_quotient(x, d, p) == rn(x / d, p), (x, d, p)


def test_rounding_helper_matches_ieee_doubles():
    rng = np.random.default_rng(7)
    a, b = rng.normal(size=200), rng.normal(size=200) + 3.0
    for x, y in zip(a, b):
        assert float(rn(Fraction(x) / Fraction(y), 53)) == x / y
        assert float(rn(Fraction(x) * Fraction(y), 53)) == x * y
