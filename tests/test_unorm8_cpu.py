"""The kernels' colour channel c = u / 255 (u an 8-bit value) is formed as
q = u r with r = RN(1/255), then c = fma(fma(-q, 255, u), r, q): three FP32
operations in place of an IEEE division.  This test replays those operations
for every u in exact rational arithmetic, each rounded once to FP32, and
requires the IEEE quotient RN(u / 255) every time."""
from fractions import Fraction as Fr

import numpy as np


def rn32(x):
    """x (a Fraction in FP32's normal range, or 0) rounded to the nearest float32, ties to even."""
    if x == 0:
        return Fr(0)
    s = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    while Fr(2) ** e > x:
        e -= 1
    while Fr(2) ** (e + 1) <= x:
        e += 1
    assert -126 <= e <= 127
    m = x / Fr(2) ** (e - 23)  # in [2^23, 2^24)
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and fl % 2 == 1):
        fl += 1
    return s * Fr(fl) * Fr(2) ** (e - 23)


def test_rn32_agrees_with_numpy():
    rng = np.random.default_rng(3)
    for a, b in rng.integers(1, 1 << 20, size=(500, 2)):
        assert float(rn32(Fr(int(a), int(b)))) == float(np.float32(a) / np.float32(b))


def test_every_channel_value_is_the_ieee_quotient():
    r = rn32(Fr(1, 255))
    assert float(r) == float(np.float32(1.0) / np.float32(255.0))
    for u in range(256):
        q = rn32(Fr(u) * r)
        e = rn32(Fr(u) - 255 * q)  # the inner fma: one rounding of the exact remainder
        c = rn32(e * r + q)        # the outer fma
        assert c == rn32(Fr(u, 255)), u
        assert float(c) == float(np.float32(u) / np.float32(255.0)), u
