"""The FP32 fused multiply-add of the mixed-precision brute force
(tests/bruteforce.py), against exact rational arithmetic rounded to float32
(to nearest, ties to even): random operands over many magnitudes, and sums
that fall within float64 rounding of a float32 midpoint, where rounding the
float64 sum alone would pick the wrong side."""
from fractions import Fraction

import numpy as np

from tests.bruteforce import fma32


def _round32(v: Fraction) -> np.float32:
    f = np.float32(float(v))
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    def key(x):
        even = int(np.array(x, np.float32).view(np.uint32)) & 1
        return (abs(Fraction(float(x)) - v), even)
    return min(cands, key=key)


def test_fma32_random_is_correctly_rounded():
    rng = np.random.default_rng(5)
    n = 4000
    a = (rng.normal(size=n) * 10.0 ** rng.integers(-4, 4, n)).astype(np.float32)
    b = (rng.normal(size=n) * 10.0 ** rng.integers(-4, 4, n)).astype(np.float32)
    c = (rng.normal(size=n) * 10.0 ** rng.integers(-8, 4, n)).astype(np.float32)
    got = fma32(a, b, c)
    for i in range(n):
        ex = _round32(Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i])))
        assert got[i] == ex, (a[i], b[i], c[i], got[i], ex)


def test_fma32_near_midpoints():
    # a b = 1 + 2^-24 - 2^-47 exactly; c brings the sum to 1 + 2^-24 +- 2^-60,
    # which rounds in float64 to the float32 midpoint 1 + 2^-24
    a = np.float32(1 + 2.0 ** -23)
    b = np.float32(1 - 2.0 ** -24)
    for c, want in ((2.0 ** -47 + 2.0 ** -60, 1 + 2.0 ** -23),   # just above: up
                    (2.0 ** -47 - 2.0 ** -60, 1.0),              # just below: down
                    (2.0 ** -47, 1.0)):                          # exact tie: even
        c32 = np.float32(c)
        assert float(c32) == c
        ex = _round32(Fraction(float(a)) * Fraction(float(b)) + Fraction(c))
        assert float(ex) == want
        assert fma32(a, b, c32) == ex, (c, fma32(a, b, c32), ex)
