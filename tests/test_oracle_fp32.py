"""Pins of the oracle's binary32 fused multiply-add (oracle/fp32.py) against exact
rational arithmetic: the result must be a*b + c rounded once to the nearest
binary32 value, ties to even (IEEE 754 fusedMultiplyAdd)."""
from fractions import Fraction

import numpy as np

from oracle.fp32 import fma32

f32 = np.float32


def round_exact(x):
    """Nearest binary32 to the rational x, ties to even."""
    f = f32(float(x))
    cands = [np.nextafter(f, f32(-np.inf)), f, np.nextafter(f, f32(np.inf))]
    best = None
    for c in cands:
        d = abs(Fraction(float(c)) - x)
        even = (int(np.array(c, dtype=f32).view(np.uint32)) & 1) == 0
        key = (d, not even)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


def exact_fma(a, b, c):
    return round_exact(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def test_double_rounding_cases():
    # a*b = 2^-24 + 2^-60 (2^36 + 1 = 4097 * 16773121): 1 + a*b rounds to the binary32
    # midpoint 1 + 2^-24 in binary64, but the exact sum lies above it
    a, b = f32(4097 * 2.0 ** -36), f32(16773121 * 2.0 ** -24)
    assert float(a) * float(b) == 2.0 ** -24 + 2.0 ** -60
    assert np.float32(float(a) * float(b) + 1.0) == f32(1.0)            # rounding twice goes wrong
    assert fma32(a, b, f32(1.0)) == f32(1.0 + 2.0 ** -23) == exact_fma(a, b, f32(1.0))
    assert fma32(-a, b, f32(-1.0)) == f32(-1.0 - 2.0 ** -23)
    # a*b = 2^-24 - 2^-60 (2^36 - 1 = 262143 * 262145): exact sum below the midpoint
    a2, b2 = f32(262143 * 2.0 ** -36), f32(262145 * 2.0 ** -24)
    assert fma32(a2, b2, f32(1.0)) == f32(1.0) == exact_fma(a2, b2, f32(1.0))
    # a true tie stays a tie: 1 + 2^-24 exactly rounds to even (1.0), 1 + 3*2^-24 to 1 + 2^-22
    assert fma32(f32(2.0 ** -24), f32(1.0), f32(1.0)) == f32(1.0)
    assert fma32(f32(3 * 2.0 ** -24), f32(1.0), f32(1.0)) == f32(1.0 + 2.0 ** -22)


def test_random_against_exact():
    rng = np.random.Generator(np.random.PCG64(11))
    n = 4000
    mag = lambda: (10.0 ** rng.uniform(-6, 6, n)) * rng.choice([-1.0, 1.0], n)
    a, b, c = mag().astype(f32), mag().astype(f32), mag().astype(f32)
    # half of the cases with c close to -a*b (cancellation)
    c[: n // 2] = (-(a[: n // 2].astype(np.float64) * b[: n // 2]) * (1 + rng.uniform(-1e-6, 1e-6, n // 2))).astype(f32)
    got = fma32(a, b, c)
    for k in range(n):
        assert got[k] == exact_fma(a[k], b[k], c[k]), (a[k], b[k], c[k])


def test_special_cases():
    rng = np.random.Generator(np.random.PCG64(12))
    a = rng.uniform(-100, 100, 500).astype(f32)
    b = rng.uniform(-100, 100, 500).astype(f32)
    # with c = 0 it is the correctly rounded product; with a = 1 the correctly rounded sum
    assert np.array_equal(fma32(a, b, f32(0.0)), (a.astype(np.float64) * b).astype(f32))
    assert np.array_equal(fma32(f32(1.0), a, b), a + b)
    assert np.isnan(fma32(f32(np.nan), f32(1.0), f32(1.0)))
