"""The resampling kernels count the thresholds theta_j = (j + u) / n below a
cumulative weight c without divisions when c n - u lies more than 2^-10 from
an integer (the count is then ceil(c n - u)), and compare the two thresholds
next to the nearest integer otherwise. This checks that rule, written here in
binary64 as the kernels evaluate it (one fma, correctly rounded), against
counting the thresholds one by one, on the thresholds themselves, their
neighbours one ulp away, and random values, for target sizes up to 2^32 - 1.
The thresholds are the definition of systematic resampling's parents (Alg.
SIR, resampling step): s(j) = min{ l : C_l > theta_j }, so a particle's
offspring are the j counted between its C_{l-1} and C_l."""
import math
from fractions import Fraction

import numpy as np
import pytest

G = 2.0 ** -10


def fma(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))  # one rounding to nearest


def theta(j: int, u: float, n: int) -> float:
    return (float(j) + u) / float(n)  # two roundings, as the kernels form it


def count_exact(c: float, u: float, n: int) -> int:
    """#{j in [0, n): theta_j < c} by bisection on the monotone thresholds."""
    lo, hi = 0, n  # answer in [lo, hi]
    while lo < hi:
        mid = (lo + hi) // 2
        if theta(mid, u, n) < c:
            lo = mid + 1
        else:
            hi = mid
    return lo


def count_fast(c: float, u: float, n: int) -> int:
    if not c > 0.0:
        return 0
    if not c < 2.0:
        return n
    dn = float(n)
    x = fma(c, dn, -u)
    f = float(math.ceil(x))
    if f - x > G and f - x < 1.0 - G:
        return int(0.0 if f < 0.0 else min(f, dn))
    J = float(round(x))  # nearest integer (ties either way: both neighbours are compared)
    r = 0 if J < 1.0 else int(min(J - 1.0, dn))
    for d in (-1.0, 0.0):
        j = J + d
        if 0.0 <= j < dn and (j + u) / dn < c:
            r += 1
    return r


@pytest.mark.parametrize("n", [1, 2, 7, 1000, 21_655, 1_000_000, 2**24 + 3, 2**31 - 1, 2**32 - 1])
def test_fast_count_equals_the_threshold_count(n):
    rng = np.random.default_rng(n % 1000 + 17)
    cases = 0
    for u in [0.0, 0.5, float(np.nextafter(1.0, 0.0)), *rng.uniform(0.0, 1.0, 6)]:
        js = set(int(v) for v in rng.integers(0, n, 40)) | {0, n - 1, n // 2}
        cs = [0.0, -0.0, 1.0, float(np.nextafter(1.0, 2.0)), 2.0, 5e-324, float("nan")]
        for j in js:
            th = theta(j, u, n)
            cs += [th, float(np.nextafter(th, 0.0)), float(np.nextafter(th, 2.0)),
                   float(np.nextafter(np.nextafter(th, 2.0), 2.0))]
        cs += list(rng.uniform(0.0, 1.0, 40))
        for c in cs:
            want = count_exact(c, u, n) if c == c else 0
            assert count_fast(c, u, n) == want, (n, u, c)
            cases += 1
    assert cases > 100
