"""Pins of the oracle's adaptive bin rule (CPU only).

The paper names adaptive bin sizes as future work without a rule; the rule
read here sets, per target and spatial axis, m = ceil(c / sd) cells per pixel
clamped to [1, m_max], sd the standard deviation of the propagated positions.
Pinned: the variance against numpy's two-pass one (within the rounding of
the one-pass form), m at constructed spreads (including a
spread that makes c / sd an integer), the clamps at sd = 0 and at large
spreads, and NaN positions taken as 2^24 like the cell index takes them.
"""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def test_variance_matches_numpy(orc):
    rng = np.random.default_rng(3)
    for sd in (0.05, 0.3, 2.0, 40.0):
        st = np.zeros((5, 5000), np.float32)
        st[0] = 500.0 + sd * rng.standard_normal(5000)
        st[1] = 20.0 + 0.5 * sd * rng.standard_normal(5000)
        m, var = orc.adaptive_bins(st, 2, 2.0, 16)
        for a in range(2):
            xa = st[a].astype(np.float64)
            ref = np.var(xa)
            # the one-pass form S2/n - mean^2 loses up to a few ulp of S2/n
            assert abs(var[a] - ref) <= 8 * 2.0 ** -53 * np.mean(xa * xa)
            want = 16 if 2.0 / math.sqrt(ref) >= 16 else max(1, math.ceil(2.0 / math.sqrt(ref)))
            assert m[a] == want
        assert m[2] == 1


def test_constructed_spreads(orc):
    def m_of(d, c=2.0, m_max=8, dim=2):
        st = np.zeros((2 * dim + 1, 2), np.float32)
        st[0] = [100.0 - d, 100.0 + d]   # population sd = d on x
        st[1] = [7.0, 7.0]               # sd = 0 on y
        if dim == 3:
            st[2] = [0.0, 3.0]           # sd = 1.5 on z
        return orc.adaptive_bins(st, dim, c, m_max)[0]
    assert m_of(0.3) == (7, 8, 1)        # ceil(2 / 0.3) = 7; sd = 0 -> m_max
    assert m_of(0.5) == (4, 8, 1)        # 2 / 0.5 = 4 exactly
    assert m_of(0.25) == (8, 8, 1)       # 2 / 0.25 = 8 = m_max
    assert m_of(0.125) == (8, 8, 1)      # above m_max
    assert m_of(50.0) == (1, 8, 1)       # ceil(0.04) = 1
    assert m_of(0.3, dim=3) == (7, 8, 2)  # ceil(2 / 1.5) = 2


def test_nan_positions_count_as_far_away(orc):
    st = np.zeros((5, 4), np.float32)
    st[0] = [10.0, 10.1, 10.2, np.nan]
    st[1] = [3.0, 3.0, 3.1, 3.0]
    m, var = orc.adaptive_bins(st, 2, 2.0, 8)
    assert m[0] == 1 and var[0] > 1e13
