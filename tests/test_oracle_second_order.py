"""Pins of the oracle's second-order dummies (CPU only).

Sec. 4 notes that a dummy could carry higher moments of its members than the
mean. The reading here: the bin's log-likelihood is the log of its members'
mean likelihood to second order in their spread, ell(mu) + tr(H S)/2 +
g'S g/2, with S the members' position covariance and g, H the gradient and
Hessian of the log-likelihood in the bin's window (central differences of
half a cell). Pinned: a bin with one member (S = 0) keeps the first-order
value exactly; and over the bins of a cloud, the second-order value is
closer than the first-order one to the members' exact log-mean likelihood,
computed member by member in the bin's window (an independent route).
"""
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def _mdl(orc, m, mode, sxi):
    return orc.Model(dim=2, m=(m, m, 1), patch=11, quad=2, sigma_psf=1.5, i_bg=10.0, sigma_xi=sxi, seed=2,
                     dummy_mode=mode, proc_sigma=(0.5, 0.5, 0.1, 0.1, 2.0))


@pytest.fixture(scope="module")
def scene():
    w = synth.preset("single-2d-64", K=2)
    tr = synth.truth(w, seed=4)
    fr = synth.frames(w, tr, seed=4)
    return w, tr, fr


def test_single_member_bins_keep_first_order(orc, scene):
    w, tr, fr = scene
    st = synth.random_cloud(w, tr[1, 0], 40, 3.0, seed=5)
    st[0] = tr[1, 0, 0] + np.arange(40, dtype=np.float32)   # one particle per pixel column
    a = orc.weigh(_mdl(orc, 4, 0, 10.0), fr[1], st, sir=False)
    b = orc.weigh(_mdl(orc, 4, 2, 10.0), fr[1], st, sir=False)
    assert np.all(a["bin_n"] == 1)
    np.testing.assert_array_equal(a["ll"], b["ll"])


def _errors(orc, fr, st, m, sxi):
    """|first - exact| and |second - exact| per bin of 20 members or more."""
    first = orc.weigh(_mdl(orc, m, 0, sxi), fr, st, sir=False)
    second = orc.weigh(_mdl(orc, m, 2, sxi), fr, st, sir=False)
    mdl = _mdl(orc, m, 0, sxi)
    e1, e2 = [], []
    for b in range(first["B"]):
        mem = np.flatnonzero(first["bin_of"] == b)
        if mem.size < 20:
            continue
        c0, r0 = int(first["bin_key"][0, b]) // m, int(first["bin_key"][1, b]) // m
        ls = np.array([orc.loglik(mdl, fr, c0, r0, float(st[0, i]), float(st[1, i]), 0.0,
                                  float(first["bin_mean"][4, b])) for i in mem])
        exact = ls.max() + math.log(np.mean(np.exp(ls - ls.max())))
        e1.append(abs(first["ll"][b] - exact))
        e2.append(abs(second["ll"][b] - exact))
    return np.array(e1), np.array(e2)


@pytest.mark.parametrize("m,sxi,factor", [(2, 40.0, 0.1), (4, 10.0, 0.7)])
def test_second_order_approaches_the_members_mean(orc, scene, m, sxi, factor):
    """Where the log-likelihood varies by well under a nat across a bin
    (sigma_xi = 40, half-pixel bins) the second-order value is over ten times
    closer to the members' mean; with a few nats of variation (sigma_xi = 10,
    quarter-pixel bins) it is still closer. Across whole pixels of a bright
    spot the expansion does not hold, which the design notes state."""
    w, tr, fr = scene
    st = synth.random_cloud(w, tr[1, 0], 20000, 1.2, seed=7)
    e1, e2 = _errors(orc, fr[1], st, m, sxi)
    assert e1.size >= 50
    assert e2.mean() < factor * e1.mean(), (e1.mean(), e2.mean())
    assert np.median(e2) < np.median(e1)
