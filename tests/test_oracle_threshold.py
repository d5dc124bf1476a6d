"""Pins of the oracle's resampling threshold and weighted dummies (CPU only).

Alg. SIR and Alg. pcSIR resample only when N_eff falls below a threshold; in
between, particles carry their normalised weights, and the pcSIR dummy is the
centre of mass of its members weighted by them (Sec. 4). Pinned here:
- an infinite threshold is the every-frame step, bit for bit;
- a zero threshold never resamples, so SIR accumulates the sequential
  importance-sampling weights, checked against per-particle likelihoods
  computed one by one over the frames (an independent route);
- the weighted dummy: equal weights give the plain mean bit for bit, one
  dominant weight gives that particle, and any weights give a convex
  combination of the members;
- the decision follows N_eff < fraction * N, and a target that does not
  resample keeps its propagated particles and log w_i.
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


def _mdl(**kw):
    import oracle
    base = dict(dim=2, m=(2, 2, 1), patch=11, quad=2, sigma_psf=1.5, i_bg=10.0, sigma_xi=10.0, seed=4,
                proc_sigma=(0.5, 0.5, 0.1, 0.1, 2.0))
    base.update(kw)
    return oracle.Model(**base)


@pytest.fixture(scope="module")
def scene():
    w = synth.preset("single-2d-64", K=5)
    tr = synth.truth(w)
    fr = synth.frames(w, tr)
    cloud = synth.random_cloud(w, tr[0, 0], 1500, 0.8, seed=8)
    return w, tr, fr, cloud


@pytest.mark.parametrize("sir", [False, True])
def test_infinite_threshold_is_the_every_frame_step(orc, scene, sir):
    w, tr, fr, cloud = scene
    mdl = _mdl()
    a = cloud.copy()
    b, lw, uni = cloud.copy(), None, True
    for k in range(1, 5):
        a, est_a, neff_a = orc.step(mdl, fr[k], a, k, 0, sir)
        b, lw, uni, est_b, neff_b, res = orc.step_thr(mdl, fr[k], b, lw, uni, k, 0, sir, float("inf"))
        assert res and uni
        assert np.array_equal(a, b) and np.array_equal(est_a, est_b) and neff_a == neff_b


def test_never_resampling_accumulates_sis_weights(orc, scene):
    """SIR with threshold 0: log w_K(i) = sum_k l_k(x_i^k) - logsumexp(.)."""
    w, tr, fr, cloud = scene
    mdl = _mdl()
    x = cloud[:, :300].copy()
    lw, uni = None, True
    ref_x = x.copy()
    acc = np.zeros(x.shape[1])
    for k in range(1, 4):
        x, lw, uni, est, neff, res = orc.step_thr(mdl, fr[k], x, lw, uni, k, 0, True, 0.0)
        assert not res and not uni
        ref_x = orc.propagate(mdl, ref_x, k, 0).astype(np.float32)
        assert np.array_equal(x, ref_x)   # never resampled: the particles only move
        for i in range(x.shape[1]):
            c0 = int(orc.bin_key(ref_x[0, i], 1)[0])
            r0 = int(orc.bin_key(ref_x[1, i], 1)[0])
            acc[i] += orc.loglik(mdl, fr[k], c0, r0, float(ref_x[0, i]), float(ref_x[1, i]), 0.0,
                                 float(ref_x[4, i]))
    mx = acc.max()
    expect = acc - (mx + math.log(np.exp(acc - mx).sum()))
    np.testing.assert_allclose(lw, expect, rtol=1e-12, atol=1e-9)


def test_weighted_dummy(orc):
    mdl = _mdl(m=(1, 1, 1))
    fr = np.full((48, 48), 10.0, np.float32)
    st = np.zeros((5, 6), np.float32)
    st[0] = [10.1, 10.2, 10.3, 20.1, 20.2, 20.4]
    st[1] = [30.0, 30.1, 29.8, 30.2, 30.0, 29.9]
    st[2] = [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    st[3] = [0.5, 0.4, 0.3, 0.2, 0.1, 0.0]
    st[4] = [40.0, 50.0, 60.0, 70.0, 80.0, 90.0]
    plain = orc.weigh(mdl, fr, st, sir=False)
    same = orc.weigh(mdl, fr, st, sir=False, logw_prev=np.full(6, -3.75))
    assert plain["B"] == 2 and np.array_equal(plain["bin_mean"], same["bin_mean"])
    # one dominant weight in the first bin: its dummy is that particle
    dom = orc.weigh(mdl, fr, st, sir=False, logw_prev=np.array([0.0, -1e3, -1e3, -2.0, -2.0, -2.0]))
    np.testing.assert_array_equal(dom["bin_mean"][:, 0], st[:, 0].astype(np.float64))
    np.testing.assert_allclose(dom["bin_mean"][:, 1], st[:, 3:].astype(np.float64).mean(axis=1), rtol=1e-15)
    # any weights: a convex combination of the members, component by component
    rng = np.random.default_rng(2)
    for _ in range(20):
        lp = rng.normal(0.0, 3.0, 6)
        r = orc.weigh(mdl, fr, st, sir=False, logw_prev=lp)
        for b, mem in enumerate((slice(0, 3), slice(3, 6))):
            lo = st[:, mem].min(axis=1) - 1e-12
            hi = st[:, mem].max(axis=1) + 1e-12
            assert np.all(r["bin_mean"][:, b] >= lo) and np.all(r["bin_mean"][:, b] <= hi)


@pytest.mark.parametrize("sir", [False, True])
def test_threshold_decision_and_kept_weights(orc, scene, sir):
    w, tr, fr, cloud = scene
    mdl = _mdl()
    N = cloud.shape[1]
    # N_eff of frame 1 from the same step with an infinite threshold
    _, _, _, _, neff, _ = orc.step_thr(mdl, fr[1], cloud, None, True, 1, 0, sir, float("inf"))
    frac = neff / N
    above = orc.step_thr(mdl, fr[1], cloud, None, True, 1, 0, sir, frac * (1 + 1e-9))
    below = orc.step_thr(mdl, fr[1], cloud, None, True, 1, 0, sir, frac * (1 - 1e-9))
    assert above[5] and above[2]
    assert not below[5] and not below[2]
    prop = orc.propagate(mdl, cloud, 1, 0).astype(np.float32)
    assert np.array_equal(below[0], prop)
    r = orc.weigh(mdl, fr[1], prop, sir=sir)
    np.testing.assert_array_equal(below[1], r["ll"][r["bin_of"]] - (r["M"] + math.log(r["S"])))
    np.testing.assert_allclose(np.exp(below[1]), r["w"], rtol=1e-13, atol=0)
    assert abs(np.exp(below[1]).sum() - 1.0) < 1e-12


def test_kept_log_weights_stay_finite_where_weights_underflow(orc, scene):
    """pcSIR without resampling over several frames: normalised weights fall
    below the smallest binary64 value (exp underflows to 0), yet the kept
    log-weights stay finite and equal the running sum of each particle's
    dummy log-likelihoods minus its log-sum-exp, recomputed here frame by
    frame from the dummies the oracle reports; every N_eff stays finite."""
    w = synth.preset("tiny", H=96, W=96, T=1, n=(1500,), K=5, i0=(40.0, 100.0))
    tr = synth.truth(w, seed=3)
    fr = np.concatenate([np.zeros((1, 96, 96), np.float32), synth.frames(w, tr, seed=3)])  # fr[k]: frame k
    mdl = _mdl()
    x, lw, uni = synth.random_cloud(w, tr[0, 0], 1500, 3.0, seed=22), None, True
    acc = np.zeros(x.shape[1])
    for k in range(1, 6):
        prev = None if uni else lw.copy()
        x, lw, uni, est, neff, res = orc.step_thr(mdl, fr[k], x, lw, uni, k, 0, False, 0.0)
        assert not res and np.isfinite(neff) and np.all(np.isfinite(lw))
        r = orc.weigh(mdl, fr[k], x, sir=False, logw_prev=prev)
        acc += r["ll"][r["bin_of"]]
        mx = acc.max()
        np.testing.assert_allclose(lw, acc - (mx + math.log(np.exp(acc - mx).sum())), rtol=1e-12, atol=1e-9)
    assert lw.min() < -746.0   # the weights themselves underflow
