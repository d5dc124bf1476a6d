"""Sec. 5.5's pseudo-tracking experiment on the oracle (CPU only).

The reference, the exact posterior mean under a fixed prior, is pinned by:
- a flat frame (the likelihood is constant): the prior's own mean;
- a noise-free object at a pixel centre with the prior centred there: the
  pixel centre, by the mirror symmetry of the likelihood about it;
- halving the quadrature cell: a change below 2e-5 px (second order);
- a Monte-Carlo estimate with 4e5 prior draws: within 4 standard errors.
Then the experiment itself, at small sizes: the estimators' RMSE against that
reference falls as N^(-1/2) for SIR, pcSIR-CoM and pcSIR-CoC, and pcSIR stays
within 15% of SIR at every N.
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


def _mdl(orc, m=1, dummy=0):
    w = synth.pseudo_workload(1, 1, m)
    return orc.Model(dim=2, m=(m, m, 1), patch=w.patch, quad=w.quad, sigma_psf=w.sigma_psf, i_bg=w.i_bg,
                     sigma_xi=w.sigma_xi, proc_sigma=tuple(w.proc_sigma), seed=1, dummy_mode=dummy)


@pytest.mark.parametrize("kind,par", synth.PSEUDO_PRIORS)
def test_flat_frame_gives_the_prior_mean(orc, kind, par):
    fr = np.full((32, 32), 10.0, np.float32)
    c = np.array([14.63, 15.21])
    got = orc.posterior_mean(_mdl(orc), fr, kind, par, c, 0.0)
    np.testing.assert_allclose(got, c, atol=1e-9)


@pytest.mark.parametrize("kind,par", [("uniform", 3.0), ("gauss", 0.5)])
def test_symmetric_object_gives_the_pixel_centre(orc, kind, par):
    w = synth.pseudo_workload(1, 1)
    fr = synth.expected_image(w, np.array([[15.0, 15.0, 0.0, 0.0, w.i0[0]]]), 32, 32).astype(np.float32)
    got = orc.posterior_mean(_mdl(orc), fr, kind, par, (15.0, 15.0), w.i0[0])
    np.testing.assert_allclose(got, [15.0, 15.0], atol=1e-10)


def test_quadrature_refinement_and_monte_carlo(orc):
    w = synth.pseudo_workload(1, 1)
    fr, xy = synth.pseudo_frame()
    mdl = _mdl(orc)
    for kind, par in (("uniform", 3.0), ("gauss", 0.8)):
        a = orc.posterior_mean(mdl, fr, kind, par, xy, w.i0[0])
        b = orc.posterior_mean(mdl, fr, kind, par, xy, w.i0[0], delta=1.0 / 64)
        assert np.abs(a - b).max() < 2e-5
        st = synth.pseudo_particles(kind, par, xy, 1, 400_000, seed=5)
        r = orc.weigh(mdl, fr, st, sir=True)
        wts = r["w"]
        pos = st[:2].astype(np.float64)
        # standard error of a self-normalised importance estimate
        se = np.sqrt(np.sum(wts ** 2 * (pos - r["est"][:2, None]) ** 2, axis=1))
        assert np.all(np.abs(r["est"][:2] - a) <= 4 * se), (r["est"][:2], a, se)


def test_convergence_rate_small(orc):
    w = synth.pseudo_workload(1, 1)
    fr, xy = synth.pseudo_frame()
    kind, par = "uniform", 3.0
    ref = orc.posterior_mean(_mdl(orc), fr, kind, par, xy, w.i0[0])
    models = {"sir": (_mdl(orc), True), "com": (_mdl(orc, 1, 0), False), "coc": (_mdl(orc, 1, 1), False)}
    Ns = (100, 400, 1600)
    reps = 100
    rmse = {k: [] for k in models}
    for N in Ns:
        st = synth.pseudo_particles(kind, par, xy, reps, N, seed=100 + N)
        err = {k: [] for k in models}
        for r in range(reps):
            s = st[:, r * N:(r + 1) * N]
            for k, (mdl, sir) in models.items():
                err[k].append(orc.weigh(mdl, fr, s, sir=sir)["est"][:2] - ref)
        for k in models:
            rmse[k].append(math.sqrt(np.mean(np.sum(np.square(err[k]), axis=1))))
    for k in models:
        slope = np.polyfit(np.log(Ns), np.log(rmse[k]), 1)[0]
        assert -0.65 <= slope <= -0.35, (k, slope, rmse[k])
    for i in range(len(Ns)):
        for k in ("com", "coc"):
            assert abs(rmse[k][i] / rmse["sir"][i] - 1.0) <= 0.15, (k, Ns[i], rmse)
