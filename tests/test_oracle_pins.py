"""Pins of the FP64 oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: the
generator's published known-answer vectors, exact rational arithmetic, closed forms (Poisson
summation of Gaussian sums, constant frames), brute force on small inputs at 50
digits, invariants stated by the paper (one particle per cell recovers SIR,
Sec. 4.2; all members of a bin share the dummy's weight, Alg. pcSIR), and the
midpoint-rule error of the Appendix.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import synth

# --------------------------------------------------------------------------- RNG


# Known-answer vectors published with the generator (Salmon et al., SC'11,
# Random123 distribution) for Philox4x32 with 10 rounds: (counter, key, output).
PHILOX4X32_10_KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX4X32_10_KAT)
def test_philox_known_answers(orc, ctr, key, want):
    assert [int(v) for v in orc.philox(ctr, key)] == list(want)


def test_uniform_open_interval_and_exact_in_binary32(orc):
    for wd in (0, 1, 2**9 - 1, 2**9, 2**31, 2**32 - 1, 0x01234567, 0xFFFFFE00, 0x1FF):
        u = orc.uniform(wd)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # 24 significant bits at most
        assert u == float(Fraction(2 * (wd >> 9) + 1, 2**24))


def test_box_muller_invariant_and_moments(orc):
    seed = 77
    # invariant of the Box-Muller map: z0^2 + z1^2 = -2 ln u1 for each pair,
    # and atan2(z1, z0) = 2 pi u2 (mod 2 pi)
    for i in range(50):
        z = orc.normals(seed, i, 3, 1)
        words = np.concatenate([orc.philox((i, 3, 1, 0), (seed, 0)), orc.philox((i, 3, 1, 1), (seed, 0))])
        for p in range(4):
            u1 = orc.uniform(int(words[2 * p]))
            u2 = orc.uniform(int(words[2 * p + 1]))
            assert z[2 * p] ** 2 + z[2 * p + 1] ** 2 == pytest.approx(-2.0 * math.log(u1), rel=1e-12)
            ang = math.atan2(z[2 * p + 1], z[2 * p]) % (2 * math.pi)
            assert min(abs(ang - 2 * math.pi * u2), 2 * math.pi - abs(ang - 2 * math.pi * u2)) < 1e-9
    # moments over many draws: every slot is N(0, 1) and slots are uncorrelated
    Z = np.array([orc.normals(seed, i, 1, 0) for i in range(40000)])
    n = Z.shape[0]
    assert np.all(np.abs(Z.mean(0)) < 5 / math.sqrt(n))
    assert np.all(np.abs(Z.var(0) - 1) < 5 * math.sqrt(2 / n))
    cc = np.corrcoef(Z.T)
    assert np.all(np.abs(cc[np.triu_indices(8, 1)]) < 5 / math.sqrt(n))


# --------------------------------------------------------------------------- keys


def _exact_key(x: np.float32, m: int) -> int:
    xf = float(x)
    if math.isnan(xf):
        xf = 2.0**24
    xf = min(max(xf, -2.0**24), 2.0**24)
    k = math.floor((Fraction(xf) + Fraction(1, 2)) * m)
    return max(-(2**30), min(2**30, k))


def _adversarial(m: int, hi: float) -> np.ndarray:
    vals = [0.0, -0.0, 2.0**-149, -(2.0**-149), 2.0**-60, -(2.0**-60), 2.0**-30, -(2.0**-30),
            2.0**-31, -(2.0**-31), 2.0**-20, -(2.0**-20), 1e30, -1e30, 2.0**24, -(2.0**24), 3e7, -3e7]
    edges = [j / m - 0.5 for j in range(-3 * m, 3 * m + 1)]
    edges += [j / m - 0.5 for j in np.linspace(hi * m - 3 * m, hi * m + 3, 40).round()]
    out = []
    for e in edges:
        f = np.float32(e)
        out.append(f)
        a, b = f, f
        for _ in range(3):
            a = np.nextafter(a, np.float32(np.inf))
            b = np.nextafter(b, np.float32(-np.inf))
            out += [a, b]
    return np.array(vals + out, dtype=np.float32)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 10, 20, 64, 4096])
def test_bin_key_is_exact_floor(orc, m):
    xs = _adversarial(m, 1024.0)
    rng = np.random.default_rng(m)
    xs = np.concatenate([xs, rng.uniform(-1030, 1030, 3000).astype(np.float32)])
    got = orc.bin_key(xs, m)
    want = np.array([_exact_key(x, m) for x in xs])
    assert np.array_equal(got, want)
    assert orc.bin_key(np.array([np.nan], np.float32), m)[0] == _exact_key(np.float32(np.nan), m)


def test_pixels_are_unions_of_cells(orc):
    rng = np.random.default_rng(1)
    xs = rng.uniform(-50, 600, 20000).astype(np.float32)
    px = orc.bin_key(xs, 1)
    for m in (2, 4, 10, 20):
        k = orc.bin_key(xs, m)
        assert np.array_equal(np.floor_divide(k, m), px)


# --------------------------------------------------------------------------- propagation


def test_propagate_zero_noise_is_exact_ncv(orc):
    w = synth.preset("tiny")
    mdl = orc.Model(proc_sigma=(0, 0, 0, 0, 0), seed=9)
    st = synth.random_cloud(w, np.array([20.3, 11.7, 1.25, -0.5, 50.0]), 500, 2.0, seed=2)
    out = orc.propagate(mdl, st, k=4)
    want = st.copy()
    want[0] = (st[0].astype(np.float64) + st[2].astype(np.float64)).astype(np.float32)
    want[1] = (st[1].astype(np.float64) + st[3].astype(np.float64)).astype(np.float32)
    assert np.array_equal(out, want)
    mdl3 = orc.Model(dim=3, proc_sigma=(0,) * 7, seed=9)
    w3 = synth.preset("3d-astig")
    st3 = synth.random_cloud(w3, np.array([5.0, 6.0, 0.5, 1.0, 2.0, -0.25, 40.0]), 100, 1.0, seed=3)
    out3 = orc.propagate(mdl3, st3, k=1)
    for a in range(3):
        assert np.array_equal(out3[a], (st3[a].astype(np.float64) + st3[3 + a]).astype(np.float32))
    assert np.array_equal(out3[3:], st3[3:])


def test_propagate_noise_moments_and_counter(orc):
    sig = (0.5, 0.7, 0.1, 0.2, 2.0)
    mdl = orc.Model(proc_sigma=sig, seed=11)
    n = 60000
    st = np.zeros((5, n), np.float32)
    st[2] = 1.0
    st[3] = -2.0
    st[4] = 30.0
    out = orc.propagate(mdl, st, k=5, t=2).astype(np.float64)
    resid = np.stack([out[0] - 1.0, out[1] + 2.0, out[2] - 1.0, out[3] + 2.0, out[4] - 30.0])
    for d in range(5):
        zd = resid[d] / sig[d]
        assert abs(zd.mean()) < 5 / math.sqrt(n)
        assert abs(zd.var() - 1) < 5 * math.sqrt(2 / n)
    # the noise of particle i at (k, t) is the Box-Muller normal of counter (i, k, t)
    for i in (0, 17, n - 1):
        z = orc.normals(11, i, 5, 2)
        assert out[4, i] == pytest.approx(float(np.float32(30.0 + 2.0 * z[4])), abs=0)
    out_other_t = orc.propagate(mdl, st, k=5, t=3).astype(np.float64)
    assert not np.array_equal(out, out_other_t)


# --------------------------------------------------------------------------- likelihood


def _mdl(**kw):
    import oracle
    base = dict(dim=2, m=(2, 2, 1), patch=11, quad=2, sigma_psf=1.5, i_bg=10.0, sigma_xi=10.0, seed=1)
    base.update(kw)
    return oracle.Model(**base)


def test_loglik_constant_frame_closed_form(orc):
    H = W = 64
    c = 3.0
    fr = np.full((H, W), 10.0 + c, np.float32)
    for P in (1, 9, 11, 15):
        mdl = _mdl(patch=P, sigma_xi=7.0)
        ll = orc.loglik(mdl, fr, 30, 31, 30.2, 30.9, 0.0, 0.0)
        assert ll == pytest.approx(-P * P * c * c / (2 * 49.0), rel=1e-14)
    # window partly outside: outside pixels read as background and add nothing
    mdl = _mdl(patch=11, sigma_xi=7.0)
    ll = orc.loglik(mdl, fr, 2, 62, 2.0, 62.0, 0.0, 0.0)
    inside = (2 + 5 + 1) * (1 + 5 + 1)  # cols 0..7, rows 57..63
    assert ll == pytest.approx(-inside * c * c / (2 * 49.0), rel=1e-14)


@pytest.mark.parametrize("q", [1, 2, 3, 8])
def test_loglik_linear_part_sums_to_gaussian_integral(orc, q):
    """sum_window mu = P^2 I_bg + I0 * 2 pi sigma^2 (Poisson summation; sub-sample
    grid of spacing 1/q), read from two constant frames through the quadratic."""
    H = W = 128
    P, s, I0, ibg, sxi = 31, 1.5, 40.0, 10.0, 10.0
    mdl = _mdl(patch=P, quad=q, sigma_psf=s, i_bg=ibg, sigma_xi=sxi)
    x, y = 63.3, 64.45
    l0 = orc.loglik(mdl, np.zeros((H, W), np.float32), 63, 64, x, y, 0.0, I0)
    cst = 5.0
    l1 = orc.loglik(mdl, np.full((H, W), cst, np.float32), 63, 64, x, y, 0.0, I0)
    sum_mu = (l1 - l0) * sxi * sxi / cst + P * P * cst / 2.0
    assert sum_mu == pytest.approx(P * P * ibg + I0 * 2 * math.pi * s * s, rel=1e-11)


def test_loglik_point_sampled_square_sum(orc):
    """q = 1 is Eq. object sampled at pixel centres; sum of its square over a
    large window is pi sigma_x sigma_y (Poisson summation)."""
    H = W = 128
    mdl = _mdl(patch=41, quad=1, sigma_psf=1.7, i_bg=0.0, sigma_xi=1.0)
    ll = orc.loglik(mdl, np.zeros((H, W), np.float32), 60, 61, 60.37, 61.1, 0.0, 1.0)
    assert -2.0 * ll == pytest.approx(math.pi * 1.7 * 1.7, rel=1e-9)


@pytest.mark.parametrize("z", [-2.0, 0.0, 1.3])
def test_loglik_astigmatic_widths(orc, z):
    s0, g, d = 1.5, 2.0, 4.0
    mdl = _mdl(dim=3, psf=1, patch=61, quad=1, sigma_psf=s0, astig_gamma=g, astig_d=d, i_bg=0.0, sigma_xi=1.0)
    sx = s0 * math.sqrt(1 + ((z - g) / d) ** 2)
    sy = s0 * math.sqrt(1 + ((z + g) / d) ** 2)
    ll = orc.loglik(mdl, np.zeros((160, 160), np.float32), 80, 79, 80.2, 79.4, z, 1.0)
    assert -2.0 * ll == pytest.approx(math.pi * sx * sy, rel=1e-9)


def test_loglik_converges_to_pixel_average_closed_form(orc):
    """As q grows the model pixel value tends to the erf closed form of the
    pixel-averaged Gaussian, with the midpoint rule's O(q^-2) rate."""
    from scipy.special import erf
    H = W = 64
    s, I0 = 1.5, 50.0
    x, y = 30.27, 33.61
    P = 15

    def avg(c, p):
        a = s * math.sqrt(2.0)
        return s * math.sqrt(math.pi / 2.0) * (erf((c + 0.5 - p) / a) - erf((c - 0.5 - p) / a))

    cols = np.arange(30 - 7, 30 + 8)
    rows = np.arange(34 - 7, 34 + 8)
    mu = I0 * np.outer([avg(r, y) for r in rows], [avg(c, x) for c in cols])
    fr = np.zeros((H, W), np.float32)
    errs = []
    for q in (4, 8, 16, 32):
        mdl = _mdl(patch=P, quad=q, sigma_psf=s, i_bg=0.0, sigma_xi=1.0)
        ll = orc.loglik(mdl, fr, 30, 34, x, y, 0.0, I0)
        errs.append(abs(-2.0 * ll - float(np.sum(mu * mu))))
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5


def test_loglik_peaks_at_truth_not_transposed(orc):
    w = synth.preset("tiny", i_bg=10.0)
    tr = np.array([[21.3, 26.8, 0.0, 0.0, 50.0]])
    mu = synth.expected_image(w, tr, 48, 48).astype(np.float32)
    mdl = _mdl(patch=11, quad=16)
    best = orc.loglik(mdl, mu, 21, 27, 21.3, 26.8, 0.0, 50.0)
    assert abs(best) < 1e-3
    assert orc.loglik(mdl, mu, 27, 21, 26.8, 21.3, 0.0, 50.0) < best - 10
    assert orc.loglik(mdl, mu, 21, 27, 21.5, 26.8, 0.0, 50.0) < best
    assert orc.loglik(mdl, mu, 21, 27, 21.3, 26.8, 0.0, 45.0) < best


# --------------------------------------------------------------------------- weighting


@pytest.fixture(scope="module")
def scene():
    w = synth.preset("single-2d-64")
    tr = synth.truth(w)
    fr = synth.frames(w, tr)
    return w, tr, fr


def test_bins_partition_particles(orc, scene):
    w, tr, fr = scene
    cloud = synth.random_cloud(w, tr[1, 0], 5000, 0.8, seed=4)
    for m in (1, 2, 4, 20):
        r = orc.weigh(_mdl(m=(m, m, 1)), fr[0], cloud, sir=False)
        B = r["B"]
        assert int(r["bin_n"].sum()) == cloud.shape[1]
        # the bins are distinct cells in ascending (ky, kx) order
        kk = r["bin_key"][1].astype(np.int64) * 2**32 + r["bin_key"][0]
        assert np.all(np.diff(kk) > 0)
        # each particle lies in its bin's cell
        for a in range(2):
            k = r["bin_key"][a][r["bin_of"]]
            assert np.array_equal(k, r["keys"][a])
            x = cloud[a].astype(np.float64)
            assert np.all(x >= k / m - 0.5) and np.all(x < (k + 1) / m - 0.5)
        # segmented means: sum_b n_b xbar_b = sum_i x_i
        for d in range(5):
            assert np.sum(r["bin_n"] * r["bin_mean"][d]) == pytest.approx(np.sum(cloud[d].astype(np.float64)),
                                                                         rel=1e-12)
        assert B == len(set(zip(r["keys"][0], r["keys"][1])))


def test_weights_brute_force_50_digits(orc, scene):
    w, tr, fr = scene
    mpmath.mp.dps = 50
    cloud = synth.random_cloud(w, tr[1, 0], 48, 1.0, seed=8)
    for sir in (True, False):
        r = orc.weigh(_mdl(m=(2, 2, 1)), fr[0], cloud, sir=sir)
        lw = [mpmath.mpf(float(r["ll"][r["bin_of"][i]])) for i in range(48)]
        Z = mpmath.fsum(mpmath.exp(v) for v in lw)
        wx = [mpmath.exp(v) / Z for v in lw]
        for i in range(48):
            assert float(wx[i]) == pytest.approx(r["w"][i], rel=1e-13, abs=1e-300)
        neff = 1 / mpmath.fsum(v * v for v in wx)
        assert float(neff) == pytest.approx(r["neff"], rel=1e-13)
        for d in range(5):
            e = mpmath.fsum(wx[i] * mpmath.mpf(float(cloud[d, i])) for i in range(48))
            assert float(e) == pytest.approx(r["est"][d], rel=1e-13, abs=1e-13)


def test_weights_sum_to_one_and_shift_invariant(orc, scene):
    w, tr, fr = scene
    cloud = synth.random_cloud(w, tr[1, 0], 4000, 1.2, seed=9)
    for sir in (True, False):
        r = orc.weigh(_mdl(), fr[0], cloud, sir=sir)
        assert abs(r["w"].sum() - 1.0) < 1e-12
        r2 = orc.weigh(_mdl(), fr[0], cloud, sir=sir, logw_prev=np.full(4000, -123.25))
        np.testing.assert_allclose(r2["w"], r["w"], rtol=1e-12)
        # members of a bin share one weight (Alg. pcSIR, copy of the dummy's weight)
        if not sir:
            for b in range(r["B"]):
                ww = r["w"][r["bin_of"] == b]
                assert np.all(ww == ww[0])


def test_one_particle_per_cell_recovers_sir(orc, scene):
    """Sec. 4.2: with one particle per cell pcSIR is SIR (bit for bit here)."""
    w, tr, fr = scene
    cloud = synth.random_cloud(w, tr[1, 0], 3000, 3.0, seed=10)
    m = 4096
    pc = orc.weigh(_mdl(m=(m, m, 1)), fr[0], cloud, sir=False)
    assert pc["B"] == 3000 and pc["bin_n"].max() == 1
    si = orc.weigh(_mdl(m=(m, m, 1)), fr[0], cloud, sir=True)
    order = pc["bin_of"]
    assert np.array_equal(pc["ll"][order], si["ll"])
    assert np.array_equal(pc["w"], si["w"])
    assert np.array_equal(pc["est"], si["est"])
    u = orc.resample_u(1, 1, 0)
    assert np.array_equal(orc.resample(pc["w"], u)[1], orc.resample(si["w"], u)[1])


def test_all_in_one_bin_gives_uniform_weights(orc, scene):
    w, tr, fr = scene
    N = 2000
    rng = np.random.default_rng(3)
    cloud = synth.random_cloud(w, tr[1, 0], N, 1.0, seed=11)
    cloud[0] = np.float32(30.0) + rng.uniform(-0.49, 0.49, N).astype(np.float32)
    cloud[1] = np.float32(31.0) + rng.uniform(-0.49, 0.49, N).astype(np.float32)
    r = orc.weigh(_mdl(m=(1, 1, 1)), fr[0], cloud, sir=False)
    assert r["B"] == 1
    assert np.all(np.abs(r["w"] * N - 1.0) <= 4 * 2.0**-52)
    u = orc.resample_u(1, 2, 0)
    cdf, s = orc.resample(r["w"], u)
    theta = (np.arange(N) + u) / N
    near = np.abs(cdf - theta) < 1e-12
    assert np.all((s == np.arange(N)) | near)


# --------------------------------------------------------------------------- resampling


def test_systematic_resampling_definition_and_offspring(orc):
    rng = np.random.default_rng(5)
    for N in (1, 2, 7, 64, 1000):
        for trial in range(5):
            wts = rng.exponential(size=N) ** 3
            if N > 3 and trial == 2:
                wts[::3] = 0.0
            wts /= wts.sum()
            u = float(rng.uniform())
            cdf, s = orc.resample(wts, u)
            # the definition, brute force
            theta = (np.arange(N) + u) / N
            want = np.minimum(np.searchsorted(cdf, theta, side="right"), N - 1)
            assert np.array_equal(s, want)
            assert np.all(np.diff(s) >= 0)
            # zero-weight particles get no offspring; counts within one of N w_l
            cnt = np.bincount(s, minlength=N)
            assert np.all(cnt[wts == 0] == 0)
            assert np.all(np.abs(cnt - N * wts) < 1.0 + 1e-9)


def test_systematic_resampling_marginals(orc):
    rng = np.random.default_rng(6)
    N = 10
    wts = rng.uniform(size=N)
    wts /= wts.sum()
    R = 20000
    hits = np.zeros(N)
    for r in range(R):
        _, s = orc.resample(wts, float(rng.uniform()))
        hits += np.bincount(s, minlength=N)
    freq = hits / (R * N)
    assert np.all(np.abs(freq - wts) < 4 * np.sqrt(wts / (R * N)) + 1e-4)


def test_resample_and_check_uniform_counters(orc):
    seed = (7 << 32) | 31   # both key words in use
    blk = orc.philox((0, 4, 9, 2), (31, 7))
    assert orc.resample_u(seed, 4, 9) == float(Fraction(((int(blk[1]) << 32) | int(blk[0])) >> 11, 2**53))
    blk = orc.philox((12, 4, 9, 3), (31, 7))
    assert orc.check_u(seed, 12, 4, 9) == float(Fraction(((int(blk[1]) << 32) | int(blk[0])) >> 11, 2**53))
    # the frame index enters modulo 2^32
    assert orc.resample_u(seed, 4 + 2**32, 9) == orc.resample_u(seed, 4, 9)


# --------------------------------------------------------------------------- bin size


def test_error_shrinks_with_bin_size(orc, scene):
    """Finer cells bring pcSIR's estimate to SIR's; the centre of mass beats the
    cell centre (Sec. 5.5) and converges at second order (the mean cancels the
    linear Taylor term, first-order multipole)."""
    w, tr, fr = scene
    cloud = synth.random_cloud(w, tr[1, 0], 20000, 0.6, seed=5)
    cloud[4, :] = cloud[4, 0]  # intensity is not binned: hold it fixed to isolate the position error
    si = orc.weigh(_mdl(m=(1, 1, 1)), fr[0], cloud, sir=True)
    hs, com, coc = [1, 2, 4, 10, 20], [], []
    for m in hs:
        for mode, acc in ((0, com), (1, coc)):
            r = orc.weigh(_mdl(m=(m, m, 1), dummy_mode=mode), fr[0], cloud, sir=False)
            acc.append(np.abs(r["est"][:2] - si["est"][:2]).max())
    assert all(a > b for a, b in zip(com, com[1:]))
    assert all(a <= b for a, b in zip(com, coc))
    slope = math.log(com[2] / com[4]) / math.log(20 / 4)
    assert slope >= 1.5


def test_appendix_midpoint_error(orc):
    """Appendix: over a cell of sides (lx, ly) the integral of f - f(centre) is
    (lx^3 ly f_xx + lx ly^3 f_yy)/24 to higher order; the cell and its centre are
    the oracle's (bin_key and the CoC dummy)."""
    from scipy.integrate import dblquad
    f = lambda x, y: math.exp(-((x - 0.3) ** 2 + 0.5 * (y + 0.2) ** 2))
    fxx = lambda x, y: (4 * (x - 0.3) ** 2 - 2) * f(x, y)
    fyy = lambda x, y: ((y + 0.2) ** 2 - 1) * f(x, y)
    prev = None
    for m in (4, 8, 16):
        kx, ky = int(orc.bin_key([0.41], m)[0]), int(orc.bin_key([-0.13], m)[0])
        x0, x1 = kx / m - 0.5, (kx + 1) / m - 0.5
        y0, y1 = ky / m - 0.5, (ky + 1) / m - 0.5
        assert orc.bin_key([np.float32(x0)], m)[0] == kx and orc.bin_key([np.float32(x1)], m)[0] == kx + 1
        # CoC dummy of a one-particle bin sits at the cell centre
        cl = np.zeros((5, 1), np.float32)
        cl[0], cl[1], cl[4] = 0.41, -0.13, 1.0
        r = orc.weigh(_mdl(m=(m, m, 1), dummy_mode=1), np.zeros((8, 8), np.float32), cl, sir=False)
        a, b = r["bin_mean"][0, 0], r["bin_mean"][1, 0]
        assert a == pytest.approx((x0 + x1) / 2, abs=1e-15) and b == pytest.approx((y0 + y1) / 2, abs=1e-15)
        l = 1.0 / m
        err, _ = dblquad(lambda y, x: f(x, y) - f(a, b), x0, x1, y0, y1, epsabs=1e-15, epsrel=1e-13)
        pred = (l**3 * l * fxx(a, b) + l * l**3 * fyy(a, b)) / 24.0
        rel = abs(err - pred) / abs(pred)
        assert rel < 2.0 * l * l
        bound = (l**4 / 24.0) * (abs(fxx(a, b)) + abs(fyy(a, b)))
        assert abs(err) <= bound * (1 + 2 * l * l)
        if prev is not None:
            assert 12 < prev / abs(err) < 20  # fourth order in l
        prev = abs(err)


# --------------------------------------------------------------------------- tracking (parity unpinned)


def test_tracking_rmse_sanity(orc, scene):
    """Tracking RMSE is 'parity unpinned' (the paper's data are not available):
    both filters must track the synthetic spot to well under a pixel."""
    w, tr, fr = scene
    n = w.counts()
    st = synth.initial_particles(w, tr[0], n)
    mdl = _mdl(m=(2, 2, 1), proc_sigma=w.proc_sigma, seed=1500)
    for sir in (True, False):
        _, est, neff = orc.track(mdl, fr, n, st, k0=1, sir=sir)
        assert synth.rmse(est, tr, 2)[0] < 1.0
        assert np.all(neff >= 1.0) and np.all(neff <= n[0] * (1 + 1e-12))
