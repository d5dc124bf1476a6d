"""GPU parity of resampling with an N_eff threshold (kept weights) against the oracle.

Alg. SIR and Alg. pcSIR resample only when N_eff falls below a threshold; a
target that does not resample keeps its propagated particles and their
normalised log-weights, and each pcSIR dummy is then the centre of mass of its
members weighted by them (Sec. 4). Every frame is checked stage by stage: the
oracle weighs the GPU's propagated states with the log-weights the GPU carried
into that frame (so errors do not accumulate across frames), and the decision,
the weights, the kept log-weights and the resampling indices are compared.

Tolerances are those of the every-frame step (gpu_helpers); in addition:
  weighted bin means  FP64 sums of binary32 states in any order: positions
                      1e-7 px, velocities 1e-7, intensity 1e-6 (as the exact
                      fixed-point sums of the unweighted means)
  kept log-weights    the weight bound in the log domain, tol(l_i) + sum_j w_j
                      tol(l_j), everywhere
  decision            equal unless N_eff lies within 1e-5 (relative) of the
                      threshold
"""
import math

import numpy as np
import pytest

import synth
from gpu_helpers import exempt_mask, ll_tol, log, oracle_model, w_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_5541_amd import lib
    lib()


def _scene(dim=2):
    if dim == 2:
        counts = (3000, 257, 2049, 1)
        w = synth.preset("tiny", H=96, W=96, T=4, n=counts, m=(2, 2, 1), K=5, mid_lo=15.0, mid_hi=81.0,
                         i0=(40.0, 100.0))
        spreads = (0.4, 1.5, 3.0, 0.5)
        seed = 3
    else:
        counts = (2500, 1, 700)
        w = synth.preset("3d-astig", H=48, W=48, T=3, n=counts, K=4, m=(2, 2, 2))
        spreads = (0.6, 0.5, 1.5)
        seed = 4
    tr = synth.truth(w, seed=seed)
    fr = synth.frames(w, tr, seed=seed)
    cloud = np.ascontiguousarray(np.concatenate(
        [synth.random_cloud(w, tr[0, t], counts[t], spreads[t], 20 + t) for t in range(len(counts))], axis=1))
    return w, fr, cloud


def _frame(cfg, fr, k, t):
    f = fr[k - 1]
    return f[t] if cfg.per_target_frames else f


def _run(cfg, fr, cloud, K, sir, lik_check=True):
    """Runs K frames on the GPU and checks each against the oracle; returns
    the per-frame decisions [K][T] (True: resampled)."""
    import torch

    import oracle
    from paper_1310_5541_amd import Filter

    T, dim = cfg.T, cfg.dim
    n = np.asarray(cfg.n_particles, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(n)])
    thr = cfg.neff_threshold
    mdl = oracle_model(cfg)
    f = Filter(cfg, torch.from_numpy(cloud).cuda())
    fr_d = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
    decisions = []
    try:
        lw_in = None
        for k in range(1, K + 1):
            start = f.get_particles().cpu().numpy()
            f.step(fr_d[k - 1], k, sir=sir)
            est, neff = f.estimate()
            prop = f.dump("propagated").cpu().numpy()
            ll_gpu = f.dump("loglik").cpu().numpy()
            w_gpu = f.dump("weights").cpu().numpy()
            tgt = f.dump("target").cpu().numpy()
            s_gpu = f.dump("resample").cpu().numpy().astype(np.int64)
            lw_out = f.dump("logw").cpu().numpy()
            if not sir:
                b_n = f.dump("bin_n").cpu().numpy()
                b_mean = f.dump("bin_mean").cpu().numpy()
            after = f.get_particles().cpu().numpy()
            row = []
            bofs = 0
            for t in range(T):
                a, b = off[t], off[t + 1]
                N = b - a
                fr_t = _frame(cfg, fr, k, t)
                op = oracle.propagate(mdl, start[:, a:b], k, t)
                err = np.abs(prop[:, a:b].astype(np.float64) - op)
                assert np.all(err <= 1e-6 * np.abs(op) + 2e-6), f"k={k} t={t}: propagate"
                prev = None
                if lw_in is not None and not np.all(lw_in[a:b] == -math.log(N)):
                    prev = lw_in[a:b]
                r = oracle.weigh(mdl, fr_t, prop[:, a:b], sir=sir, logw_prev=prev)
                B = r["B"]
                if sir:
                    ll_g, ll_o = ll_gpu[a:b], r["ll"]
                else:
                    gsl = slice(bofs, bofs + B)
                    assert np.array_equal(b_n[gsl], r["bin_n"]), f"k={k} t={t}: bin counts"
                    gm, om = b_mean[:, gsl], r["bin_mean"]
                    assert np.abs(gm[:dim] - om[:dim]).max() <= 1e-7, f"k={k} t={t}: dummy positions"
                    assert np.abs(gm[dim:2 * dim] - om[dim:2 * dim]).max() <= 1e-7, f"k={k} t={t}: velocities"
                    assert np.abs(gm[2 * dim] - om[2 * dim]).max() <= 1e-6, f"k={k} t={t}: intensity"
                    ll_g, ll_o = ll_gpu[gsl], r["ll"]
                    bofs += B
                if lik_check:
                    d_ll = np.abs(ll_g - ll_o)
                    assert np.all(d_ll <= ll_tol(cfg, sir, ll_o)), f"k={k} t={t}: ll off {d_ll.max()}"
                wg, wo = w_gpu[a:b], r["w"]
                bound = w_bound(cfg, sir, r["ll"][r["bin_of"]], wo)
                assert np.all(np.abs(wg - wo) <= bound), f"k={k} t={t}: weights"
                e_est = np.abs(est[t] - r["est"]) / np.maximum(np.abs(r["est"]), 1.0)
                assert np.all(e_est <= 1e-5), f"k={k} t={t}: estimate off {e_est.max()}"
                assert abs(neff[t] - r["neff"]) <= 1e-5 * r["neff"], f"k={k} t={t}: N_eff"
                u = oracle.resample_u(cfg.seed, k, t)
                assert tgt[t, 3] == u
                # the GPU resampled a target iff it carries uniform log-weights
                # into the next frame (one particle: N_eff = N, never below)
                want = bool(r["neff"] < thr * N)
                got = N > 1 and bool(np.all(lw_out[a:b] == -math.log(N)))
                if abs(r["neff"] - thr * N) > 1e-5 * r["neff"]:
                    assert got == want, f"k={k} t={t}: decision (N_eff {r['neff']}, threshold {thr * N})"
                row.append(got)
                sg = s_gpu[a:b]
                if got:
                    theta = (np.arange(N, dtype=np.float64) + u) / N
                    cdf_o, s_o = oracle.resample(wo, u)
                    diff = sg != s_o
                    ex = exempt_mask(cdf_o, s_o, theta, 1e-6)
                    assert not np.any(diff & ~ex), f"k={k} t={t}: resampling indices"
                    assert np.all(lw_out[a:b] == -math.log(N))
                    assert np.array_equal(after[:, a:b], prop[:, a:b][:, sg])
                else:
                    assert np.array_equal(sg, np.arange(N)), f"k={k} t={t}: kept target was resampled"
                    assert np.array_equal(after[:, a:b], prop[:, a:b])
                    lg = lw_out[a:b]
                    lo = (0.0 if prev is None else prev) + r["ll"][r["bin_of"]] - (r["M"] + math.log(r["S"]))
                    assert np.all(np.isfinite(lg))
                    assert np.all(np.abs(np.exp(lg) - wo) <= bound), f"k={k} t={t}: kept weights"
                    tl = ll_tol(cfg, sir, r["ll"][r["bin_of"]])
                    lbound = 1.01 * (tl + np.sum(wo * tl)) + 1e-9
                    assert np.all(np.abs(lg - lo) <= lbound), f"k={k} t={t}: kept log-weights"
            decisions.append(row)
            lw_in = lw_out
    finally:
        f.close()
    return decisions


def _cfg(w, **kw):
    from paper_1310_5541_amd import Config
    return Config.from_workload(w, **kw)


@pytest.mark.parametrize("sir", [False, True])
def test_never_resampling_keeps_weights(sir):
    """Threshold 0: no target ever resamples; weights accumulate over five
    frames until most of them underflow binary64 (the log-weights stay finite)."""
    w, fr, cloud = _scene()
    cfg = _cfg(w, seed=5, lik_mode=1, neff_threshold=0.0)
    log(f"case never_resampling sir={sir}")
    dec = _run(cfg, fr, cloud, 5, sir)
    assert not any(any(r) for r in dec)


@pytest.mark.parametrize("sir", [False, True])
def test_threshold_mixes_kept_and_resampled_targets(sir):
    """A threshold of 2% of N: per frame, some targets resample and others keep
    their weights, so kept and uniform targets share every launch."""
    w, fr, cloud = _scene()
    cfg = _cfg(w, seed=5, lik_mode=1, neff_threshold=0.02)
    log(f"case threshold_mix sir={sir}")
    dec = _run(cfg, fr, cloud, 5, sir)
    flat = [d for r in dec for d in r]
    assert any(flat) and not all(flat), dec
    log(f"  decisions {dec}")


def test_threshold_3d_direct():
    w, fr, cloud = _scene(dim=3)
    cfg = _cfg(w, seed=19, lik_mode=0, quad=4, neff_threshold=0.05)
    log("case threshold_3d")
    _run(cfg, fr, cloud, 4, False)


def test_threshold_one_resamples_like_every_frame():
    """Threshold 1 with many particles per target: every target resamples
    (N_eff < N), through the per-particle normalisation of the kept-weight
    mode; the checks are those of the every-frame step."""
    w, fr, cloud = _scene()
    resamples = np.asarray(w.counts()) > 1   # one particle: N_eff = N
    cfg = _cfg(w, seed=7, lik_mode=1, neff_threshold=1.0)
    log("case threshold_one")
    dec = _run(cfg, fr, cloud, 2, False)
    assert all(d == bool(x) for r in dec for d, x in zip(r, resamples))


def test_set_particles_resets_to_uniform_weights():
    """After set_particles a step weighs as from uniform weights: bit for bit
    the step of a fresh context started from the same particles."""
    import torch

    from paper_1310_5541_amd import Filter
    w, fr, cloud = _scene()
    cfg = _cfg(w, seed=5, lik_mode=1, neff_threshold=0.0)
    fr_d = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
    log("case set_particles_resets")
    a = Filter(cfg, torch.from_numpy(cloud).cuda())
    a.step(fr_d[0], 1)
    a.step(fr_d[1], 2)
    mid = a.get_particles().clone()
    a.set_particles(mid)
    a.step(fr_d[2], 3)
    ea, na = a.estimate()
    wa, la = a.dump("weights").cpu().numpy(), a.dump("logw").cpu().numpy()
    a.close()
    b = Filter(cfg, mid)
    b.step(fr_d[2], 3)
    eb, nb = b.estimate()
    wb, lb = b.dump("weights").cpu().numpy(), b.dump("logw").cpu().numpy()
    b.close()
    assert np.array_equal(ea, eb) and np.array_equal(na, nb)
    assert np.array_equal(wa, wb) and np.array_equal(la, lb)


def test_default_carries_uniform_log_weights():
    import torch

    from paper_1310_5541_amd import Filter
    w, fr, cloud = _scene()
    cfg = _cfg(w, seed=5, lik_mode=1)
    assert math.isinf(cfg.neff_threshold)
    f = Filter(cfg, torch.from_numpy(cloud).cuda())
    f.step(torch.from_numpy(fr[0]).cuda(), 1)
    lw = f.dump("logw").cpu().numpy()
    f.close()
    n = np.asarray(w.counts())
    assert np.array_equal(lw, np.repeat(-np.log(n.astype(np.float64)), n))
