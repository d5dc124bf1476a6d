"""Stage-wise parity of one GPU filter step against the FP64 oracle.

The GPU and the oracle share no code. Propagation is compared on the same
parent states and counters; every later stage is compared by running the
oracle on the GPU's propagated (binary32) states, so that keys, counts and
resampling indices can be required bit-exact.

Tolerances (derived in the design notes from the FP32 arithmetic of the path):
  propagate      |d| <= 1e-6 * |x| + 2e-6
  keys, bins     bit-exact (keys, counts, bin order, targets)
  bin means      positions 1e-7 px, velocities 1e-7, intensity 1e-6
  log-likelihood separable form (model image in FP32 pairs; also the surrogate's exact
                 check and fallback, and SIR in those modes): |d| <= 2e-6 + 1e-9 |l|.
                 Per-sub-sample form (one FP32 word per model value):
                 |d| <= 5e-6 + 3e-7 |l|; the rounding of each model value (6e-8 of
                 it) times residuals of tens of counts gives errors that grow with
                 the window's sum of squares S = -2 sigma_xi^2 l.
  weights        separable form: |dw_i| <= 1e-5 w_i + 1e-10 max w (relative 1e-5,
                 with a floor for weights that are negligible next to the largest).
                 Per-sub-sample form: inherited from its l bound, w_i = exp(l_i - M) / S,
                 so to first order dw_i / w_i = dl_i - sum_j w_j dl_j and
                 |dw_i| <= 1.01 (tol(l_i) + sum_j w_j tol(l_j)) w_i + 1e-12 max w
  estimates      rel 1e-5 (abs 1e-5); N_eff rel 1e-5
  resampling u   bit-exact
  s(j)           bit-exact except where the oracle's cumulative weight lies
                 within 1e-6 of theta_j; and, from the GPU's own weights,
                 bit-exact except within 1e-9.
"""
from __future__ import annotations

import dataclasses
import math
import sys

import numpy as np

LL_ATOL = 5e-6          # per-sub-sample form
LL_RTOL = 3e-7
LL_SEP_ATOL = 2e-6      # separable form (pairs)
LL_SEP_RTOL = 1e-9
W_RTOL = 1e-5           # weights, separable form: 1e-5 w + 1e-10 max w
W_FLOOR = 1e-10


def pair_form(cfg, sir):
    """True when the step's exact log-likelihoods come from the separable pair form."""
    return cfg.lik_mode != 0


def ll_tol(cfg, sir, ll):
    ll = np.abs(np.asarray(ll, dtype=np.float64))
    if pair_form(cfg, sir):
        return LL_SEP_ATOL + LL_SEP_RTOL * ll
    return LL_ATOL + LL_RTOL * ll


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_model(cfg, seed=None):
    import oracle
    return oracle.Model(dim=cfg.dim, m=tuple(cfg.bins_per_px), patch=cfg.patch, quad=cfg.quad, psf=cfg.psf,
                        dummy_mode=cfg.dummy_mode, sigma_psf=cfg.sigma_psf, astig_gamma=cfg.astig_gamma,
                        astig_d=cfg.astig_d, i_bg=cfg.i_bg, sigma_xi=cfg.sigma_xi,
                        proc_sigma=tuple(cfg.proc_sigma), seed=cfg.seed if seed is None else seed)


def exempt_mask(cdf, s, theta, eps):
    """j whose threshold lies within eps of a cumulative weight bracketing it."""
    N = cdf.shape[0]
    hi = cdf[s]
    lo = np.where(s > 0, cdf[np.maximum(s - 1, 0)], 0.0)
    return (np.abs(hi - theta) <= eps) | (np.abs(lo - theta) <= eps)


def weight_bound(ll_of_particle, wo, tl=None):
    """Largest |w_gpu - w_oracle| per particle that the log-likelihood tolerance
    (tl per particle; by default that of the log-likelihood row) allows."""
    if tl is None:
        tl = LL_ATOL + LL_RTOL * np.abs(ll_of_particle)
    return 1.01 * (tl + np.sum(wo * tl)) * wo + 1e-12 * wo.max()


def w_bound(cfg, sir, ll_of_particle, wo):
    """Largest |w_gpu - w_oracle| per particle for the step's likelihood form."""
    if pair_form(cfg, sir):
        return W_RTOL * wo + W_FLOOR * wo.max()
    return weight_bound(ll_of_particle, wo)


def run_step_parity(cfg, cloud, frames, k, sir, check_prop=True, report=None, surrogate=None, on_filter=None,
                    targets=None, tuning=None):
    """cloud: [D, NT] float32 (host); frames: [H, W] or [T, H, W] float32 (host).
    Runs one GPU step from `cloud` and checks every stage against the oracle.
    surrogate: (params, act_scale, check_fraction, tol) installed before the step
    (a surrogate lik_mode); on_filter(f) runs after the dumps, before close.
    targets: the targets to check (all by default); tuning: launch shapes.
    Returns a dict of the largest deviations."""
    import torch

    import oracle
    from paper_1310_5541_amd import Filter

    T, D, dim = cfg.T, cfg.D, cfg.dim
    n = np.asarray(cfg.n_particles, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(n)])
    mdl = oracle_model(cfg)
    f = Filter(cfg, torch.from_numpy(np.ascontiguousarray(cloud)).cuda())
    f.set_debug(True)
    if tuning is not None:
        f.set_tuning(**tuning)
    if surrogate is not None:
        f.set_surrogate(*surrogate)
    fr_t = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    f.step(fr_t, k, sir=sir)
    est, neff = f.estimate()
    prop = f.dump("propagated").cpu().numpy()
    keys = f.dump("keys").cpu().numpy()
    ll_gpu = f.dump("loglik").cpu().numpy()
    w_gpu = f.dump("weights").cpu().numpy()
    tgt = f.dump("target").cpu().numpy()
    cdf_gpu = f.dump("cdf").cpu().numpy()
    s_gpu = f.dump("resample").cpu().numpy().astype(np.int64)
    if not sir:
        m_gpu = f.dump("bins_per_px").cpu().numpy()
        counts = f.dump("counts").cpu().numpy()
        b_t = f.dump("bin_target").cpu().numpy()
        b_key = f.dump("bin_key").cpu().numpy()
        b_n = f.dump("bin_n").cpu().numpy()
        b_mean = f.dump("bin_mean").cpu().numpy()
    after = f.get_particles().cpu().numpy()
    if on_filter is not None:
        on_filter(f)
    f.close()

    dev = dict(prop=0.0, mean_pos=0.0, mean_vel=0.0, mean_int=0.0, ll=0.0, w=0.0, est=0.0, neff=0.0,
               exempt=0, mismatch=0, B=0)
    check = range(T) if targets is None else sorted(set(int(t) for t in targets))
    if not sir:
        # bins are ordered by target: each target's first bin
        bfirst = np.searchsorted(b_t, np.arange(T + 1), side="left")
        assert np.all(np.diff(b_t) >= 0), "bins not ordered by target"
    for t in check:
        a, b = off[t], off[t + 1]
        fr = frames[t] if cfg.per_target_frames else frames
        if check_prop:
            op = oracle.propagate(mdl, cloud[:, a:b], k, t)
            err = np.abs(prop[:, a:b].astype(np.float64) - op)
            tol = 1e-6 * np.abs(op.astype(np.float64)) + 2e-6
            assert np.all(err <= tol), f"target {t}: propagate off by {err.max()}"
            dev["prop"] = max(dev["prop"], float(err.max()))
        mdl_t = mdl
        if not sir and cfg.bins_per_sigma > 0:
            # adaptive bins: the GPU's cells per pixel against the rule; a
            # variance within rounding of a step of the rule may go either way
            m_o, var = oracle.adaptive_bins(prop[:, a:b], dim, cfg.bins_per_sigma, cfg.bins_max)
            for ax in range(dim):
                if m_gpu[t, ax] != m_o[ax]:
                    sd = math.sqrt(var[ax])
                    step = cfg.bins_per_sigma / min(m_gpu[t, ax], m_o[ax])
                    assert abs(sd - step) <= 1e-6 * step, f"target {t} axis {ax}: m {m_gpu[t, ax]} vs {m_o[ax]}"
            dev["adaptive_m"] = dev.get("adaptive_m", []) + [tuple(int(v) for v in m_gpu[t])]
            mdl_t = dataclasses.replace(mdl, m=tuple(int(v) for v in m_gpu[t]))
        r = oracle.weigh(mdl_t, fr, prop[:, a:b], sir=sir)
        assert np.array_equal(keys[:dim, a:b], r["keys"][:dim]), f"target {t}: keys differ"
        B = r["B"]
        if sir:
            ll_o = r["ll"]
            ll_g = ll_gpu[a:b].astype(np.float64)
        else:
            gsl = slice(int(bfirst[t]), int(bfirst[t + 1]))
            assert bfirst[t + 1] - bfirst[t] == B, f"target {t}: {bfirst[t + 1] - bfirst[t]} bins, oracle {B}"
            assert np.all(b_t[gsl] == t), f"target {t}: bin targets"
            assert np.array_equal(b_key[:dim, gsl], r["bin_key"][:dim]), f"target {t}: bin keys"
            assert np.array_equal(b_n[gsl], r["bin_n"]), f"target {t}: bin counts"
            gm, om = b_mean[:, gsl], r["bin_mean"]
            e_pos = np.abs(gm[:dim] - om[:dim]).max()
            e_vel = np.abs(gm[dim:2 * dim] - om[dim:2 * dim]).max()
            e_int = np.abs(gm[2 * dim] - om[2 * dim]).max()
            if cfg.dummy_mode == 0:
                assert e_pos <= 1e-7, f"target {t}: bin mean positions off by {e_pos}"
            assert e_vel <= 1e-7 and e_int <= 1e-6, (e_vel, e_int)
            dev["mean_pos"] = max(dev["mean_pos"], float(e_pos))
            dev["mean_vel"] = max(dev["mean_vel"], float(e_vel))
            dev["mean_int"] = max(dev["mean_int"], float(e_int))
            ll_o = r["ll"]
            ll_g = ll_gpu[gsl].astype(np.float64)
            dev["B"] += B
        d_ll = np.abs(ll_g - ll_o)
        tol_ll = ll_tol(cfg, sir, ll_o)
        if not sir and cfg.dummy_mode == 2:
            # second-order dummies: nine evaluations, each within tol, enter through
            # central differences of step delta = half a cell, with |S| <= delta^2:
            # |error| <= 6 tol + 2 tol delta (|g_x| + |g_y|); g from the oracle's stencil
            mx, my = mdl_t.m[0], mdl_t.m[1]
            gsum = np.zeros(B)
            for bi in range(B):
                c0, r0 = int(r["bin_key"][0, bi]) // mx, int(r["bin_key"][1, bi]) // my
                ux, uy = float(r["bin_mean"][0, bi]), float(r["bin_mean"][1, bi])
                I0 = float(r["bin_mean"][2 * dim, bi])
                dx, dy = 0.5 / mx, 0.5 / my
                lx = [oracle.loglik(mdl_t, fr, c0, r0, ux + sx * dx, uy, 0.0, I0) for sx in (-1, 1)]
                ly = [oracle.loglik(mdl_t, fr, c0, r0, ux, uy + sy * dy, 0.0, I0) for sy in (-1, 1)]
                gsum[bi] = abs(lx[1] - lx[0]) / 2.0 + abs(ly[1] - ly[0]) / 2.0   # delta (|g_x| + |g_y|)
            tol_ll = 1.2 * (6.0 * tol_ll + 2.0 * tol_ll * gsum)
        bad = d_ll > tol_ll
        assert not np.any(bad), (f"target {t}: log-likelihood off by {d_ll[bad].max()} at l = "
                                 f"{ll_o[bad][np.argmax(d_ll[bad])]}")
        dev["ll"] = max(dev["ll"], float(d_ll.max()))
        dev["ll_rel"] = max(dev.get("ll_rel", 0.0), float(np.max(d_ll / np.maximum(np.abs(ll_o), 1.0))))
        wg, wo = w_gpu[a:b], r["w"]
        if pair_form(cfg, sir) and cfg.dummy_mode != 2:
            wb = W_RTOL * wo + W_FLOOR * wo.max()
        else:
            tl_p = tol_ll[r["bin_of"]] if (not sir and cfg.dummy_mode == 2) else None
            wb = weight_bound(r["ll"][r["bin_of"]], wo, tl_p)
        e_w = np.abs(wg - wo) - wb
        worst = int(np.argmax(e_w))
        assert np.all(e_w <= 0), (f"target {t}: weights off, worst excess {e_w[worst]} at w = {wo[worst]} "
                                  f"(GPU {wg[worst]}), l = {r['ll'][r['bin_of'][worst]]}, max w = {wo.max()}")
        dev["w"] = max(dev["w"], float(np.max(np.abs(wg - wo) / np.maximum(wo, 1e-300))))
        # relative weight error where the weight is not negligible (above the floor)
        big = wo > W_FLOOR * wo.max() / W_RTOL
        dev["w_rel"] = max(dev.get("w_rel", 0.0), float(np.max(np.abs(wg - wo)[big] / wo[big])))
        assert abs(wg.sum() - 1.0) < 1e-12
        e_est = np.abs(est[t] - r["est"]) / np.maximum(np.abs(r["est"]), 1.0)
        assert np.all(e_est <= 1e-5), f"target {t}: estimate off by {e_est.max()}"
        dev["est"] = max(dev["est"], float(e_est.max()))
        e_neff = abs(neff[t] - r["neff"]) / r["neff"]
        assert e_neff <= 1e-5, f"target {t}: N_eff off by {e_neff}"
        dev["neff"] = max(dev["neff"], float(e_neff))
        u = oracle.resample_u(cfg.seed, k, t)
        assert tgt[t, 3] == u, f"target {t}: resampling uniform"
        N = b - a
        theta = (np.arange(N, dtype=np.float64) + u) / N
        # (1) from the oracle's weights: exact except near a threshold
        cdf_o, s_o = oracle.resample(wo, u)
        sg = s_gpu[a:b]
        diff = sg != s_o
        ex = exempt_mask(cdf_o, s_o, theta, 1e-6)
        assert not np.any(diff & ~ex), f"target {t}: {int(np.sum(diff & ~ex))} resampling indices differ"
        dev["exempt"] += int(np.sum(ex))
        dev["mismatch"] += int(np.sum(diff))
        # (2) from the GPU's own weights: the scan and the search
        cdf_g, s_g = oracle.resample(wg, u)
        e_cdf = np.abs(cdf_gpu[a:b] - cdf_g).max()
        # two FP64 prefix sums of the same non-negative weights (total 1) in
        # different orders: recursive summation errs by at most (N - 1) u each
        # (u = 2^-53); an element taken twice or dropped would err by ~1/N
        tol_cdf = 2.0 * N * 2.0 ** -53
        assert e_cdf <= tol_cdf, f"target {t}: cumulative weights off by {e_cdf} (bound {tol_cdf})"
        diff2 = sg != s_g
        ex2 = exempt_mask(cdf_g, s_g, theta, 1e-9)
        assert not np.any(diff2 & ~ex2), f"target {t}: resampling from the GPU's weights differs"
        assert np.all((sg >= 0) & (sg < N)) and np.all(np.diff(sg) >= 0)
        # the resampled set is the gather of the propagated states
        assert np.array_equal(after[:, a:b], prop[:, a:b][:, sg])
    if not sir:
        assert int(counts[0]) == b_t.size
        if targets is None:
            assert int(counts[0]) == dev["B"]
    if report is not None:
        report.update(dev)
    return dev, after
