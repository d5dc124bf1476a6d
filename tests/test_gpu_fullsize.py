"""GPU parity at the full sizes the benchmark runs, in its launch configuration.

The single target (10^6 particles, 512 x 512, 15 x 15 window, 8 x 8
quadrature), the batched workload (1000 targets, 21 654 239 particles,
1024 x 1024) and the 3D workload (200 targets x 5 x 10^4 particles, D = 7)
step from a state three frames into tracking, at h = 0.25, with graph
launches and the launch shapes the benchmark's autotuner picks; the batched
workload runs with both exact likelihood forms (separable, the benchmark's,
and per sub-sample). The oracle checks every stage (propagation, keys, bins,
bin means, log-likelihoods, weights, estimates, N_eff, resampling) for the
whole single target and, of the others, for 50 targets: the 10 with the most
bins of this frame (lost, spread-out clouds, whose bin sums span the most
chunks) and 40 spread over the particle counts from the smallest to the
largest, to the tolerances of gpu_helpers. Every target is checked through
properties that hold at any size: bins ordered by target, member counts
summing to N_t, weights summing to 1 and non-decreasing parents.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import log, run_step_parity

pytestmark = pytest.mark.gpu

TUNING = dict(bin_tile=4096, list_blocks=512, digit_bits=11, grid_per_cu=32)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_5541_amd import lib
    lib()


def _start(w, cfg, frames, k0):
    """The particle set after k0 - 1 frames of tracking from the truth."""
    import torch

    from paper_1310_5541_amd import Filter
    tr = synth.truth(w)
    f = Filter(cfg, torch.from_numpy(synth.initial_particles(w, tr[0], w.counts())).cuda())
    f.set_tuning(**TUNING)
    fr = torch.from_numpy(frames).cuda()
    for k in range(1, k0):
        f.step(fr[k - 1], k)
    st = f.get_particles().cpu().numpy()
    f.close()
    return st


def _properties(cfg, frames, start, k):
    """Size-independent properties of one step over every target."""
    import torch

    from paper_1310_5541_amd import Filter
    n = np.asarray(cfg.n_particles, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(n)])
    f = Filter(cfg, torch.from_numpy(start).cuda())
    f.set_tuning(**TUNING)
    f.step(torch.from_numpy(frames).cuda(), k)
    f.estimate()
    b_t = f.dump("bin_target").cpu().numpy()
    b_n = f.dump("bin_n").cpu().numpy()
    w = f.dump("weights").cpu().numpy()
    s = f.dump("resample").cpu().numpy().astype(np.int64)
    f.close()
    assert np.all(np.diff(b_t) >= 0)
    bins = np.bincount(b_t, minlength=len(n))
    assert np.array_equal(np.bincount(b_t, weights=b_n, minlength=len(n)).astype(np.int64), n)
    sums = np.add.reduceat(w, off[:-1])
    assert np.all(np.abs(sums - 1.0) < 1e-12), np.abs(sums - 1.0).max()
    for t in range(len(n)):
        st = s[off[t]:off[t + 1]]
        assert st.min() >= 0 and st.max() < n[t] and np.all(np.diff(st) >= 0), t
    return bins


def _sample(n, bins, most=10, spread=40):
    """The targets with the most bins, then targets spread over the particle counts."""
    T = len(n)
    pick = list(np.argsort(-bins, kind="stable")[:most])
    order = np.argsort(n, kind="stable")
    for i in np.unique(np.linspace(0, T - 1, spread).round().astype(int)):
        if order[i] not in pick:
            pick.append(order[i])
    return sorted(int(t) for t in pick)


@pytest.mark.parametrize("workload,lik,extra", [("single-2d-512", 1, None), ("batched-2d-1024", 1, None),
                                                ("3d-astig", 1, None), ("batched-2d-1024", 0, None),
                                                ("batched-2d-1024", 1, dict(resample_light=0)),
                                                ("single-2d-512", 1, dict(resample_light=0)),
                                                ("batched-2d-1024", 1, dict(sort_bins=1)),
                                                ("3d-astig", 1, dict(sort_bins=1))])
def test_full_size_step(workload, lik, extra):
    """extra: launch shapes beyond the benchmark's. resample_light = 0: every
    scan tile with offspring leaves them to the search over blocks of new
    particles (the path of tiles holding much of their target's weight);
    sort_bins = 1: bins numbered by the radix sort instead of the occupancy
    bitmap; both at full size."""
    from paper_1310_5541_amd import Config
    w = synth.preset(workload, K=4)
    frames = synth.frames(w, synth.truth(w))
    m = 4
    cfg = Config.from_workload(w, bins_per_px=(m, m, m if w.dim == 3 else 1), lik_mode=lik, seed=w.seed + 500)
    start = _start(w, cfg, frames, 4)
    n = w.counts()
    log(f"case full_size {workload} lik_mode={lik} {extra}: {int(n.sum())} particles, {len(n)} targets")
    bins = _properties(cfg, frames[3], start, 4)
    sample = _sample(n, bins)
    log(f"  checked {len(sample)} targets: {sample}; most bins {int(bins.max())}")
    tuning = dict(TUNING, **(extra or {}))
    dev, _ = run_step_parity(cfg, start, frames[3], 4, False, targets=sample, tuning=tuning)
    log(f"  deviations {dev}")
