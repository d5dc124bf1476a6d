"""GPU parity of large likelihood windows against the FP64 oracle.

The large-object workload of Sec. 5 (sigma_PSF = 13, a 65 x 65 support) puts
more window pixels on every axis than a wave has lanes: the separable form
then keeps two per-axis sums per lane. Cases: the large-object workload with
point sampling and with q = 2, a window that leaves the frame, the largest
window (127 x 127, larger than the frame), and a window between 33 and 63
pixels wide (one per-axis sum per lane). Tolerances as in gpu_helpers.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import log, run_step_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_5541_amd import lib
    lib()


def _cfg(w, **kw):
    from paper_1310_5541_amd import Config
    return Config.from_workload(w, **kw)


def _clouds(w, counts, centres, spread, seed):
    parts = [synth.random_cloud(w, np.asarray(c, np.float64), int(n), spread, seed + t)
             for t, (n, c) in enumerate(zip(counts, centres))]
    return np.ascontiguousarray(np.concatenate(parts, axis=1))


@pytest.mark.parametrize("sir", [False, True])
@pytest.mark.parametrize("lik,quad", [(0, 1), (1, 1), (1, 2)])
def test_large_object(sir, lik, quad):
    """Three sequences of the large-object workload in one 512 x 512 frame,
    one of them 12 px from the frame's edge."""
    counts = (3000, 1, 2049)
    w = synth.preset("large-2d-512", T=3, n=counts, K=2, quad=quad)
    tr = synth.truth(w, seed=6)
    tr[:, 2, 0] += 12.0 - tr[1, 2, 0]   # third object near the left edge at frame 1
    fr = synth.frames(w, tr, seed=6)
    cfg = _cfg(w, seed=31, lik_mode=lik, bins_per_px=(2, 2, 1))
    cloud = _clouds(w, counts, [tr[1, t] for t in range(3)], 3.0, 13)
    log(f"case large_object sir={sir} lik={lik} quad={quad}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 2, sir)
    log(f"  deviations {dev}")


@pytest.mark.parametrize("sir", [False, True])
@pytest.mark.parametrize("lik", [0, 1])
def test_largest_window_exceeds_the_frame(sir, lik):
    counts = (700, 300)
    w = synth.preset("large-2d-512", H=96, W=80, T=2, n=counts, K=2, patch=127, sigma_psf=9.0, mid_lo=30.0,
                     mid_hi=50.0)
    tr = synth.truth(w, seed=2)
    fr = synth.frames(w, tr, seed=2)
    cfg = _cfg(w, seed=3, lik_mode=lik)
    cloud = _clouds(w, counts, [tr[1, t] for t in range(2)], 2.0, 5)
    log(f"case largest_window sir={sir} lik={lik}")
    run_step_parity(cfg, cloud, fr[1], 2, sir)


@pytest.mark.parametrize("sir", [False, True])
def test_window_wider_than_half_a_wave(sir):
    counts = (2500, 257)
    w = synth.preset("tiny", H=128, W=128, T=2, n=counts, K=2, patch=41, quad=2, sigma_psf=6.0, mid_lo=40.0,
                     mid_hi=88.0, m=(2, 2, 1))
    tr = synth.truth(w, seed=8)
    fr = synth.frames(w, tr, seed=8)
    cfg = _cfg(w, seed=17, lik_mode=1)
    cloud = _clouds(w, counts, [tr[1, t] for t in range(2)], 1.5, 21)
    log(f"case window_41 sir={sir}")
    run_step_parity(cfg, cloud, fr[1], 2, sir)
