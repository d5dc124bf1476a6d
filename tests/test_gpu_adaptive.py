"""GPU parity of adaptive bin sizes against the oracle.

With bins_per_sigma > 0 every target picks, per frame and spatial axis,
m = ceil(bins_per_sigma / sd) cells per pixel in [1, bins_max] from the
spread of its propagated positions (a rule read for the adaptive bins the
paper names as future work). Checked: the cells per pixel the GPU used
against the oracle's rule, then every stage of the step with the oracle run
at each target's m (gpu_helpers); targets of very different spreads in one
launch, 2D and 3D; and a rule that gives bins_max everywhere, which must
reproduce the fixed-bin step with bins_per_px = bins_max bit for bit.
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


def _scene(dim=2):
    if dim == 2:
        counts = (3000, 700, 2049, 1, 257)
        w = synth.preset("tiny", H=128, W=128, T=len(counts), n=counts, K=2, mid_lo=20.0, mid_hi=108.0,
                         i0=(40.0, 100.0))
        spreads = (0.15, 0.4, 1.0, 0.5, 6.0)
    else:
        counts = (2500, 1, 700)
        w = synth.preset("3d-astig", H=48, W=48, T=3, n=counts, K=2)
        spreads = (0.2, 0.5, 1.2)
    tr = synth.truth(w, seed=5)
    fr = synth.frames(w, tr, seed=5)
    cloud = np.ascontiguousarray(np.concatenate(
        [synth.random_cloud(w, tr[1, t], counts[t], spreads[t], 40 + t) for t in range(len(counts))], axis=1))
    return w, fr, cloud


def test_adaptive_bins_2d():
    w, fr, cloud = _scene()
    cfg = _cfg(w, seed=13, lik_mode=1, bins_per_sigma=2.0, bins_max=8)
    log("case adaptive_bins_2d")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 2, False)
    ms = dev["adaptive_m"]
    log(f"  cells per pixel {ms}")
    assert len(set(ms)) >= 3, ms   # the spreads lead to different bin sizes


@pytest.mark.parametrize("dummy", [0, 1])
def test_adaptive_bins_3d(dummy):
    w, fr, cloud = _scene(dim=3)
    cfg = _cfg(w, seed=19, lik_mode=0, quad=4, bins_per_sigma=1.5, bins_max=6, dummy_mode=dummy)
    log(f"case adaptive_bins_3d dummy={dummy}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 2, False)
    log(f"  cells per pixel {dev['adaptive_m']}")


def test_saturated_rule_is_the_fixed_step():
    import torch

    from paper_1310_5541_amd import Filter
    w, fr, cloud = _scene()
    out = []
    for kw in (dict(bins_per_sigma=1e9, bins_max=3), dict(bins_per_px=(3, 3, 1))):
        f = Filter(_cfg(w, seed=13, lik_mode=1, **kw), torch.from_numpy(cloud).cuda())
        frd = torch.from_numpy(np.ascontiguousarray(fr)).cuda()
        for k in (1, 2):
            f.step(frd[k - 1], k)
        est, neff = f.estimate()
        out.append((est, neff, f.dump("weights").cpu().numpy(), f.dump("resample").cpu().numpy(),
                    f.dump("bins_per_px").cpu().numpy()))
        f.close()
    a, b = out
    assert np.all(a[4][:, :2] == 3)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
