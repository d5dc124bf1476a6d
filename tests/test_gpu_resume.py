"""Checkpoint and resume: the particle set read after frame k (pcsir_get_particles)
and loaded into a fresh context (pcsir_set_particles) continues bit for bit
like the uninterrupted run, in pcSIR and SIR, 2D and 3D. Resampling every
frame leaves uniform weights, so the particle set is the whole filter state;
the random numbers of frame k depend only on (seed, particle, k, target)."""
import numpy as np
import pytest

import synth
from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_5541_amd import lib
    lib()


def _run(cfg, start, frames, ks, sir):
    import torch

    from paper_1310_5541_amd import Filter
    f = Filter(cfg, torch.from_numpy(start).cuda())
    out = []
    for k in ks:
        f.step(frames[k - 1], k, sir=sir)
        est, neff = f.estimate()
        out.append((est, neff))
    st = f.get_particles().cpu().numpy()
    f.close()
    return out, st


@pytest.mark.parametrize("dim,sir", [(2, False), (2, True), (3, False)])
def test_resume_from_particles_is_bit_identical(dim, sir):
    import torch

    from paper_1310_5541_amd import Config
    if dim == 2:
        w = synth.preset("tiny", T=3, n=(3000, 1, 2500), K=6)
    else:
        w = synth.preset("3d-astig", H=48, W=48, T=2, n=(2000, 777), K=6)
    tr = synth.truth(w)
    fr = torch.from_numpy(synth.frames(w, tr)).cuda()
    cfg = Config.from_workload(w, seed=33, lik_mode=1)
    start = synth.initial_particles(w, tr[0], w.counts())
    log(f"case resume dim={dim} sir={sir}")
    full, st_full = _run(cfg, start, fr, range(1, 7), sir)
    first, st_mid = _run(cfg, start, fr, range(1, 4), sir)
    rest, st_end = _run(cfg, st_mid, fr, range(4, 7), sir)
    for (e1, n1), (e2, n2) in zip(full, first + rest):
        assert np.array_equal(e1, e2) and np.array_equal(n1, n2)
    assert np.array_equal(st_full, st_end)
