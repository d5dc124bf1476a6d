"""The benchmark's CPU-baseline sample (host logic, no GPU): whole targets one
after another, frame after frame, each target continuing from its previous
step, until the time budget is used; its count of particle-steps and its
final states must equal a plain run of the same frames."""
import numpy as np

import bench
import oracle
import synth


def _model(w):
    return oracle.Model(dim=2, m=w.m, patch=w.patch, quad=w.quad, sigma_psf=w.sigma_psf, i_bg=w.i_bg,
                        sigma_xi=w.sigma_xi, proc_sigma=w.proc_sigma, seed=21)


def test_cpu_sample_walks_frames_and_counts_particle_steps():
    w = synth.preset("tiny")
    tr = synth.truth(w)
    fr = synth.frames(w, tr)
    counts = w.counts()
    st = synth.initial_particles(w, tr[0], counts)
    r = bench.cpu_oracle_rate(oracle, _model(w), w, fr, counts, st, seconds=1e9)  # budget never reached
    # every frame of the single target, once each
    assert r["sample"].startswith(f"{w.K} target-steps over frames 1..{w.K} ({w.K * int(counts[0])} particle-steps")
    assert r["value"] > 0 and r["cores"] == 1 and r["kind"] == "oracle"


def test_cpu_sample_stops_after_one_step_with_no_budget():
    w = synth.preset("tiny")
    tr = synth.truth(w)
    fr = synth.frames(w, tr)
    counts = w.counts()
    st = synth.initial_particles(w, tr[0], counts)
    r = bench.cpu_oracle_rate(oracle, _model(w), w, fr, counts, st, seconds=0.0)
    assert r["sample"].startswith(f"1 target-steps over frames 1..1 ({int(counts[0])} particle-steps")


def test_cpu_sample_steps_match_a_plain_track():
    """The sample tracks frame by frame from each target's previous state, as
    one multi-frame run does."""
    w = synth.preset("tiny")
    tr = synth.truth(w)
    fr = synth.frames(w, tr)
    counts = w.counts()
    st = synth.initial_particles(w, tr[0], counts)
    mdl = _model(w)
    s_all, _, _ = oracle.track(mdl, fr, counts, st, k0=1)
    s = np.array(st, dtype=np.float32, copy=True)
    for k in range(1, w.K + 1):
        s, _, _ = oracle.track(mdl, fr[k - 1:k], counts, s, k0=k)
    np.testing.assert_array_equal(s, s_all)
