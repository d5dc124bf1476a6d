"""The benchmark's CPU-baseline sample (host logic, no GPU): a stride-selected
subset of targets tracked frame after frame from frame 1 until the time
budget is used; its count of particle-steps and its final states must equal a
plain run of the same frames, whatever the number of OpenMP threads."""
import numpy as np

import bench
import oracle
import synth


def _model(w):
    return oracle.Model(dim=2, m=w.m, patch=w.patch, quad=w.quad, sigma_psf=w.sigma_psf, i_bg=w.i_bg,
                        sigma_xi=w.sigma_xi, proc_sigma=w.proc_sigma, seed=21)


def _inputs(T=1):
    w = synth.preset("tiny", T=T) if T > 1 else synth.preset("tiny")
    tr = synth.truth(w)
    fr = synth.frames(w, tr)
    counts = w.counts()
    return w, fr, counts, synth.initial_particles(w, tr[0], counts)


def test_cpu_sample_walks_frames_and_counts_particle_steps():
    w, fr, counts, st = _inputs()
    r = bench.cpu_oracle_rate(oracle, _model(w), w, fr, counts, st, seconds=1e9)  # budget never reached
    # every frame of the single target, once each
    assert f"frames 1..{w.K} ({w.K * int(counts[0])} particle-steps" in r["sample"], r["sample"]
    assert r["value"] > 0 and r["cores"] == 1 and r["kind"] == "oracle"


def test_cpu_sample_stops_after_one_frame_with_no_budget():
    w, fr, counts, st = _inputs()
    r = bench.cpu_oracle_rate(oracle, _model(w), w, fr, counts, st, seconds=0.0)
    assert f"frames 1..1 ({int(counts[0])} particle-steps" in r["sample"], r["sample"]


def test_cpu_subset_is_every_stride_th_target():
    assert list(bench.cpu_subset(25, 10)) == [0, 10, 20]
    assert list(bench.cpu_subset(7, 10)) == list(range(7))


def test_cpu_sample_uses_the_threads_asked_for():
    w, fr, counts, st = _inputs()
    r = bench.cpu_oracle_rate(oracle, _model(w), w, fr, counts, st, seconds=0.0, threads=3)
    assert r["cores"] == 3 and "3 threads" in r["sample"]


def test_oracle_tracking_is_independent_of_threads():
    """Targets run in parallel on private copies: states, estimates and N_eff
    are bit-identical for 1 and 4 threads."""
    w, fr, counts, st = _inputs(T=6)
    mdl = _model(w)
    try:
        oracle.set_threads(1)
        a = oracle.track(mdl, fr[:3], counts, st, k0=1)
        oracle.set_threads(4)
        b = oracle.track(mdl, fr[:3], counts, st, k0=1)
    finally:
        oracle.set_threads(1)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_cpu_sample_steps_match_a_plain_track():
    """The sample tracks frame by frame from each target's previous state, as
    one multi-frame run does."""
    w, fr, counts, st = _inputs()
    mdl = _model(w)
    s_all, _, _ = oracle.track(mdl, fr, counts, st, k0=1)
    s = np.array(st, dtype=np.float32, copy=True)
    for k in range(1, w.K + 1):
        s, _, _ = oracle.track(mdl, fr[k - 1:k], counts, s, k0=k)
    np.testing.assert_array_equal(s, s_all)
