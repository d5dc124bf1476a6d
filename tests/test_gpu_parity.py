"""GPU parity of the HIP filter step against the FP64 oracle (through the C ABI).

Sizes span several tiles of every kernel (256-particle propagate tiles,
2048-particle scan tiles, 4096-key sort chunks) with ragged tails; edge cases
cover single-particle targets, one particle per cell (pcSIR must equal SIR),
everything in one cell (uniform weights), windows that leave the frame, 3D
with per-target frames, the cell-centre dummy, the separable likelihood, and
several consecutive frames (the pending resampling gather).
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
    parts = []
    for t, (n, c) in enumerate(zip(counts, centres)):
        parts.append(synth.random_cloud(w, np.asarray(c, np.float64), int(n), spread, seed + t))
    return np.ascontiguousarray(np.concatenate(parts, axis=1))


def _scene(w, seed=5):
    tr = synth.truth(w, seed=seed)
    fr = synth.frames(w, tr, seed=seed)
    return tr, fr


@pytest.mark.parametrize("sir", [False, True])
@pytest.mark.parametrize("lik", [0, 1])
def test_single_target_small(sir, lik):
    w = synth.preset("single-2d-64", n=(10_000,))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=21, lik_mode=lik)
    cloud = _clouds(w, [10_000], [tr[1, 0]], 0.8, 7)
    log(f"case single_target_small sir={sir} lik={lik}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 2, sir)
    log(f"  deviations {dev}")


def _separated_mids(T, lo, hi, gap, seed):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < T:
        p = rng.uniform(lo, hi, 2)
        if all(np.hypot(*(p - q)) >= gap for q in pts):
            pts.append(p)
    return np.array(pts)


@pytest.mark.parametrize("sir", [False, True])
def test_ragged_multi_target(sir):
    """Eight targets, particle counts around every tile size, one spot per window."""
    counts = (1, 255, 256, 257, 2047, 2049, 4097, 5000)
    w = synth.preset("tiny", H=160, W=160, T=len(counts), n=counts, m=(4, 4, 1), K=2, i0=(20.0, 100.0),
                     speed=(0.5, 1.0))
    tr = synth.truth(w, seed=9)
    mids = _separated_mids(len(counts), 15.0, 145.0, 30.0, 9)
    tr[:, :, :2] += (mids - tr[1, :, :2])[None]  # place the spots apart (frame 1 at the mid-points)
    fr = synth.frames(w, tr, seed=9)
    cfg = _cfg(w, seed=5, lik_mode=1)
    cloud = _clouds(w, counts, [tr[1, t] for t in range(len(counts))], 0.6, 11)
    log(f"case ragged_multi_target sir={sir}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 3, sir)
    log(f"  deviations {dev}")


@pytest.mark.parametrize("sir", [False, True])
def test_overlapping_bright_spots(sir):
    """Windows that hold other targets' bright spots: |l| reaches several hundred,
    and the weights carry the log-likelihood's relative tolerance."""
    counts = (1, 255, 256, 257, 2047, 2049, 4097, 5000)
    w = synth.preset("tiny", H=96, W=96, T=len(counts), n=counts, m=(4, 4, 1), mid_lo=10.0, mid_hi=86.0,
                     i0=(20.0, 100.0))
    tr, fr = _scene(w, seed=9)
    cfg = _cfg(w, seed=5, lik_mode=1)
    cloud = _clouds(w, counts, [tr[1, t] for t in range(len(counts))], 0.6, 11)
    log(f"case overlapping_bright_spots sir={sir}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 3, sir)
    log(f"  deviations {dev}")


@pytest.mark.parametrize("sort_bins", [0, 1])
def test_one_particle_per_cell_equals_sir(sort_bins):
    """Sec. 4.2: one particle per cell recovers SIR. On the GPU the dummy of a
    one-member bin is that particle exactly, so the log-likelihoods agree bit
    for bit; the weights differ only by summation order. With 2048 cells per
    pixel the key range (about 10^8 cells) is wider than the sorted list's
    cell -> bin table, so the sort path's bin sums search each chunk's keys."""
    import torch

    from paper_1310_5541_amd import Filter
    w = synth.preset("single-2d-64", n=(3000,), m=(2048, 2048, 1))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=33, proc_sigma=(0, 0, 0, 0, 0))
    cloud = _clouds(w, [3000], [tr[1, 0]], 3.0, 2)
    log(f"case one_particle_per_cell sort_bins={sort_bins}")
    run_step_parity(cfg, cloud, fr[1], 1, False, tuning=dict(sort_bins=sort_bins))
    out = {}
    for sir in (False, True):
        f = Filter(cfg, torch.from_numpy(cloud).cuda())
        f.set_tuning(sort_bins=sort_bins)
        f.step(torch.from_numpy(fr[1]).cuda(), 1, sir=sir)
        f.estimate()
        if not sir:
            assert int(f.dump("bin_n").max().item()) == 1
        out[sir] = (f.dump("loglik").cpu().numpy(), f.dump("weights").cpu().numpy(),
                    f.dump("resample").cpu().numpy(), f.dump("propagated").cpu().numpy())
        f.close()
    # bins are in key order; map them back to particles through the keys
    prop = out[True][3]
    order = np.lexsort((np.floor((prop[0].astype(np.float64) + 0.5) * 2048),
                        np.floor((prop[1].astype(np.float64) + 0.5) * 2048)))
    assert np.array_equal(out[False][0], out[True][0][order])
    np.testing.assert_allclose(out[False][1], out[True][1], rtol=1e-12, atol=0)


def test_all_in_one_cell_gives_uniform_weights():
    w = synth.preset("single-2d-64", n=(5000,), m=(1, 1, 1))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=3, proc_sigma=(0, 0, 0.1, 0.1, 2.0))
    rng = np.random.default_rng(1)
    cloud = _clouds(w, [5000], [tr[1, 0]], 0.5, 4)
    cloud[0] = np.float32(30.0) + rng.uniform(-0.45, 0.45, 5000).astype(np.float32)
    cloud[1] = np.float32(31.0) + rng.uniform(-0.45, 0.45, 5000).astype(np.float32)
    cloud[2:4] = 0.0
    log("case all_in_one_cell")
    dev, after = run_step_parity(cfg, cloud, fr[1], 1, False)
    assert dev["B"] == 1


def test_window_leaves_the_frame():
    w = synth.preset("tiny", H=40, W=52, n=(3000,), m=(2, 2, 1))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=8)
    cloud = _clouds(w, [3000], [[1.0, 38.5, 0.5, -0.2, 40.0]], 1.5, 3)
    log("case window_leaves_frame")
    for sir in (False, True):
        run_step_parity(cfg, cloud, fr[0], 1, sir)


def test_cell_centre_dummy():
    w = synth.preset("single-2d-64", n=(6000,), m=(4, 4, 1))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=12, dummy_mode=1)
    cloud = _clouds(w, [6000], [tr[1, 0]], 0.9, 5)
    log("case cell_centre_dummy")
    run_step_parity(cfg, cloud, fr[1], 2, False)


@pytest.mark.parametrize("sir", [False, True])
def test_3d_astigmatic_per_target_frames(sir):
    counts = (3000, 1, 2500)
    w = synth.preset("3d-astig", H=48, W=48, T=3, n=counts, K=2)
    tr, fr = _scene(w, seed=4)
    cfg = _cfg(w, seed=19, lik_mode=0, quad=4)
    cloud = _clouds(w, counts, [tr[1, t] for t in range(3)], 0.5, 9)
    log(f"case 3d_astigmatic sir={sir}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 2, sir)
    log(f"  deviations {dev}")


@pytest.mark.parametrize("sir", [False, True])
def test_consecutive_frames(sir):
    """Three frames in a row: each step starts from the GPU's resampled set
    (the gather is fused into the next propagation)."""
    import torch

    from paper_1310_5541_amd import Filter
    w = synth.preset("single-2d-64", n=(7000,), K=4)
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=44)
    cloud = synth.initial_particles(w, tr[0], w.counts())
    f = Filter(cfg, torch.from_numpy(cloud).cuda())
    for k in range(1, 4):
        f.step(torch.from_numpy(fr[k - 1]).cuda(), k, sir=sir)
    f.estimate()
    start = f.get_particles().cpu().numpy()
    f.close()
    log(f"case consecutive_frames sir={sir}")
    run_step_parity(cfg, start, fr[3], 4, sir)


def test_bit_reproducible():
    import torch

    from paper_1310_5541_amd import Filter
    w = synth.preset("tiny", n=(20_000,), T=1)
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=2, bins_per_px=(10, 10, 1))
    cloud = _clouds(w, [20_000], [tr[1, 0]], 1.0, 1)
    res = []
    for _ in range(2):
        f = Filter(cfg, torch.from_numpy(cloud).cuda())
        for k in (1, 2):
            f.step(torch.from_numpy(fr[k]).cuda(), k)
        est, neff = f.estimate()
        res.append((est, neff, f.dump("resample").cpu().numpy(), f.dump("weights").cpu().numpy(),
                    f.get_particles().cpu().numpy()))
        f.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_nonfinite_frame_is_reported_and_particles_kept():
    import torch

    from paper_1310_5541_amd import Filter, PcsirError
    w = synth.preset("tiny", n=(3000,))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=2)
    cloud = _clouds(w, [3000], [tr[1, 0]], 1.0, 1)
    bad = fr[1].copy()
    bad[:, :] = np.nan
    f = Filter(cfg, torch.from_numpy(cloud).cuda())
    f.step(torch.from_numpy(bad).cuda(), 1)
    with pytest.raises(PcsirError) as ei:
        f.estimate()
    assert ei.value.status == -5
    s = f.dump("resample").cpu().numpy()
    assert np.array_equal(s, np.arange(3000))
    f.close()


@pytest.mark.parametrize("sort_bins", [0, 1])
def test_key_range_overflow_is_reported(sort_bins):
    """A frame whose occupied cell range does not fit 32-bit keys (4096 cells
    per pixel over a cloud of about 100 px: about 10^11 cells) gets no bins,
    whichever numbering is chosen, and the step reports the cell range
    instead of binning with wrapped keys."""
    import torch

    from paper_1310_5541_amd import Filter, PcsirError
    w = synth.preset("tiny", n=(2000,), m=(4096, 4096, 1))
    tr, fr = _scene(w)
    cfg = _cfg(w, seed=4)
    cloud = _clouds(w, [2000], [tr[1, 0]], 20.0, 3)
    log(f"case key_range_overflow sort_bins={sort_bins}")
    f = Filter(cfg, torch.from_numpy(cloud).cuda())
    f.set_tuning(sort_bins=sort_bins)
    f.step(torch.from_numpy(fr[1]).cuda(), 1)
    with pytest.raises(PcsirError) as ei:
        f.estimate()
    assert "cell range" in str(ei.value)
    f.close()


def test_api_state_errors():
    import torch

    from paper_1310_5541_amd import Filter, PcsirError
    w = synth.preset("tiny", n=(300,))
    cfg = _cfg(w)
    f = Filter(cfg, torch.zeros((5, 300), dtype=torch.float32, device="cuda"))
    with pytest.raises(PcsirError) as ei:
        f.estimate()
    assert ei.value.status == -4
    wrong = torch.zeros((w.H + 1, w.W), dtype=torch.float32, device="cuda")
    from paper_1310_5541_amd._lib import lib
    import ctypes as C
    assert lib().pcsir_step(f._ctx, C.c_void_p(wrong.data_ptr()), w.H + 1, w.W, 1) == -4
    assert lib().pcsir_step(f._ctx, C.c_void_p(wrong.data_ptr()), w.H, w.W, 0) == -1
    f.close()


@pytest.mark.parametrize("sir", [False, True])
def test_graph_replays_match_eager_launches(sir):
    """Each step replays a captured HIP graph; over several frames, with eager
    work and synchronisation in between, every replay must give the same bytes
    as launching the kernels one by one."""
    import torch

    from paper_1310_5541_amd import Filter
    counts = (3000, 700, 4100)
    w = synth.preset("tiny", H=96, W=96, T=3, n=counts, K=5, mid_lo=20.0, mid_hi=76.0)
    tr, fr = _scene(w, seed=3)
    cfg = _cfg(w, seed=7)
    init = torch.from_numpy(synth.initial_particles(w, tr[0], np.array(counts))).cuda()
    fg, fe = Filter(cfg, init), Filter(cfg, init)
    fe.set_graphs(False)
    for k in range(1, 6):
        frame = torch.from_numpy(fr[k - 1]).cuda()
        fg.step(frame, k, sir=sir)
        fe.step(frame, k, sir=sir)
        eg, ng = fg.estimate()
        ee, ne = fe.estimate()
        assert np.array_equal(eg, ee) and np.array_equal(ng, ne), k
        for what in ("resample", "weights", "propagated"):
            assert torch.equal(fg.dump(what), fe.dump(what)), (k, what)
        _ = (frame * 2).sum().item()  # unrelated eager work between replays
    assert torch.equal(fg.get_particles(), fe.get_particles())
    fg.close()
    fe.close()


@pytest.mark.parametrize("m", [1, 2, 4, 5, 10, 20])
def test_cell_index_at_adversarial_positions(m):
    """Cells of positions within a few ulp of every cell edge j/m - 1/2, tiny
    values around the 2^-17 switch of the GPU's method, signed zeros and
    negatives; compared with the oracle's exact floor. Zero process noise and
    zero velocity leave the positions unchanged by propagation."""
    import torch

    import oracle
    from paper_1310_5541_amd import Config, Filter
    edges = (np.arange(-30 * m, 30 * m + 1) / m - 0.5).astype(np.float32)
    vals = [edges]
    for d in (1, 2, 3):
        up, dn = edges.copy(), edges.copy()
        for _ in range(d):
            up = np.nextafter(up, np.float32(np.inf))
            dn = np.nextafter(dn, np.float32(-np.inf))
        vals += [up, dn]
    tiny = np.array([2.0 ** -60, 2.0 ** -30, 2.0 ** -18, 2.0 ** -17, 2.0 ** -16, 1e-6, 0.0], np.float32)
    t17 = np.float32(2.0 ** -17)
    tiny = np.concatenate([tiny, -tiny, [np.nextafter(t17, np.float32(0)), np.nextafter(t17, np.float32(1)),
                                         -np.nextafter(t17, np.float32(0)), -np.nextafter(t17, np.float32(1)),
                                         np.float32(-0.0)]]).astype(np.float32)
    x = np.concatenate(vals + [tiny]).astype(np.float32)
    n = x.size
    rng = np.random.default_rng(m)
    y = rng.permutation(x)
    state = np.zeros((5, n), np.float32)
    state[0], state[1], state[4] = x, y, 50.0
    w = synth.preset("tiny", H=64, W=64, n=(n,), m=(m, m, 1), proc_sigma=(0.0, 0.0, 0.0, 0.0, 0.0))
    cfg = _cfg(w, seed=3, lik_mode=1)
    f = Filter(cfg, torch.from_numpy(state).cuda())
    f.set_debug(True)
    frame = torch.full((64, 64), 10.0, dtype=torch.float32, device="cuda")
    log(f"case cell_index_adversarial m={m} n={n}")
    f.pcsir_step(frame, 1)
    prop = f.dump("propagated").cpu().numpy()
    keys = f.dump("keys").cpu().numpy()
    f.close()
    np.testing.assert_array_equal(prop[0], x + np.float32(0.0))
    np.testing.assert_array_equal(keys[0], oracle.bin_key(prop[0], m))
    np.testing.assert_array_equal(keys[1], oracle.bin_key(prop[1], m))


def test_launch_shapes_do_not_change_results_and_autotune_restores_particles():
    """Every pcsir_tuning setting gives bit-identical steps (bins are the
    distinct keys in ascending order whether the occupancy bitmap or the sort
    numbers them, sums are exact integers, no reduction depends on the grid,
    and a scan tile's offspring get the same parents whether the tile resolves
    them itself or leaves them to the search blocks: resample_light 0 sends
    every tile with offspring to the search, 4096 only tiles with more than
    4096); SIR steps too. The
    autotuner returns a valid setting and leaves the particles as they were."""
    import torch

    from paper_1310_5541_amd import Filter
    counts = (1, 255, 2049, 5000, 9000)
    w = synth.preset("tiny", H=128, W=128, T=len(counts), n=counts, m=(4, 4, 1), K=4, i0=(20.0, 100.0),
                     speed=(0.5, 1.0), patch=15, quad=4)
    tr = synth.truth(w, seed=12)
    mids = _separated_mids(len(counts), 15.0, 113.0, 25.0, 12)
    tr[:, :, :2] += (mids - tr[1, :, :2])[None]
    fr = torch.from_numpy(synth.frames(w, tr, seed=12)).cuda()
    cloud = torch.from_numpy(_clouds(w, counts, [tr[1, t] for t in range(len(counts))], 1.2, 5)).cuda()
    cfg = _cfg(w, seed=13, lik_mode=1)
    shapes = [None, dict(bin_tile=1024, list_blocks=64, digit_bits=6, grid_per_cu=4, resample_light=0, sort_bins=1),
              dict(bin_tile=2048, list_blocks=512, digit_bits=8, grid_per_cu=16, resample_light=1024, sort_bins=1),
              dict(bin_tile=1024, list_blocks=64, digit_bits=11, grid_per_cu=8, resample_light=2048, sort_bins=0)]
    outs = []
    for sh in shapes:
        log(f"case launch_shapes {sh}")
        f = Filter(cfg, cloud)
        f.set_debug(True)
        if sh:
            f.set_tuning(**sh)
            assert f.get_tuning() == sh
        for k in range(1, 4):
            f.pcsir_step(fr[k], k)
        outs.append({n: f.dump(n).cpu().numpy()
                     for n in ("loglik", "weights", "resample", "cdf", "bin_key", "bin_n")}
                    | {"after": f.get_particles().cpu().numpy(), "passes": int(f.dump("counts")[1].item())})
        f.sir_step(fr[3], 4)
        outs[-1] |= {"sir_" + n: f.dump(n).cpu().numpy() for n in ("weights", "resample", "cdf")}
        f.close()
    for o in outs[1:]:
        for n in ("loglik", "weights", "resample", "cdf", "bin_key", "bin_n", "after",
                  "sir_weights", "sir_resample", "sir_cdf"):
            assert np.array_equal(o[n], outs[0][n]), n
    log(f"  sort passes per shape: {[o['passes'] for o in outs]}")
    assert [o["passes"] > 0 for o in outs] == [False, True, True, False]
    # autotune
    f = Filter(cfg, cloud)
    f.pcsir_step(fr[1], 1)
    before = f.get_particles().cpu().numpy()
    best, ms, n = f.autotune(fr[2], 2, reps=2)
    log(f"  autotune: {best}, {ms:.4f} ms/step, {n} trials")
    assert n >= 9 and ms > 0
    assert best["bin_tile"] in (1024, 2048, 4096) and 6 <= best["digit_bits"] <= 11 and best["sort_bins"] in (0, 1)
    assert f.get_tuning() == best
    assert np.array_equal(f.get_particles().cpu().numpy(), before)
    f.pcsir_step(fr[2], 2)
    f.estimate()
    f.close()


def test_bin_numbering_across_steps_with_changing_key_ranges():
    """The occupancy bitmap keeps no stale bits between steps: on one filter,
    particle sets with wide and narrow clouds alternate (the key range grows
    and shrinks by orders of magnitude) while the bin numbering switches
    between the bitmap and the sort, and every step equals the same step on a
    fresh filter bit for bit (the bits a step sets are cleared by the next
    step's propagation, over the previous key range)."""
    import torch

    from paper_1310_5541_amd import Filter
    counts = (3000, 700, 4000)
    w = synth.preset("tiny", H=128, W=128, T=len(counts), n=counts, m=(8, 8, 1), K=2, i0=(20.0, 100.0))
    tr, fr = _scene(w, seed=17)
    cfg = _cfg(w, seed=19, lik_mode=1)
    centres = [tr[1, t] for t in range(len(counts))]
    wide = torch.from_numpy(_clouds(w, counts, centres, 12.0, 7)).cuda()
    narrow = torch.from_numpy(_clouds(w, counts, centres, 0.3, 8)).cuda()
    frame = torch.from_numpy(fr[1]).cuda()
    names = ("bin_key", "bin_n", "loglik", "weights", "resample")
    f = Filter(cfg, narrow)
    for i, (cl, sb) in enumerate([(wide, 0), (narrow, 0), (wide, 1), (narrow, 1), (wide, 0), (narrow, 0), (wide, 0)]):
        log(f"case bin_numbering_across_steps step {i} {'wide' if cl is wide else 'narrow'} sort_bins={sb}")
        f.set_particles(cl)
        f.set_tuning(sort_bins=sb)
        f.pcsir_step(frame, 1)
        got = {n: f.dump(n).cpu().numpy() for n in names}
        g = Filter(cfg, cl)
        g.pcsir_step(frame, 1)
        ref = {n: g.dump(n).cpu().numpy() for n in names}
        g.close()
        for n in names:
            assert np.array_equal(got[n], ref[n]), (i, n)
    f.close()


@pytest.mark.parametrize("lik", [0, 1])
def test_second_order_dummies(lik):
    """Dummies that carry their members' position covariance: nine shifted
    evaluations per dummy, combined to second order (tolerance in gpu_helpers)."""
    counts = (4000, 1, 1500)
    w = synth.preset("tiny", H=96, W=96, T=3, n=counts, K=2, mid_lo=20.0, mid_hi=76.0, m=(2, 2, 1),
                     sigma_xi=40.0)
    tr, fr = _scene(w, seed=6)
    cfg = _cfg(w, seed=23, lik_mode=lik, dummy_mode=2)
    cloud = _clouds(w, counts, [tr[1, t] for t in range(3)], 0.8, 31)
    log(f"case second_order_dummies lik={lik}")
    dev, _ = run_step_parity(cfg, cloud, fr[1], 2, False)
    log(f"  deviations {dev}")
