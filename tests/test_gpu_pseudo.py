"""Sec. 5.5's pseudo-tracking experiment on the GPU.

Repetitions run batched as targets that share one frame; with no motion, one
step weighs the prior draws as they are. Checked here:
- stage parity with the oracle for SIR, pcSIR-CoM and pcSIR-CoC (the
  propagation is the identity);
- the experiment: against the oracle's exact posterior mean, the RMSE of SIR
  and of pcSIR (CoM and CoC) falls as N^(-1/2) while the Monte-Carlo error
  dominates, and pcSIR stays within 15% of SIR there.
"""
import math

import numpy as np
import pytest

import synth
from gpu_helpers import log, oracle_model, run_step_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_5541_amd import lib
    lib()


def _cfg(reps, n, m=1, dummy=0, lik=1):
    from paper_1310_5541_amd import Config
    return Config.from_workload(synth.pseudo_workload(reps, n, m), dummy_mode=dummy, lik_mode=lik, seed=9)


@pytest.mark.parametrize("mode", ["sir", "com", "coc"])
def test_pseudo_step_parity(mode):
    fr, xy = synth.pseudo_frame()
    reps, n = 6, 2000
    cfg = _cfg(reps, n, dummy=1 if mode == "coc" else 0, lik=0)
    st = synth.pseudo_particles("uniform", 3.0, xy, reps, n, seed=3)
    log(f"case pseudo_step_parity {mode}")
    run_step_parity(cfg, st, fr, 1, mode == "sir")


MODES = {"sir": (1, 0), "com1": (1, 0), "coc1": (1, 1), "com2": (2, 0), "coc2": (2, 1)}


def _experiment(kind, par, Ns, reps):
    """RMSE and |mean error| of every estimator against the exact posterior mean."""
    import torch

    import oracle
    from paper_1310_5541_amd import Filter
    fr, xy = synth.pseudo_frame()
    w = synth.pseudo_workload(1, 1)
    ref = oracle.posterior_mean(oracle_model(_cfg(1, 1)), fr, kind, par, xy, w.i0[0])
    frd = torch.from_numpy(fr).cuda()
    rmse = {k: [] for k in MODES}
    bias = {k: [] for k in MODES}
    for N in Ns:
        st = torch.from_numpy(synth.pseudo_particles(kind, par, xy, reps, N, seed=1000 + N)).cuda()
        for mode, (m, dummy) in MODES.items():
            f = Filter(_cfg(reps, N, m=m, dummy=dummy), st)
            f.step(frd, 1, sir=mode == "sir")
            est, _ = f.estimate()
            f.close()
            d = est[:, :2] - ref[None]
            rmse[mode].append(math.sqrt(float(np.mean(np.sum(d * d, axis=1)))))
            bias[mode].append(float(np.linalg.norm(d.mean(axis=0))))
        del st
    return rmse, bias


@pytest.mark.parametrize("kind,par", synth.PSEUDO_PRIORS)
def test_pseudo_tracking_convergence(kind, par):
    """1000 repetitions per N. Asserted where the Monte-Carlo error dominates
    (N <= 16 000): SIR and pcSIR with half-pixel bins converge as N^(-1/2)
    and stay within 15% of each other, and SIR's mean error is consistent
    with zero. Pixel-sized bins carry an approximation error of a few
    thousandths of a pixel that the larger N expose; it is logged."""
    Ns = (1000, 4000, 16000, 64000)
    reps = 1000
    rmse, bias = _experiment(kind, par, Ns, reps)
    log(f"case pseudo_convergence {kind} {par}: N {Ns}, {reps} repetitions")
    for k in MODES:
        log(f"  {k}: rmse {[round(x, 6) for x in rmse[k]]} |mean error| {[round(x, 6) for x in bias[k]]}")
    small = slice(0, 3)
    for k in ("sir", "com2", "coc2"):
        slope = np.polyfit(np.log(Ns[small]), np.log(rmse[k][small]), 1)[0]
        assert -0.6 <= slope <= -0.4, (k, slope, rmse[k])
    for i in range(3):
        for k in ("com2", "coc2"):
            assert abs(rmse[k][i] / rmse["sir"][i] - 1.0) <= 0.15, (k, Ns[i], rmse)
        assert bias["sir"][i] <= 4.0 * rmse["sir"][i] / math.sqrt(reps), (Ns[i], bias["sir"])
