"""Training and evaluation of the learned log-likelihood surrogate, on the GPU.

The surrogate stands in for the model-image terms of the dummies'
log-likelihood (Sec. 5.2, Eq. likelihood) in Alg. pcSIR; the decomposition,
features and target are described in include/pcsir_mlp.h. Here:

* rows: training rows (features, exact l + A) of every dummy of exact pcSIR
  steps over a frame sequence, gathered by the library
  (pcsir_surrogate_features) into one device buffer;
* train: Adam on the mean squared error with the library's BF16 MFMA forward /
  backward kernels (pcsir_mlp_train_step), one shuffle per epoch, linear
  learning-rate decay;
* calibrate: FP8 input scales of the three layers from the BF16 activations of
  a sample of rows; optionally, quantisation-aware epochs after the BF16 ones
  (pcsir_mlp_train_step_fp8) fit the network to the FP8 mode's quantisers;
* evaluate: |l_surrogate - l_exact| in nats through the fused inference kernel.

torch provides device memory, the row shuffle and the reductions of the error
statistics; every network evaluation runs in the library's kernels.
"""
from __future__ import annotations

import math
import time

import numpy as np

from ._lib import Filter, MLPTrainer, SurrogateNet, mlp_param_count

N_HIDDEN = 256
N_FEAT = 256


def init_params(seed: int, n_in: int, y_mean: float = 0.0) -> np.ndarray:
    """He-initialised FP32 parameter vector (layout of pcsir_mlp.h); input rows beyond n_in are 0."""
    rng = np.random.default_rng(seed)
    H, F = N_HIDDEN, N_FEAT
    W1 = rng.standard_normal((F, H)) * math.sqrt(2.0 / n_in)
    W1[n_in:] = 0.0
    W2 = rng.standard_normal((H, H)) * math.sqrt(2.0 / H)
    W3 = rng.standard_normal((H, H)) * math.sqrt(2.0 / H)
    w4 = rng.standard_normal(H) * math.sqrt(1.0 / H)
    parts = [W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(H), w4, [y_mean]]
    th = np.concatenate([np.asarray(p, np.float64).ravel() for p in parts]).astype(np.float32)
    assert th.size == mlp_param_count()
    return th


def rows(f: Filter, frames, k0: int, n_frames: int, cap: int, X=None, y=None, start: int = 0):
    """Step `f` (an exact-likelihood filter) over frames[k0-1 .. k0+n_frames-2] and append
    the dummies' training rows to X, y from row `start` on, at most `cap` rows in all.
    Returns the number of rows written (start included)."""
    import torch
    if X is None:
        X = torch.empty((cap, N_FEAT), dtype=torch.bfloat16, device=f.device)
        y = torch.empty(cap, dtype=torch.float32, device=f.device)
    n = start
    for k in range(k0, k0 + n_frames):
        if n >= cap:
            break
        f.pcsir_step(frames[k - 1], k)
        _, _, B = f.surrogate_features(cap - n, X=X[n:], y=y[n:])
        n += min(B, cap - n)
    return n


def train(X, y, epochs: int = 4, batch: int = 1024, lr: float = 1e-3, lr_end: float = 5e-5, seed: int = 0,
          n_in: int = 230, log=None, qat_epochs: int = 0, qat_lr: float = 1e-4):
    """Train on rows X [n, 256] BF16, y [n] FP32 (device). Returns (params FP32 device, history).

    qat_epochs > 0: after the BF16 epochs, calibrate the FP8 input scales on the
    trained network and train a copy of it for qat_epochs more epochs with the
    FP8 inference's quantisers in the forward pass (pcsir_mlp_train_step_fp8,
    learning rate qat_lr decaying to lr_end). The returned parameters stay
    those of the BF16 epochs (for the BF16 mode); the history then holds the
    FP8 mode's parameters ("fp8_params") and the scales they were trained
    with ("fp8_scales"), which must be used together."""
    import torch
    n = (X.shape[0] // batch) * batch
    ym = float(y[:n].mean().item())
    params = torch.from_numpy(init_params(seed, n_in, ym)).to(X.device)
    tr = MLPTrainer(params, batch)
    steps_per_epoch = n // batch
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    hist, hist_q = [], []
    t0 = time.perf_counter()
    step = 0

    def run(n_ep, lr0, out, act_scale, tag):
        nonlocal step
        total = n_ep * steps_per_epoch
        s0 = step
        for ep in range(n_ep):
            perm = torch.randperm(X.shape[0], device=X.device, generator=g)[:n]
            Xs = X[perm].contiguous()
            ys = y[perm].contiguous()
            acc = torch.zeros((), dtype=torch.float32, device=X.device)
            for b in range(steps_per_epoch):
                frac = (step - s0) / max(total - 1, 1)
                cur = lr0 * (1.0 - frac) + lr_end * frac
                loss = tr.step(Xs[b * batch:(b + 1) * batch], ys[b * batch:(b + 1) * batch], cur, act_scale)
                acc += loss[0]
                step += 1
            mse = float(acc.item()) / steps_per_epoch
            out.append(mse)
            if log:
                log(f"{tag} epoch {ep + 1}/{n_ep}: mse {mse:.5f} (rms {math.sqrt(mse) * 100:.3f} nats), "
                    f"{time.perf_counter() - t0:.1f} s")

    run(epochs, lr, hist, None, "bf16")
    params_bf16 = tr.params.clone()
    info = {"mse_per_epoch": hist, "steps": step, "batch": batch, "rows": n}
    if qat_epochs > 0:
        scales = calibrate(params_bf16, X)
        sc = torch.tensor([float(v) for v in scales], dtype=torch.float32, device=X.device)
        run(qat_epochs, qat_lr, hist_q, sc, "fp8-aware")
        info.update({"qat_mse_per_epoch": hist_q, "fp8_scales": [float(v) for v in scales], "steps": step,
                     "fp8_params": tr.params.clone()})
    torch.cuda.synchronize()
    info["train_s"] = time.perf_counter() - t0
    return params_bf16, info


def calibrate(params, X, n: int = 65536, margin: float = 1.0):
    """FP8 input scales s_l = margin * max|input_l| / 448 from the BF16 activations of n rows."""
    net = SurrogateNet(params)
    return net.calibrate(X[:n].contiguous(), margin)


def evaluate(params, X, y, act_scale=None, fp8: bool = False) -> dict:
    """Error statistics of l_surrogate - l_exact in nats on rows X, y (network scale 100 / unit)."""
    import torch
    net = SurrogateNet(params, act_scale=act_scale)
    f = net.rows(X.contiguous(), fp8=fp8)
    e = (f - y).double() * 100.0
    a = e.abs()
    q = torch.quantile(a[: min(a.numel(), 1 << 24)].float(), torch.tensor([0.5, 0.9, 0.99], device=a.device))
    return {"rows": int(X.shape[0]), "bias": float(e.mean()), "rms": float(e.pow(2).mean().sqrt()),
            "median_abs": float(q[0]), "p90_abs": float(q[1]), "p99_abs": float(q[2]), "max_abs": float(a.max())}
