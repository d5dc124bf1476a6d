"""GPU checks of the quantisation-aware training step (pcsir_mlp_train_step_fp8).

Its forward pass must be the FP8 inference kernel's network: the loss it
reports equals the mean squared error of that kernel's outputs. Its
gradients must be the straight-through gradients of that network: a numpy
reference takes the same operands (BF16 input layer; E4M3 values of the
scaled hidden inputs and weights; BF16 output activations), works in float64
and treats each quantiser as the identity where it does not clamp. And a few
quantisation-aware epochs must lower the FP8 mode's error on held-out rows.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from fp_emul import bf16_round, e4m3_round

pytestmark = pytest.mark.gpu

FP8_MAX = 448.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def _gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _quant(g, s):
    """E4M3 value of clamp(g * (1 / s)) in the kernels' binary32 arithmetic, and the in-range mask."""
    inv = np.float32(1.0) / np.float32(s)
    v = (np.asarray(g, np.float32) * inv).astype(np.float32)
    inside = np.abs(v) <= FP8_MAX
    return e4m3_round(np.clip(v, -FP8_MAX, FP8_MAX)).astype(np.float64), inside


def _wquant(W):
    W32 = np.asarray(W, np.float32)
    sw = np.float32(np.float32(np.abs(W32).max()) / np.float32(FP8_MAX))
    return e4m3_round(np.clip((W32 / sw).astype(np.float32), -FP8_MAX, FP8_MAX)).astype(np.float64), float(sw)


def _reference(th, Xo, y, sx):
    """Loss and straight-through gradients of the quantised network (float64)."""
    from oracle import mlp
    p = mlp.unpack(th.astype(np.float64))
    M = Xo.shape[0]
    W1 = bf16_round(p["W1"].astype(np.float32)).astype(np.float64)
    W2q, sw2 = _wquant(p["W2"])
    W3q, sw3 = _wquant(p["W3"])
    a2 = float(np.float32(sx[1]) * np.float32(sw2))
    a3 = float(np.float32(sx[2]) * np.float32(sw3))
    Z1 = Xo @ W1 + p["b1"]
    Q1, m1 = _quant(_gelu(Z1), sx[1])
    Z2 = (Q1 @ W2q) * a2 + p["b2"]
    Q2, m2 = _quant(_gelu(Z2), sx[2])
    Z3 = (Q2 @ W3q) * a3 + p["b3"]
    H3 = bf16_round(_gelu(Z3).astype(np.float32)).astype(np.float64)
    f = H3 @ p["w4"] + p["b4"][0]
    r = f - y
    loss = float(np.mean(r * r))
    df = 2.0 * r / M
    g = {"w4": H3.T @ df, "b4": np.array([df.sum()])}
    dZ3 = np.outer(df, p["w4"]) * _gelu_grad(Z3)
    g["W3"], g["b3"] = (float(sx[2]) * Q2).T @ dZ3, dZ3.sum(0)
    dZ2 = (dZ3 @ (sw3 * W3q).T) * _gelu_grad(Z2) * m2
    g["W2"], g["b2"] = (float(sx[1]) * Q1).T @ dZ2, dZ2.sum(0)
    dZ1 = (dZ2 @ (sw2 * W2q).T) * _gelu_grad(Z1) * m1
    g["W1"], g["b1"] = Xo.T @ dZ1, dZ1.sum(0)
    return loss, g, f


def _setup(seed, B):
    import torch

    from oracle import mlp
    rng = np.random.default_rng(seed)
    X = np.zeros((B, 256))
    X[:, :230] = rng.standard_normal((B, 230)) * 0.5
    y = rng.standard_normal(B) * 0.3
    th = mlp.init_params(seed + 1).astype(np.float32)
    Xb = torch.from_numpy(X.astype(np.float32)).cuda().to(torch.bfloat16)
    return th, Xb, Xb.float().cpu().numpy().astype(np.float64), y


def test_fp8_aware_loss_is_the_fp8_inference_loss():
    import torch

    from paper_1310_5541_amd._lib import MLPTrainer, SurrogateNet
    B = 256
    th, Xb, Xo, y = _setup(5, B)
    params = torch.from_numpy(th).cuda()
    sx = SurrogateNet(params).calibrate(Xb)
    yt = torch.from_numpy(y.astype(np.float32)).cuda()
    tr = MLPTrainer(params, B)
    _, loss = tr.gradients(Xb, yt, torch.tensor(sx, dtype=torch.float32, device="cuda"))
    f8 = SurrogateNet(params, act_scale=sx).rows(Xb, fp8=True).double().cpu().numpy()
    loss_inf = float(np.mean((f8 - y) ** 2))
    print(f"case fp8_aware_loss: train-path loss {loss:.6e}, inference loss {loss_inf:.6e}", flush=True)
    assert loss == pytest.approx(loss_inf, rel=2e-3)


def test_fp8_aware_gradients_are_straight_through():
    import torch

    from oracle import mlp
    from paper_1310_5541_amd._lib import MLPTrainer, SurrogateNet
    B = 128
    th, Xb, Xo, y = _setup(7, B)
    params = torch.from_numpy(th).cuda()
    sx = SurrogateNet(params).calibrate(Xb)
    tr = MLPTrainer(params, B)
    g, loss = tr.gradients(Xb, torch.from_numpy(y.astype(np.float32)).cuda(),
                           torch.tensor(sx, dtype=torch.float32, device="cuda"))
    g = g.cpu().numpy().astype(np.float64)
    loss_r, g_r, _ = _reference(th, Xo, y, sx)
    print(f"case fp8_aware_gradients: loss {loss:.6e} vs reference {loss_r:.6e}", flush=True)
    assert loss == pytest.approx(loss_r, rel=1e-2)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SIZES])
    for i, (name, _) in enumerate(mlp.SIZES):
        a, b = g[offs[i]:offs[i + 1]], np.asarray(g_r[name]).ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(f"  {name}: relative gradient error {rel:.2e}", flush=True)
        assert rel <= 2e-2, (name, rel)


def test_fp8_aware_epochs_lower_the_fp8_error():
    """From one BF16-trained network, four more epochs either in BF16 or
    quantisation-aware (same learning rate); the latter must give the lower
    FP8-mode error on held-out rows."""
    import torch

    from paper_1310_5541_amd import surrogate as sg
    from paper_1310_5541_amd._lib import MLPTrainer, SurrogateNet
    rng = np.random.default_rng(11)
    n, n_in, B = 65536, 16, 1024
    X = np.zeros((n, 256), np.float32)
    X[:, :n_in] = rng.uniform(-1, 1, (n, n_in))
    y = (np.sin(2 * X[:, 0]) * X[:, 1] + 0.5 * X[:, 2] * X[:, 3] - 0.3 * X[:, 4] ** 2).astype(np.float32)
    Xt = torch.from_numpy(X).cuda().to(torch.bfloat16)
    yt = torch.from_numpy(y).cuda()
    ntr = 57344
    p0, _ = sg.train(Xt[:ntr], yt[:ntr], epochs=20, n_in=n_in, lr=2e-3, lr_end=1e-4)
    sx = sg.calibrate(p0, Xt[:ntr])
    sxt = torch.tensor(sx, dtype=torch.float32, device="cuda")

    def more(act_scale):
        tr = MLPTrainer(p0, B)
        for _ in range(4):
            for b in range(ntr // B):
                tr.step(Xt[b * B:(b + 1) * B], yt[b * B:(b + 1) * B], 1e-4, act_scale)
        return tr.params.clone()

    def rms(p, s, fp8=True):
        f = SurrogateNet(p, act_scale=s).rows(Xt[ntr:].contiguous(), fp8=fp8).double()
        return float((f - yt[ntr:].double()).pow(2).mean().sqrt())

    pa, pb = more(None), more(sxt)
    e_bf16 = rms(pa, None, fp8=False)
    e_a, e_b = rms(pa, sg.calibrate(pa, Xt[:ntr])), rms(pb, sx)
    print(f"case fp8_aware_epochs: held-out rms: BF16 network {e_bf16:.4e}; FP8 mode after BF16 epochs "
          f"{e_a:.4e}, after FP8-aware epochs {e_b:.4e}", flush=True)
    assert e_b < e_a
