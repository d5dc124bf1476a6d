"""GPU checks of the surrogate network's MFMA kernels against numpy / the FP64 oracle.

The GEMM test fixes the gfx950 MFMA lane layout the kernels assume (every
transposition case, several tiles); the gradient test compares one training
step's gradients with the oracle's reverse mode on the same BF16-rounded
weights and inputs (relative error of each tensor's norm <= 1e-2; BF16
activations and gradients bound the agreement)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bf(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda().to(torch.bfloat16)


@pytest.mark.parametrize("a_t,b_t", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_bf16_matches_numpy(a_t, b_t):
    from paper_1310_5541_amd._lib import gemm_bf16
    rng = np.random.default_rng(1)
    M, N, K = 128, 192, 96
    A = rng.standard_normal((K, M) if a_t else (M, K))
    B = rng.standard_normal((N, K) if b_t else (K, N))
    Ab, Bb = _bf(A), _bf(B)
    C = gemm_bf16(Ab, Bb, a_t, b_t).cpu().numpy().astype(np.float64)
    A64 = Ab.float().cpu().numpy().astype(np.float64)
    B64 = Bb.float().cpu().numpy().astype(np.float64)
    ref = (A64.T if a_t else A64) @ (B64.T if b_t else B64)
    np.testing.assert_allclose(C, ref, rtol=1e-5, atol=1e-4 * np.abs(ref).max())


def test_training_gradients_match_oracle():
    import torch

    from oracle import mlp
    from paper_1310_5541_amd._lib import MLPTrainer
    rng = np.random.default_rng(2)
    B = 128
    X = np.zeros((B, 256))
    X[:, :230] = rng.standard_normal((B, 230)) * 0.5
    y = rng.standard_normal(B)
    th = mlp.init_params(3)
    # the GPU multiplies BF16 weights and inputs: give the oracle the same values
    P = mlp.unpack(th.copy())
    for k in ("W1", "W2", "W3"):
        P[k] = torch.tensor(P[k], dtype=torch.float32).to(torch.bfloat16).double().numpy()
    thb = mlp.pack(P)
    Xb = _bf(X)
    Xo = Xb.float().cpu().numpy().astype(np.float64)
    tr = MLPTrainer(torch.from_numpy(thb.astype(np.float32)).cuda(), B)
    g, loss = tr.gradients(Xb, torch.from_numpy(y.astype(np.float32)).cuda())
    g = g.cpu().numpy().astype(np.float64)
    loss_o, g_o = mlp.loss_and_grad(thb, Xo, y)
    assert loss == pytest.approx(loss_o, rel=1e-2)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SIZES])
    for i, (name, _) in enumerate(mlp.SIZES):
        a, b = g[offs[i]:offs[i + 1]], g_o[offs[i]:offs[i + 1]]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 1e-2, (name, rel)
    f = tr.forward(Xb).cpu().numpy()
    fo, _ = mlp.forward(thb, Xo)
    assert np.linalg.norm(f - fo) / np.linalg.norm(fo) <= 1e-2


def test_adam_steps_reduce_loss():
    import torch

    from oracle import mlp
    from paper_1310_5541_amd._lib import MLPTrainer
    rng = np.random.default_rng(4)
    B = 512
    X = np.zeros((B, 256))
    X[:, :8] = rng.uniform(-1, 1, (B, 8))
    y = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    tr = MLPTrainer(torch.from_numpy(mlp.init_params(9, n_in=8).astype(np.float32)).cuda(), B)
    Xb, yt = _bf(X), torch.from_numpy(y.astype(np.float32)).cuda()
    l0 = float(tr.step(Xb, yt, 1e-3).item())
    for _ in range(300):
        loss = tr.step(Xb, yt, 1e-3)
    assert float(loss.item()) < 0.05 * l0
