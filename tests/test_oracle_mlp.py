"""Pins of the FP64 surrogate-network oracle (CPU only).

The reverse-mode gradient is checked against central finite differences of
the loss, coordinate by coordinate on a sample of every parameter tensor; GELU
against its closed form at known points; the Adam step against the published
update rule evaluated on scalars.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_closed_form_points():
    # u Phi(u): Phi(0) = 1/2, Phi(1) = 0.841344746..., Phi(-1) = 0.158655253...
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-14)
    assert mlp.gelu(np.array([-1.0]))[0] == pytest.approx(-0.15865525393145707, rel=1e-14)
    u = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (mlp.gelu(u + h) - mlp.gelu(u - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(u), fd, rtol=1e-8, atol=1e-9)


def test_pack_roundtrip_and_size():
    th = mlp.init_params(1)
    assert th.shape == (mlp.N_PARAMS,) and mlp.N_PARAMS == 3 * 256 * 256 + 4 * 256 + 1
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(th)), th)
    assert np.all(mlp.unpack(th)["W1"][230:] == 0.0)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    n = 24
    X = np.zeros((n, 256))
    X[:, :230] = rng.standard_normal((n, 230)) * 0.5
    y = rng.standard_normal(n)
    th = mlp.init_params(7) * 0.7
    th[mlp.N_PARAMS - 1] = 0.1
    loss, g = mlp.loss_and_grad(th, X, y)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SIZES])
    h = 1e-6
    for ti, (name, shape) in enumerate(mlp.SIZES):
        size = int(np.prod(shape))
        picks = rng.choice(size, size=min(12, size), replace=False)
        if name == "W1":
            picks = np.array([p for p in picks if p // 256 < 230][:8])
        for p in picks:
            i = offs[ti] + p
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            fd = (mlp.loss_and_grad(tp, X, y)[0] - mlp.loss_and_grad(tm, X, y)[0]) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), (name, p)


def test_forward_is_the_composition():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((5, 256))
    th = mlp.init_params(2)
    p = mlp.unpack(th)
    f, _ = mlp.forward(th, X)
    for r in range(5):
        h = X[r]
        for W, b in (("W1", "b1"), ("W2", "b2"), ("W3", "b3")):
            z = np.array([sum(h[k] * p[W][k, n] for k in range(256)) for n in range(256)]) + p[b]
            h = np.array([zi * 0.5 * (1 + math.erf(zi / math.sqrt(2))) for zi in z])
        assert f[r] == pytest.approx(float(h @ p["w4"] + p["b4"][0]), rel=1e-12)


def test_adam_step_scalar_rule():
    th = np.array([0.3, -1.2])
    g = np.array([0.5, -0.25])
    m = np.array([0.1, 0.0])
    v = np.array([0.01, 0.02])
    t, lr = 3, 1e-3
    th2, m2, v2 = mlp.adam_step(th, m, v, g, t, lr)
    for i in range(2):
        mi = 0.9 * m[i] + 0.1 * g[i]
        vi = 0.999 * v[i] + 0.001 * g[i] ** 2
        upd = lr * (mi / (1 - 0.9**t)) / (math.sqrt(vi / (1 - 0.999**t)) + 1e-8)
        assert th2[i] == pytest.approx(th[i] - upd, rel=1e-15)
        assert m2[i] == pytest.approx(mi) and v2[i] == pytest.approx(vi)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(5)
    X = np.zeros((256, 256))
    X[:, :8] = rng.uniform(-1, 1, (256, 8))
    y = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    th = mlp.init_params(9, n_in=8)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss_and_grad(th, X, y)[0]
    for t in range(1, 201):
        loss, g = mlp.loss_and_grad(th, X, y)
        th, m, v = mlp.adam_step(th, m, v, g, t, 1e-3)
    assert loss < 0.05 * l0
