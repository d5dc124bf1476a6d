"""FP64 reference of the log-likelihood surrogate network — TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this module; the GPU library shares no code with it.

The surrogate is not part of the paper; it is an extension that replaces the
expensive model-image terms of the log-likelihood (Sec. 5.2, Eq. likelihood)
for the dummy particles of Alg. pcSIR:

    l(z, x) = -A(z) + 100 * f(features(z, x)),   A(z) = sum_window (z - I_bg)^2 / (2 sigma_xi^2)

where A(z) depends on the frame only (computed exactly) and f is a multilayer
perceptron with three hidden layers of 256 units and exact GELU, g(u) = u Phi(u).
Layout of the parameter vector (float32 on the GPU, float64 here), all
matrices row-major with the input index first (W[k][n]: input k -> unit n):
    W1 [256][256], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
    w4 [256], b4 [1]
Inputs are padded to 256 features (unused features are zero). Training
minimises the mean squared error of f against (l + A) / 100 with Adam.

Parity: the gradients are pinned by central finite differences
(tests/test_oracle_mlp.py); the Adam step is pinned against its published
update rule written out on scalars.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 256           # hidden width
F = 256           # padded input width
SIZES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
         ("w4", (H,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(seed: int, n_in: int = 230) -> np.ndarray:
    """He-style initialisation; rows of W1 beyond the n_in used inputs are zero."""
    rng = np.random.default_rng(seed)
    p = {}
    p["W1"] = rng.standard_normal((F, H)) * math.sqrt(2.0 / n_in)
    p["W1"][n_in:] = 0.0
    p["b1"] = np.zeros(H)
    p["W2"] = rng.standard_normal((H, H)) * math.sqrt(2.0 / H)
    p["b2"] = np.zeros(H)
    p["W3"] = rng.standard_normal((H, H)) * math.sqrt(2.0 / H)
    p["b3"] = np.zeros(H)
    p["w4"] = rng.standard_normal(H) * math.sqrt(1.0 / H)
    p["b4"] = np.zeros(1)
    return pack(p)


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    # d/du [u Phi(u)] = Phi(u) + u phi(u)
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def forward(theta: np.ndarray, X: np.ndarray):
    """Network output f [n] and the cache for the backward pass."""
    p = unpack(theta)
    Z1 = X @ p["W1"] + p["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = gelu(Z2)
    Z3 = H2 @ p["W3"] + p["b3"]
    H3 = gelu(Z3)
    y = H3 @ p["w4"] + p["b4"][0]
    return y, (X, Z1, H1, Z2, H2, Z3, H3)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, y: np.ndarray):
    """Mean squared error and its gradient with respect to theta (reverse mode)."""
    p = unpack(theta)
    f, (X, Z1, H1, Z2, H2, Z3, H3) = forward(theta, X)
    n = X.shape[0]
    r = f - y
    loss = float(np.mean(r * r))
    df = 2.0 * r / n
    g = {}
    g["w4"] = H3.T @ df
    g["b4"] = np.array([df.sum()])
    dZ3 = np.outer(df, p["w4"]) * gelu_grad(Z3)
    g["W3"] = H2.T @ dZ3
    g["b3"] = dZ3.sum(0)
    dZ2 = (dZ3 @ p["W3"].T) * gelu_grad(Z2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ p["W2"].T) * gelu_grad(Z1)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(0)
    return loss, pack(g)


def adam_step(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v
