"""Fit the polynomial p(f) ~ 2^f on [-1/2, 1/2] used by exp2_neg() in kernels.h.

Least squares on the relative error over a dense Chebyshev grid, in float64,
with p(0) = 1 held exact. The coefficients are then rounded to binary32 one at
a time, lowest order first, refitting the higher ones after each rounding, so
that the rounding of a coefficient is absorbed by the ones above it.
Prints the coefficients and the relative error of the binary32 polynomial.
"""
import numpy as np

DEG = 6


def fit(fixed):
    # relative-error least squares: minimise sum ((p(f) - 2^f) / 2^f)^2
    k0 = len(fixed)
    x = 0.5 * np.cos(np.pi * (np.arange(4000) + 0.5) / 4000)
    y = 2.0 ** x
    rhs = y - sum(c * x**i for i, c in enumerate(fixed))
    A = np.stack([x**i for i in range(k0, DEG + 1)], axis=1)
    wgt = 1.0 / y
    sol, *_ = np.linalg.lstsq(A * wgt[:, None], rhs * wgt, rcond=None)
    return list(fixed) + list(sol)


coef = [1.0]
for k in range(1, DEG + 1):
    c = fit(coef)
    coef.append(float(np.float32(c[k])))
x = np.linspace(-0.5, 0.5, 200001)
p = np.zeros_like(x)
for c in reversed(coef):
    p = p * x + c
rel = np.abs(p / 2.0**x - 1.0)
for i, c in enumerate(coef):
    print(f"c{i} = {np.float32(c).hex() if False else repr(np.float32(c))}  ({float(np.float32(c)).hex()})")
print("max relative error of the binary32-coefficient polynomial (exact arithmetic):", rel.max())
