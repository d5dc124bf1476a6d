"""Numpy emulation of the narrow floating-point formats the surrogate kernels use.

bfloat16: the upper 16 bits of binary32, rounded to nearest, ties to even.
E4M3 (OCP 8-bit floating point, "FN" variant): 1 sign, 4 exponent (bias 7),
3 mantissa bits; subnormals m 2^-9; largest finite 448 (S.1111.110);
S.1111.111 is NaN and there is no infinity. Rounding to nearest, ties to the
code with an even mantissa.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """binary32 -> bfloat16 (RNE) -> binary32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def e4m3_values() -> np.ndarray:
    """Value of each of the 256 codes (NaN for the two NaN codes)."""
    v = np.empty(256, np.float64)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e = (c >> 3) & 0xF
        m = c & 7
        if e == 15 and m == 7:
            v[c] = np.nan
        elif e == 0:
            v[c] = s * m * 2.0 ** -9
        else:
            v[c] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return v


_POS = None


def e4m3_round(x) -> np.ndarray:
    """binary32 values (|x| <= 448, finite) -> nearest E4M3 value, ties to even mantissa."""
    global _POS
    if _POS is None:
        _POS = e4m3_values()[:127]   # codes 0x00 .. 0x7E, increasing
    a = np.abs(np.asarray(x, dtype=np.float64))
    assert np.all(a <= 448.0), "values beyond the largest finite E4M3 are not emulated"
    i = np.searchsorted(_POS, a, side="left")           # _POS[i-1] < a <= _POS[i]
    i = np.clip(i, 1, 126)
    lo, hi = _POS[i - 1], _POS[i]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & (i % 2 == 0))
    code = np.where(a <= _POS[0], 0, np.where(pick_hi, i, i - 1))
    out = _POS[code]
    return np.where(np.asarray(x) < 0, -out, out)
