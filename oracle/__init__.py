"""FP64 CPU oracle of the SIR and pcSIR filter steps — TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (``paper_1310_5541_amd``)
never imports it and shares no code with it.

This module is a thin ctypes loader around ``liboracle.so`` (built from
``pcsir_oracle.cpp`` by :func:`build`). Each function names the passage of the
paper it follows in the C source. Parity pins live in ``tests/test_oracle_*.py``;
the tracking-RMSE level is "parity unpinned" (no data from the paper).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcsir_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile the oracle with g++ (plain -O2, IEEE semantics, no fast-math;
    OpenMP only for the loop over independent targets in orc_track)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-o", _LIB_PATH + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Model(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("m", C.c_int32 * 3), ("patch", C.c_int32), ("quad", C.c_int32),
        ("psf", C.c_int32), ("dummy_mode", C.c_int32),
        ("sigma_psf", C.c_double), ("astig_gamma", C.c_double), ("astig_d", C.c_double),
        ("i_bg", C.c_double), ("sigma_xi", C.c_double), ("proc_sigma", C.c_double * 7),
        ("seed", C.c_uint64),
    ]


class _WeighOut(C.Structure):
    _fields_ = [
        ("keys", C.c_void_p), ("bin_of", C.c_void_p), ("bin_key", C.c_void_p), ("bin_n", C.c_void_p),
        ("bin_mean", C.c_void_p), ("ll", C.c_void_p), ("w", C.c_void_p), ("scal", C.c_void_p),
        ("est", C.c_void_p),
    ]


@dataclass
class Model:
    """Model parameters of the oracle (same meaning as the library's config)."""
    dim: int = 2
    m: tuple = (2, 2, 1)
    patch: int = 11
    quad: int = 2
    psf: int = 0
    dummy_mode: int = 0
    sigma_psf: float = 1.5
    astig_gamma: float = 2.0
    astig_d: float = 4.0
    i_bg: float = 10.0
    sigma_xi: float = 10.0
    proc_sigma: tuple = (0.5, 0.5, 0.1, 0.1, 2.0)
    seed: int = 1

    @property
    def D(self) -> int:
        return 2 * self.dim + 1

    def _c(self) -> _Model:
        s = _Model()
        s.dim = self.dim
        m = list(self.m) + [1] * (3 - len(self.m))
        for a in range(3):
            s.m[a] = int(m[a])
        s.patch, s.quad, s.psf, s.dummy_mode = self.patch, self.quad, self.psf, self.dummy_mode
        s.sigma_psf, s.astig_gamma, s.astig_d = self.sigma_psf, self.astig_gamma, self.astig_d
        s.i_bg, s.sigma_xi = self.i_bg, self.sigma_xi
        ps = list(self.proc_sigma) + [0.0] * (7 - len(self.proc_sigma))
        for d in range(7):
            s.proc_sigma[d] = float(ps[d])
        s.seed = int(self.seed) & (2**64 - 1)
        return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p]
        L.orc_resample_u.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_resample_u.restype = C.c_double
        L.orc_check_u.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_check_u.restype = C.c_double
        L.orc_bin_key.argtypes = [C.c_float, C.c_int32]
        L.orc_bin_key.restype = C.c_int32
        L.orc_propagate.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int64]
        L.orc_loglik.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                                 C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_loglik.restype = C.c_double
        L.orc_weigh.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_int32, C.c_void_p]
        L.orc_weigh.restype = C.c_int64
        L.orc_step_thr.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_int32), C.c_int64, C.c_int64, C.c_int32, C.c_double, C.c_void_p,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.orc_resample.argtypes = [C.c_int64, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_void_p,
                               C.c_int64, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_track.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_void_p,
                                C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_set_threads.restype = C.c_int32
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of :func:`track` (targets in parallel; 1 = one core). Returns the
    count in effect; n <= 0 only queries it."""
    return int(lib().orc_set_threads(int(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: four 32-bit counter words, two key words."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c), _p(k), _p(out))
    return out


def uniform(word: int) -> float:
    return lib().orc_uniform(C.c_uint32(int(word)))


def normals(seed: int, i: int, k: int, t: int) -> np.ndarray:
    z = np.zeros(8, dtype=np.float64)
    lib().orc_normals(seed, i, k, t, _p(z))
    return z


def resample_u(seed: int, k: int, t: int) -> float:
    return lib().orc_resample_u(seed, k, t)


def check_u(seed: int, dummy: int, k: int, t: int) -> float:
    return lib().orc_check_u(seed, dummy, k, t)


def bin_key(x, m: int) -> np.ndarray:
    xs = np.asarray(x, dtype=np.float32).ravel()
    f = lib().orc_bin_key
    return np.array([f(C.c_float(float(v)), m) for v in xs], dtype=np.int32)


def propagate(model: Model, state: np.ndarray, k: int, t: int = 0) -> np.ndarray:
    s = np.ascontiguousarray(state, dtype=np.float32).copy()
    D, N = s.shape
    assert D == model.D
    mc = model._c()
    lib().orc_propagate(C.byref(mc), N, _p(s), k, t)
    return s


def loglik(model: Model, frame: np.ndarray, c0: int, r0: int, x: float, y: float, z: float, I0: float) -> float:
    fr = np.ascontiguousarray(frame, dtype=np.float32)
    H, W = fr.shape
    mc = model._c()
    return lib().orc_loglik(C.byref(mc), _p(fr), H, W, int(c0), int(r0), float(x), float(y), float(z), float(I0))


def weigh(model: Model, frame: np.ndarray, state: np.ndarray, sir: bool, logw_prev=None) -> dict:
    """Weighting stage of one target; returns keys, bins, likelihoods, weights, N_eff, estimate."""
    fr = np.ascontiguousarray(frame, dtype=np.float32)
    H, W = fr.shape
    s = np.ascontiguousarray(state, dtype=np.float32)
    D, N = s.shape
    keys = np.zeros((3, N), np.int32)
    bin_of = np.zeros(N, np.int64)
    bin_key = np.zeros((3, N), np.int32)
    bin_n = np.zeros(N, np.int64)
    bin_mean = np.zeros((D, N), np.float64)
    ll = np.zeros(N, np.float64)
    w = np.zeros(N, np.float64)
    scal = np.zeros(3, np.float64)
    est = np.zeros(D, np.float64)
    o = _WeighOut(_p(keys).value, _p(bin_of).value, _p(bin_key).value, _p(bin_n).value,
                  _p(bin_mean).value, _p(ll).value, _p(w).value, _p(scal).value, _p(est).value)
    lp = None
    if logw_prev is not None:
        lp = np.ascontiguousarray(logw_prev, dtype=np.float64)
    mc = model._c()
    B = lib().orc_weigh(C.byref(mc), _p(fr), H, W, N, _p(s), _p(lp) if lp is not None else None,
                        1 if sir else 0, C.byref(o))
    return dict(keys=keys, bin_of=bin_of, B=B, bin_key=bin_key[:, :B].copy(), bin_n=bin_n[:B].copy(),
                bin_mean=bin_mean[:, :B].copy(), ll=ll[:B].copy(), w=w, M=scal[0], S=scal[1],
                neff=scal[2], est=est)


def resample(w: np.ndarray, u: float):
    ww = np.ascontiguousarray(w, dtype=np.float64)
    N = ww.shape[0]
    cdf = np.zeros(N, np.float64)
    s = np.zeros(N, np.int64)
    lib().orc_resample(N, _p(ww), float(u), _p(cdf), _p(s))
    return cdf, s


def step(model: Model, frame: np.ndarray, state: np.ndarray, k: int, t: int = 0, sir: bool = False):
    fr = np.ascontiguousarray(frame, dtype=np.float32)
    H, W = fr.shape
    s = np.ascontiguousarray(state, dtype=np.float32).copy()
    D, N = s.shape
    est = np.zeros(D, np.float64)
    neff = np.zeros(1, np.float64)
    mc = model._c()
    lib().orc_step(C.byref(mc), _p(fr), H, W, N, _p(s), k, t, 1 if sir else 0, _p(est), _p(neff))
    return s, est, float(neff[0])


def step_thr(model: Model, frame: np.ndarray, state: np.ndarray, logw, uniform: bool, k: int, t: int = 0,
             sir: bool = False, neff_frac: float = float("inf")):
    """One step with a resampling threshold (orc_step_thr). Returns
    (state, logw, uniform, est [D], neff, resampled)."""
    fr = np.ascontiguousarray(frame, dtype=np.float32)
    H, W = fr.shape
    s = np.ascontiguousarray(state, dtype=np.float32).copy()
    D, N = s.shape
    lw = np.ascontiguousarray(np.zeros(N) if logw is None else logw, dtype=np.float64).copy()
    uni = C.c_int32(1 if uniform else 0)
    est = np.zeros(D, np.float64)
    neff = C.c_double(0.0)
    res = C.c_int32(0)
    mc = model._c()
    lib().orc_step_thr(C.byref(mc), _p(fr), H, W, N, _p(s), _p(lw), C.byref(uni), int(k), int(t), 1 if sir else 0,
                       float(neff_frac), _p(est), C.byref(neff), C.byref(res))
    return s, lw, bool(uni.value), est, float(neff.value), bool(res.value)


def track(model: Model, frames: np.ndarray, n_per_target, state: np.ndarray, k0: int = 1,
          sir: bool = False, per_target: bool = False):
    """Run frames k0..k0+K-1 over all targets; returns (state, est [K,T,D], neff [K,T])."""
    fr = np.ascontiguousarray(frames, dtype=np.float32)
    n = np.ascontiguousarray(n_per_target, dtype=np.int64)
    T = n.shape[0]
    if per_target:
        K, T2, H, W = fr.shape
        assert T2 == T
    else:
        K, H, W = fr.shape
    s = np.ascontiguousarray(state, dtype=np.float32).copy()
    D = s.shape[0]
    est = np.zeros((K, T, D), np.float64)
    neff = np.zeros((K, T), np.float64)
    mc = model._c()
    lib().orc_track(C.byref(mc), _p(fr), H, W, 1 if per_target else 0, T, _p(n), _p(s), k0, K,
                    1 if sir else 0, _p(est), _p(neff))
    return s, est, neff


def posterior_mean(model: Model, frame: np.ndarray, kind: str, par: float, centre, I0: float,
                   delta: float = 1.0 / 32) -> np.ndarray:
    """Exact posterior mean of the position (x, y) for a fixed prior, the
    reference of Sec. 5.5's convergence experiment: the integral of
    x prior(x) p(z | x) over the integral of prior(x) p(z | x), with p(z | x)
    the Eq. likelihood at intensity I0 (velocity 0).

    Midpoint quadrature on square cells of side delta (1 / delta an integer)
    aligned with the pixel edges, where the likelihood's window changes, so it
    is smooth inside every cell. Each cell carries the prior's exact mass in it:
    the overlap with the par x par square ("uniform") or the product of normal
    CDF differences ("gauss", sigma par, cells out to 6 sigma). The weighting
    itself is the oracle's SIR weighting of the cell midpoints with those
    masses as previous weights."""
    from scipy.special import ndtr
    c = np.asarray(centre, np.float64)
    half = par / 2.0 if kind == "uniform" else 6.0 * par
    lo = np.floor(c - half + 0.5) - 0.5
    hi = np.ceil(c + half - 0.5) + 0.5
    axes, masses = [], []
    for a in range(2):
        n = int(round((hi[a] - lo[a]) / delta))
        e0 = lo[a] + np.arange(n) * delta
        e1 = e0 + delta
        if kind == "uniform":
            m = np.clip(np.minimum(e1, c[a] + half) - np.maximum(e0, c[a] - half), 0.0, None) / par
        else:
            m = ndtr((e1 - c[a]) / par) - ndtr((e0 - c[a]) / par)
        keep = m > 0.0
        axes.append((e0 + 0.5 * delta)[keep])
        masses.append(m[keep])
    X, Y = np.meshgrid(axes[0], axes[1])
    P = np.outer(masses[1], masses[0]).ravel()
    st = np.zeros((model.D, P.size), np.float32)
    st[0] = X.ravel()
    st[1] = Y.ravel()
    st[model.D - 1] = I0
    r = weigh(model, frame, st, sir=True, logw_prev=np.log(P))
    return r["est"][:2]


def adaptive_bins(state: np.ndarray, dim: int, bins_per_sigma: float, bins_max: int):
    """Cells per pixel of one target with adaptive bins. The paper names
    adaptive bin sizes as future work without a rule; the rule here: per
    spatial axis, m = ceil(bins_per_sigma / sd) clamped to [1, bins_max]
    (bins_max when sd = 0), sd the population standard deviation of the
    target's positions, S2/n - (S1/n)^2 in binary64 with each sum correctly
    rounded, positions taken through the clamp of the cell index (NaN -> 2^24,
    then into [-2^24, 2^24]). Returns (m [3] with 1 for unused axes, variances [dim])."""
    m = [1, 1, 1]
    var = []
    for a in range(dim):
        x = np.asarray(state[a], dtype=np.float32).astype(np.float64)
        x = np.where(np.isnan(x), 2.0 ** 24, np.clip(x, -(2.0 ** 24), 2.0 ** 24))
        n = x.size
        s1 = math.fsum(x.tolist())
        s2 = math.fsum((x * x).tolist())   # squares of binary32 values are exact in binary64
        mean = s1 / n
        v = max(s2 / n - mean * mean, 0.0)
        var.append(v)
        sd = math.sqrt(v)
        q = bins_per_sigma / sd if sd > 0.0 else math.inf
        m[a] = int(bins_max) if not q < bins_max else max(1, int(math.ceil(q)))
    return tuple(m), var
