"""Seeded synthetic inputs: workload presets, truth trajectories and microscopy-like frames.

This module is the only code that the oracle side and the GPU side both use. It
holds none of the filter's arithmetic: it simulates the "microscope" that the
filter observes (the paper's synthetic sequences, Sec. 5.3, are not available,
so these stand in for them) and builds the initial particle sets.

Data-generating process (the readings are listed in the design notes):
  * truth follows nearly-constant-velocity motion (Sec. 5.1) with position noise
    0.5 px and velocity noise 0.1 px per frame; its intensity stays constant;
  * the start is placed so that the nominal straight path is centred on a chosen
    mid-point; heading uniform on [0, 2 pi), speed uniform in a preset range;
  * a pixel's expected value is I_bg + I0 times the Gaussian PSF averaged over
    the pixel's area (closed form with erf, i.e. the limit of infinitely many
    sub-samples); the observed value is a Poisson draw of it, stored as float32.
All randomness comes from numpy's PCG64 seeded by the caller.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np
from scipy.special import erf


@dataclass
class Workload:
    name: str
    dim: int = 2                  # spatial dimension (2 or 3)
    H: int = 64
    W: int = 64
    K: int = 20                   # frames
    T: int = 1                    # targets
    n: tuple = (10_000,)          # particles per target (or a rule, see n_rule)
    n_rule: str = "fixed"         # "fixed" | "loguniform" (floor(10**U[lo, hi]))
    n_lo: float = 3.0
    n_hi: float = 5.0
    m: tuple = (2, 2, 1)          # bins per pixel along x, y, z
    patch: int = 11
    quad: int = 2
    sigma_psf: float = 1.5
    astig_gamma: float = 2.0
    astig_d: float = 4.0
    i_bg: float = 10.0
    i0: tuple = (50.0, 50.0)      # truth intensity range (uniform)
    sigma_xi: float = 10.0
    proc_sigma: tuple = (0.5, 0.5, 0.1, 0.1, 2.0)
    speed: tuple = (1.0, 2.0)
    mid_lo: float | None = None   # truth mid-points uniform in [mid_lo, mid_hi]^2 (None: frame centre)
    mid_hi: float | None = None
    z_range: tuple = (-2.0, 2.0)  # 3D: truth depth range
    vz_range: tuple = (-0.1, 0.1)
    per_target_frames: bool = False
    truth_sigma_pos: float = 0.5
    truth_sigma_v: float = 0.1
    seed: int = 1000

    @property
    def D(self) -> int:
        return 2 * self.dim + 1

    def counts(self) -> np.ndarray:
        if self.n_rule == "fixed":
            n = np.asarray(self.n, dtype=np.int64)
            if n.size == 1 and self.T > 1:
                n = np.full(self.T, int(n[0]), dtype=np.int64)
            return n
        rng = np.random.Generator(np.random.PCG64(self.seed + 7))
        return np.floor(10.0 ** rng.uniform(self.n_lo, self.n_hi, size=self.T)).astype(np.int64)


# Peak intensity above a background of 10 at SNR 2, with the Poisson SNR read
# as I0 / sqrt(I0 + I_bg): I0 = 2 + sqrt(4 + 4 I_bg).
SNR2_I0 = 2.0 + math.sqrt(44.0)


def preset(name: str, **kw) -> Workload:
    """Named workloads. 'single-2d-64' .. '3d-astig' follow the configurations the
    benchmark is quoted on; 'tiny' is a fast case for tests."""
    p = {
        "tiny": Workload(name="tiny", H=48, W=48, K=4, n=(3000,), patch=11, quad=2, speed=(1.0, 2.0)),
        "single-2d-64": Workload(name="single-2d-64", H=64, W=64, K=20, n=(10_000,), m=(2, 2, 1),
                                 patch=11, quad=2, speed=(1.0, 2.0)),
        "single-2d-512": Workload(name="single-2d-512", H=512, W=512, K=100, n=(1_000_000,), m=(2, 2, 1),
                                  patch=15, quad=8, speed=(2.0, 4.0)),
        "batched-2d-1024": Workload(name="batched-2d-1024", H=1024, W=1024, K=50, T=1000, n_rule="loguniform",
                                    n_lo=3.0, n_hi=5.0, m=(2, 2, 1), patch=15, quad=8, i0=(20.0, 100.0),
                                    speed=(2.0, 4.0), mid_lo=100.0, mid_hi=924.0),
        # surrogate training data: 512x512 frames (the single-target workload's
        # frame size, PSF, window and quadrature) holding spots at the batched
        # workload's density (250 in the central 412^2), intensities U[20, 100]
        "train-2d-512": Workload(name="train-2d-512", H=512, W=512, K=60, T=250, n_rule="loguniform", n_lo=3.0,
                                 n_hi=4.0, m=(2, 2, 1), patch=15, quad=8, i0=(20.0, 100.0), speed=(2.0, 4.0),
                                 mid_lo=50.0, mid_hi=462.0, seed=7000),
        "train-3d": Workload(name="train-3d", dim=3, H=256, W=256, K=20, T=40, n=(50_000,), m=(4, 4, 4), patch=15,
                             quad=8, i0=(20.0, 100.0), speed=(2.0, 4.0),
                             proc_sigma=(0.5, 0.5, 0.5, 0.1, 0.1, 0.1, 2.0), per_target_frames=True, seed=8000),
        # large objects (Sec. 5): sigma_PSF = 13, a 65 x 65 likelihood support,
        # speeds U[2, 7], SNR 2 (peak I0 with I0 / sqrt(I0 + I_bg) = 2), 12 800
        # particles per sequence; sigma_xi = 30 as for the large-object kernels
        # of the likelihood figure; the pixel value is point-sampled (q = 1)
        "large-2d-512": Workload(name="large-2d-512", H=512, W=512, K=50, n=(12_800,), m=(1, 1, 1), patch=65,
                                 quad=1, sigma_psf=13.0, i_bg=10.0, i0=(SNR2_I0, SNR2_I0), sigma_xi=30.0,
                                 speed=(2.0, 7.0), mid_lo=128.0, mid_hi=384.0),
        "3d-astig": Workload(name="3d-astig", dim=3, H=256, W=256, K=20, T=200, n=(50_000,), m=(4, 4, 4),
                             patch=15, quad=8, i0=(20.0, 100.0), speed=(2.0, 4.0),
                             proc_sigma=(0.5, 0.5, 0.5, 0.1, 0.1, 0.1, 2.0), per_target_frames=True),
    }[name]
    return replace(p, **kw) if kw else p


def truth(w: Workload, seed: int | None = None) -> np.ndarray:
    """Truth states for frames 0..K: array [K+1, T, D] float64."""
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    T, D, dim, K = w.T, w.D, w.dim, w.K
    out = np.zeros((K + 1, T, D), np.float64)
    head = rng.uniform(0.0, 2.0 * math.pi, size=T)
    speed = rng.uniform(w.speed[0], w.speed[1], size=T)
    if w.mid_lo is None:
        mid = np.tile(np.array([(w.W - 1) / 2.0, (w.H - 1) / 2.0]), (T, 1))
    else:
        mid = rng.uniform(w.mid_lo, w.mid_hi, size=(T, 2))
    vx, vy = speed * np.cos(head), speed * np.sin(head)
    out[0, :, 0] = mid[:, 0] - 0.5 * K * vx
    out[0, :, 1] = mid[:, 1] - 0.5 * K * vy
    out[0, :, dim + 0] = vx
    out[0, :, dim + 1] = vy
    if dim == 3:
        out[0, :, 2] = rng.uniform(w.z_range[0], w.z_range[1], size=T)
        out[0, :, 5] = rng.uniform(w.vz_range[0], w.vz_range[1], size=T)
    out[0, :, 2 * dim] = rng.uniform(w.i0[0], w.i0[1], size=T)
    for k in range(1, K + 1):
        prev = out[k - 1]
        cur = prev.copy()
        cur[:, :dim] = prev[:, :dim] + prev[:, dim:2 * dim] + w.truth_sigma_pos * rng.standard_normal((T, dim))
        cur[:, dim:2 * dim] = prev[:, dim:2 * dim] + w.truth_sigma_v * rng.standard_normal((T, dim))
        if dim == 3:  # keep the truth depth inside the modelled range
            cur[:, 2] = np.clip(cur[:, 2], w.z_range[0] - 1.0, w.z_range[1] + 1.0)
        out[k] = cur
    return out


def _pixel_avg(centres: np.ndarray, pos: float, sigma: float) -> np.ndarray:
    """Average of exp(-(u-pos)^2 / 2 sigma^2) over [c - 1/2, c + 1/2] (closed form)."""
    s = sigma * math.sqrt(2.0)
    return (sigma * math.sqrt(math.pi / 2.0)) * (erf((centres + 0.5 - pos) / s) - erf((centres - 0.5 - pos) / s))


def _sigmas(w: Workload, z: float) -> tuple:
    if w.dim == 3:
        ax = (z - w.astig_gamma) / w.astig_d
        ay = (z + w.astig_gamma) / w.astig_d
        return w.sigma_psf * math.sqrt(1 + ax * ax), w.sigma_psf * math.sqrt(1 + ay * ay)
    return w.sigma_psf, w.sigma_psf


def expected_image(w: Workload, states: np.ndarray, H: int, W: int) -> np.ndarray:
    """Noise-free image of the given truth states [T, D] (sum of spots over the background)."""
    img = np.full((H, W), w.i_bg, np.float64)
    dim = w.dim
    for st in states:
        x, y, i0 = st[0], st[1], st[2 * dim]
        sx, sy = _sigmas(w, st[2] if dim == 3 else 0.0)
        rad = int(math.ceil(7 * max(sx, sy))) + 2
        c_lo, c_hi = max(0, int(math.floor(x)) - rad), min(W, int(math.floor(x)) + rad + 1)
        r_lo, r_hi = max(0, int(math.floor(y)) - rad), min(H, int(math.floor(y)) + rad + 1)
        if c_lo >= c_hi or r_lo >= r_hi:
            continue
        ax = _pixel_avg(np.arange(c_lo, c_hi, dtype=np.float64), x, sx)
        ay = _pixel_avg(np.arange(r_lo, r_hi, dtype=np.float64), y, sy)
        img[r_lo:r_hi, c_lo:c_hi] += i0 * np.outer(ay, ax)
    return img


def frames(w: Workload, tr: np.ndarray, seed: int | None = None, noise: bool = True) -> np.ndarray:
    """Frames for k = 1..K. Shared frame: [K, H, W]; per-target regions: [K, T, H, W]."""
    rng = np.random.Generator(np.random.PCG64((w.seed if seed is None else seed) + 1))
    K = tr.shape[0] - 1
    if w.per_target_frames:
        out = np.zeros((K, w.T, w.H, w.W), np.float32)
        for k in range(1, K + 1):
            for t in range(w.T):
                mu = expected_image(w, tr[k, t:t + 1], w.H, w.W)
                out[k - 1, t] = rng.poisson(mu) if noise else mu
        return out
    out = np.zeros((K, w.H, w.W), np.float32)
    for k in range(1, K + 1):
        mu = expected_image(w, tr[k], w.H, w.W)
        out[k - 1] = rng.poisson(mu) if noise else mu
    return out


def initial_particles(w: Workload, tr0: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """All particles of target t at its truth state at frame 0: SoA [D, sum(counts)] float32."""
    D = w.D
    total = int(np.sum(counts))
    out = np.zeros((D, total), np.float32)
    off = 0
    for t, n in enumerate(counts):
        out[:, off:off + int(n)] = tr0[t].astype(np.float32)[:, None]
        off += int(n)
    return out


def random_cloud(w: Workload, centre: np.ndarray, n: int, spread: float, seed: int) -> np.ndarray:
    """A particle cloud [D, n] float32 around a state: positions ~ N(centre, spread^2),
    velocities ~ N(v, 0.3^2), intensity ~ N(I0, 3^2). For stage-level tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D, dim = w.D, w.dim
    out = np.empty((D, n), np.float64)
    for d in range(D):
        sd = spread if d < dim else (0.3 if d < 2 * dim else 3.0)
        out[d] = centre[d] + sd * rng.standard_normal(n)
    return out.astype(np.float32)


def rmse(est: np.ndarray, tr: np.ndarray, dim: int) -> np.ndarray:
    """Per-target tracking RMSE over frames 1..K of the positions: est [K, T, D], truth [K+1, T, D]."""
    d = est[:, :, :dim] - tr[1:, :, :dim]
    return np.sqrt(np.mean(np.sum(d * d, axis=2), axis=0))


# ---------------------------------------------------------------- pseudo-tracking
# Sec. 5.5's convergence experiment: the prior p(x_k | Z^{k-1}) is fixed (a
# uniform square of 3 or 5 pixels, or an isotropic Gaussian of sigma 0.5 or
# 0.8 px), the object is one spot of sigma_PSF = 1.16 at SNR 2, and the
# likelihood has sigma_xi = 20. Readings: the prior is centred on the object;
# one noisy frame is drawn and kept, and the repetitions differ in the particle
# draws only, so the RMSE over repetitions measures the estimator's error
# against the exact posterior mean of that frame.
PSEUDO_PRIORS = (("uniform", 3.0), ("uniform", 5.0), ("gauss", 0.5), ("gauss", 0.8))


def pseudo_workload(reps: int, n: int, m: int = 1) -> Workload:
    """Model constants of the pseudo-tracking experiment: `reps` repetitions of
    n particles as targets sharing one 32 x 32 frame; no motion (velocity 0 and
    no process noise, so a step weighs the prior draws as they are)."""
    return Workload(name="pseudo-2d-32", H=32, W=32, K=1, T=reps, n=(n,), m=(m, m, 1), patch=9, quad=2,
                    sigma_psf=1.16, i_bg=10.0, i0=(SNR2_I0, SNR2_I0), sigma_xi=20.0,
                    proc_sigma=(0.0, 0.0, 0.0, 0.0, 0.0))


def pseudo_frame(seed: int = 11) -> tuple:
    """(frame [32, 32] float32, object position (x, y)): the object uniformly
    placed in the central pixel's area, Poisson noise."""
    w = pseudo_workload(1, 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    xy = np.array([15.0, 15.0]) + rng.uniform(-0.5, 0.5, 2)
    st = np.array([[xy[0], xy[1], 0.0, 0.0, w.i0[0]]])
    mu = expected_image(w, st, w.H, w.W)
    return rng.poisson(mu).astype(np.float32), xy


def pseudo_particles(kind: str, par: float, centre, reps: int, n: int, seed: int) -> np.ndarray:
    """Prior draws [5, reps * n] float32 (repetition after repetition): positions
    uniform on the par x par square or Gaussian with sigma par around centre,
    velocity 0, intensity the object's."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = reps * n
    out = np.zeros((5, N), np.float64)
    for a in range(2):
        if kind == "uniform":
            out[a] = centre[a] + rng.uniform(-par / 2.0, par / 2.0, N)
        else:
            out[a] = centre[a] + par * rng.standard_normal(N)
    out[4] = SNR2_I0
    return out.astype(np.float32)
