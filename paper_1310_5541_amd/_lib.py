"""ctypes binding of ``libpcsir.so`` (the C ABI declared in include/pcsir.h).

Names follow the C ABI. Device memory comes from torch (``torch.empty`` on the
current CUDA/HIP device) and work goes to torch's current stream; every step of
the filter runs in the library's kernels. If the library is not built the
binding raises :class:`LibraryMissing`: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libpcsir.so")

ABI_VERSION = 3

DUMP = dict(propagated=0, keys=1, counts=2, bin_target=3, bin_key=4, bin_n=5, bin_mean=6, loglik=7,
            weights=8, target=9, cdf=10, resample=11, logw=12, bins_per_px=13)

_STATUS = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_HIP", -4: "E_STATE", -5: "E_NUMERIC",
           -6: "E_UNSUPPORTED"}


class LibraryMissing(RuntimeError):
    pass


class PcsirError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pcsir {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Cfg(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("dim", C.c_int32), ("n_targets", C.c_int32),
        ("n_particles", C.POINTER(C.c_int64)), ("bins_per_px", C.c_int32 * 3), ("patch", C.c_int32),
        ("quad", C.c_int32), ("psf", C.c_int32), ("dummy_mode", C.c_int32), ("lik_mode", C.c_int32),
        ("per_target_frames", C.c_int32), ("frame_h", C.c_int32), ("frame_w", C.c_int32),
        ("sigma_psf", C.c_float), ("astig_gamma", C.c_float), ("astig_d", C.c_float), ("i_bg", C.c_float),
        ("sigma_xi", C.c_float), ("proc_sigma", C.c_float * 7), ("seed", C.c_uint64),
        ("neff_threshold", C.c_double), ("bins_per_sigma", C.c_double), ("bins_max", C.c_int32),
    ]


_lib = None


class Tuning(C.Structure):
    """Python mirror of ``pcsir_tuning`` (launch shapes; results do not depend on them)."""
    _fields_ = [("bin_tile", C.c_int32), ("list_blocks", C.c_int32), ("digit_bits", C.c_int32),
                ("grid_per_cu", C.c_int32), ("resample_light", C.c_int32),
                ("sort_bins", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def lib_path() -> str:
    return _LIB


def lib():
    """Load libpcsir.so (built by ``__graft_entry__.build()``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise LibraryMissing(f"{_LIB} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(_LIB)
    vp, i32, i64, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
    L.pcsir_workspace_bytes.argtypes = [C.POINTER(_Cfg)]
    L.pcsir_workspace_bytes.restype = sz
    L.pcsir_init.argtypes = [C.POINTER(_Cfg), vp, vp, sz, vp, C.POINTER(vp)]
    L.pcsir_step.argtypes = [vp, vp, i32, i32, i64]
    L.sir_step.argtypes = [vp, vp, i32, i32, i64]
    L.pcsir_estimate.argtypes = [vp, vp, vp]
    L.pcsir_destroy.argtypes = [vp]
    L.pcsir_last_error.argtypes = [vp]
    L.pcsir_last_error.restype = C.c_char_p
    L.pcsir_get_particles.argtypes = [vp, vp]
    L.pcsir_set_particles.argtypes = [vp, vp]
    L.pcsir_debug_dump.argtypes = [vp, i32, vp, sz]
    L.pcsir_set_debug.argtypes = [vp, i32]
    L.pcsir_set_graphs.argtypes = [vp, i32]
    L.pcsir_set_timing.argtypes = [vp, i32]
    L.pcsir_kernel_times.argtypes = [vp, C.POINTER(C.c_char_p), C.POINTER(C.c_float), i32, C.POINTER(i32)]
    L.pcsir_mlp_param_count.argtypes = []
    L.pcsir_mlp_param_count.restype = sz
    L.pcsir_mlp_train_bytes.argtypes = [i32]
    L.pcsir_mlp_train_bytes.restype = sz
    L.pcsir_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, i32, vp, sz, vp, vp, vp]
    L.pcsir_mlp_train_step_static.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, i32, vp, vp, vp]
    L.pcsir_mlp_train_step_fp8.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, i32, vp, vp, sz, vp, vp, vp]
    L.pcsir_mlp_forward_train_path.argtypes = [vp, vp, i32, vp, vp, sz, vp]
    L.pcsir_mlp_gemm_bf16.argtypes = [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, vp]
    L.pcsir_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.pcsir_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.pcsir_autotune.argtypes = [vp, vp, i32, i32, i64, i32, vp, C.POINTER(Tuning), C.POINTER(C.c_float),
                                 C.POINTER(i32)]
    L.pcsir_surr_bytes.argtypes = []
    L.pcsir_surr_bytes.restype = sz
    L.pcsir_surr_prepare.argtypes = [vp, vp, vp, sz, vp]
    L.pcsir_surr_rows.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.pcsir_set_surrogate.argtypes = [vp, vp, vp, C.c_float, C.c_float]
    L.pcsir_surrogate_features.argtypes = [vp, vp, vp, i32, C.POINTER(i32)]
    L.pcsir_surrogate_stats.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_float), i32]
    for f in ("pcsir_mlp_train_step", "pcsir_mlp_train_step_static", "pcsir_mlp_train_step_fp8",
              "pcsir_mlp_forward_train_path", "pcsir_mlp_gemm_bf16", "pcsir_surr_prepare",
              "pcsir_surr_rows", "pcsir_set_surrogate", "pcsir_surrogate_features", "pcsir_surrogate_stats",
              "pcsir_get_tuning", "pcsir_set_tuning", "pcsir_autotune"):
        getattr(L, f).restype = i32
    for f in ("pcsir_init", "pcsir_step", "sir_step", "pcsir_estimate", "pcsir_destroy", "pcsir_get_particles",
              "pcsir_set_particles", "pcsir_debug_dump", "pcsir_set_debug", "pcsir_set_graphs", "pcsir_set_timing",
              "pcsir_kernel_times"):
        getattr(L, f).restype = i32
    _lib = L
    return L


@dataclass
class Config:
    """Python mirror of ``pcsir_config`` (include/pcsir.h)."""
    n_particles: tuple
    dim: int = 2
    bins_per_px: tuple = (2, 2, 1)
    patch: int = 11
    quad: int = 2
    psf: int = 0
    dummy_mode: int = 0
    lik_mode: int = 0          # 0 DIRECT, 1 SEPARABLE, 2 surrogate BF16, 3 surrogate FP8
    per_target_frames: bool = False
    frame_h: int = 64
    frame_w: int = 64
    sigma_psf: float = 1.5
    astig_gamma: float = 2.0
    astig_d: float = 4.0
    i_bg: float = 10.0
    sigma_xi: float = 10.0
    proc_sigma: tuple = (0.5, 0.5, 0.1, 0.1, 2.0)
    seed: int = 1
    neff_threshold: float = float("inf")   # <= 1: resample only when N_eff < fraction * N
    bins_per_sigma: float = 0.0            # > 0: adaptive bins, about this many per standard deviation
    bins_max: int = 8                      # adaptive bins: largest cells per pixel

    @property
    def D(self) -> int:
        return 2 * self.dim + 1

    @property
    def T(self) -> int:
        return len(self.n_particles)

    @property
    def NT(self) -> int:
        return int(np.sum(np.asarray(self.n_particles, dtype=np.int64)))

    def _c(self):
        n = np.ascontiguousarray(np.asarray(self.n_particles, dtype=np.int64))
        c = _Cfg()
        c.abi_version = ABI_VERSION
        c.dim = self.dim
        c.n_targets = int(n.shape[0])
        c.n_particles = n.ctypes.data_as(C.POINTER(C.c_int64))
        m = list(self.bins_per_px) + [1] * (3 - len(self.bins_per_px))
        for a in range(3):
            c.bins_per_px[a] = int(m[a])
        c.patch, c.quad, c.psf, c.dummy_mode, c.lik_mode = self.patch, self.quad, self.psf, self.dummy_mode, self.lik_mode
        c.per_target_frames = 1 if self.per_target_frames else 0
        c.frame_h, c.frame_w = self.frame_h, self.frame_w
        c.sigma_psf, c.astig_gamma, c.astig_d = self.sigma_psf, self.astig_gamma, self.astig_d
        c.i_bg, c.sigma_xi = self.i_bg, self.sigma_xi
        ps = list(self.proc_sigma) + [0.0] * (7 - len(self.proc_sigma))
        for d in range(7):
            c.proc_sigma[d] = float(ps[d])
        c.seed = int(self.seed) & (2**64 - 1)
        c.neff_threshold = float(self.neff_threshold)
        c.bins_per_sigma = float(self.bins_per_sigma)
        c.bins_max = int(self.bins_max)
        return c, n  # keep n alive while c is used

    @classmethod
    def from_workload(cls, w, **kw) -> "Config":
        """Config for a ``synth.Workload`` (sizes and model constants only)."""
        base = dict(n_particles=tuple(int(v) for v in w.counts()), dim=w.dim, bins_per_px=tuple(w.m),
                    patch=w.patch, quad=w.quad, psf=1 if w.dim == 3 else 0, frame_h=w.H, frame_w=w.W,
                    per_target_frames=w.per_target_frames, sigma_psf=w.sigma_psf, astig_gamma=w.astig_gamma,
                    astig_d=w.astig_d, i_bg=w.i_bg, sigma_xi=w.sigma_xi, proc_sigma=tuple(w.proc_sigma))
        base.update(kw)
        return cls(**base)


class Filter:
    """One library context: T targets advanced by pcsir_step / sir_step."""

    def __init__(self, cfg: Config, init_state, stream=None):
        import torch
        self._torch = torch
        L = lib()
        self.cfg = cfg
        c, self._n = cfg._c()
        nbytes = L.pcsir_workspace_bytes(C.byref(c))
        if nbytes == 0:
            raise PcsirError(-1, "invalid config")
        assert init_state.is_cuda and init_state.dtype == torch.float32
        assert tuple(init_state.shape) == (cfg.D, cfg.NT), (tuple(init_state.shape), (cfg.D, cfg.NT))
        self.device = init_state.device
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        init = init_state.contiguous()
        ctx = C.c_void_p()
        st = L.pcsir_init(C.byref(c), C.c_void_p(init.data_ptr()), C.c_void_p(self.workspace.data_ptr()),
                          nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != 0:
            raise PcsirError(st, "pcsir_init failed (see stderr)")
        self._ctx = ctx
        self.workspace_bytes = int(nbytes)

    # -- helpers
    def _check(self, st: int):
        if st != 0:
            msg = lib().pcsir_last_error(self._ctx)
            raise PcsirError(st, msg.decode() if msg else "")

    def _frame(self, frame):
        t = self._torch
        assert frame.is_cuda and frame.dtype == t.float32 and frame.is_contiguous()
        H, W = self.cfg.frame_h, self.cfg.frame_w
        want = (self.cfg.T, H, W) if self.cfg.per_target_frames else (H, W)
        assert tuple(frame.shape) == want, (tuple(frame.shape), want)
        return C.c_void_p(frame.data_ptr()), H, W

    # -- C ABI
    def pcsir_step(self, frame, k: int):
        fp, H, W = self._frame(frame)
        self._check(lib().pcsir_step(self._ctx, fp, H, W, int(k)))

    def sir_step(self, frame, k: int):
        fp, H, W = self._frame(frame)
        self._check(lib().sir_step(self._ctx, fp, H, W, int(k)))

    def step(self, frame, k: int, sir: bool = False):
        (self.sir_step if sir else self.pcsir_step)(frame, k)

    def pcsir_estimate(self):
        T, D = self.cfg.T, self.cfg.D
        est = np.zeros((T, D), np.float64)
        neff = np.zeros(T, np.float64)
        self._check(lib().pcsir_estimate(self._ctx, est.ctypes.data_as(C.c_void_p), neff.ctypes.data_as(C.c_void_p)))
        return est, neff

    estimate = pcsir_estimate

    def get_particles(self):
        out = self._torch.empty((self.cfg.D, self.cfg.NT), dtype=self._torch.float32, device=self.device)
        self._check(lib().pcsir_get_particles(self._ctx, C.c_void_p(out.data_ptr())))
        return out

    def set_particles(self, state):
        s = state.contiguous()
        assert tuple(s.shape) == (self.cfg.D, self.cfg.NT) and s.dtype == self._torch.float32 and s.is_cuda
        self._check(lib().pcsir_set_particles(self._ctx, C.c_void_p(s.data_ptr())))
        self._hold = s

    def set_debug(self, on: bool = True):
        self._check(lib().pcsir_set_debug(self._ctx, 1 if on else 0))

    # -- launch shapes
    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib().pcsir_get_tuning(self._ctx, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{**self.get_tuning(), **kw})
        self._check(lib().pcsir_set_tuning(self._ctx, C.byref(t)))

    def autotune(self, frame, k: int, reps: int = 3):
        """Search the launch shapes on `frame` (pcsir_autotune); returns (tuning, ms per step, trials).
        The particles are left as they were."""
        fp, H, W = self._frame(frame)
        scratch = self._torch.empty((self.cfg.D, self.cfg.NT), dtype=self._torch.float32, device=self.device)
        best, ms, n = Tuning(), C.c_float(0.0), C.c_int32(0)
        self._check(lib().pcsir_autotune(self._ctx, fp, H, W, int(k), int(reps), _ptr(scratch), C.byref(best),
                                         C.byref(ms), C.byref(n)))
        self._hold = scratch
        return best.as_dict(), float(ms.value), int(n.value)

    # -- learned surrogate (lik_mode 2 / 3)
    def set_surrogate(self, params, act_scale=None, check_fraction: float = 0.01, tol_nats: float = 1.0):
        """Install surrogate weights (FP32 device vector) on a filter made with a surrogate lik_mode."""
        assert params.dtype == self._torch.float32 and params.is_cuda and params.numel() == mlp_param_count()
        sc = None if act_scale is None else (C.c_float * 3)(*[float(v) for v in act_scale])
        self._check(lib().pcsir_set_surrogate(self._ctx, _ptr(params.contiguous()), sc, float(check_fraction),
                                              float(tol_nats)))

    def surrogate_features(self, cap: int, X=None, y=None):
        """(X bf16 [n, 256], y fp32 [n], B) training rows from the dummies of the last pcsir_step,
        n = min(B, cap); written into X[:n], y[:n] when those are given (contiguous, >= cap rows)."""
        t = self._torch
        if X is None:
            X = t.empty((max(cap, 1), 256), dtype=t.bfloat16, device=self.device)
            y = t.empty(max(cap, 1), dtype=t.float32, device=self.device)
        assert X.dtype == t.bfloat16 and X.is_contiguous() and X.shape[0] >= cap and X.shape[1] == 256
        assert y.dtype == t.float32 and y.is_contiguous() and y.shape[0] >= cap
        cnt = C.c_int32(0)
        self._check(lib().pcsir_surrogate_features(self._ctx, _ptr(X), _ptr(y), int(cap), C.byref(cnt)))
        n = min(cnt.value, cap)
        return X[:n], y[:n], cnt.value

    def surrogate_stats(self, reset: bool = False):
        """(dummies checked, target-frames that fell back, largest |error| in nats), cumulative."""
        a, b, m = C.c_uint64(0), C.c_uint64(0), C.c_float(0.0)
        self._check(lib().pcsir_surrogate_stats(self._ctx, C.byref(a), C.byref(b), C.byref(m), 1 if reset else 0))
        return int(a.value), int(b.value), float(m.value)

    def dump(self, what: str):
        """Debug / parity view of the last step as a torch tensor (see PCSIR_DUMP_* in pcsir.h)."""
        t = self._torch
        NT, T, D = self.cfg.NT, self.cfg.T, self.cfg.D
        if what in ("bin_target", "bin_key", "bin_n", "bin_mean", "loglik"):
            B = int(self.dump("counts")[0].item())
        shapes = dict(propagated=((D, NT), t.float32), keys=((3, NT), t.int32), counts=((3,), t.int64),
                      weights=((NT,), t.float64), target=((T, 4), t.float64), cdf=((NT,), t.float64),
                      resample=((NT,), t.int32), logw=((NT,), t.float64), bins_per_px=((T, 3), t.int32))
        if what in shapes:
            shape, dt = shapes[what]
        elif what == "bin_target":
            shape, dt = (B,), t.int32
        elif what == "bin_key":
            shape, dt = (3, B), t.int32
        elif what == "bin_n":
            shape, dt = (B,), t.int64
        elif what == "bin_mean":
            shape, dt = (D, B), t.float64
        elif what == "loglik":
            shape, dt = (B,), t.float64
        else:
            raise KeyError(what)
        out = t.zeros(shape, dtype=dt, device=self.device)
        nbytes = out.numel() * out.element_size()
        self._check(lib().pcsir_debug_dump(self._ctx, DUMP[what], C.c_void_p(out.data_ptr()), max(nbytes, 1)))
        self.stream.synchronize()
        return out

    def set_graphs(self, on: bool = True):
        self._check(lib().pcsir_set_graphs(self._ctx, 1 if on else 0))

    def set_timing(self, on: bool = True):
        self._check(lib().pcsir_set_timing(self._ctx, 1 if on else 0))

    def kernel_times(self):
        cap = 8192
        names = (C.c_char_p * cap)()
        ms = (C.c_float * cap)()
        n = C.c_int32()
        self._check(lib().pcsir_kernel_times(self._ctx, names, ms, cap, C.byref(n)))
        return [(names[i].decode(), float(ms[i])) for i in range(n.value)]

    def close(self):
        if getattr(self, "_ctx", None):
            st = lib().pcsir_destroy(self._ctx)
            self._ctx = None
            if st not in (0, -5):
                raise PcsirError(st, "pcsir_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- surrogate network
def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device=None):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def mlp_param_count() -> int:
    return int(lib().pcsir_mlp_param_count())


def gemm_bf16(A, B, a_trans: bool = False, b_trans: bool = False):
    """C = op(A) op(B) with the library's BF16 MFMA GEMM (tests)."""
    import torch
    assert A.dtype == torch.bfloat16 and B.dtype == torch.bfloat16 and A.is_contiguous() and B.is_contiguous()
    M = A.shape[1] if a_trans else A.shape[0]
    K = A.shape[0] if a_trans else A.shape[1]
    N = B.shape[0] if b_trans else B.shape[1]
    assert (B.shape[1] if b_trans else B.shape[0]) == K
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    st = lib().pcsir_mlp_gemm_bf16(M, N, K, _ptr(A), A.shape[1], 1 if a_trans else 0, _ptr(B), B.shape[1],
                                   1 if b_trans else 0, _ptr(Cm), N, _stream(A.device))
    if st != 0:
        raise PcsirError(st, "pcsir_mlp_gemm_bf16")
    return Cm


class MLPTrainer:
    """FP32 master parameters, Adam moments and a training workspace on the device."""

    def __init__(self, params, batch: int):
        import torch
        self._torch = torch
        n = mlp_param_count()
        assert params.dtype == torch.float32 and params.numel() == n and params.is_cuda
        self.params = params.contiguous().clone()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.batch = batch
        nb = lib().pcsir_mlp_train_bytes(batch)
        if nb == 0:
            raise PcsirError(-1, "batch must be a positive multiple of 64")
        self.ws = torch.empty(int(nb), dtype=torch.uint8, device=self.params.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.params.device)
        self.t = 0

    def _run(self, X, y, lr, adam: bool, act_scale=None):
        assert X.dtype == self._torch.bfloat16 and X.shape == (self.batch, 256) and X.is_contiguous()
        assert y.dtype == self._torch.float32 and y.shape == (self.batch,)
        if adam:
            self.t += 1
        common = (_ptr(self.params), _ptr(self.m) if adam else None, _ptr(self.v) if adam else None, _ptr(X),
                  _ptr(y), self.batch, float(lr), self.t if adam else 0)
        tail = (_ptr(self.ws), self.ws.numel(), _stream(X.device), _ptr(self.loss), _ptr(self.grad))
        if act_scale is None:
            st = lib().pcsir_mlp_train_step(*common, *tail)
            name = "pcsir_mlp_train_step"
        else:
            assert act_scale.dtype == self._torch.float32 and act_scale.numel() == 3 and act_scale.is_cuda
            st = lib().pcsir_mlp_train_step_fp8(*common, _ptr(act_scale), *tail)
            name = "pcsir_mlp_train_step_fp8"
        if st != 0:
            raise PcsirError(st, name)

    def step(self, X, y, lr: float, act_scale=None):
        """One Adam step on a batch; returns the loss tensor (device, before the step).
        act_scale (device FP32 [3]): quantisation-aware step with the FP8 inference's
        quantisers (pcsir_mlp_train_step_fp8)."""
        self._run(X, y, lr, True, act_scale)
        return self.loss

    def step_static(self, X, y, lr: float):
        """One Adam step through pcsir_mlp_train_step_static (no workspace; batch
        rows up to PCSIR_MLP_STATIC_MAX_BATCH, any multiple of 64); returns the status."""
        assert X.dtype == self._torch.bfloat16 and X.dim() == 2 and X.shape[1] == 256 and X.is_contiguous()
        assert y.dtype == self._torch.float32 and y.shape == (X.shape[0],)
        self.t += 1
        return lib().pcsir_mlp_train_step_static(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(X), _ptr(y),
                                                 int(X.shape[0]), float(lr), self.t, _stream(X.device),
                                                 _ptr(self.loss), _ptr(self.grad))

    def gradients(self, X, y, act_scale=None):
        """Gradient of the batch loss without updating the parameters (act_scale:
        of the quantisation-aware forward pass, as in step)."""
        self._run(X, y, 0.0, False, act_scale)
        return self.grad.clone(), float(self.loss.item())

    def forward(self, X, params=None):
        import torch
        n = X.shape[0]
        assert n % 64 == 0 and X.dtype == torch.bfloat16
        nb = lib().pcsir_mlp_train_bytes(n)
        ws = torch.empty(int(nb), dtype=torch.uint8, device=X.device)
        f = torch.empty(n, dtype=torch.float32, device=X.device)
        p = self.params if params is None else params
        st = lib().pcsir_mlp_forward_train_path(_ptr(p), _ptr(X), n, _ptr(f), _ptr(ws), ws.numel(),
                                                _stream(X.device))
        if st != 0:
            raise PcsirError(st, "pcsir_mlp_forward_train_path")
        return f


class SurrogateNet:
    """Inference form of the surrogate network (fused BF16 / FP8 MFMA kernel)."""

    def __init__(self, params, act_scale=None):
        import torch
        self._torch = torch
        assert params.dtype == torch.float32 and params.is_cuda and params.numel() == mlp_param_count()
        self.device = params.device
        self.block = torch.empty(int(lib().pcsir_surr_bytes()), dtype=torch.uint8, device=self.device)
        self.act_scale = None if act_scale is None else [float(v) for v in act_scale]
        sc = None if act_scale is None else (C.c_float * 3)(*self.act_scale)
        st = lib().pcsir_surr_prepare(_ptr(params.contiguous()), sc, _ptr(self.block), self.block.numel(),
                                      _stream(self.device))
        if st != 0:
            raise PcsirError(st, "pcsir_surr_prepare")

    def rows(self, X, fp8: bool = False, absmax=None):
        """f for BF16 feature rows X [n, 256]; absmax: optional fp32 [3] device tensor (max-accumulated)."""
        t = self._torch
        assert X.dtype == t.bfloat16 and X.is_contiguous() and X.shape[1] == 256
        f = t.empty(X.shape[0], dtype=t.float32, device=self.device)
        st = lib().pcsir_surr_rows(_ptr(self.block), _ptr(X), X.shape[0], 1 if fp8 else 0, _ptr(f),
                                   _ptr(absmax), _stream(self.device))
        if st != 0:
            raise PcsirError(st, "pcsir_surr_rows")
        return f

    def calibrate(self, X, margin: float = 1.0):
        """FP8 input scales of the three layers from the BF16 activations of rows X."""
        a = self._torch.zeros(3, dtype=self._torch.float32, device=self.device)
        self.rows(X, fp8=False, absmax=a)
        return [max(float(v), 1e-30) * margin / 448.0 for v in a.cpu()]
