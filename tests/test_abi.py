"""C ABI checks that need no GPU: the library loads, exports every function that
include/pcsir.h declares, and its host-side config validation and workspace
planning behave as documented."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    """Every function that a header under include/ declares."""
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if not h.endswith(".h"):
            continue
        src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:pcsir_status|size_t|const char\s*\*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    import paper_1310_5541_amd as P
    if not os.path.exists(P.lib_path()):
        from paper_1310_5541_amd import build
        build.build()
    return P.lib()


def test_every_declared_symbol_is_exported(L):
    import paper_1310_5541_amd as P
    names = _declared()
    assert {"pcsir_init", "pcsir_step", "sir_step", "pcsir_estimate", "pcsir_workspace_bytes",
            "pcsir_mlp_train_step", "pcsir_mlp_train_step_static", "pcsir_surr_rows"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", P.lib_path()], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(L, n)


def test_library_is_built_for_gfx950_only():
    import paper_1310_5541_amd as P
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", P.lib_path()], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls not available")
    targets = set(re.findall(r"gfx\w+", out.stdout))
    assert targets == {"gfx950"}, targets


def _cfg(**kw):
    from paper_1310_5541_amd import Config
    base = dict(n_particles=(1000, 37), frame_h=64, frame_w=64)
    base.update(kw)
    return Config(**base)


def test_workspace_bytes_and_validation(L):
    c, keep = _cfg()._c()
    b = L.pcsir_workspace_bytes(C.byref(c))
    assert b > 0 and b % 256 == 0
    # a fixed part (the occupancy bitmap over every 32-bit cell key: 2^26
    # 16-byte entries of a 64-bit word and its first bin), and a part that
    # grows with the particle count, roughly linearly
    fixed = 16 * 2 ** 26
    assert b > fixed
    c2, keep2 = _cfg(n_particles=(100000, 3700))._c()
    b2 = L.pcsir_workspace_bytes(C.byref(c2))
    assert 50 * (b - fixed) < b2 - fixed < 150 * (b - fixed)
    bad = [dict(dim=4), dict(n_particles=(0,)), dict(bins_per_px=(0, 2, 1)), dict(bins_per_px=(5000, 2, 1)),
           dict(patch=10), dict(patch=129), dict(quad=0), dict(quad=17), dict(psf=1), dict(lik_mode=7),
           dict(sigma_xi=0.0), dict(sigma_psf=-1.0), dict(frame_h=0), dict(dummy_mode=3),
           dict(proc_sigma=(-1, 0, 0, 0, 0)), dict(neff_threshold=float("nan")), dict(neff_threshold=-1.0),
           dict(bins_per_sigma=-1.0), dict(bins_per_sigma=float("inf")), dict(bins_per_sigma=2.0, bins_max=0),
           dict(dummy_mode=2, neff_threshold=0.5), dict(dummy_mode=2, lik_mode=2),
           dict(dummy_mode=2, dim=3, psf=1, bins_per_px=(4, 4, 4), proc_sigma=(0.5,) * 7)]
    for kw in bad:
        cb, kb = _cfg(**kw)._c()
        assert L.pcsir_workspace_bytes(C.byref(cb)) == 0, kw
    cb, kb = _cfg()._c()
    cb.abi_version = 99
    assert L.pcsir_workspace_bytes(C.byref(cb)) == 0
    for kw in (dict(dummy_mode=2), dict(bins_per_sigma=2.0, bins_max=8), dict(neff_threshold=0.3)):
        cg, kg = _cfg(**kw)._c()
        assert L.pcsir_workspace_bytes(C.byref(cg)) > 0, kw
    # 3D with the astigmatic PSF is valid
    c3, k3 = _cfg(dim=3, psf=1, bins_per_px=(4, 4, 4), proc_sigma=(0.5,) * 7)._c()
    assert L.pcsir_workspace_bytes(C.byref(c3)) > 0


def test_null_arguments_are_rejected_without_a_device(L):
    c, keep = _cfg()._c()
    out = C.c_void_p()
    assert L.pcsir_init(C.byref(c), None, None, 0, None, C.byref(out)) == -1
    assert L.pcsir_step(None, None, 64, 64, 1) == -1
    assert L.sir_step(None, None, 64, 64, 1) == -1
    assert L.pcsir_estimate(None, None, None) == -1
    assert L.pcsir_destroy(None) == -1
    # surrogate calls
    assert L.pcsir_surr_bytes() > 0 and L.pcsir_surr_bytes() % 256 == 0
    assert L.pcsir_surr_prepare(None, None, None, 0, None) == -1
    assert L.pcsir_surr_rows(None, None, 0, 0, None, None, None) == -1
    assert L.pcsir_set_surrogate(None, None, None, C.c_float(0.01), C.c_float(1.0)) == -1
    cnt = C.c_int32(0)
    assert L.pcsir_surrogate_features(None, None, None, 0, C.byref(cnt)) == -1
    assert L.pcsir_surrogate_stats(None, None, None, None, 0) == -1
    # a surrogate mode with a window too large for the 256 features is refused
    bad, keep2 = _cfg(lik_mode=2, patch=17)._c()
    assert L.pcsir_workspace_bytes(C.byref(bad)) == 0
    ok, keep3 = _cfg(lik_mode=3, patch=15)._c()
    assert L.pcsir_workspace_bytes(C.byref(ok)) > 0


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1310_5541_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "pcsir_oracle" not in txt, f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1310_5541_amd._lib as lib
    monkeypatch.setattr(lib, "_LIB", str(tmp_path / "absent.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(lib.LibraryMissing):
        lib.lib()
