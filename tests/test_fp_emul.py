"""Pins of the narrow-format emulation used by the surrogate GPU tests (CPU)."""
import numpy as np
import torch

from fp_emul import bf16_round, e4m3_round, e4m3_values


def test_bf16_round_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100_000) * 10.0 ** rng.uniform(-8, 8, 100_000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(bf16_round(x), ref)
    assert bf16_round(np.float32(1 + 2.0 ** -8)) == 1.0               # tie -> even mantissa
    assert bf16_round(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6  # tie -> even mantissa


def test_e4m3_table_and_rounding():
    v = e4m3_values()
    assert v[0x38] == 1.0 and v[0x7E] == 448.0 and v[0x01] == 2.0 ** -9 and np.isnan(v[0x7F])
    assert v[0x08] == 2.0 ** -6 and v[0x07] == 7 * 2.0 ** -9            # smallest normal, largest subnormal
    assert np.all(np.diff(v[:127]) > 0) and np.sum(np.isfinite(v)) == 254
    cases = {1.0: 1.0, 448.0: 448.0, 2.0 ** -10: 0.0, 3 * 2.0 ** -10: 2.0 ** -8, 1.0625: 1.0, 1.1875: 1.25,
             -1.1875: -1.25, 1.07: 1.125, 300.0: 288.0, 0.3: 0.3125}
    for a, b in cases.items():
        assert e4m3_round(np.float32(a)) == b, (a, e4m3_round(np.float32(a)), b)
    # every representable value maps to itself; midpoints between neighbours go to the even code
    fin = v[:127]
    np.testing.assert_array_equal(e4m3_round(fin), fin)
    mid = 0.5 * (fin[:-1] + fin[1:])
    got = e4m3_round(mid)
    even = np.where(np.arange(126) % 2 == 0, fin[:-1], fin[1:])
    np.testing.assert_array_equal(got, even)


def test_branch_free_normal_cdf_of_the_gelu_kernels():
    """The GELU of the surrogate kernels takes Phi from Abramowitz & Stegun
    7.1.26 (erf within 1.5e-7). Written out here in binary32 as the kernels
    evaluate it, it stays within 3e-7 of the exact Phi (the formula's 0.75e-7 plus
    the binary32 roundings), and g = u Phi(u) and g' = Phi + u phi within
    3e-7 (1 + |u|) of the exact values, for |u| <= 12."""
    import math

    from scipy.special import ndtr
    f32 = np.float32
    u = np.linspace(-12.0, 12.0, 200_001).astype(f32)
    x = np.abs(u) * f32(0.70710678118654752)
    t = f32(1.0) / (f32(0.3275911) * x + f32(1.0))
    poly = t * ((((f32(1.061405429) * t + f32(-1.453152027)) * t + f32(1.421413741)) * t + f32(-0.284496736)) * t
                + f32(0.254829592))
    e = np.exp2((u * u) * f32(-0.72134752044448170)).astype(f32)
    h = f32(0.5) * (poly * e)
    phi_c = np.where(u < 0, h, f32(1.0) - h).astype(np.float64)
    ud = u.astype(np.float64)
    exact = ndtr(ud)
    assert np.max(np.abs(phi_c - exact)) <= 3e-7
    g_err = np.abs(ud * phi_c - ud * exact)
    assert np.all(g_err <= 3e-7 * (1.0 + np.abs(ud)))
    dens = np.exp(-0.5 * ud * ud) / math.sqrt(2.0 * math.pi)
    gp = phi_c + ud * e.astype(np.float64) * 0.39894228040143268
    assert np.all(np.abs(gp - (exact + ud * dens)) <= 3e-7 * (1.0 + np.abs(ud)))
