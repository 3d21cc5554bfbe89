"""Pins of the oracle's 2LPT initial conditions and their derivatives
(no GPU)."""
import numpy as np
import pytest

from oracle import cosmology as C
from oracle import lpt
from paper_2211_09815_amd import inputs


def _grid(n):
    return np.stack(np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij"))


def _unit_amp(n):
    _, _, k2, _ = lpt.lattice_wavenumbers(n)
    return (k2 > 0).astype(float)


def test_single_plane_wave_has_no_second_order():
    n = 16
    q = _grid(n)
    k = 2 * np.pi * 3 / n
    delta1 = 0.01 * np.cos(k * q[0] + 0.3)
    s1, s2, _ = lpt.lpt_fields(delta1, 1.0, None, amp=_unit_amp(n))
    # s1 = -grad phi1 with laplacian phi1 = delta1 -> s1_x = -0.01 sin(k q + 0.3) / k
    np.testing.assert_allclose(s1[0], -0.01 * np.sin(k * q[0] + 0.3) / k, atol=1e-15)
    assert np.abs(s1[1:]).max() < 1e-16
    assert np.abs(s2).max() < 1e-18


def test_two_orthogonal_waves_second_order_closed_form():
    # phi1 = A cos(k1 x) + B cos(k2 y):  S = phi_xx phi_yy = A B k1^2 k2^2 cos cos,
    # phi2 = -S / (k1^2 + k2^2),  s2 = -grad phi2
    n = 16
    q = _grid(n)
    k1, k2 = 2 * np.pi * 2 / n, 2 * np.pi * 3 / n
    A, B = 0.3, -0.2
    delta1 = -A * k1 ** 2 * np.cos(k1 * q[0]) - B * k2 ** 2 * np.cos(k2 * q[1])
    _, s2, H = lpt.lpt_fields(delta1, 1.0, None, amp=_unit_amp(n))
    np.testing.assert_allclose(H[(0, 0)], -A * k1 ** 2 * np.cos(k1 * q[0]), atol=1e-14)
    np.testing.assert_allclose(H[(0, 1)], 0.0, atol=1e-14)
    c = A * B * k1 ** 2 * k2 ** 2 / (k1 ** 2 + k2 ** 2)
    # phi2 = -c cos(k1 x) cos(k2 y);  s2 = grad(c cos cos)
    np.testing.assert_allclose(s2[0], -c * k1 * np.sin(k1 * q[0]) * np.cos(k2 * q[1]), atol=1e-14)
    np.testing.assert_allclose(s2[1], -c * k2 * np.cos(k1 * q[0]) * np.sin(k2 * q[1]), atol=1e-14)
    np.testing.assert_allclose(s2[2], 0.0, atol=1e-14)


def test_linear_field_variance_matches_power_sum():
    # <delta1(q)^2> = (1/V) sum_k P(k) over the lattice modes (statistical pin of
    # the sqrt(P / V_cell) normalisation)
    n, box = 48, 200.0
    cos = C.Cosmo()
    omega = inputs.white_noise(n, 4)
    A = lpt.amplitude(n, box, cos)
    delta1 = np.fft.irfftn(A * np.fft.rfftn(omega), s=omega.shape)
    _, _, k2, _ = lpt.lattice_wavenumbers(n)
    kph = np.sqrt(k2) * n / box
    P = np.zeros_like(kph)
    nz = k2 > 0
    P[nz] = C.linear_power(kph[nz], cos.omega_m, cos.omega_b, cos.h, cos.n_s, cos.sigma8)
    w = np.full(k2.shape, 2.0)
    w[..., 0] = 1.0
    w[..., -1] = 1.0
    expect = np.sum(w * P) / box ** 3
    assert np.mean(delta1 ** 2) == pytest.approx(expect, rel=0.03)


def test_lpt_vjp_matches_finite_difference():
    n, box, a0, r = 8, 64.0, 0.1, 2.0
    cos = C.Cosmo()
    om = inputs.white_noise(n, 0)
    s0, p0 = lpt.lpt(om, box, cos, a0, r)
    xb = inputs.normal(s0.shape, 30)
    pb = inputs.normal(p0.shape, 31)
    g = lpt.lpt_vjp(om, box, cos, a0, r, xb, pb)
    h = 1e-5
    for seed in (32, 33):
        d = inputs.normal(om.shape, seed)
        sp, pp = lpt.lpt(om + h * d, box, cos, a0, r)
        sm, pmn = lpt.lpt(om - h * d, box, cos, a0, r)
        fd = (np.sum(xb * (sp - sm)) + np.sum(pb * (pp - pmn))) / (2 * h)
        assert np.sum(g * d) == pytest.approx(fd, rel=1e-8)


def test_lpt_theta_tangents_match_finite_difference():
    n, box, a0, r = 8, 64.0, 0.1, 2.0
    cos = C.Cosmo()
    om = inputs.white_noise(n, 0)
    ds, dp = lpt.lpt_jvp_omega_m(om, box, cos, a0, r)
    h = 1e-5
    sp, pp = lpt.lpt(om, box, cos.replace(omega_m=0.3 + h), a0, r)
    sm, pmn = lpt.lpt(om, box, cos.replace(omega_m=0.3 - h), a0, r)
    np.testing.assert_allclose(ds, (sp - sm) / (2 * h), atol=1e-8 * np.abs(ds).max())
    np.testing.assert_allclose(dp, (pp - pmn) / (2 * h), atol=1e-8 * np.abs(dp).max())
    ds8, dp8 = lpt.lpt_dsigma8(om, box, cos, a0, r)
    sp, pp = lpt.lpt(om, box, cos.replace(sigma8=0.8 + h), a0, r)
    sm, pmn = lpt.lpt(om, box, cos.replace(sigma8=0.8 - h), a0, r)
    np.testing.assert_allclose(ds8, (sp - sm) / (2 * h), atol=1e-8 * np.abs(ds8).max())
    np.testing.assert_allclose(dp8, (pp - pmn) / (2 * h), atol=1e-8 * np.abs(dp8).max())
