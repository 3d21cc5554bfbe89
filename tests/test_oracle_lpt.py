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


# ---------------------------------------------------------------------------
# Momentum factors and the lattice scaling of eq. lpt, pinned by closed forms.
# Each helper returns an error measure; the tests check it is at rounding for
# the oracle and that a planted mistake (a wrong power of a in P_m, r^2 for r,
# a momentum without the factor r) is caught.
# ---------------------------------------------------------------------------


def _eds_time_factor_error(factors):
    """Einstein-de Sitter (Omega_m = 1): D1 = a, D2 = 3/7 a^2 and, with
    D' = dD/dln a and E = a^(-3/2), P1 = a^2 E D1' = a^(3/2) and
    P2 = a^2 E D2' = 6/7 a^(5/2)."""
    err = 0.0
    for a in (0.02, 0.1, 0.5, 1.0):
        D1, D2, P1, P2 = factors(a, 1.0)
        want = (a, 3.0 / 7.0 * a * a, a ** 1.5, 6.0 / 7.0 * a ** 2.5)
        err = max(err, max(abs(g - w) / abs(w) for g, w in zip((D1, D2, P1, P2), want)))
    return err


def _lcdm_momentum_factor_error(factors, om=0.3):
    """P_m / (a^2 E) must be dD_m/dln a: compared with a central difference
    of D_m(a) in ln a (D_1 itself is pinned by the Heath integral)."""
    err = 0.0
    h = 1e-4
    for a in (1.0 / 64, 0.1, 0.5):
        D1, D2, P1, P2 = factors(a, om)
        Dp = factors(a * np.exp(h), om)
        Dm = factors(a * np.exp(-h), om)
        e = C.E(a, om)
        for m, P in ((0, P1), (1, P2)):
            fd = (Dp[m] - Dm[m]) / (2 * h)
            err = max(err, abs(P / (a * a * e) - fd) / abs(fd))
    return err


def test_ic_time_factors_eds_closed_form():
    assert _eds_time_factor_error(lpt.ic_time_factors) < 1e-10


def test_ic_momentum_factors_are_growth_rates():
    assert _lcdm_momentum_factor_error(lpt.ic_time_factors) < 1e-7


def test_ic_time_factor_pins_catch_planted_mistakes():
    # P_m with a^3 instead of a^2, and with D_m instead of dD_m/dln a
    def a_cubed(a0, om):
        D1, D2, P1, P2 = lpt.ic_time_factors(a0, om)
        return D1, D2, P1 * a0, P2 * a0

    def no_rate(a0, om):
        g = C.growth(np.array([a0]), om)
        e = C.E(a0, om)
        return g["D1"][0], g["D2"][0], a0 * a0 * e * g["D1"][0], a0 * a0 * e * g["D2"][0]

    for bad in (a_cubed, no_rate):
        assert _eds_time_factor_error(bad) > 1e-2
        assert _lcdm_momentum_factor_error(bad) > 1e-2


def _plane_wave_noise(n, box, cos, eps, phase=0.3):
    """White noise whose linear field delta1 = irfft(A rfft(omega)) is the
    single plane wave eps cos(2 pi q_x / n + phase) on the lattice."""
    A = lpt.amplitude(n, box, cos)
    q = _grid(n)
    delta1 = eps * np.cos(2 * np.pi * q[0] / n + phase)
    X = np.fft.rfftn(delta1)
    X = np.where(A != 0, X / np.where(A != 0, A, 1.0), 0.0)
    return np.fft.irfftn(X, s=delta1.shape, axes=(0, 1, 2))


def _lpt_plane_wave_error(lpt_fn, n=8, r=2.0, a0=0.1, eps=1e-3, phase=0.3):
    """eq. lpt for one plane wave in EdS: s1 = -grad phi1 with laplacian
    phi1 = delta1 gives s1_x = -eps sin(k q + phase) / k (k = 2 pi / n per
    lattice spacing), s2 = 0, so s0 = r a0 s1 and p0 = r a0^(3/2) s1 in mesh
    cells (r cells per lattice spacing)."""
    cos = C.Cosmo().replace(omega_m=1.0)
    box = 4.0 * n
    omega = _plane_wave_noise(n, box, cos, eps, phase)
    s0, p0 = lpt_fn(omega, box, cos, a0, r)
    k = 2 * np.pi / n
    q = _grid(n)
    s1x = (-eps * np.sin(k * q[0] + phase) / k).ravel()
    want_s = np.zeros_like(s0)
    want_s[:, 0] = r * a0 * s1x
    want_p = np.zeros_like(p0)
    want_p[:, 0] = r * a0 ** 1.5 * s1x
    return max(np.abs(s0 - want_s).max() / np.abs(want_s).max(),
               np.abs(p0 - want_p).max() / np.abs(want_p).max())


def test_lpt_plane_wave_closed_form_with_lattice_scaling():
    assert _lpt_plane_wave_error(lpt.lpt) < 1e-11
    assert _lpt_plane_wave_error(lpt.lpt, r=1.0, a0=0.5) < 1e-11


def test_lpt_plane_wave_pin_catches_planted_mistakes():
    def r_squared(omega, box, cos, a0, r):
        s, p = lpt.lpt(omega, box, cos, a0, r)
        return s * r, p * r

    def p_without_r(omega, box, cos, a0, r):
        s, p = lpt.lpt(omega, box, cos, a0, r)
        return s, p / r

    def p_a_cubed(omega, box, cos, a0, r):
        s, p = lpt.lpt(omega, box, cos, a0, r)
        return s, p * a0

    for bad in (r_squared, p_without_r, p_a_cubed):
        assert _lpt_plane_wave_error(bad) > 0.1
