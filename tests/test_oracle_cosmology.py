"""Pins of the oracle's background, growth, FastPM factors, step coefficients
and power-spectrum normalisation against closed forms and independent
integrals (no GPU)."""
import math

import numpy as np
import pytest

from oracle import cosmology as C


A_TEST = np.array([0.01, 0.0625, 0.1, 0.3, 0.5, 0.8, 1.0])


def test_growth_D1_matches_heath_integral():
    # Heath closed form for flat LambdaCDM, normalised to D1 -> a (Appendix A ICs)
    for om in (0.3, 0.15, 0.5):
        g = C.growth(A_TEST, om)
        heath = C.heath_D1(A_TEST, om)
        np.testing.assert_allclose(g["D1"], heath, rtol=1e-9)


def test_growth_einstein_de_sitter_exact():
    # Omega_m = 1: D1 = a, D2 = 3/7 a^2 exactly (Appendix A growing mode)
    g = C.growth(A_TEST, 1.0)
    np.testing.assert_allclose(g["D1"], A_TEST, rtol=1e-12)
    np.testing.assert_allclose(g["dD1"], A_TEST, rtol=1e-12)
    np.testing.assert_allclose(g["ddD1"], A_TEST, rtol=1e-12)
    np.testing.assert_allclose(g["D2"], 3.0 / 7.0 * A_TEST ** 2, rtol=1e-12)
    np.testing.assert_allclose(g["dD2"], 6.0 / 7.0 * A_TEST ** 2, rtol=1e-12)


def test_growth_D2_bouchet_approximation():
    # D2 ~ 3/7 D1^2 Omega_m(a)^(-1/143) (Bouchet et al. 1995), good to ~1e-3
    g = C.growth(A_TEST, 0.3)
    approx = 3.0 / 7.0 * g["D1"] ** 2 * C.omega_m_a(A_TEST, 0.3) ** (-1.0 / 143.0)
    np.testing.assert_allclose(g["D2"], approx, rtol=1e-2)


def test_growth_second_derivative_consistent():
    # dD1 and ddD1 from the product rule agree with finite differences in ln a
    a = np.array([0.05, 0.2, 0.7])
    h = 1e-4
    g = C.growth(a, 0.3)
    gp = C.growth(a * math.exp(h), 0.3)
    gm = C.growth(a * math.exp(-h), 0.3)
    np.testing.assert_allclose(g["dD1"], (gp["D1"] - gm["D1"]) / (2 * h), rtol=1e-7)
    np.testing.assert_allclose(g["ddD1"], (gp["dD1"] - gm["dD1"]) / (2 * h), rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(g["dD2"], (gp["D2"] - gm["D2"]) / (2 * h), rtol=1e-7)


def test_GK_equals_1p5_omega_m_D1():
    # G_K = a^3 H^2 [D1'' + (2 + H'/H) D1'] = 1.5 Omega_m D1 by the D1 ODE
    for om in (0.3, 0.7, 1.0):
        D1, GD, GK = C.fastpm_factors(A_TEST, om)
        np.testing.assert_allclose(GK, 1.5 * om * D1, rtol=1e-10)


def test_fastpm_factors_eds():
    D1, GD, GK = C.fastpm_factors(A_TEST, 1.0)
    np.testing.assert_allclose(GD, A_TEST ** 1.5, rtol=1e-12)
    np.testing.assert_allclose(GK, 1.5 * A_TEST, rtol=1e-12)


def test_drift_kick_antisymmetry():
    # D(tc, ta, tb) = -D(tc, tb, ta), same for K (Sec. 3.6)
    for (ac, aa, ab) in [(0.3, 0.2, 0.4), (0.75, 0.5, 1.0)]:
        assert C.drift_factor(ac, aa, ab, 0.3) == pytest.approx(-C.drift_factor(ac, ab, aa, 0.3), rel=1e-14)
        assert C.kick_factor(ac, aa, ab, 0.3) == pytest.approx(-C.kick_factor(ac, ab, aa, 0.3), rel=1e-14)


def test_step_coefficients_eds_closed_form():
    grid = C.linear_a_grid(1.0 / 16, 1.0, 10)
    c = C.step_coefficients(grid, 1.0)
    a0, a1 = grid[:-1], grid[1:]
    ah = 0.5 * (a0 + a1)
    Ka = (ah ** 1.5 - a0 ** 1.5) / (1.5 * a0)
    D = (a1 - a0) / ah ** 1.5
    Kb = (a1 ** 1.5 - ah ** 1.5) / (1.5 * a1)
    np.testing.assert_allclose(c[:, 0], Ka, rtol=1e-11)
    np.testing.assert_allclose(c[:, 1], D, rtol=1e-11)
    np.testing.assert_allclose(c[:, 2], Kb, rtol=1e-11)


def test_step_coefficient_derivatives_converge_to_complex_step():
    grid = C.linear_a_grid(1.0 / 16, 1.0, 10)
    _, dc = C.step_coefficients_with_derivative(grid, 0.3)
    errs = []
    for h in (1e-3, 1e-4):
        fd = (C.step_coefficients(grid, 0.3 + h) - C.step_coefficients(grid, 0.3 - h)) / (2 * h)
        errs.append(np.max(np.abs(fd - dc) / np.abs(dc)))
    # central differences converge as h^2 toward the complex-step value
    assert errs[1] < 2e-7
    assert errs[0] / errs[1] == pytest.approx(100.0, rel=0.1)


def test_eh_nowiggle_limits():
    # T(k -> 0) -> 1 and T decreases monotonically; beyond these limits the
    # transfer function values are parity unpinned (no tabulated values here)
    k = np.logspace(-6, 2, 200)
    T = C.eh_nowiggle(k, 0.3, 0.05, 0.7)
    assert abs(T[0] - 1.0) < 1e-5
    assert np.all(np.diff(T) < 0)
    # large-k asymptote L0 / (C0 q^2) with C0 -> 14.2
    assert T[-1] * k[-1] ** 2 / np.log(k[-1]) < 1.0


def test_sigma8_quadrature_converged_and_independent():
    from scipy.integrate import quad
    om, ob, h, ns = 0.3, 0.05, 0.7, 0.96
    I1 = C.sigma_r_shape_integral(om, ob, h, ns, panels=4096)
    I2 = C.sigma_r_shape_integral(om, ob, h, ns, panels=8192)
    assert abs(I1 - I2) / I1 < 1e-10
    # independent adaptive quadrature in k (not ln k)

    def f(k):
        T = C.eh_nowiggle(np.array([k]), om, ob, h)[0]
        W = C.tophat_window(np.array([8.0 * k]))[0]
        return k * k * k ** ns * T * T * W * W / (2 * math.pi ** 2)
    edges = np.concatenate([[1e-5], np.logspace(-4, 2, 61)])
    I3 = sum(quad(f, edges[i], edges[i + 1], epsabs=0, epsrel=1e-12, limit=200)[0]
             for i in range(len(edges) - 1))
    assert abs(I1 - I3) / I1 < 1e-8


def test_power_amplitude_reproduces_sigma8():
    om = 0.3
    A = C.power_amplitude(om, 0.05, 0.7, 0.96, 0.8)
    D1 = C.growth(np.array([1.0]), om)["D1"][0]
    I = C.sigma_r_shape_integral(om, 0.05, 0.7, 0.96)
    assert math.sqrt(A * D1 ** 2 * I) == pytest.approx(0.8, rel=1e-12)
    # sigma8 scales the amplitude quadratically
    A2 = C.power_amplitude(om, 0.05, 0.7, 0.96, 1.6)
    assert A2 / A == pytest.approx(4.0, rel=1e-13)
