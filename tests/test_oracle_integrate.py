"""Pins of the oracle's KDK integrator, adjoints and end-to-end gradient
(no GPU)."""
import numpy as np
import pytest

from oracle import cosmology as C
from oracle import integrate, lpt, pm, simulate
from paper_2211_09815_amd import inputs


def _za_plane_wave_residual(n, steps=10, eps=1e-4, compensate=False):
    """Relative deviation of s(a_n)/s(a_0) from D1(a_n)/D1(a_0) for a 1LPT
    plane wave at the box scale, r = 1, lattice offset 0.5 cell.

    FastPM's kick and drift factors make KDK exact in the Zel'dovich
    approximation (Sec. 2.3).  On the mesh, CIC paint followed by CIC readout of
    this wave scales the force by sin(k)/k (k in cell units); with
    `compensate` the force coefficient is divided by that factor, which leaves
    only O(eps k) nonlinearity and roundoff."""
    om = 0.3
    q = pm.lattice_positions((n, n, n), 1.0, 0.5)
    s1 = np.zeros_like(q)
    k = 2 * np.pi / n
    s1[:, 0] = eps * np.sin(k * q[:, 0])
    grid = C.linear_a_grid(0.1, 1.0, steps)
    g = C.growth(grid[[0, -1]], om)
    e0 = C.E(grid[0], om)
    s0 = g["D1"][0] * s1
    p0 = grid[0] ** 2 * e0 * g["dD1"][0] * s1
    coefs = C.step_coefficients(grid, om)
    F = integrate.ForceModel((n, n, n), n ** 3, om)
    if compensate:
        F.coef = F.coef * k / np.sin(k)
    s, p, _, _ = integrate.forward(q, s0, p0, coefs, F, store=False)
    ratio = g["D1"][1] / g["D1"][0]
    sel = np.abs(s1[:, 0]) > 0.5 * eps
    return np.max(np.abs(s[sel, 0] / s0[sel, 0] - ratio)) / ratio


def test_za_exact_for_any_step_count():
    # with the mesh response divided out the integrator is exact in ZA
    for steps in (1, 3, 20):
        assert _za_plane_wave_residual(16, steps=steps, eps=1e-5, compensate=True) < 1e-5


def test_za_plane_wave_mesh_response():
    # without compensation the growth is short by about eps_mesh = 1 - sin(k)/k,
    # which falls 4x per doubling of the mesh
    res = {}
    for n in (16, 32):
        k = 2 * np.pi / n
        eps_mesh = 1 - np.sin(k) / k
        res[n] = _za_plane_wave_residual(n, steps=10)
        assert 0.5 * eps_mesh < res[n] < 1.5 * eps_mesh
    assert 3.5 < res[16] / res[32] < 4.5


def _small_run(n=8, nm=16, steps=4, seed=0):
    cfg = simulate.SimConfig(n, nm, 32.0, 1.0 / 16, 1.0, steps)
    omega = inputs.white_noise(n, seed)
    return cfg, omega


def test_time_reversibility_fp64():
    cfg, omega = _small_run(steps=6)
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    coefs = C.step_coefficients(cfg.a_grid(), cfg.cosmo.omega_m)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, cfg.cosmo.omega_m)
    s, p, a, _ = integrate.forward(q, s0, p0, coefs, F, store=False)
    sb, pb = integrate.backward_only(q, s, p, a, coefs, F)
    assert np.sqrt(np.mean((sb - s0) ** 2)) / np.std(s0) < 1e-12
    assert np.sqrt(np.mean((pb - p0) ** 2)) / np.std(p0) < 1e-12


def test_reverse_time_adjoint_matches_stored_trajectory():
    cfg, omega = _small_run(steps=5)
    target = simulate.final_density(inputs.white_noise(cfg.n_ptcl, 1), cfg)
    J1, g1, t1 = simulate.value_and_grad(omega, cfg, target, mode="stored")
    J2, g2, t2 = simulate.value_and_grad(omega, cfg, target, mode="reverse")
    assert J1 == J2
    assert np.linalg.norm(g1 - g2) / np.linalg.norm(g1) < 1e-8
    np.testing.assert_allclose(t1, t2, rtol=1e-8)


def test_checkpoints_hold_the_states_of_the_stored_trajectory():
    # checkpoint j is (s_j, p_{j-1/2}): the positions after step j and the
    # momentum its drift used
    cfg, omega = _small_run(steps=5)
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    coefs = C.step_coefficients(cfg.a_grid(), cfg.cosmo.omega_m)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, cfg.cosmo.omega_m)
    ck = {1: None, 3: None, 5: None}
    integrate.forward(q, s0, p0, coefs, F, store=True, checkpoints=ck)
    _, _, _, traj = integrate.forward(q, s0, p0, coefs, F, store=True)
    for j, (s_j, p_j) in ck.items():
        np.testing.assert_array_equal(q + s_j, traj["x"][j])
        np.testing.assert_array_equal(p_j, traj["p_half"][j - 1])


@pytest.mark.parametrize("steps_ck", [(2,), (1, 3, 5), (1, 2, 3, 4, 5)])
def test_piecewise_reverse_matches_stored_trajectory(steps_ck):
    # resuming (x, p) from checkpoints leaves the gradient of the discrete
    # map unchanged; a checkpoint restored one step early or late would move
    # the positions by a whole drift and fail this by orders of magnitude
    cfg, omega = _small_run(steps=5)
    target = simulate.final_density(inputs.white_noise(cfg.n_ptcl, 1), cfg)
    J1, g1, t1 = simulate.value_and_grad(omega, cfg, target, mode="stored")
    J2, g2, t2 = simulate.value_and_grad(omega, cfg, target, mode="reverse", checkpoint_steps=steps_ck)
    assert J1 == J2
    assert np.linalg.norm(g1 - g2) / np.linalg.norm(g1) < 1e-8
    np.testing.assert_allclose(t1, t2, rtol=1e-8)


def test_checkpoint_at_last_step_replaces_the_reconstructed_momentum():
    # with a checkpoint at step n the reverse pass takes p_{n-1/2} from it, so
    # a wrong final momentum has no effect at all; without it, it does
    cfg, omega = _small_run(steps=4)
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    om = cfg.cosmo.omega_m
    coefs, dcoefs = C.step_coefficients_with_derivative(cfg.a_grid(), om)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, om)
    ck = {4: None}
    s, p, a, _ = integrate.forward(q, s0, p0, coefs, F, store=False, checkpoints=ck)
    xi = inputs.normal(s.shape, 70)
    pi = inputs.normal(s.shape, 71, 0.1)
    wrong = p + inputs.normal(p.shape, 72)
    good = integrate.adjoint_reverse(q, s, p, a, xi, pi, coefs, dcoefs, F, checkpoints=ck)
    bad = integrate.adjoint_reverse(q, s, wrong, a, xi, pi, coefs, dcoefs, F, checkpoints=ck)
    for u, v in zip(good, bad):
        np.testing.assert_array_equal(u, v)
    plain = integrate.adjoint_reverse(q, s, wrong, a, xi, pi, coefs, dcoefs, F)
    assert np.linalg.norm(plain[2] - good[2]) > 1e-3 * np.linalg.norm(good[2])


@pytest.mark.slow
def test_end_to_end_gradient_brute_force_fd():
    # every one of the 8^3 white-noise entries and both theta components
    cfg, omega = _small_run(n=8, nm=16, steps=3)
    target = simulate.final_density(inputs.white_noise(cfg.n_ptcl, 1), cfg)
    J, g, gt = simulate.value_and_grad(omega, cfg, target, mode="stored")
    Jw = simulate.FixedThetaObjective(cfg, target)
    assert Jw(omega) == pytest.approx(J, rel=1e-14)
    # This box is very nonlinear, so a probe can straddle a CIC kink (a particle
    # crossing a mesh node), where the central difference is not a derivative.
    # Two step sizes flag those probes; all others must agree tightly.
    flat = omega.ravel()
    fds = []
    for h in (1e-5, 5e-6):
        fd = np.zeros(omega.size)
        for i in range(omega.size):
            e = np.zeros_like(flat)
            e[i] = h
            fd[i] = (Jw((flat + e).reshape(omega.shape)) - Jw((flat - e).reshape(omega.shape))) / (2 * h)
        fds.append(fd)
    scale = np.abs(fds[0]).max()
    smooth = np.abs(fds[0] - fds[1]) < 1e-7 * scale
    assert smooth.mean() > 0.97
    gs = g.ravel()[smooth]
    assert np.linalg.norm(gs - fds[1][smooth]) / np.linalg.norm(gs) < 1e-7
    for k, (name, val) in enumerate([("omega_m", 0.3), ("sigma8", 0.8)]):
        vals = []
        for hh in (3e-6, 1e-6):
            cp = cfg.with_cosmo(cfg.cosmo.replace(**{name: val + hh}))
            cm = cfg.with_cosmo(cfg.cosmo.replace(**{name: val - hh}))
            vals.append((simulate.objective_value(omega, cp, target)
                         - simulate.objective_value(omega, cm, target)) / (2 * hh))
        assert vals[0] == pytest.approx(vals[1], rel=1e-7)     # no kink straddled
        assert gt[k] == pytest.approx(vals[1], rel=1e-7)
