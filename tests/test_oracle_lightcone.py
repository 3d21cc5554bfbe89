"""Pins of the oracle's light-cone observation (Sec. 2.4), its VJP and the
exact gradient of an objective on the observables (Sec. 3.4, eq.
explicit_adj).  No GPU."""
import numpy as np
import pytest

from oracle import cosmology
from oracle import cosmology as C
from oracle import integrate
from oracle import lightcone as L
from oracle import simulate
from paper_2211_09815_amd import inputs


# ---- light front: closed forms at Omega_m = 1 and Omega_m = 0 --------------

@pytest.mark.parametrize("a", [1.0 / 64, 0.3, 0.77, 1.0])
def test_light_front_einstein_de_sitter(a):
    # E = a^{-3/2}: chi = 2 (c/H0) (1 - sqrt a), dchi/da = -(c/H0) a^{-1/2};
    # d/dOmega_m of the integrand at Omega_m = 1 is -(a^{-1/2} - a^{5/2}) / 2
    cell = 2.0
    kc = L.C_OVER_H0 / cell
    chi, dchi, chi_om, dchi_om = L.light_front(a, 1.0, cell)
    assert chi == pytest.approx(2 * kc * (1 - np.sqrt(a)), rel=1e-13, abs=1e-10)
    assert dchi == pytest.approx(-kc / np.sqrt(a), rel=1e-14)
    ref_om = -0.5 * kc * ((2 - 2.0 / 7) - (2 * np.sqrt(a) - 2.0 / 7 * a ** 3.5))
    assert chi_om == pytest.approx(ref_om, rel=1e-12, abs=1e-10)
    assert dchi_om == pytest.approx(0.5 * kc * (a ** -0.5 - a ** 2.5), rel=1e-13, abs=1e-12)


def test_light_front_pure_lambda():
    # Omega_m = 0: E = 1, chi = (c/H0) (1/a - 1)
    for a in (0.05, 0.5, 0.9):
        chi, dchi, _, _ = L.light_front(a, 0.0, 1.0)
        assert chi == pytest.approx(L.C_OVER_H0 * (1 / a - 1), rel=1e-13)
        assert dchi == pytest.approx(-L.C_OVER_H0 / a ** 2, rel=1e-14)


# ---- Hermite basis ----------------------------------------------------------

def test_hermite_reproduces_cubics():
    rng = np.random.default_rng(5)
    c = rng.standard_normal(4)
    P = lambda u: c[0] + c[1] * u + c[2] * u ** 2 + c[3] * u ** 3
    dP = lambda u: c[1] + 2 * c[2] * u + 3 * c[3] * u ** 2
    ddP = lambda u: 2 * c[2] + 6 * c[3] * u
    u = np.linspace(0, 1, 11)
    h, d, dd = L.hermite(u)
    ends = (P(0.0), dP(0.0), P(1.0), dP(1.0))
    np.testing.assert_allclose(sum(b * e for b, e in zip(h, ends)), P(u), rtol=0, atol=1e-14)
    np.testing.assert_allclose(sum(b * e for b, e in zip(d, ends)), dP(u), rtol=0, atol=1e-13)
    np.testing.assert_allclose(sum(b * e for b, e in zip(dd, ends)), ddP(u), rtol=0, atol=1e-12)


# ---- one step ----------------------------------------------------------------

OM, CELL = 0.3, 2.0
A0, A1 = 0.85, 0.85 + 1.0 / 32


def _step(observer=(0.0, 0.0, 0.0)):
    return L.Step(A0, A1, OM, CELL, observer)


def _cubic_particles(st, m=64, seed=7):
    """Particles on trajectories cubic in a, placed so that they cross the
    front inside the step: x(a) = x_c + B (a - a_m) + Cc (a - a_m)^2 + Dd (a - a_m)^3."""
    rng = np.random.default_rng(seed)
    am = 0.5 * (st.a0 + st.a1)
    chi_m = L.light_front(am, OM, CELL)[0]
    dirs = rng.standard_normal((m, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    xc = st.X + dirs * chi_m * (1 + 0.002 * rng.uniform(-1, 1, (m, 1)))
    B, Cc, Dd = (rng.standard_normal((m, 3)) * s for s in (40.0, 200.0, 800.0))
    x = lambda a: xc + B * (a - am) + Cc * (a - am) ** 2 + Dd * (a - am) ** 3
    dx = lambda a: B + 2 * Cc * (a - am) + 3 * Dd * (a - am) ** 2
    S = lambda a: a ** 3 * np.sqrt(OM * a ** -3 + 1 - OM)
    return x, dx, S


def test_observation_reproduces_cubic_trajectories():
    st = _step()
    x, dx, S = _cubic_particles(st)
    x0, x1 = x(st.a0), x(st.a1)
    p0, p1 = dx(st.a0) * S(st.a0), dx(st.a1) * S(st.a1)
    m, xh, ph, ah, u = L.observe_step(st, x0, p0, x1, p1)
    assert m.sum() >= 40
    assert np.all((ah >= st.a0) & (ah <= st.a1))
    a = ah[:, None]
    np.testing.assert_allclose(xh, x(a)[m], rtol=1e-13)
    np.testing.assert_allclose(ph, (dx(a) * S(a))[m], rtol=1e-10, atol=1e-9)
    # on the root, the distance equals the cubic light front
    h, _, _ = L.hermite(u)
    front = h[0] * st.c0 + h[1] * st.da * st.dc0 + h[2] * st.c1 + h[3] * st.da * st.dc1
    np.testing.assert_allclose(np.linalg.norm(xh - st.X, axis=1), front, rtol=1e-13)
    # and the cubic front is close to the exact one (interpolation error only)
    exact = np.array([L.light_front(v, OM, CELL)[0] for v in ah[:5]])
    np.testing.assert_allclose(front[:5], exact, rtol=1e-6)


def test_particle_at_rest_and_crossing_test():
    st = _step()
    chi_m = L.light_front(0.5 * (A0 + A1), OM, CELL)[0]
    x = np.array([[chi_m, 0, 0], [st.c0 * 1.01, 0, 0], [st.c1 * 0.99, 0, 0]], dtype=float)
    p = np.zeros_like(x)
    m, xh, ph, ah, u = L.observe_step(st, x, p, x, p)
    assert m.tolist() == [True, False, False]   # outside at a0 / inside at a1: not observed
    np.testing.assert_allclose(xh[0], x[0], rtol=1e-15, atol=0)
    np.testing.assert_allclose(ph[0], 0.0, atol=1e-12)
    assert st.a0 < ah[0] < st.a1


def _observe_all(st_fn, x0, p0, x1, p1, om):
    st = st_fn(om)
    m, xh, ph, ah, _ = L.observe_step(st, x0, p0, x1, p1)
    assert m.all()
    return np.concatenate([xh, ph, ah[:, None]], axis=1)


def test_observation_vjp_matches_central_differences():
    st = _step(observer=(3.0, -2.0, 1.0))
    x, dx, S = _cubic_particles(st, m=8, seed=11)
    x0, x1 = x(st.a0), x(st.a1)
    p0, p1 = dx(st.a0) * S(st.a0), dx(st.a1) * S(st.a1)
    m = L.crossing_mask(st, x0, x1)
    x0, p0, x1, p1 = x0[m], p0[m], x1[m], p1[m]
    rng = np.random.default_rng(3)
    g = rng.standard_normal((len(x0), 7))
    v0, v1 = L._tangents(st, p0, p1)
    u = L.crossing_root(st, x0, v0, x1, v1)
    bars = L.observe_step_vjp(st, x0, p0, x1, p1, u, g[:, 0:3], g[:, 3:6], g[:, 6])
    st_fn = lambda om: L.Step(A0, A1, om, CELL, st.X)
    J = lambda a, b, c, d, om=OM: float(np.sum(g * _observe_all(st_fn, a, b, c, d, om)))
    args = [x0, p0, x1, p1]
    for k in range(4):
        for (i, j) in [(0, 0), (1, 2), (len(x0) - 1, 1)]:
            h = 1e-6 * max(1.0, abs(args[k][i, j]))
            ap = [a.copy() for a in args]
            am = [a.copy() for a in args]
            ap[k][i, j] += h
            am[k][i, j] -= h
            fd = (J(*ap) - J(*am)) / (2 * h)
            assert bars[k][i, j] == pytest.approx(fd, rel=2e-6, abs=1e-7 * np.abs(g).max())
    h = 1e-6
    fd = (J(*args, om=OM + h) - J(*args, om=OM - h)) / (2 * h)
    assert bars[4] == pytest.approx(fd, rel=1e-6)


# ---- a whole run ----------------------------------------------------------------

def lightcone_setup(n=8, nm=16, box=32.0, steps=4, split_step=None):
    """A small run and an observer placed so that the light front sweeps the
    box across the boundary a_{split_step} (default: the step before last)."""
    cfg = simulate.SimConfig(n, nm, box, 1.0 / 16, 1.0, steps)
    grid = cfg.a_grid()
    k = steps - 1 if split_step is None else split_step
    cell = box / nm
    chi_k = L.light_front(grid[k], cfg.cosmo.omega_m, cell)[0]
    observer = np.array([nm / 2.0 - chi_k, nm / 2.0, nm / 2.0])
    return cfg, observer


def test_run_observes_every_particle_once_across_two_steps():
    cfg, X = lightcone_setup()
    omega = inputs.white_noise(cfg.n_ptcl, 0)
    w = inputs.normal((cfg.n_particles, 7), inputs.SEED_COTANGENT)
    J, g, gt, obs, step = L.value_and_grad(omega, cfg, X, w)
    n = cfg.n_steps
    counts = np.bincount(step, minlength=n + 1)
    assert counts[0] == 0 and counts[n - 1] > 50 and counts[n] > 50
    grid = cfg.a_grid()
    assert np.all((obs[:, 6] > grid[step - 1]) & (obs[:, 6] <= grid[step]))


@pytest.mark.slow
def test_run_gradient_matches_central_differences():
    cfg, X = lightcone_setup()
    omega = inputs.white_noise(cfg.n_ptcl, 0)
    w = inputs.normal((cfg.n_particles, 7), inputs.SEED_COTANGENT)
    J, g, gt, _, _ = L.value_and_grad(omega, cfg, X, w)
    assert L.objective_value(omega, cfg, X, w) == pytest.approx(J, rel=1e-14)
    flat = omega.ravel()
    idx = inputs.probe_indices(flat.size, 48)
    fds = []
    for h in (1e-5, 5e-6):
        fd = np.zeros(len(idx))
        for t, i in enumerate(idx):
            e = np.zeros_like(flat)
            e[i] = h
            fd[t] = (L.objective_value((flat + e).reshape(omega.shape), cfg, X, w)
                     - L.objective_value((flat - e).reshape(omega.shape), cfg, X, w)) / (2 * h)
        fds.append(fd)
    # probes that straddle a CIC kink show up as disagreement of the two steps
    scale = np.abs(fds[0]).max()
    smooth = np.abs(fds[0] - fds[1]) < 1e-7 * scale
    assert smooth.mean() > 0.9
    gs = g.ravel()[idx][smooth]
    assert np.linalg.norm(gs - fds[1][smooth]) / np.linalg.norm(gs) < 1e-7
    for k, (name, val) in enumerate([("omega_m", 0.3), ("sigma8", 0.8)]):
        vals = []
        for hh in (3e-6, 1e-6):
            cp = cfg.with_cosmo(cfg.cosmo.replace(**{name: val + hh}))
            cm = cfg.with_cosmo(cfg.cosmo.replace(**{name: val - hh}))
            vals.append((L.objective_value(omega, cp, X, w) - L.objective_value(omega, cm, X, w)) / (2 * hh))
        assert vals[0] == pytest.approx(vals[1], rel=1e-6)
        assert gt[k] == pytest.approx(vals[1], rel=1e-6)


def _objective_sourcing_frozen(omega, cfg, observer, weights, step, ref_x):
    """J of the forward map in which the force at t_m takes the particles
    observed in steps 1..m at their positions ref_x[m] in the unperturbed run
    instead of their own: the map whose exact gradient the truncated adjoint
    of reading L7 is.  NaN if the perturbation moved a crossing to another
    step."""
    q = simulate.lattice(cfg)
    s, p = simulate.initial_state(omega, cfg)
    om = cfg.cosmo.omega_m
    a_grid = cfg.a_grid()
    coefs = cosmology.step_coefficients(a_grid, om)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, om)

    def acc(x, m):
        xh = x.copy()
        frozen = (step > 0) & (step <= m)
        xh[frozen] = ref_x[m][frozen]
        return F(xh)

    xs, P = [q + s], [p.copy()]
    a = acc(q + s, 0)
    for i, (Ka, D, Kb) in enumerate(coefs, start=1):
        p = p + a * Ka
        s = s + p * D
        a = acc(q + s, i)
        p = p + a * Kb
        xs.append(q + s)
        P.append(p.copy())
    obs, st = L.observe_run({"x": xs}, P, a_grid, om, cfg.box / cfg.n_mesh, observer)
    if not np.array_equal(st, step):
        return float("nan")
    return L.linear_objective(obs, st, weights)


def test_truncated_gradient_is_the_gradient_with_observed_sources_frozen():
    # reading L7 against central differences of the map it differentiates;
    # first, that the truncation matters here
    cfg, X = lightcone_setup()
    omega = inputs.white_noise(cfg.n_ptcl, 0)
    w = inputs.normal((cfg.n_particles, 7), inputs.SEED_COTANGENT)
    J, g, gt, _, step = L.value_and_grad(omega, cfg, X, w)
    Jt, g_tr, gt_tr, _, step_t = L.value_and_grad(omega, cfg, X, w, truncate=True)
    assert Jt == J and np.array_equal(step_t, step)
    assert np.linalg.norm(g_tr - g) > 1e-4 * np.linalg.norm(g)
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    coefs = cosmology.step_coefficients(cfg.a_grid(), cfg.cosmo.omega_m)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, cfg.cosmo.omega_m)
    ref_x = integrate.forward(q, s0, p0, coefs, F, store=True)[3]["x"]
    Jf = lambda om_, c=cfg: _objective_sourcing_frozen(om_, c, X, w, step, ref_x)   # noqa: E731
    assert Jf(omega) == pytest.approx(J, rel=1e-14)
    flat = omega.ravel()
    idx = inputs.probe_indices(flat.size, 24)
    fds = []
    for h in (1e-5, 5e-6):
        fd = np.zeros(len(idx))
        for t, i in enumerate(idx):
            e = np.zeros_like(flat)
            e[i] = h
            fd[t] = (Jf((flat + e).reshape(omega.shape)) - Jf((flat - e).reshape(omega.shape))) / (2 * h)
        fds.append(fd)
    scale = np.abs(fds[0]).max()
    smooth = np.abs(fds[0] - fds[1]) < 1e-7 * scale
    assert smooth.mean() > 0.9
    gs = g_tr.ravel()[idx][smooth]
    assert np.linalg.norm(gs - fds[1][smooth]) / np.linalg.norm(gs) < 1e-7
    # and the exact gradient is not the gradient of this map
    ge = g.ravel()[idx][smooth]
    assert np.linalg.norm(ge - fds[1][smooth]) / np.linalg.norm(gs) > 1e-5
    hh = 1e-6
    for k, (name, val) in enumerate([("omega_m", 0.3), ("sigma8", 0.8)]):
        cp = cfg.with_cosmo(cfg.cosmo.replace(**{name: val + hh}))
        cm = cfg.with_cosmo(cfg.cosmo.replace(**{name: val - hh}))
        fd = (Jf(omega, cp) - Jf(omega, cm)) / (2 * hh)
        assert gt_tr[k] == pytest.approx(fd, rel=1e-6)


def test_vjp_is_finite_for_a_particle_at_the_observer():
    # a particle that reaches the observer's position at a = 1 crosses there
    # (f(1) = 0); the distance has no gradient at that point (reading L3)
    st = L.Step(1.0 - 1.0 / 32, 1.0, OM, CELL, (5.0, 6.0, 7.0))
    x1 = np.array([[5.0, 6.0, 7.0]])
    p = np.array([[3.0, -2.0, 1.0]])
    x0 = x1 - st.da * st.w0 * p
    m, xh, ph, ah, u = L.observe_step(st, x0, p, x1, p)
    assert m.tolist() == [True] and ah[0] == pytest.approx(1.0, abs=1e-15)
    bars = L.observe_step_vjp(st, x0, p, x1, p, u, np.ones((1, 3)), np.ones((1, 3)), np.ones(1))
    assert all(np.all(np.isfinite(b)) for b in bars)
