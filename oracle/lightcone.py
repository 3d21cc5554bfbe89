"""Light-cone observation operator, its VJP, and the gradient of an objective
on the observables -- plain FP64 reference.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * Sec. 2.4 (observation): every particle is recorded at the time it crosses
    the past light cone of an observer.  Between the states z = (x, p) at
    t_{i-1} and t_i its trajectory is a cubic Hermite spline; the light front
    is approximated cubically in the same way, so the crossing is the root of
    a smooth function of one variable on the step.
  * Sec. 3.4 (objective on the observables): the cotangent of an observed
    state enters the adjoint only at that particle's crossing; before (in
    reverse time: after) it the particle's adjoint is zero.
  * eq. explicit_adj (Sec. 3.5): in the discrete setting this is the chain
    rule through the interpolation, which hands the cotangent of an observed
    state to the two states of the step that brackets its crossing; the
    partial objective derivatives dJ/dz_i are added to the adjoint at t_i.

Readings (the paper gives no formulas for these; each is ours):
  L1  Spline variable: the scale factor a.  The tangent is dx/da =
      p / (a^3 E(a)), from dx/dt = p / a^2 (Sec. 2.3) and dt = da / (a H),
      H0 = 1.  On step i, u = (a - a_{i-1}) / (a_i - a_{i-1}).
  L2  Light front: comoving distance chi(a) = (c/H0) int_a^1 da' / (a'^2 E(a'))
      in mesh cells (c/H0 = 2997.92458 Mpc/h divided by the cell size),
      interpolated on each step by the cubic Hermite spline through chi and
      dchi/da at both ends.
  L3  Crossing: f(u) = |x(u) - x_obs| - chi(u).  A particle is observed in
      step i when f(0) < 0 <= f(1), at the root u* of f in [0, 1].  One copy
      of the periodic box is observed (unwrapped positions x = q + s, no
      images); a particle outside the front at a_0 is never observed.  If a
      particle satisfied the test in two steps, the later one wins.  At the
      observer itself (distance 0, possible only at a = 1) the distance's
      gradient is taken as zero.
  L4  Observed state: x^ = x(u*), p^ = a^3 E(a^) dx/da (u*) (so p^ equals the
      integer-time momentum at either end of the step), a^ = a_{i-1} + u* da.
  L5  Integer-time momenta of the KDK scheme: p_i = p_{i-1/2} + a_i Kb_i.
  L6  The gradient is exact for the discrete map, including the dependence of
      u* on the states and on Omega_m (implicit function theorem).  The paper
      drops d t^/d theta in its continuous derivation, where that term
      vanishes on the true trajectory; on the spline it does not vanish
      exactly, so it is kept.
  L7  The paper's own adjoint sets a particle's adjoint to zero after its
      crossing (Sec. 3.4), which drops the gravitational coupling of an
      observed particle to the particles observed after it.  As an option
      (truncate), the discrete form of that: the force at integer time t_m
      (the one evaluation that both half-kicks at t_m use) takes the
      positions of the particles observed in steps 1..m as constants.  Its
      VJP then gives those particles nothing: what they would receive is
      discarded, while their own momentum cotangent still reaches the other
      particles through it.  The result is the exact gradient of that
      modified forward map; a particle observed in step s keeps its exact
      adjoint up to t_s, the end of its crossing step.
"""
import numpy as np
from scipy.integrate import quad

from . import cosmology, integrate, lpt

C_OVER_H0 = 2997.92458  # Mpc/h


# ----------------------------------------------------------------------------
# background pieces (flat LambdaCDM, H0 = 1)
# ----------------------------------------------------------------------------


def _E(a, om):
    return np.sqrt(om * a ** -3.0 + (1.0 - om))


def _dE_dom(a, om):
    return (a ** -3.0 - 1.0) / (2.0 * _E(a, om))


def _dE_da(a, om):
    return -1.5 * om * a ** -4.0 / _E(a, om)


def light_front(a, om, cell):
    """(chi, dchi/da, dchi/dOmega_m, d(dchi/da)/dOmega_m) at scale factor a,
    in mesh cells of `cell` Mpc/h (reading L2).  The integrals are adaptive
    quadratures of the integrand and of its analytic Omega_m derivative."""
    kc = C_OVER_H0 / cell
    f = lambda x: 1.0 / (x * x * _E(x, om))
    fo = lambda x: -_dE_dom(x, om) / (x * x * _E(x, om) ** 2)
    chi = kc * quad(f, a, 1.0, epsabs=0.0, epsrel=2e-14, limit=200)[0]
    chi_om = kc * quad(fo, a, 1.0, epsabs=0.0, epsrel=2e-14, limit=200)[0]
    return chi, -kc * f(a), chi_om, -kc * fo(a)


def velocity_factor(a, om):
    """w(a) = 1 / (a^3 E(a)) with dw/dOmega_m (reading L1)."""
    e = _E(a, om)
    return 1.0 / (a ** 3 * e), -_dE_dom(a, om) / (a ** 3 * e * e)


# ----------------------------------------------------------------------------
# cubic Hermite basis on [0, 1]
# ----------------------------------------------------------------------------


def hermite(u):
    """(h00, h10, h01, h11) and their first and second derivatives in u."""
    u2, u3 = u * u, u * u * u
    h = (2 * u3 - 3 * u2 + 1, u3 - 2 * u2 + u, -2 * u3 + 3 * u2, u3 - u2)
    d = (6 * u2 - 6 * u, 3 * u2 - 4 * u + 1, -6 * u2 + 6 * u, 3 * u2 - 2 * u)
    dd = (12 * u - 6, 6 * u - 4, -12 * u + 6, 6 * u - 2)
    return h, d, dd


def _spline(b, y0, t0, y1, t1):
    """b[0] y0 + b[1] t0 + b[2] y1 + b[3] t1 with broadcasting over particles."""
    return b[0] * y0 + b[1] * t0 + b[2] * y1 + b[3] * t1


class Step:
    """The scalars of one step from a0 to a1 that do not depend on particles."""

    def __init__(self, a0, a1, om, cell, observer):
        self.a0, self.a1, self.om = float(a0), float(a1), float(om)
        self.da = self.a1 - self.a0
        self.X = np.asarray(observer, dtype=np.float64)
        self.c0, self.dc0, self.c0_om, self.dc0_om = light_front(self.a0, om, cell)
        self.c1, self.dc1, self.c1_om, self.dc1_om = light_front(self.a1, om, cell)
        self.w0, self.w0_om = velocity_factor(self.a0, om)
        self.w1, self.w1_om = velocity_factor(self.a1, om)


def _tangents(st, p0, p1):
    return st.da * st.w0 * p0, st.da * st.w1 * p1


def _front(st, b):
    """chi spline (or its u-derivative with the derivative basis) at u."""
    return b[0] * st.c0 + b[1] * (st.da * st.dc0) + b[2] * st.c1 + b[3] * (st.da * st.dc1)


def crossing_mask(st, x0, x1):
    """Particles observed in this step (reading L3): f(0) < 0 <= f(1)."""
    r0 = np.linalg.norm(x0 - st.X, axis=1)
    r1 = np.linalg.norm(x1 - st.X, axis=1)
    return (r0 < st.c0) & (r1 >= st.c1)


def crossing_root(st, x0, v0, x1, v1, iters=64):
    """Root u* of f on [0, 1] by bisection (f(0) < 0 <= f(1) is assumed)."""
    lo = np.zeros(len(x0))
    hi = np.ones(len(x0))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        h, _, _ = hermite(mid[:, None])
        pos = _spline(h, x0, v0, x1, v1)
        hs, _, _ = hermite(mid)
        fm = np.linalg.norm(pos - st.X, axis=1) - _front(st, hs)
        neg = fm < 0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def observe_step(st, x0, p0, x1, p1):
    """Observation of one step (readings L1-L4).  x, p: (N, 3) positions and
    integer-time momenta at a0 and a1.  Returns (mask, xhat, phat, ahat, u)
    for the observed particles (rows of mask)."""
    m = crossing_mask(st, x0, x1)
    x0, p0, x1, p1 = x0[m], p0[m], x1[m], p1[m]
    v0, v1 = _tangents(st, p0, p1)
    u = crossing_root(st, x0, v0, x1, v1)
    h, d, _ = hermite(u[:, None])
    ahat = st.a0 + u * st.da
    xhat = _spline(h, x0, v0, x1, v1)
    S = ahat ** 3 * _E(ahat, st.om)
    phat = S[:, None] * _spline(d, x0, v0, x1, v1) / st.da
    return m, xhat, phat, ahat, u


def observe_step_vjp(st, x0, p0, x1, p1, u, gx, gp, ga):
    """Transpose of observe_step for the observed particles (rows already
    selected), at their root u.  gx, gp: (M, 3) cotangents of x^ and p^, ga:
    (M,) cotangent of a^.  Returns (x0_bar, p0_bar, x1_bar, p1_bar, om_bar)
    (reading L6)."""
    da = st.da
    v0, v1 = _tangents(st, p0, p1)
    h, d, dd = hermite(u[:, None])
    hs, ds, _ = hermite(u)
    pos = _spline(h, x0, v0, x1, v1)
    vel = _spline(d, x0, v0, x1, v1)          # dx/du
    acc = _spline(dd, x0, v0, x1, v1)         # d2x/du2
    rel = pos - st.X
    r = np.linalg.norm(rel, axis=1)
    # |x - X| has no gradient at the observer itself; reading L3 takes it as zero there
    rhat = np.divide(rel, r[:, None], out=np.zeros_like(rel), where=r[:, None] > 0)
    ahat = st.a0 + u * da
    E = _E(ahat, st.om)
    S = ahat ** 3 * E
    dS_da = 3 * ahat ** 2 * E + ahat ** 3 * _dE_da(ahat, st.om)
    dS_dom = ahat ** 3 * _dE_dom(ahat, st.om)
    # d(observables)/du contracted with the cotangents, and df/du
    G_u = (np.sum(gx * vel, axis=1) + np.sum(gp * (dS_da[:, None] * vel + S[:, None] * acc / da), axis=1)
           + ga * da)
    f_u = np.sum(rhat * vel, axis=1) - _front(st, ds)
    lam = -G_u / f_u
    # direct dependence at fixed u, plus lam * df/d(input)
    cx = gx + lam[:, None] * rhat                      # multiplies the basis h
    cp = gp * (S / da)[:, None]                        # multiplies the basis d
    x0b = h[0] * cx + d[0] * cp
    v0b = h[1] * cx + d[1] * cp
    x1b = h[2] * cx + d[2] * cp
    v1b = h[3] * cx + d[3] * cp
    p0b = da * st.w0 * v0b
    p1b = da * st.w1 * v1b
    om_b = np.sum(np.sum(gp * vel, axis=1) / da * dS_dom)
    om_b += np.sum(-lam * (hs[0] * st.c0_om + hs[1] * da * st.dc0_om + hs[2] * st.c1_om + hs[3] * da * st.dc1_om))
    om_b += np.sum(da * p0 * v0b) * st.w0_om + np.sum(da * p1 * v1b) * st.w1_om
    return x0b, p0b, x1b, p1b, om_b


# ----------------------------------------------------------------------------
# a whole run: forward with observation, and the exact gradient
# ----------------------------------------------------------------------------


def integer_momenta(p0, traj, coefs):
    """p_0 and p_i = p_{i-1/2} + a_i Kb_i, i = 1..n (reading L5)."""
    return [np.array(p0, dtype=np.float64)] + [traj["p_half"][i - 1] + traj["a"][i] * coefs[i - 1][2]
                                               for i in range(1, len(coefs) + 1)]


def observe_run(traj, P, a_grid, om, cell, observer):
    """Observation over all steps of a stored trajectory.  Returns (obs, step)
    with obs (N, 7) = (x^, p^, a^) (zeros where never observed) and step (N,)
    the step of the crossing (0 = never observed)."""
    N = traj["x"][0].shape[0]
    obs = np.zeros((N, 7))
    step = np.zeros(N, dtype=np.int64)
    for i in range(1, len(a_grid)):
        st = Step(a_grid[i - 1], a_grid[i], om, cell, observer)
        m, xh, ph, ah, _ = observe_step(st, traj["x"][i - 1], P[i - 1], traj["x"][i], P[i])
        obs[m, 0:3], obs[m, 3:6], obs[m, 6] = xh, ph, ah
        step[m] = i
    return obs, step


def linear_objective(obs, step, weights):
    """J = sum over observed particles of weights . (x^, p^, a^) (the test
    objective on the observables; weights (N, 7))."""
    seen = step > 0
    return float(np.sum(weights[seen] * obs[seen]))


def observation_cotangents(traj, P, a_grid, om, cell, observer, step, obs_bar):
    """dJ/dx_k and dJ/dp_k (k = 0..n) from the observations, and the direct
    Omega_m part, for cotangents obs_bar (N, 7) of the observed states."""
    n = len(a_grid) - 1
    N = traj["x"][0].shape[0]
    xb = [np.zeros((N, 3)) for _ in range(n + 1)]
    pb = [np.zeros((N, 3)) for _ in range(n + 1)]
    om_b = 0.0
    for i in range(1, n + 1):
        sel = step == i
        if not np.any(sel):
            continue
        st = Step(a_grid[i - 1], a_grid[i], om, cell, observer)
        x0, p0, x1, p1 = traj["x"][i - 1][sel], P[i - 1][sel], traj["x"][i][sel], P[i][sel]
        v0, v1 = _tangents(st, p0, p1)
        u = crossing_root(st, x0, v0, x1, v1)
        g = obs_bar[sel]
        x0b, p0b, x1b, p1b, ob = observe_step_vjp(st, x0, p0, x1, p1, u, g[:, 0:3], g[:, 3:6], g[:, 6])
        xb[i - 1][sel] += x0b
        pb[i - 1][sel] += p0b
        xb[i][sel] += x1b
        pb[i][sel] += p1b
        om_b += ob
    return xb, pb, om_b


def adjoint_stored_with_observations(traj, coefs, dcoefs, xb, pb, F, step=None):
    """Reverse accumulation through eq. KDFK along the stored trajectory with
    the partial derivatives dJ/dx_k, dJ/dp_k added at every integer time k
    (eq. explicit_adj).  Returns (xi_0, pi_0, dJ/dOmega_m from the steps).
    With `step` (the crossing step of each particle, 0 = never observed) the
    adjoint is truncated as in reading L7."""
    n = len(coefs)
    xi = np.array(xb[n], dtype=np.float64)
    pi = np.array(pb[n], dtype=np.float64)
    th = 0.0
    for i in range(n, 0, -1):
        Ka, D, Kb = coefs[i - 1]
        dKa, dD, dKb = dcoefs[i - 1]
        x_i, a_i = traj["x"][i], traj["a"][i]
        p_half = traj["p_half"][i - 1]
        x_im1, a_im1 = traj["x"][i - 1], traj["a"][i - 1]
        # p_i = p_{i-1/2} + a(x_i) Kb_i
        g, ob, _ = F.vjp(x_i, pi * Kb)
        th += np.sum(pi * a_i) * dKb + ob
        if step is not None:
            g[(step > 0) & (step <= i)] = 0.0         # frozen at t_i (reading L7)
        xi = xi + g
        # x_i = x_{i-1} + p_{i-1/2} D_i
        th += np.sum(xi * p_half) * dD
        pi = pi + xi * D
        # p_{i-1/2} = p_{i-1} + a(x_{i-1}) Ka_i
        g, ob, _ = F.vjp(x_im1, pi * Ka)
        th += np.sum(pi * a_im1) * dKa + ob
        if step is not None:
            g[(step > 0) & (step <= i - 1)] = 0.0     # frozen at t_{i-1}
        xi = xi + g
        # the observations' partial derivatives at t_{i-1}
        xi = xi + xb[i - 1]
        pi = pi + pb[i - 1]
    return xi, pi, th


def value_and_grad(omega, cfg, observer, weights, truncate=False):
    """J = linear_objective of the light-cone observation of the run from
    white noise omega, and (dJ/domega, dJ/dOmega_m, dJ/dsigma8), exact or
    (truncate) with the adjoint of reading L7.  Returns (J, g_omega,
    g_theta, obs, step)."""
    from . import simulate
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    om = cfg.cosmo.omega_m
    a_grid = cfg.a_grid()
    cell = cfg.box / cfg.n_mesh
    coefs, dcoefs = cosmology.step_coefficients_with_derivative(a_grid, om)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, om)
    _, _, _, traj = integrate.forward(q, s0, p0, coefs, F, store=True)
    P = integer_momenta(p0, traj, coefs)
    obs, step = observe_run(traj, P, a_grid, om, cell, observer)
    J = linear_objective(obs, step, weights)
    xb, pb, om_obs = observation_cotangents(traj, P, a_grid, om, cell, observer, step, weights)
    xi0, pi0, th = adjoint_stored_with_observations(traj, coefs, dcoefs, xb, pb, F, step if truncate else None)
    g_omega = lpt.lpt_vjp(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r, xi0, pi0)
    ds, dp = lpt.lpt_jvp_omega_m(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r)
    g_om = th + om_obs + np.sum(xi0 * ds) + np.sum(pi0 * dp)
    ds8, dp8 = lpt.lpt_dsigma8(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r)
    g_s8 = np.sum(xi0 * ds8) + np.sum(pi0 * dp8)
    return J, g_omega, np.array([g_om, g_s8]), obs, step


def objective_value(omega, cfg, observer, weights):
    """J alone (for finite differences)."""
    from . import simulate
    q = simulate.lattice(cfg)
    s0, p0 = simulate.initial_state(omega, cfg)
    om = cfg.cosmo.omega_m
    a_grid = cfg.a_grid()
    coefs = cosmology.step_coefficients(a_grid, om)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, om)
    _, _, _, traj = integrate.forward(q, s0, p0, coefs, F, store=True)
    P = integer_momenta(p0, traj, coefs)
    obs, step = observe_run(traj, P, a_grid, om, cfg.box / cfg.n_mesh, observer)
    return linear_objective(obs, step, weights)
