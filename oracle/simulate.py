"""End-to-end forward model J(omega, theta) and its gradients -- plain FP64
reference.

Test infrastructure only (see oracle/__init__.py).

Follows Fig. 1 of the paper: Boltz (growth, transfer function) -> LPT ->
Integ (KDK leapfrog, eq. KDFK) -> Obs/Obj (final-snapshot density MSE); the
gradient follows eq. KDFKO_grad:
    dJ/dtheta = xi_0 . dx_0/dtheta + pi_0 . dp_0/dtheta + (step terms)
    dJ/domega = xi_0 . dx_0/domega + pi_0 . dp_0/domega
with theta = (Omega_m, sigma8).
"""
import numpy as np

from . import cosmology, integrate, lpt, objective, pm


class SimConfig:
    def __init__(self, n_ptcl, n_mesh, box, a_start, a_end, n_steps, cosmo=None, offset=0.0):
        self.n_ptcl = n_ptcl
        self.n_mesh = n_mesh
        self.box = box
        self.a_start = a_start
        self.a_end = a_end
        self.n_steps = n_steps
        self.cosmo = cosmo if cosmo is not None else cosmology.Cosmo()
        self.offset = offset

    @property
    def r(self):
        return self.n_mesh / self.n_ptcl

    @property
    def n_particles(self):
        return self.n_ptcl ** 3

    @property
    def mesh_shape(self):
        return (self.n_mesh,) * 3

    def a_grid(self):
        return cosmology.linear_a_grid(self.a_start, self.a_end, self.n_steps)

    def with_cosmo(self, cosmo):
        return SimConfig(self.n_ptcl, self.n_mesh, self.box, self.a_start, self.a_end,
                         self.n_steps, cosmo, self.offset)


def lattice(cfg):
    return pm.lattice_positions((cfg.n_ptcl,) * 3, cfg.r, cfg.offset)


def initial_state(omega, cfg):
    return lpt.lpt(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r)


def final_state(omega, cfg):
    """Run the forward model; returns (q, s_n, p_n, a_n)."""
    q = lattice(cfg)
    s0, p0 = initial_state(omega, cfg)
    coefs = cosmology.step_coefficients(cfg.a_grid(), cfg.cosmo.omega_m)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, cfg.cosmo.omega_m)
    s, p, a, _ = integrate.forward(q, s0, p0, coefs, F, store=False)
    return q, s, p, a


def final_density(omega, cfg):
    q, s, _, _ = final_state(omega, cfg)
    return pm.density_contrast(q + s, cfg.mesh_shape, cfg.n_particles)


def objective_value(omega, cfg, target):
    q, s, _, _ = final_state(omega, cfg)
    J, _ = objective.density_mse(q + s, target, cfg.n_particles)
    return J


class FixedThetaObjective:
    """omega -> J at fixed theta, with the theta-only tables (step coefficients,
    initial-condition time factors, amplitude A(k)) computed once; used for
    brute-force finite differences over many white-noise entries."""

    def __init__(self, cfg, target):
        self.cfg = cfg
        self.target = target
        cos = cfg.cosmo
        self.q = lattice(cfg)
        self.coefs = cosmology.step_coefficients(cfg.a_grid(), cos.omega_m)
        self.tf = lpt.ic_time_factors(cfg.a_start, cos.omega_m)
        self.amp = lpt.amplitude(cfg.n_ptcl, cfg.box, cos)
        self.F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, cos.omega_m)

    def __call__(self, omega):
        s1, s2, _ = lpt.lpt_fields(omega, self.cfg.box, self.cfg.cosmo, amp=self.amp)
        D1, D2, P1, P2 = self.tf
        r = self.cfg.r
        s0 = (r * (D1 * s1 + D2 * s2)).reshape(3, -1).T
        p0 = (r * (P1 * s1 + P2 * s2)).reshape(3, -1).T
        s, _, _, _ = integrate.forward(self.q, s0, p0, self.coefs, self.F, store=False)
        J, _ = objective.density_mse(self.q + s, self.target, self.cfg.n_particles)
        return J


def value_and_grad(omega, cfg, target, mode="stored", final_state_out=None, checkpoint_steps=()):
    """J and (dJ/domega, dJ/dOmega_m, dJ/dsigma8).

    mode = "stored": discrete adjoint along the stored trajectory (plain chain
    rule, Sec. 3.5); mode = "reverse": adjoint with reverse-time integration
    (eq. KDFKO_adj), resumed from forward checkpoints at `checkpoint_steps`
    (Sec. 3.5) if any.  If `final_state_out` is a dict, the final forward
    state is stored in it as "s" and "p" ((N, 3) arrays)."""
    q = lattice(cfg)
    s0, p0 = initial_state(omega, cfg)
    om = cfg.cosmo.omega_m
    coefs, dcoefs = cosmology.step_coefficients_with_derivative(cfg.a_grid(), om)
    F = integrate.ForceModel(cfg.mesh_shape, cfg.n_particles, om)
    ck = {int(j): None for j in checkpoint_steps}
    s, p, a, traj = integrate.forward(q, s0, p0, coefs, F, store=(mode == "stored"), checkpoints=ck)
    if final_state_out is not None:
        final_state_out["s"], final_state_out["p"] = s.copy(), p.copy()
    J, xbar = objective.density_mse(q + s, target, cfg.n_particles)
    pbar = np.zeros_like(xbar)
    if mode == "stored":
        xi0, pi0, th = integrate.adjoint_stored(traj, coefs, dcoefs, xbar, pbar, F)
    else:
        _, _, xi0, pi0, th = integrate.adjoint_reverse(q, s, p, a, xbar, pbar, coefs, dcoefs, F, checkpoints=ck)
    g_omega = lpt.lpt_vjp(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r, xi0, pi0)
    ds, dp = lpt.lpt_jvp_omega_m(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r)
    g_om = th + np.sum(xi0 * ds) + np.sum(pi0 * dp)
    ds8, dp8 = lpt.lpt_dsigma8(omega, cfg.box, cfg.cosmo, cfg.a_start, cfg.r)
    g_s8 = np.sum(xi0 * ds8) + np.sum(pi0 * dp8)
    return J, g_omega, np.array([g_om, g_s8])
