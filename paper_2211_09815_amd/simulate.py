"""Differentiable forward model on the GPU: 2LPT -> KDK leapfrog -> final
density MSE, with the adjoint pass of the paper (reverse-time integration,
eq. KDFKO_adj) giving dJ/domega and dJ/d(Omega_m, sigma8) (eq. KDFKO_grad).

Everything numeric runs in libpm through the binding in api.py; this module
only sequences the library calls and owns the device buffers.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import api


@dataclass
class SimConfig:
    n_ptcl: int            # particles per side
    n_mesh: int            # mesh cells per side
    box: float             # Mpc/h
    a_start: float
    a_end: float
    n_steps: int
    mesh_dtype: torch.dtype = torch.float32
    state_dtype: torch.dtype = torch.float64
    lattice_offset: float = 0.0
    # steps j (1..n_steps) whose forward state (s_j, p_{j-1/2}) is saved for
    # the piecewise reverse pass (Sec. 3.5); empty: plain reverse integration
    checkpoint_steps: tuple = ()
    # fixed-point paint (bitwise reproducible) or floating-point LDS atomics
    deterministic: bool = True

    @property
    def n_particles(self):
        return self.n_ptcl ** 3

    def a_grid(self):
        """Steps linearly spaced in a (Sec. 4)."""
        return np.linspace(self.a_start, self.a_end, self.n_steps + 1)


class Simulation:
    def __init__(self, cfg: SimConfig):
        self.cfg = cfg
        self.plan = api.Plan(cfg.n_mesh, cfg.n_ptcl, box=cfg.box, lattice_offset=cfg.lattice_offset,
                             mesh_dtype=cfg.mesh_dtype, state_dtype=cfg.state_dtype,
                             deterministic=cfg.deterministic)
        dev = self.plan.device
        n = cfg.n_particles
        self.s = torch.zeros((3, n), dtype=self.plan.sdt, device=dev)
        self.p = torch.zeros((3, n), dtype=self.plan.sdt, device=dev)
        self.acc = torch.zeros((3, n), dtype=self.plan.mdt, device=dev)
        self.xi = torch.zeros((3, n), dtype=self.plan.mdt, device=dev)
        self.pi = torch.zeros((3, n), dtype=self.plan.mdt, device=dev)
        self.theta_bar = torch.zeros(2, dtype=torch.float64, device=dev)
        self.checkpoints = self.plan.new_checkpoints(cfg.checkpoint_steps) if cfg.checkpoint_steps else None

    def state(self):
        return {"s": self.s, "p": self.p, "acc": self.acc}

    def adj(self):
        return {"xi": self.xi, "pi": self.pi}

    def tables(self, cosmo):
        return api.tables(cosmo, self.cfg.a_grid())

    def forward(self, omega, cosmo, tables=None):
        """2LPT + n KDK steps; leaves (s_n, p_n, a_n) in the simulation buffers."""
        coefs, ic = tables if tables is not None else self.tables(cosmo)
        st = self.state()
        self.plan.lpt(omega, cosmo, ic, st)
        if self.checkpoints is None:
            self.plan.run_fwd(st, coefs, cosmo.omega_m)
        else:
            self.plan.run_fwd_ckpt(st, coefs, cosmo.omega_m, self.checkpoints)
        return coefs, ic

    def final_density(self, omega, cosmo):
        self.forward(omega, cosmo)
        return self.plan.density(self.s)

    def value_and_grad(self, omega, cosmo, target, tables=None):
        """(J, dJ/domega, dJ/d(Omega_m, sigma8)) as device tensors."""
        coefs, ic = self.forward(omega, cosmo, tables)
        J, xbar = self.plan.density_mse(self.s, target)
        self.xi.copy_(xbar)
        self.pi.zero_()
        self.theta_bar.zero_()
        if self.checkpoints is None:
            self.plan.run_adj(self.state(), self.adj(), coefs, cosmo.omega_m, self.theta_bar)
        else:
            self.plan.run_adj_ckpt(self.state(), self.adj(), coefs, cosmo.omega_m, self.checkpoints,
                                   self.theta_bar)
        g_omega = self.plan.lpt_vjp(omega, cosmo, ic, self.adj(), self.theta_bar)
        return J, g_omega, self.theta_bar.clone()


class Simulate(torch.autograd.Function):
    """J = Simulate.apply(omega, theta, sim, target, base_cosmo) with
    theta = (Omega_m, sigma8); backward returns dJ/domega and dJ/dtheta from
    the adjoint pass (no automatic differentiation through the steps)."""

    @staticmethod
    def forward(ctx, omega, theta, sim, target, base_cosmo):
        th = theta.detach().cpu().double().numpy()
        cosmo = base_cosmo.replace(omega_m=float(th[0]), sigma8=float(th[1]))
        J, g_omega, g_theta = sim.value_and_grad(omega.detach().contiguous(), cosmo, target)
        ctx.save_for_backward(g_omega, g_theta.to(theta.dtype).to(theta.device))
        return J.reshape(()).to(omega.dtype)

    @staticmethod
    def backward(ctx, gJ):
        g_omega, g_theta = ctx.saved_tensors
        return gJ * g_omega, gJ * g_theta, None, None, None
