"""KDK leapfrog and its discrete adjoint -- plain FP64 reference.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * eq. KDFK (Sec. 2.3): from t_{i-1} to t_i,
        p_{i-1/2} = p_{i-1} + a_{i-1} Ka_i,   x_i = x_{i-1} + p_{i-1/2} D_i,
        a_i = F(x_i),                          p_i = p_{i-1/2} + a_i Kb_i,
    with a_0 = F(x_0) before the first step.  Kicks are applied separately
    (not merged) so that each line of the scheme is visible.
  * eq. explicit_adj / explicit_grad (Sec. 3.5, discretize-then-optimize):
    the discrete adjoint along the stored forward trajectory is plain reverse
    accumulation of the chain rule through every line of eq. KDFK.
  * eq. KDFKO_adj and KDFKO_grad (Sec. 3.6): the adjoint KDK stepping from t_i
    to t_{i-1}, which re-integrates (x, p) backward together with (xi, pi) and
    caches alpha = pi . da/dx and zeta = pi . da/dtheta; the objective gradient
    with respect to theta accumulates the kick and drift factor derivatives.
  * Sec. 3.5 (end): when the backward evolution drifts from the forward one,
    it can be resumed piecewise from states saved during the forward pass.
    Checkpoint j holds s_j and p_{j-1/2}, the values the reverse step j starts
    from; the reverse pass takes s_j from it when its drift reaches t_j and
    p_{j-1/2} when its kick does.

theta here is Omega_m only (the step coefficients and the force coefficient
1.5 Omega_m depend on nothing else); sigma8 enters through the initial
conditions only.  K(t_i, t_i, t_{i-1/2}) = -Kb_i and D(t_{i-1/2}, t_i,
t_{i-1}) = -D_i (antisymmetry of the factors), which turns the paper's leading
minus signs into the plus signs below.
"""
import numpy as np

from . import pm

FORCE_COEF_PER_OMEGA_M = 1.5  # coef = 1.5 Omega_m (H0 = 1)


class ForceModel:
    """F(x) on a periodic mesh; x are absolute positions in cell units."""

    def __init__(self, mesh_shape, n_particles, omega_m):
        self.shape = tuple(mesh_shape)
        self.n = n_particles
        self.om = omega_m
        self.coef = FORCE_COEF_PER_OMEGA_M * omega_m

    def __call__(self, x):
        return pm.force(x, self.shape, self.n, self.coef)

    def vjp(self, x, cot):
        """(cot . da/dx, cot . da/dOmega_m, a)."""
        xbar, coef_bar, a = pm.force_vjp(x, cot, self.shape, self.n, self.coef)
        return xbar, coef_bar * FORCE_COEF_PER_OMEGA_M, a


def forward(q, s0, p0, coefs, F, store=True, checkpoints=None):
    """KDK forward (eq. KDFK).  Returns (s_n, p_n, a_n, traj) where traj holds
    x_i (i = 0..n), p_{i-1/2} (i = 1..n) and a_i (i = 0..n) if store.  If
    `checkpoints` is a dict whose keys are steps j (1..n), each value is set to
    (s_j, p_{j-1/2})."""
    s = np.array(s0, dtype=np.float64)
    p = np.array(p0, dtype=np.float64)
    a = F(q + s)
    traj = {"x": [q + s], "p_half": [], "a": [a]} if store else None
    for i, (Ka, D, Kb) in enumerate(coefs, start=1):
        p = p + a * Ka
        if store:
            traj["p_half"].append(p.copy())
        s = s + p * D
        if checkpoints is not None and i in checkpoints:
            checkpoints[i] = (s.copy(), p.copy())
        a = F(q + s)
        p = p + a * Kb
        if store:
            traj["x"].append(q + s)
            traj["a"].append(a)
    return s, p, a, traj


def adjoint_stored(traj, coefs, dcoefs, xbar_n, pbar_n, F):
    """Reverse accumulation of the chain rule through eq. KDFK along the stored
    trajectory (the 'AD' gradient of Sec. 4.2).

    Returns (xi_0, pi_0, dJ/dOmega_m from the steps)."""
    xi = np.array(xbar_n, dtype=np.float64)
    pi = np.array(pbar_n, dtype=np.float64)
    th = 0.0
    n = len(coefs)
    for i in range(n, 0, -1):
        Ka, D, Kb = coefs[i - 1]
        dKa, dD, dKb = dcoefs[i - 1]
        x_i, a_i = traj["x"][i], traj["a"][i]
        p_half = traj["p_half"][i - 1]
        x_im1, a_im1 = traj["x"][i - 1], traj["a"][i - 1]
        # p_i = p_{i-1/2} + a(x_i) Kb_i
        xb, ob, _ = F.vjp(x_i, pi * Kb)
        th += np.sum(pi * a_i) * dKb + ob
        xi = xi + xb
        # x_i = x_{i-1} + p_{i-1/2} D_i
        th += np.sum(xi * p_half) * dD
        pi = pi + xi * D
        # p_{i-1/2} = p_{i-1} + a(x_{i-1}) Ka_i
        xb, ob, _ = F.vjp(x_im1, pi * Ka)
        th += np.sum(pi * a_im1) * dKa + ob
        xi = xi + xb
    return xi, pi, th


def adjoint_reverse(q, s_n, p_n, a_n, xi_n, pi_n, coefs, dcoefs, F, checkpoints=None):
    """Adjoint KDK with reverse-time integration (eq. KDFKO_adj, KDFKO_grad).

    (x, p) are re-integrated backward jointly with (xi, pi); a and the VJP
    caches alpha, zeta are recomputed at each x_{i-1}.  a_n comes from the
    forward pass; alpha_n, zeta_n from one VJP at x_n.  `checkpoints` ({j:
    (s_j, p_{j-1/2})}, as filled by forward) resumes (x, p) from the saved
    states.  Returns (s_0, p_0, xi_0, pi_0, dJ/dOmega_m from the steps)."""
    ck = checkpoints or {}
    s = np.array(s_n, dtype=np.float64)
    p = np.array(p_n, dtype=np.float64)
    xi = np.array(xi_n, dtype=np.float64)
    pi = np.array(pi_n, dtype=np.float64)
    a = np.array(a_n, dtype=np.float64)
    alpha, zeta, _ = F.vjp(q + s, pi)
    th = 0.0
    n = len(coefs)
    for i in range(n, 0, -1):
        Ka, D, Kb = coefs[i - 1]
        dKa, dD, dKb = dcoefs[i - 1]
        # K_i^{i-1/2}
        p = p - a * Kb
        if i in ck:
            p = np.array(ck[i][1], dtype=np.float64)
        xi = xi + alpha * Kb
        th += np.sum(pi * a) * dKb + zeta * Kb
        # D_i^{i-1}
        th += np.sum(xi * p) * dD
        s = s - p * D
        if i - 1 in ck:
            s = np.array(ck[i - 1][0], dtype=np.float64)
        pi = pi + xi * D
        # F_{i-1}
        alpha, zeta, a = F.vjp(q + s, pi)
        # K_{i-1/2}^{i-1}
        p = p - a * Ka
        xi = xi + alpha * Ka
        th += np.sum(pi * a) * dKa + zeta * Ka
    return s, p, xi, pi, th


def backward_only(q, s_n, p_n, a_n, coefs, F):
    """Reverse-time integration of (x, p) alone (the first lines of the K and
    D operators of eq. KDFKO_adj), used for the reversibility pin."""
    s = np.array(s_n, dtype=np.float64)
    p = np.array(p_n, dtype=np.float64)
    a = np.array(a_n, dtype=np.float64)
    for i in range(len(coefs), 0, -1):
        Ka, D, Kb = coefs[i - 1]
        p = p - a * Kb
        s = s - p * D
        a = F(q + s)
        p = p - a * Ka
    return s, p
