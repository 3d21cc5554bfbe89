"""Light-cone observation during the forward pass, and the gradient of an
objective on the observables by the adjoint with reverse-time integration
(Sec. 2.4, Sec. 3.4, eq. explicit_adj).

Every numeric step runs in libpm (api.py); this module only sequences the
calls and owns the buffers.

Forward: the light front moves inward at the speed of light, so a particle
outside it stays outside, and no particle crosses before the front has come
within reach of one.  The steps before that run as the native loop
(pm_run_fwd, merged kicks), up to the last step m whose front lies further
from the observer than any lattice site plus a displacement margin; then
pm_lightcone_reach checks that every particle is inside the front of a_m (if
one is not, the forward pass starts again and observes every step).  From
there the kicks are not merged, so that the state holds the integer-time
momenta p_i that the Hermite splines need: pm_step_fwd(i) without a next step
leaves (s_i, p_i, a_i), pm_lightcone observes step i from the saved (s_{i-1},
p_{i-1}), and pm_kick applies the first half kick of step i + 1.

Reverse: the objective's cotangent reaches the states (x_k, p_k) of the two
ends of each particle's crossing step.  A cotangent of p_k also reaches a_k
(p_k = p_{k-1/2} + a_k Kb_k), and through the force VJP at x_k the position
adjoint; pm_adj_bump adds both at t_k, right after pm_step_adj(k + 1) has
brought the reverse integration to t_k.  The observation of step k needs the
state at t_{k-1} before the reverse integration gets there, so one step ahead
the driver reconstructs x_{k-1} (pm_drift) and a_{k-1} (pm_force).  Steps in
which no particle crosses, and the steps next to them, skip all of this;
below the first observed step the rest of the reverse pass is the native loop
(pm_run_adj_from).  The gradient is the exact gradient of the discrete
forward map, up to the reversibility of the reconstruction.

With truncate, the gradient is the truncated adjoint of Sec. 3.4 in the
library's discrete form (pm_lightcone_truncate): every force VJP at t_m gives
the particles observed in steps 1..m nothing.  Those VJPs are pm_adj_init's
at t_n, each pm_step_adj(m + 1)'s at x_m and each bump's; the position
cotangent of the observation at t_n is added after pm_adj_init's.
"""
import numpy as np
import torch

from . import api


class LightCone:
    """Observer at `observer` (mesh cells, the frame of q + s) of the run of
    Simulation `sim`."""

    def __init__(self, sim, observer):
        self.sim = sim
        self.observer = [float(v) for v in observer]
        plan = sim.plan
        dev, n = plan.device, sim.cfg.n_particles
        sd = lambda: torch.empty((3, n), dtype=plan.sdt, device=dev)   # noqa: E731
        md = lambda: torch.zeros((3, n), dtype=plan.mdt, device=dev)   # noqa: E731
        self.obs = torch.zeros((7, n), dtype=plan.sdt, device=dev)
        self.obs_step = torch.zeros(n, dtype=torch.int32, device=dev)
        self.counts = torch.zeros(sim.cfg.n_steps + 1, dtype=torch.float64, device=dev)
        self.x_tmp, self.p_tmp, self.p_int = sd(), sd(), sd()
        self.xb = [md(), md()]      # position cotangents of z_k (cur) and z_{k-1} (pending)
        self.pb = [md(), md()]
        self.a = [md(), md()]       # a_k (cur) and a_{k-1} (ahead)
        self.c = md()
        self.cb = torch.zeros(1, dtype=torch.float64, device=dev)
        self.n_obs = None

    def tables(self, cosmo):
        coefs, ic = self.sim.tables(cosmo)
        cell = self.sim.cfg.box / self.sim.cfg.n_mesh
        return coefs, ic, api.lightcone_tables(cosmo, self.sim.cfg.a_grid(), cell)

    def _step(self, lc, cosmo, i):
        return api.lc_step(lc[i - 1], lc[i], cosmo.omega_m, self.observer, i)

    def quiet_steps(self, lc, margin):
        """The last step m < n whose light front (lc[m].chi, mesh cells) lies
        further from the observer than every lattice site by more than
        `margin` cells, or 0.  Host arithmetic on the lattice's extent."""
        cfg = self.sim.cfg
        r = cfg.n_mesh / cfg.n_ptcl
        ends = np.array([cfg.lattice_offset, (cfg.n_ptcl - 1) * r + cfg.lattice_offset])
        reach = np.sqrt(sum(np.max(np.abs(ends - x)) ** 2 for x in self.observer)) + margin
        m = 0
        for i in range(1, len(lc) - 1):
            if lc[i].chi > reach:
                m = i
        return m

    def forward(self, omega, cosmo, tables=None, margin=None):
        """2LPT, n KDK steps and the observation of every step.  Leaves
        (s_n, p_n, a_n) in the simulation and (x^, p^, a^) in self.obs;
        returns the host array of particles observed per step (index 1..n).
        The steps before the front can reach a particle (quiet_steps with a
        displacement margin, default a quarter of the mesh side; checked)
        run as the native loop without observation."""
        sim, plan = self.sim, self.sim.plan
        coefs, ic, lc = tables if tables is not None else self.tables(cosmo)
        n = len(coefs)
        om = cosmo.omega_m
        st = sim.state()
        self.obs.zero_()
        self.obs_step.zero_()
        self.counts.zero_()
        s_prev, p_prev = self.x_tmp, self.p_tmp
        m = self.quiet_steps(lc, sim.cfg.n_mesh / 4 if margin is None else margin)
        plan.lpt(omega, cosmo, ic, st)
        if m > 0:
            plan.run_fwd(st, coefs[:m], om)                  # (s_m, p_m, a_m)
            if not float(plan.lightcone_reach(sim.s, self.observer).item()) < lc[m].chi:
                m = 0                                        # a particle is out already: observe every step
                plan.lpt(omega, cosmo, ic, st)
        self.native_steps = m
        s_prev.copy_(sim.s)
        p_prev.copy_(sim.p)
        if m > 0:
            plan.kick(sim.p, sim.acc, coefs[m][0], out=sim.p)   # first half kick of step m + 1
        else:
            plan.fwd_init(st, coefs[0], om)
        for i in range(m + 1, n + 1):
            plan.step_fwd(st, coefs[i - 1], None, om)
            plan.lightcone(self._step(lc, cosmo, i), s_prev, p_prev, sim.s, sim.p, self.obs, self.obs_step,
                           self.counts[i:i + 1])
            if i < n:
                s_prev.copy_(sim.s)
                p_prev.copy_(sim.p)
                plan.kick(sim.p, sim.acc, coefs[i][0], out=sim.p)
        self.n_obs = self.counts.cpu().numpy().round().astype(np.int64)
        return self.n_obs

    def _swap(self):
        self.xb.reverse()
        self.pb.reverse()
        self.xb[1].zero_()
        self.pb[1].zero_()

    def gradient(self, omega, cosmo, obs_bar, tables=None, truncate=False):
        """dJ/domega and dJ/d(Omega_m, sigma8) for the cotangent obs_bar
        ([7, N_p] mesh dtype) of the observed (x^, p^, a^), after forward()
        with the same arguments; truncate: the truncated adjoint (module
        docstring).  Returns (g_omega, theta_bar) on the device."""
        sim, plan = self.sim, self.sim.plan
        coefs, ic, lc = tables if tables is not None else self.tables(cosmo)
        n = len(coefs)
        cnt = np.concatenate([self.n_obs, [0]])        # cnt[n + 1] = 0
        om = cosmo.omega_m
        st, adj = sim.state(), sim.adj()
        thb = sim.theta_bar.zero_()
        sim.xi.zero_()
        sim.pi.zero_()
        for t in self.xb + self.pb:
            t.zero_()
        need = lambda k: cnt[k] > 0 or cnt[k + 1] > 0   # noqa: E731  cotangents on z_k
        observed = [j for j in range(1, n + 1) if cnt[j] > 0]
        first = observed[0] if observed else n + 1       # reverse steps below it are plain
        self.a[0].copy_(sim.acc)                         # a_n
        s, p = sim.s, sim.p

        def ahead(k, p_half):
            # x_{k-1}, a_{k-1}, p_{k-1} from (s_k, p_{k-1/2})
            Ka, D = coefs[k - 1][0], coefs[k - 1][1]
            plan.drift(s, p_half, -D, out=self.x_tmp)
            plan.force(self.x_tmp, om, out=self.a[1])
            plan.kick(p_half, self.a[1], -Ka, out=self.p_tmp)

        # t_n: pm_adj_init's own VJP at x_n already carries Kb_n pi_n
        init_ahead = cnt[n] > 0 or (n >= 2 and cnt[n - 1] > 0)
        if init_ahead:
            plan.kick(p, self.a[0], -coefs[n - 1][2], out=self.p_int)    # p_{n-1/2}
            ahead(n, self.p_int)
        x1b = sim.xi
        if truncate:
            self.c.zero_()
            x1b = self.c      # added after pm_adj_init's VJP, which freezes the observed
        if cnt[n] > 0:
            plan.lightcone_vjp(self._step(lc, cosmo, n), self.x_tmp, self.p_tmp, s, p, self.obs_step, obs_bar,
                               self.xb[1], self.pb[1], x1b, sim.pi, thb)
        plan.adj_init(st, adj, coefs[n - 1], om, thb)
        if truncate and first <= n:
            plan.lightcone_truncate(sim.xi, self.obs_step, n)
            plan.adj_bump(sim.xi, None, self.c, None, None, 0.0, 0.0, None, None, thb)
        self._swap()
        if init_ahead:
            self.a.reverse()
        for i in range(n, 0, -1):
            if i < first:
                # nothing observed in steps 1..i+1: the native reverse loop
                plan.run_adj_from(st, adj, coefs[:i], om, thb)
                break
            plan.step_adj(st, adj, coefs[i - 1], coefs[i - 2] if i > 1 else None, om, thb)
            k = i - 1
            frozen = truncate and k >= first     # particles observed in steps 1..k
            if frozen:
                plan.lightcone_truncate(sim.xi, self.obs_step, k)
            if k == 0:
                if cnt[1] > 0:
                    plan.adj_bump(sim.xi, sim.pi, self.xb[0], self.pb[0], None, 0.0, 0.0, None, None, thb)
                break
            go_ahead = cnt[k] > 0 or (k >= 2 and cnt[k - 1] > 0)
            if need(k):
                plan.kick(p, self.a[0], coefs[k - 1][2], out=self.p_int)   # p_k
            if go_ahead:
                ahead(k, p)
            if cnt[k] > 0:
                plan.lightcone_vjp(self._step(lc, cosmo, k), self.x_tmp, self.p_tmp, s, self.p_int, self.obs_step,
                                   obs_bar, self.xb[1], self.pb[1], self.xb[0], self.pb[0], thb)
            if need(k):
                self.cb.zero_()
                plan.force_vjp(s, self.pb[0], om, want_acc=False, out=self.c, omega_m_bar=self.cb)
                if frozen:
                    plan.lightcone_truncate(self.c, self.obs_step, k)
                Kb, dKb = coefs[k - 1][2], coefs[k - 1][5]
                plan.adj_bump(sim.xi, sim.pi, self.xb[0], self.pb[0], self.c, Kb, dKb, self.a[0], self.cb, thb)
                self._swap()
            if go_ahead:
                self.a.reverse()
        g_omega = plan.lpt_vjp(omega, cosmo, ic, adj, thb)
        return g_omega, thb
