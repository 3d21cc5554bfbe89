"""Thin Python binding of libpm (same names as include/pm.h).

Argument marshalling only: each method checks tensor device, dtype, shape and
contiguity, then passes raw device pointers and the current HIP stream to
the C-ABI.  Every computation happens in the library's kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (PmAdj, PmCheckpoints, PmConfig, PmCosmo, PmIcCoef, PmLcCoef, PmLcStep, PmState, PmStepCoef,
                   check, lib)

_TORCH_DT = {_lib.PM_F32: torch.float32, _lib.PM_F64: torch.float64}
_CPLX_DT = {_lib.PM_F32: torch.complex64, _lib.PM_F64: torch.complex128}


def _code(dtype):
    if dtype in (torch.float32, "f32", "float32", np.float32):
        return _lib.PM_F32
    if dtype in (torch.float64, "f64", "float64", np.float64):
        return _lib.PM_F64
    raise ValueError("dtype must be float32 or float64, got %r" % (dtype,))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def step_coef(row):
    """pm_step_coef from (Ka, D, Kb, dKa, dD, dKb)."""
    return PmStepCoef(*[float(v) for v in row])


class Cosmology:
    """theta = (Omega_m, sigma8) with Omega_b, h, n_s, T_cmb held fixed."""

    def __init__(self, omega_m=0.3, sigma8=0.8, omega_b=0.05, h=0.7, n_s=0.96, t_cmb=2.7255):
        self.omega_m, self.sigma8, self.omega_b = omega_m, sigma8, omega_b
        self.h, self.n_s, self.t_cmb = h, n_s, t_cmb

    def c_struct(self):
        return PmCosmo(self.omega_m, self.omega_b, self.h, self.n_s, self.sigma8, self.t_cmb)

    def replace(self, **kw):
        d = dict(omega_m=self.omega_m, sigma8=self.sigma8, omega_b=self.omega_b, h=self.h,
                 n_s=self.n_s, t_cmb=self.t_cmb)
        d.update(kw)
        return Cosmology(**d)


def tables(cosmo, a_grid):
    """Host FP64 tables (pm_tables): step coefficients (n, 6) as
    (Ka, D, Kb, dKa, dD, dKb) and the IC factors at a_grid[0] as a dict."""
    a = np.ascontiguousarray(np.asarray(a_grid, dtype=np.float64))
    n = len(a) - 1
    coefs = (PmStepCoef * max(n, 1))()
    ic = PmIcCoef()
    check(lib().pm_tables(ctypes.byref(cosmo.c_struct()), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                          coefs if n > 0 else None, ctypes.byref(ic)))
    arr = np.array([[c.Ka, c.D, c.Kb, c.dKa, c.dD, c.dKb] for c in coefs[:n]], dtype=np.float64).reshape(n, 6)
    icd = {f: getattr(ic, f) for f, _ in PmIcCoef._fields_}
    return arr, icd


def lightcone_tables(cosmo, a_grid, cell):
    """Host FP64 light-front and velocity factors (pm_lightcone_tables) at
    every a of a_grid for mesh cells of `cell` Mpc/h: a ctypes array of
    pm_lc_coef."""
    a = np.ascontiguousarray(np.asarray(a_grid, dtype=np.float64))
    out = (PmLcCoef * len(a))()
    check(lib().pm_lightcone_tables(ctypes.byref(cosmo.c_struct()), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    len(a) - 1, float(cell), out))
    return out


def lc_step(c0, c1, omega_m, observer, step):
    """pm_lc_step of step `step` from the factors at its two ends."""
    return PmLcStep(c0, c1, float(omega_m), (ctypes.c_double * 3)(*[float(v) for v in observer]), int(step))


def ic_struct(icd):
    return PmIcCoef(*[float(icd[f]) for f, _ in PmIcCoef._fields_])


class Plan:
    """A libpm plan: mesh/lattice geometry, precision and device scratch.
    deterministic=True (default): the fixed-point paint, bitwise
    reproducible; False: floating-point LDS atomics (see pm_config).
    lpt_scratch (default: whenever the lattice and box allow 2LPT): the plan
    allocates the 2LPT lattice scratch up front, so no later call allocates.
    lpt_keep (default True): pm_lpt keeps its second-order fields for the
    next pm_lpt_vjp of the same omega tensor and cosmology (pm_config)."""

    def __init__(self, mesh, ptcl, box=(1.0, 1.0, 1.0), lattice_offset=0.0, mesh_dtype=torch.float32,
                 state_dtype=torch.float64, deterministic=True, lpt_scratch=None, lpt_keep=True):
        mesh = tuple(int(m) for m in (mesh if np.iterable(mesh) else (mesh,) * 3))
        ptcl = tuple(int(m) for m in (ptcl if np.iterable(ptcl) else (ptcl,) * 3))
        box = tuple(float(b) for b in (box if np.iterable(box) else (box,) * 3))
        if lpt_scratch is None:
            n = ptcl[0]
            lpt_scratch = (ptcl == (n, n, n) and 4 <= n <= 1024 and n & (n - 1) == 0 and box[0] > 0
                           and box == (box[0],) * 3)
        self.cfg = PmConfig((ctypes.c_int32 * 3)(*mesh), (ctypes.c_int32 * 3)(*ptcl), (ctypes.c_double * 3)(*box),
                            float(lattice_offset), _code(mesh_dtype), _code(state_dtype), int(bool(deterministic)),
                            int(bool(lpt_scratch)), int(bool(lpt_keep)))
        self.mesh = mesh
        self.ptcl = ptcl
        self.box = box
        self.n_particles = ptcl[0] * ptcl[1] * ptcl[2]
        self.n_cells = mesh[0] * mesh[1] * mesh[2]
        self.spec_shape = (mesh[0], mesh[1], mesh[2] // 2 + 1)
        self.mdt = _TORCH_DT[self.cfg.mesh_dtype]
        self.sdt = _TORCH_DT[self.cfg.state_dtype]
        self.cdt = _CPLX_DT[self.cfg.mesh_dtype]
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        check(lib().pm_plan_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self._h = h
        self._dev_scalars = torch.zeros(4, dtype=torch.float64, device=self.device)

    @staticmethod
    def workspace_bytes(mesh, ptcl, mesh_dtype=torch.float32, state_dtype=torch.float64):
        cfg = PmConfig((ctypes.c_int32 * 3)(*mesh), (ctypes.c_int32 * 3)(*ptcl), (ctypes.c_double * 3)(1, 1, 1),
                       0.0, _code(mesh_dtype), _code(state_dtype), 0)
        return lib().pm_workspace_bytes(ctypes.byref(cfg))

    def close(self):
        if getattr(self, "_h", None):
            lib().pm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- tensor checks ----------------------------------------------------
    def _t(self, t, dtype, numel, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device.type != "cuda":
            raise ValueError("%s must be on the GPU" % name)
        if t.dtype != dtype:
            raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if numel is not None and t.numel() != numel:
            raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
        return t

    def _disp(self, disp):
        return self._t(disp, self.sdt, 3 * self.n_particles, "disp")

    def _c(self, rc):
        return check(rc, self._h)

    # ---- hot path ----------------------------------------------------------
    def paint(self, disp, weights=None, out=None):
        """CIC paint (pm_paint): (nch, n0, n1, n2) mesh, unit mass if weights is None."""
        self._disp(disp)
        nch = 1 if weights is None else weights.numel() // self.n_particles
        if weights is not None:
            self._t(weights, self.mdt, nch * self.n_particles, "weights")
        if out is None:
            out = torch.empty((nch,) + self.mesh, dtype=self.mdt, device=self.device)
        self._t(out, self.mdt, nch * self.n_cells, "out")
        self._c(lib().pm_paint(self._h, _ptr(disp), _ptr(weights), nch, _ptr(out), _stream()))
        return out

    def fft_r2c(self, x, out=None):
        """R2C (pm_fft dir=+1) of (batch, n0, n1, n2) real -> (batch, n0, n1, n2/2+1) complex."""
        batch = x.numel() // self.n_cells
        self._t(x, self.mdt, batch * self.n_cells, "x")
        if out is None:
            out = torch.empty((batch,) + self.spec_shape, dtype=self.cdt, device=self.device)
        self._t(out, self.cdt, batch * int(np.prod(self.spec_shape)), "out")
        self._c(lib().pm_fft(self._h, 1, _ptr(x), _ptr(out), batch, _stream()))
        return out

    def fft_c2r(self, X, out=None, destroy_input=False):
        """C2R (pm_fft dir=-1) with 1/N_c; the input is copied unless destroy_input."""
        nsp = int(np.prod(self.spec_shape))
        batch = X.numel() // nsp
        self._t(X, self.cdt, batch * nsp, "X")
        src = X if destroy_input else X.clone()
        if out is None:
            out = torch.empty((batch,) + self.mesh, dtype=self.mdt, device=self.device)
        self._t(out, self.mdt, batch * self.n_cells, "out")
        self._c(lib().pm_fft(self._h, -1, _ptr(src), _ptr(out), batch, _stream()))
        return out

    def poisson_grad(self, delta_k, omega_m, out=None):
        """Poisson gradient (pm_poisson_grad): [3] half spectra T_j delta_k,
        T_j = i k_j 1.5 omega_m / k^2."""
        nsp = int(np.prod(self.spec_shape))
        self._t(delta_k, self.cdt, nsp, "delta_k")
        if out is None:
            out = torch.empty((3,) + self.spec_shape, dtype=self.cdt, device=self.device)
        self._t(out, self.cdt, 3 * nsp, "out")
        self._c(lib().pm_poisson_grad(self._h, _ptr(delta_k), _ptr(out), float(omega_m), _stream()))
        return out

    def readout(self, disp, mesh, out=None):
        self._disp(disp)
        nch = mesh.numel() // self.n_cells
        self._t(mesh, self.mdt, nch * self.n_cells, "mesh")
        if out is None:
            out = torch.empty((nch, self.n_particles), dtype=self.mdt, device=self.device)
        self._t(out, self.mdt, nch * self.n_particles, "out")
        self._c(lib().pm_readout(self._h, _ptr(disp), _ptr(mesh), nch, _ptr(out), _stream()))
        return out

    def force(self, disp, omega_m, out=None):
        """PM force (pm_force): accelerations [3, N_p] at q + disp."""
        self._disp(disp)
        if out is None:
            out = torch.empty((3, self.n_particles), dtype=self.mdt, device=self.device)
        self._t(out, self.mdt, 3 * self.n_particles, "acc")
        self._c(lib().pm_force(self._h, _ptr(disp), float(omega_m), _ptr(out), _stream()))
        return out

    def force_vjp(self, disp, acc_bar, omega_m, want_acc=True, out=None, omega_m_bar=None):
        """(disp_bar, omega_m_bar (device FP64 scalar, +=), acc or None);
        `out` and `omega_m_bar` may be given to reuse buffers."""
        self._disp(disp)
        self._t(acc_bar, self.mdt, 3 * self.n_particles, "acc_bar")
        xbar = torch.empty((3, self.n_particles), dtype=self.mdt, device=self.device) if out is None else \
            self._t(out, self.mdt, 3 * self.n_particles, "out")
        acc = torch.empty_like(xbar) if want_acc else None
        cbar = torch.zeros(1, dtype=torch.float64, device=self.device) if omega_m_bar is None else \
            self._t(omega_m_bar, torch.float64, 1, "omega_m_bar")
        self._c(lib().pm_force_vjp(self._h, _ptr(disp), _ptr(acc_bar), float(omega_m), _ptr(xbar), _ptr(cbar),
                                   _ptr(acc), _stream()))
        return xbar, cbar, acc

    # ---- integration --------------------------------------------------------
    def new_state(self, s, p, with_acc=True):
        self._t(s, self.sdt, 3 * self.n_particles, "s")
        self._t(p, self.sdt, 3 * self.n_particles, "p")
        acc = torch.empty((3, self.n_particles), dtype=self.mdt, device=self.device) if with_acc else None
        return {"s": s, "p": p, "acc": acc}

    @staticmethod
    def _st(state):
        return PmState(state["s"].data_ptr(), state["p"].data_ptr(),
                       state["acc"].data_ptr() if state.get("acc") is not None else None)

    @staticmethod
    def _adj(adj):
        return PmAdj(adj["xi"].data_ptr(), adj["pi"].data_ptr())

    def fwd_init(self, state, first, omega_m):
        self._c(lib().pm_fwd_init(self._h, ctypes.byref(self._st(state)), ctypes.byref(step_coef(first)),
                                  float(omega_m), _stream()))

    def step_fwd(self, state, cur, nxt, omega_m):
        n = ctypes.byref(step_coef(nxt)) if nxt is not None else None
        self._c(lib().pm_step_fwd(self._h, ctypes.byref(self._st(state)), ctypes.byref(step_coef(cur)), n,
                                  float(omega_m), _stream()))

    def adj_init(self, state, adj, last, omega_m, theta_bar):
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        self._c(lib().pm_adj_init(self._h, ctypes.byref(self._st(state)), ctypes.byref(self._adj(adj)),
                                  ctypes.byref(step_coef(last)), float(omega_m), _ptr(theta_bar), _stream()))

    def step_adj(self, state, adj, cur, prev, omega_m, theta_bar):
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        pv = ctypes.byref(step_coef(prev)) if prev is not None else None
        self._c(lib().pm_step_adj(self._h, ctypes.byref(self._st(state)), ctypes.byref(self._adj(adj)),
                                  ctypes.byref(step_coef(cur)), pv, float(omega_m), _ptr(theta_bar), _stream()))

    def _coef_array(self, coefs):
        coefs = np.asarray(coefs, dtype=np.float64).reshape(-1, 6)
        arr = (PmStepCoef * len(coefs))(*[step_coef(r) for r in coefs])
        return arr, len(coefs)

    def run_fwd(self, state, coefs, omega_m):
        arr, n = self._coef_array(coefs)
        self._c(lib().pm_run_fwd(self._h, ctypes.byref(self._st(state)), arr, n, float(omega_m), _stream()))

    def run_adj(self, state, adj, coefs, omega_m, theta_bar):
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        arr, n = self._coef_array(coefs)
        self._c(lib().pm_run_adj(self._h, ctypes.byref(self._st(state)), ctypes.byref(self._adj(adj)), arr, n,
                                 float(omega_m), _ptr(theta_bar), _stream()))

    def run_adj_from(self, state, adj, coefs, omega_m, theta_bar):
        """pm_run_adj_from: the reverse steps len(coefs)..1 from where the
        step calls left off (no pm_adj_init)."""
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        arr, n = self._coef_array(coefs)
        self._c(lib().pm_run_adj_from(self._h, ctypes.byref(self._st(state)), ctypes.byref(self._adj(adj)), arr,
                                      n, float(omega_m), _ptr(theta_bar), _stream()))

    def new_checkpoints(self, steps):
        """Buffers for forward checkpoints at the given steps (1..n): a dict
        with "step" (sorted list), "s" and "p" (lists of [3, N_p] tensors)."""
        steps = sorted(int(j) for j in steps)
        n = self.n_particles
        mk = lambda: torch.empty((3, n), dtype=self.sdt, device=self.device)  # noqa: E731
        return {"step": steps, "s": [mk() for _ in steps], "p": [mk() for _ in steps]}

    def _ck(self, ck):
        if ck is None:
            return None, ()
        for t in list(ck["s"]) + list(ck["p"]):
            self._t(t, self.sdt, 3 * self.n_particles, "checkpoint")
        k = len(ck["step"])
        steps = (ctypes.c_int * max(k, 1))(*ck["step"])
        sp = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in ck["s"]])
        pp = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in ck["p"]])
        c = PmCheckpoints(k, ctypes.cast(steps, ctypes.POINTER(ctypes.c_int)),
                          ctypes.cast(sp, ctypes.POINTER(ctypes.c_void_p)),
                          ctypes.cast(pp, ctypes.POINTER(ctypes.c_void_p)))
        return c, (steps, sp, pp)     # keep the arrays alive for the call

    def run_fwd_ckpt(self, state, coefs, omega_m, checkpoints):
        arr, n = self._coef_array(coefs)
        c, keep = self._ck(checkpoints)
        self._c(lib().pm_run_fwd_ckpt(self._h, ctypes.byref(self._st(state)), arr, n, float(omega_m),
                                      ctypes.byref(c) if c is not None else None, _stream()))
        del keep

    def run_adj_ckpt(self, state, adj, coefs, omega_m, checkpoints, theta_bar):
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        arr, n = self._coef_array(coefs)
        c, keep = self._ck(checkpoints)
        self._c(lib().pm_run_adj_ckpt(self._h, ctypes.byref(self._st(state)), ctypes.byref(self._adj(adj)), arr,
                                      n, float(omega_m), ctypes.byref(c) if c is not None else None,
                                      _ptr(theta_bar), _stream()))
        del keep

    def density_mse(self, disp, target, want_grad=True):
        """(J device FP64 scalar, disp_bar or None)."""
        self._disp(disp)
        self._t(target, self.mdt, self.n_cells, "target")
        J = torch.zeros(1, dtype=torch.float64, device=self.device)
        xbar = torch.empty((3, self.n_particles), dtype=self.mdt, device=self.device) if want_grad else None
        self._c(lib().pm_density_mse(self._h, _ptr(disp), _ptr(target), _ptr(J), _ptr(xbar), _stream()))
        return J, xbar

    def density(self, disp, out=None):
        """delta = paint(x) N_c/N_p - 1 (pm_density), shape mesh."""
        self._disp(disp)
        if out is None:
            out = torch.empty(self.mesh, dtype=self.mdt, device=self.device)
        self._t(out, self.mdt, self.n_cells, "out")
        self._c(lib().pm_density(self._h, _ptr(disp), _ptr(out), _stream()))
        return out

    # ---- light cone -----------------------------------------------------------
    def _state3(self, t, name):
        return self._t(t, self.sdt, 3 * self.n_particles, name)

    def _mesh3(self, t, name):
        return self._t(t, self.mdt, 3 * self.n_particles, name) if t is not None else None

    def lightcone_reach(self, disp, observer, out=None):
        """pm_lightcone_reach: the largest |q + disp - observer| over the
        particles (mesh cells), a device FP64 scalar."""
        self._state3(disp, "disp")
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        self._t(out, torch.float64, 1, "r_max")
        obs = (ctypes.c_double * 3)(*[float(v) for v in observer])
        self._c(lib().pm_lightcone_reach(self._h, _ptr(disp), obs, _ptr(out), _stream()))
        return out

    def lightcone_truncate(self, x, obs_step, last):
        """pm_lightcone_truncate: x[:, n] = 0 (in place) for the particles
        observed in steps 1..last (the frozen sources of the truncated
        adjoint)."""
        self._mesh3(x, "x")
        self._t(obs_step, torch.int32, self.n_particles, "obs_step")
        self._c(lib().pm_lightcone_truncate(self._h, _ptr(x), _ptr(obs_step), int(last), _stream()))

    def lightcone(self, step, s0, p0, s1, p1, obs, obs_step, count):
        """pm_lightcone: record the particles that cross the light front in
        `step` (a pm_lc_step) into obs [7, N_p] and obs_step [N_p];
        count (device FP64, one element) += their number."""
        for t, nm in ((s0, "s0"), (p0, "p0"), (s1, "s1"), (p1, "p1")):
            self._state3(t, nm)
        self._t(obs, self.sdt, 7 * self.n_particles, "obs")
        self._t(obs_step, torch.int32, self.n_particles, "obs_step")
        self._t(count, torch.float64, 1, "count")
        self._c(lib().pm_lightcone(self._h, ctypes.byref(step), _ptr(s0), _ptr(p0), _ptr(s1), _ptr(p1), _ptr(obs),
                                   _ptr(obs_step), _ptr(count), _stream()))

    def lightcone_vjp(self, step, s0, p0, s1, p1, obs_step, obs_bar, x0_bar, p0_bar, x1_bar, p1_bar, theta_bar):
        """pm_lightcone_vjp: accumulate the cotangents of the two ends of
        `step` (any of the four outputs may be None) and theta_bar[0]."""
        for t, nm in ((s0, "s0"), (p0, "p0"), (s1, "s1"), (p1, "p1")):
            self._state3(t, nm)
        self._t(obs_step, torch.int32, self.n_particles, "obs_step")
        self._t(obs_bar, self.mdt, 7 * self.n_particles, "obs_bar")
        outs = [self._mesh3(t, nm) for t, nm in ((x0_bar, "x0_bar"), (p0_bar, "p0_bar"), (x1_bar, "x1_bar"),
                                                 (p1_bar, "p1_bar"))]
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        self._c(lib().pm_lightcone_vjp(self._h, ctypes.byref(step), _ptr(s0), _ptr(p0), _ptr(s1), _ptr(p1),
                                       _ptr(obs_step), _ptr(obs_bar), *[_ptr(t) for t in outs], _ptr(theta_bar),
                                       _stream()))

    def adj_bump(self, xi, pi, x_bar, p_bar, c, Kb, dKb, acc, omega_m_bar, theta_bar):
        """pm_adj_bump: xi += x_bar + Kb c, pi += p_bar and the theta_bar terms."""
        for t, nm in ((xi, "xi"), (pi, "pi"), (x_bar, "x_bar"), (p_bar, "p_bar")):
            self._mesh3(t, nm)
        self._mesh3(c, "c")
        self._mesh3(acc, "acc")
        if omega_m_bar is not None:
            self._t(omega_m_bar, torch.float64, 1, "omega_m_bar")
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        self._c(lib().pm_adj_bump(self._h, _ptr(xi), _ptr(pi), _ptr(x_bar), _ptr(p_bar), _ptr(c), float(Kb),
                                  float(dKb), _ptr(acc), _ptr(omega_m_bar), _ptr(theta_bar), _stream()))

    def kick(self, p, acc, K, out=None):
        """pm_kick: out = p + acc K (out may be p)."""
        self._state3(p, "p")
        self._mesh3(acc, "acc")
        out = torch.empty_like(p) if out is None else self._state3(out, "p_out")
        self._c(lib().pm_kick(self._h, _ptr(p), _ptr(acc), float(K), _ptr(out), _stream()))
        return out

    def drift(self, s, p, D, out=None):
        """pm_drift: out = s + p D (out may be s)."""
        self._state3(s, "s")
        self._state3(p, "p")
        out = torch.empty_like(s) if out is None else self._state3(out, "s_out")
        self._c(lib().pm_drift(self._h, _ptr(s), _ptr(p), float(D), _ptr(out), _stream()))
        return out

    def power_spectrum(self, field, spectrum=False):
        """Shell-averaged power spectrum (pm_power_spectrum) of a real field
        ([n, n, n] mesh dtype; transformed with pm_fft first), or of a half
        spectrum when spectrum=True.  Returns device FP64 tensors (k, P,
        count) of n/2 shells b = 1..n/2 (k in h/Mpc for a box in Mpc/h)."""
        if spectrum:
            dk = self._t(field, self.cdt, int(np.prod(self.spec_shape)), "delta_k")
        else:
            dk = self.fft_r2c(self._t(field, self.mdt, self.n_cells, "field"))
        nb = self.mesh[0] // 2
        k, P, cnt = (torch.empty(nb, dtype=torch.float64, device=self.device) for _ in range(3))
        self._c(lib().pm_power_spectrum(self._h, _ptr(dk), _ptr(k), _ptr(P), _ptr(cnt), _stream()))
        return k, P, cnt

    # ---- initial conditions -------------------------------------------------
    def lpt(self, omega, cosmo, ic, state):
        self._t(omega, self.mdt, self.n_particles, "omega")
        self._c(lib().pm_lpt(self._h, _ptr(omega), ctypes.byref(cosmo.c_struct()), ctypes.byref(ic_struct(ic)),
                             ctypes.byref(self._st(state)), _stream()))

    def lpt_vjp(self, omega, cosmo, ic, adj, theta_bar, out=None):
        self._t(omega, self.mdt, self.n_particles, "omega")
        self._t(theta_bar, torch.float64, 2, "theta_bar")
        if out is None:
            out = torch.empty_like(omega)
        self._c(lib().pm_lpt_vjp(self._h, _ptr(omega), ctypes.byref(cosmo.c_struct()), ctypes.byref(ic_struct(ic)),
                                 ctypes.byref(self._adj(adj)), _ptr(out), _ptr(theta_bar), _stream()))
        return out

    # ---- support ------------------------------------------------------------
    def check_finite(self, x):
        bad = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._c(lib().pm_check_finite(self._h, _ptr(x), x.numel(), _code(x.dtype), _ptr(bad), _stream()))
        return bad

    def stream(self, mode, src=None, dst=None):
        """pm_stream: one STREAM-like pass (read src, copy src -> dst, or
        write dst) on the current stream; returns the bytes moved."""
        t = src if src is not None else dst
        if t is None or not t.is_cuda or not t.is_contiguous():
            raise ValueError("stream needs contiguous device tensors")
        nbytes = t.numel() * t.element_size()
        if src is not None and dst is not None and dst.numel() * dst.element_size() < nbytes:
            raise ValueError("dst is smaller than src")
        self._c(lib().pm_stream(self._h, int(mode), _ptr(src), _ptr(dst), nbytes, _stream()))
        return nbytes * (2 if mode == _lib.PM_STREAM_COPY else 1)

    def timing_enable(self, kernels=()):
        """Time the given PM_K_* kernel families (empty: switch timing off)."""
        mask = 0
        for k in kernels:
            mask |= 1 << int(k)
        self._c(lib().pm_timing_enable(self._h, mask))

    def timing_read(self, kernel, method=False):
        """(total milliseconds, launches, total algorithmic bytes) of one
        PM_K_* family since timing_enable; with method=True a fourth value,
        the total method bytes (pm_timing_read)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        b = ctypes.c_double()
        mb = ctypes.c_double()
        self._c(lib().pm_timing_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                     ctypes.byref(mb)))
        return (ms.value, n.value, b.value, mb.value) if method else (ms.value, n.value, b.value)
