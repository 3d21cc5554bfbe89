"""Background cosmology, growth functions, FastPM factors, KDK step
coefficients and the linear power spectrum -- plain FP64 reference.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed:
  * Appendix A (growth equations): the second-order growth ODEs written in the
    suppression factors G_m = D_m / a^m, with growing-mode initial conditions
    G_1 = 1, G_1' = 0, G_2 = 3/7, G_2' = 0 at a_ic; ' = d/d ln a.
  * eq. G_eval: G_D = a^2 H D_1', G_K = a^3 H^2 [D_1'' + (2 + H'/H) D_1'].
    The D_m' and D_m'' lines of that equation are printed with G_1 where G_m
    is meant; we use the product rule on D_m = a^m G_m.
  * Sec. 2.3 (FastPM drift and kick factors):
        D(t_c, t_a, t_b) = (D_1(t_b) - D_1(t_a)) / G_D(t_c)
        K(t_c, t_a, t_b) = (G_D(t_b) - G_D(t_a)) / G_K(t_c)
    and the kick-drift-kick order of eq. KDFK.
  * eq. Plin: the shape of the linear power spectrum is k^{n_s} T^2(k); the
    amplitude is fixed here by sigma8 instead of A_s (our reading).
  * Sec. 2.1 cites the Eisenstein & Hu (1998) fitting formula for T(k); we use
    its no-wiggle form (EH98 Sec. 4.2).

Readings (where the paper is silent): flat LambdaCDM without radiation,
H0 = 1 (time in 1/H0), a_ic = 1e-4, half step a_{i-1/2} = (a_{i-1} + a_i)/2,
sigma8 measured at a = 1 with the top-hat of radius 8 Mpc/h.

Derivatives with respect to Omega_m are taken by the complex-step method
(f'(x) = Im f(x + i h) / h with h = 1e-30), so every function here is written
with analytic operations only (no abs, no comparisons on Omega_m).
"""
import math

import numpy as np
from scipy.integrate import solve_ivp

A_IC = 1e-4
CSTEP = 1e-30

# ----------------------------------------------------------------------------
# background (flat LambdaCDM, H0 = 1)
# ----------------------------------------------------------------------------


def E(a, om):
    """Dimensionless Hubble rate H/H0 for flat LambdaCDM."""
    return np.sqrt(om * a ** -3.0 + (1.0 - om))


def omega_m_a(a, om):
    """Omega_m(a) = Omega_m H0^2 / (a^3 H^2) (Appendix A)."""
    return om / (a ** 3 * E(a, om) ** 2)


def dlnH_dlna(a, om):
    """H'/H = d ln H / d ln a = -1.5 Omega_m(a) for flat LambdaCDM."""
    return -1.5 * omega_m_a(a, om)


# ----------------------------------------------------------------------------
# growth ODEs in suppression-factor form (Appendix A)
# ----------------------------------------------------------------------------


def _growth_rhs(lna, y, om):
    a = np.exp(lna)
    g1, dg1, g2, dg2 = y
    hh = dlnH_dlna(a, om)
    oma = omega_m_a(a, om)
    ddg1 = -(4.0 + hh) * dg1 - (3.0 + hh - 1.5 * oma) * g1
    ddg2 = -(6.0 + hh) * dg2 - (8.0 + 2.0 * hh - 1.5 * oma) * g2 + 1.5 * oma * g1 * g1
    return [dg1, ddg1, dg2, ddg2]


def growth(a, om, a_ic=A_IC, rtol=1e-13, atol=1e-15):
    """Growth functions at scale factors `a` (1-d array, a >= a_ic).

    Returns a dict of arrays: G1, dG1, ddG1, G2, dG2, ddG2 (suppression
    factors and their ln-a derivatives), D1, dD1, ddD1, D2, dD2, ddD2
    (D_m = a^m G_m and ln-a derivatives by the product rule).
    `om` may be complex (complex-step differentiation).
    """
    a = np.asarray(a, dtype=float)
    order = np.argsort(a)
    a_sorted = a[order]
    uniq, inv = np.unique(a_sorted, return_inverse=True)
    lna_eval = np.log(uniq)
    y0 = np.array([1.0, 0.0, 3.0 / 7.0, 0.0], dtype=complex if np.iscomplexobj(om) else float)
    t0 = math.log(a_ic)
    t1 = float(lna_eval[-1])
    if t1 <= t0:
        raise ValueError("growth: requested a below a_ic")
    sol = solve_ivp(_growth_rhs, (t0, t1), y0, method="DOP853", t_eval=lna_eval,
                    rtol=rtol, atol=atol, args=(om,))
    if not sol.success:
        raise RuntimeError("growth ODE failed: " + sol.message)
    y = sol.y  # (4, n_unique)
    g1, dg1, g2, dg2 = y
    rhs = np.array(_growth_rhs(lna_eval, y, om))
    ddg1, ddg2 = rhs[1], rhs[3]
    # undo the unique/sort
    out_u = dict(G1=g1, dG1=dg1, ddG1=ddg1, G2=g2, dG2=dg2, ddG2=ddg2)
    out = {}
    for key, val in out_u.items():
        v_sorted = val[inv]
        v = np.empty_like(v_sorted)
        v[order] = v_sorted
        out[key] = v
    for m in (1, 2):
        G, dG, ddG = out["G%d" % m], out["dG%d" % m], out["ddG%d" % m]
        am = a ** m
        out["D%d" % m] = am * G
        out["dD%d" % m] = am * (m * G + dG)
        out["ddD%d" % m] = am * (m * m * G + 2 * m * dG + ddG)
    return out


def fastpm_factors(a, om):
    """G_D(a) = a^2 H D_1' and G_K(a) = a^3 H^2 [D_1'' + (2 + H'/H) D_1']
    (eq. G_eval), plus D_1 itself. H0 = 1."""
    a = np.asarray(a, dtype=float)
    g = growth(a, om)
    e = E(a, om)
    GD = a ** 2 * e * g["dD1"]
    GK = a ** 3 * e ** 2 * (g["ddD1"] + (2.0 + dlnH_dlna(a, om)) * g["dD1"])
    return g["D1"], GD, GK


def drift_factor(ac, aa, ab, om):
    """D(t_c, t_a, t_b) = (D_1(t_b) - D_1(t_a)) / G_D(t_c) (Sec. 2.3)."""
    D1, GD, _ = fastpm_factors(np.array([ac, aa, ab]), om)
    return (D1[2] - D1[1]) / GD[0]


def kick_factor(ac, aa, ab, om):
    """K(t_c, t_a, t_b) = (G_D(t_b) - G_D(t_a)) / G_K(t_c) (Sec. 2.3)."""
    _, GD, GK = fastpm_factors(np.array([ac, aa, ab]), om)
    return (GD[2] - GD[1]) / GK[0]


def step_coefficients(a_grid, om):
    """KDK step coefficients for steps i = 1..n on the grid a_0..a_n (eq. KDFK).

    Row i-1 holds (Ka_i, D_i, Kb_i):
        Ka_i = K(t_{i-1}, t_{i-1}, t_{i-1/2})
        D_i  = D(t_{i-1/2}, t_{i-1}, t_i)
        Kb_i = K(t_i, t_{i-1/2}, t_i)
    with a_{i-1/2} the arithmetic midpoint (reading).
    """
    a_grid = np.asarray(a_grid, dtype=float)
    a0, a1 = a_grid[:-1], a_grid[1:]
    ah = 0.5 * (a0 + a1)
    n = len(a1)
    allA = np.concatenate([a0, ah, a1])
    D1, GD, GK = fastpm_factors(allA, om)
    D1_0, D1_h, D1_1 = D1[:n], D1[n:2 * n], D1[2 * n:]
    GD_0, GD_h, GD_1 = GD[:n], GD[n:2 * n], GD[2 * n:]
    GK_0, GK_1 = GK[:n], GK[2 * n:]
    Ka = (GD_h - GD_0) / GK_0
    Dd = (D1_1 - D1_0) / GD_h
    Kb = (GD_1 - GD_h) / GK_1
    return np.stack([Ka, Dd, Kb], axis=1)


def step_coefficients_with_derivative(a_grid, om):
    """(coefs, dcoefs/dOmega_m), each (n, 3), derivative by complex step."""
    c = step_coefficients(a_grid, om)
    dc = step_coefficients(a_grid, om + 1j * CSTEP).imag / CSTEP
    return c, dc


def linear_a_grid(a_start, a_end, n):
    """Time steps linearly spaced in a (Sec. 4)."""
    return np.linspace(a_start, a_end, n + 1)


# ----------------------------------------------------------------------------
# Heath (1977) integral for flat LambdaCDM -- used only as an independent pin
# ----------------------------------------------------------------------------


def heath_D1(a, om):
    """D_1(a) = 2.5 Omega_m E(a) int_0^a da' / (a' E(a'))^3, normalised so that
    D_1 -> a as a -> 0. Independent closed form used to pin growth()."""
    from scipy.integrate import quad
    a = np.atleast_1d(np.asarray(a, dtype=float))
    out = np.empty_like(a)
    for i, ai in enumerate(a):
        # substitute a' = u^2 to remove the a'^{3/2} endpoint behaviour
        f = lambda u: 2.0 * u / (u * u * E(u * u, om)) ** 3
        val, _ = quad(f, 0.0, math.sqrt(ai), epsabs=0.0, epsrel=1e-13, limit=200)
        out[i] = 2.5 * om * E(ai, om) * val
    return out


# ----------------------------------------------------------------------------
# transfer function and linear power spectrum (eq. Plin)
# ----------------------------------------------------------------------------


def eh_nowiggle(k, om, ob, h, t_cmb=2.7255):
    """Eisenstein & Hu (1998) no-wiggle transfer function T(k), k in h/Mpc.

    Sound horizon s and shape suppression alpha_Gamma per EH98 Sec. 4.2; the
    product k*s uses k in 1/Mpc.
    """
    k = np.asarray(k, dtype=float)
    omh2 = om * h * h
    obh2 = ob * h * h
    fb = ob / om
    theta = t_cmb / 2.7
    s = 44.5 * np.log(9.83 / omh2) / np.sqrt(1.0 + 10.0 * obh2 ** 0.75)
    alpha = 1.0 - 0.328 * np.log(431.0 * omh2) * fb + 0.38 * np.log(22.3 * omh2) * fb * fb
    ks = k * h * s
    gamma = om * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * ks) ** 4))
    q = k * theta * theta / gamma
    L0 = np.log(2.0 * math.e + 1.8 * q)
    C0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return L0 / (L0 + C0 * q * q)


def tophat_window(x):
    """Fourier transform of a unit-volume top-hat, W(x) = 3(sin x - x cos x)/x^3."""
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    small = x < 1e-3
    xs = x[small]
    out[small] = 1.0 - xs * xs / 10.0 + xs ** 4 / 280.0
    xl = x[~small]
    out[~small] = 3.0 * (np.sin(xl) - xl * np.cos(xl)) / xl ** 3
    return out


def _gauss_legendre_lnk(lnk_min, lnk_max, panels, order):
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(lnk_min, lnk_max, panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    nodes = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    weights = (half[:, None] * w[None, :]).ravel()
    return nodes, weights


def sigma_r_shape_integral(om, ob, h, ns, R=8.0, t_cmb=2.7255, panels=4096, order=8,
                           lnk_min=math.log(1e-5), lnk_max=math.log(1e2)):
    """I = int d ln k  k^3 k^{n_s} T^2(k) W^2(kR) / (2 pi^2) (composite
    Gauss-Legendre in ln k). sigma_R^2 = A D_1(1)^2 I for P = A k^{n_s} T^2."""
    lnk, w = _gauss_legendre_lnk(lnk_min, lnk_max, panels, order)
    k = np.exp(lnk)
    T = eh_nowiggle(k, om, ob, h, t_cmb)
    Wt = tophat_window(k * R)
    integrand = k ** 3 * k ** ns * T * T * Wt * Wt / (2.0 * math.pi ** 2)
    return np.sum(w * integrand)


def power_amplitude(om, ob, h, ns, sigma8, t_cmb=2.7255, **kw):
    """Amplitude A of P_lin(k) = A k^{n_s} T^2(k), where P_lin is the
    early-time normalised spectrum of eq. Plin (growth D_1 -> a kept apart),
    fixed so that the linear sigma8 at a = 1 equals `sigma8` (reading)."""
    I = sigma_r_shape_integral(om, ob, h, ns, t_cmb=t_cmb, **kw)
    D1_1 = growth(np.array([1.0]), om)["D1"][0]
    return sigma8 ** 2 / (D1_1 ** 2 * I)


def linear_power(k, om, ob, h, ns, sigma8, t_cmb=2.7255):
    """P_lin(k) in (Mpc/h)^3 for k in h/Mpc (eq. Plin, normalised by sigma8)."""
    A = power_amplitude(om, ob, h, ns, sigma8, t_cmb)
    k = np.asarray(k, dtype=float)
    return A * k ** ns * eh_nowiggle(k, om, ob, h, t_cmb) ** 2


class Cosmo:
    """Cosmological parameters theta; (Omega_m, sigma8) are the free ones."""

    def __init__(self, omega_m=0.3, sigma8=0.8, omega_b=0.05, h=0.7, n_s=0.96, t_cmb=2.7255):
        self.omega_m = omega_m
        self.sigma8 = sigma8
        self.omega_b = omega_b
        self.h = h
        self.n_s = n_s
        self.t_cmb = t_cmb

    def replace(self, **kw):
        d = dict(omega_m=self.omega_m, sigma8=self.sigma8, omega_b=self.omega_b,
                 h=self.h, n_s=self.n_s, t_cmb=self.t_cmb)
        d.update(kw)
        return Cosmo(**d)
