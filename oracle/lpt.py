"""Second-order LPT initial conditions and their derivatives -- plain FP64
reference.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed (Sec. 2.1, "Initial Conditions & Perturbation
Theories"):
  * x = q + s; eq. lpt: s = D_1 s1 + D_2 s2 and p = a^2 H (D_1' s1 + D_2' s2).
  * s1 = -grad phi1, s2 = -grad phi2 with laplacian phi1 = delta1 and
    laplacian phi2 = sum_{i<j} (phi1_ii phi1_jj - phi1_ij phi1_ji).
  * delta1(k) = sqrt(V P_lin(k)) omega(k) with omega the Fourier transform of a
    real white-noise field omega(q).

Readings: omega(q) ~ N(0, 1) i.i.d. on the N_l^3 particle lattice;
delta1(q) = irfftn( sqrt(P(k) / V_cell) rfftn(omega) ), V_cell = (L/N_l)^3,
which gives <|delta1(k)|^2> = V P(k) for the continuous transform.  Spectral
derivatives on the lattice's own k grid (radians per lattice spacing); the
first-derivative factor i k_j is zeroed on the Nyquist plane of j, the mixed
second-derivative factor -k_i k_j (i != j) on the Nyquist planes of i and j,
diagonal second derivatives and 1/k^2 keep Nyquist.  Displacements are turned
into mesh-cell units by the lattice spacing r (cells per lattice spacing);
momentum p = a^2 E(a) ds/dln a in cell units with H0 = 1.
"""
import math

import numpy as np

from . import cosmology as cosmo_mod

PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def lattice_wavenumbers(n):
    kx = 2 * np.pi * np.fft.fftfreq(n)
    kz = 2 * np.pi * np.fft.rfftfreq(n)
    K = np.meshgrid(kx, kx, kz, indexing="ij")
    nyq = []
    for ax in range(3):
        m = np.zeros(K[0].shape, dtype=bool)
        sl = [slice(None)] * 3
        sl[ax] = n // 2
        m[tuple(sl)] = True
        nyq.append(m)
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    inv_k2 = np.zeros_like(k2)
    inv_k2[k2 > 0] = 1.0 / k2[k2 > 0]
    return K, nyq, k2, inv_k2


def first_derivative_kernel(n, j):
    """i k_j on the half-spectrum, zero on the Nyquist plane of j."""
    K, nyq, _, _ = lattice_wavenumbers(n)
    T = 1j * K[j]
    T = np.where(nyq[j], 0.0, T)
    return T


def second_derivative_kernel(n, i, j):
    """-k_i k_j on the half-spectrum; for i != j zero on both Nyquist planes."""
    K, nyq, _, _ = lattice_wavenumbers(n)
    T = -K[i] * K[j]
    if i != j:
        T = np.where(nyq[i] | nyq[j], 0.0, T)
    return T.astype(complex)


def amplitude(n, box, cosmo, om=None):
    """A(k) = sqrt(P_lin(k) / V_cell) on the lattice half-spectrum, A(0) = 0.
    `om` overrides Omega_m (may be complex for complex-step derivatives)."""
    om = cosmo.omega_m if om is None else om
    _, _, k2, _ = lattice_wavenumbers(n)
    cell = box / n
    kphys = np.sqrt(k2) / cell  # h/Mpc
    Aamp = cosmo_mod.power_amplitude(om, cosmo.omega_b, cosmo.h, cosmo.n_s, cosmo.sigma8, cosmo.t_cmb)
    out = np.zeros(k2.shape, dtype=complex if np.iscomplexobj(Aamp) else float)
    nz = k2 > 0
    kk = kphys[nz]
    P = Aamp * kk ** cosmo.n_s * cosmo_mod.eh_nowiggle(kk, om, cosmo.omega_b, cosmo.h, cosmo.t_cmb) ** 2
    out[nz] = np.sqrt(P / cell ** 3)
    return out


def lpt_fields(omega, box, cosmo, amp=None):
    """s1, s2 (each (3, n, n, n), lattice-spacing units) and the Hessian of
    phi1 for white noise omega (n, n, n)."""
    n = omega.shape[0]
    _, _, _, inv_k2 = lattice_wavenumbers(n)
    A = amplitude(n, box, cosmo) if amp is None else amp
    W = np.fft.rfftn(omega)
    delta1_k = A * W
    phi1_k = -delta1_k * inv_k2
    s1 = np.stack([np.fft.irfftn(-first_derivative_kernel(n, j) * phi1_k, s=omega.shape, axes=(0, 1, 2))
                   for j in range(3)])
    H = {}
    for (i, j) in PAIRS:
        H[(i, j)] = np.fft.irfftn(second_derivative_kernel(n, i, j) * phi1_k, s=omega.shape, axes=(0, 1, 2))
    S = (H[(0, 0)] * H[(1, 1)] + H[(0, 0)] * H[(2, 2)] + H[(1, 1)] * H[(2, 2)]
         - H[(0, 1)] ** 2 - H[(0, 2)] ** 2 - H[(1, 2)] ** 2)
    phi2_k = -np.fft.rfftn(S) * inv_k2
    s2 = np.stack([np.fft.irfftn(-first_derivative_kernel(n, j) * phi2_k, s=omega.shape, axes=(0, 1, 2))
                   for j in range(3)])
    return s1, s2, H


def ic_time_factors(a0, om):
    """(D1, D2, P1, P2) at a0 with P_m = a^2 E(a) D_m' (momentum factors)."""
    g = cosmo_mod.growth(np.array([a0]), om)
    e = cosmo_mod.E(a0, om)
    return (g["D1"][0], g["D2"][0], a0 * a0 * e * g["dD1"][0], a0 * a0 * e * g["dD2"][0])


def lpt(omega, box, cosmo, a0, r):
    """2LPT displacement s0 and momentum p0 at a0, shape (N_p, 3), mesh-cell
    units, particles in row-major lattice order (eq. lpt)."""
    s1, s2, _ = lpt_fields(omega, box, cosmo)
    D1, D2, P1, P2 = ic_time_factors(a0, cosmo.omega_m)
    s = r * (D1 * s1 + D2 * s2)
    p = r * (P1 * s1 + P2 * s2)
    return s.reshape(3, -1).T.copy(), p.reshape(3, -1).T.copy()


def lpt_vjp(omega, box, cosmo, a0, r, xbar, pbar):
    """Gradient of <xbar, s0> + <pbar, p0> with respect to omega (n, n, n).

    Transpose of the map omega -> (s0, p0), derived by hand:
      s1bar = r (D1 xbar + P1 pbar),  s2bar = r (D2 xbar + P2 pbar)
      Sbar  = sum_j B_j^T s2bar_j,  B_j = irfft (-T1_j)(-1/k^2) rfft
      Hbar_ii = Sbar * sum_{j != i} H_jj,  Hbar_ij = -2 Sbar H_ij (i < j)
      delta1bar = sum_j C_j^T s1bar_j + sum_{i<=j} E_ij^T Hbar_ij
      omegabar = irfft(A rfft(delta1bar))
    where every operator is irfft(M rfft(.)) with a Hermitian multiplier M and
    hence has transpose irfft(conj(M) rfft(.)).
    """
    n = omega.shape[0]
    shp = omega.shape
    _, _, _, inv_k2 = lattice_wavenumbers(n)
    s1, s2, H = lpt_fields(omega, box, cosmo)
    D1, D2, P1, P2 = ic_time_factors(a0, cosmo.omega_m)
    xb = np.asarray(xbar, dtype=np.float64).T.reshape(3, *shp)
    pb = np.asarray(pbar, dtype=np.float64).T.reshape(3, *shp)
    s1b = r * (D1 * xb + P1 * pb)
    s2b = r * (D2 * xb + P2 * pb)
    # s2_j = irfft( M2_j rfft(S) ) with M2_j = -T1_j * (-1/k^2) = T1_j / k^2
    acc = np.zeros(inv_k2.shape, dtype=complex)
    for j in range(3):
        M2 = first_derivative_kernel(n, j) * inv_k2
        acc += np.conj(M2) * np.fft.rfftn(s2b[j])
    Sb = np.fft.irfftn(acc, s=shp, axes=(0, 1, 2))
    Hb = {}
    Hb[(0, 0)] = Sb * (H[(1, 1)] + H[(2, 2)])
    Hb[(1, 1)] = Sb * (H[(0, 0)] + H[(2, 2)])
    Hb[(2, 2)] = Sb * (H[(0, 0)] + H[(1, 1)])
    Hb[(0, 1)] = -2.0 * Sb * H[(0, 1)]
    Hb[(0, 2)] = -2.0 * Sb * H[(0, 2)]
    Hb[(1, 2)] = -2.0 * Sb * H[(1, 2)]
    # s1_j = irfft( M1_j delta1_k ),  M1_j = T1_j / k^2
    # H_ij = irfft( M_ij delta1_k ),  M_ij = second_derivative_kernel * (-1/k^2)
    acc = np.zeros(inv_k2.shape, dtype=complex)
    for j in range(3):
        M1 = first_derivative_kernel(n, j) * inv_k2
        acc += np.conj(M1) * np.fft.rfftn(s1b[j])
    for (i, j) in PAIRS:
        M = -second_derivative_kernel(n, i, j) * inv_k2
        acc += np.conj(M) * np.fft.rfftn(Hb[(i, j)])
    A = amplitude(n, box, cosmo)
    return np.fft.irfftn(np.conj(A) * acc, s=shp, axes=(0, 1, 2))


def lpt_jvp_omega_m(omega, box, cosmo, a0, r):
    """Tangent (ds0/dOmega_m, dp0/dOmega_m) of the IC map, each (N_p, 3).

    Forward-mode derivative written out: the amplitude A(k) and the time
    factors differentiate by complex step; s1 is linear in A, and
    S = sum_{i<j}(H_ii H_jj - H_ij^2) is differentiated by the product rule.
    """
    n = omega.shape[0]
    shp = omega.shape
    h = cosmo_mod.CSTEP
    om = cosmo.omega_m
    _, _, _, inv_k2 = lattice_wavenumbers(n)
    A = amplitude(n, box, cosmo)
    dA = amplitude(n, box, cosmo, om=om + 1j * h).imag / h
    W = np.fft.rfftn(omega)
    s1, s2, H = lpt_fields(omega, box, cosmo, amp=A)
    # tangent of delta1_k is dA * W; s1 and H are linear in delta1
    ds1, ds2, dH = lpt_fields(omega, box, cosmo, amp=dA)
    dS = (dH[(0, 0)] * H[(1, 1)] + H[(0, 0)] * dH[(1, 1)]
          + dH[(0, 0)] * H[(2, 2)] + H[(0, 0)] * dH[(2, 2)]
          + dH[(1, 1)] * H[(2, 2)] + H[(1, 1)] * dH[(2, 2)]
          - 2 * H[(0, 1)] * dH[(0, 1)] - 2 * H[(0, 2)] * dH[(0, 2)] - 2 * H[(1, 2)] * dH[(1, 2)])
    dphi2_k = -np.fft.rfftn(dS) * inv_k2
    ds2 = np.stack([np.fft.irfftn(-first_derivative_kernel(n, j) * dphi2_k, s=shp, axes=(0, 1, 2)) for j in range(3)])
    D1, D2, P1, P2 = ic_time_factors(a0, om)
    tf = np.array(ic_time_factors(a0, om + 1j * h))
    dD1, dD2, dP1, dP2 = (tf.imag / h)
    del W
    ds = r * (dD1 * s1 + D1 * ds1 + dD2 * s2 + D2 * ds2)
    dp = r * (dP1 * s1 + P1 * ds1 + dP2 * s2 + P2 * ds2)
    return ds.reshape(3, -1).T.copy(), dp.reshape(3, -1).T.copy()


def lpt_dsigma8(omega, box, cosmo, a0, r):
    """(ds0/dsigma8, dp0/dsigma8): s1 is proportional to sigma8 and s2 to
    sigma8^2, so ds/dsigma8 = r (D1 s1 + 2 D2 s2)/sigma8 (closed form)."""
    s1, s2, _ = lpt_fields(omega, box, cosmo)
    D1, D2, P1, P2 = ic_time_factors(a0, cosmo.omega_m)
    ds = r * (D1 * s1 + 2 * D2 * s2) / cosmo.sigma8
    dp = r * (P1 * s1 + 2 * P2 * s2) / cosmo.sigma8
    return ds.reshape(3, -1).T.copy(), dp.reshape(3, -1).T.copy()
