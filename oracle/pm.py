"""Particle-mesh force and its vector-Jacobian product -- plain FP64 reference.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed (Sec. 2.2, "Force Evaluation"):
  * eq. cic: CIC (trilinear) weight W(x, x') = prod_i max(1 - |x_i - x'_i|/l, 0).
    Positions here are in mesh-cell units (l = 1) and the mesh is periodic.
  * Poisson equation for phi~ = a phi: laplacian phi~ = 1.5 Omega_m H0^2 delta;
    in Fourier space -k^2 phi~(k) = 1.5 Omega_m delta(k), and the field
    -grad phi~ is -i k phi~(k); one forward and three inverse FFTs.
  * the accelerations are gathered from the mesh with the same weights as the
    paint.
  * Sec. 3.6 (application to simulation): the force VJPs alpha = pi . da/dx and
    zeta = pi . da/dtheta entering eq. KDFKO_adj; the scatter/gather VJPs are
    written out by hand (no automatic differentiation).

Readings: numpy FFT conventions (forward unnormalised, inverse 1/N);
k_j = 2 pi m_j / N_j in cell units; exact spectral kernels, no deconvolution;
delta(k = 0) -> 0; the i k_j factor is zeroed on the Nyquist plane of axis j
so that each gradient operator is real and exactly anti-self-adjoint.
CIC: base node floor(x), fraction f = x - floor(x) in [0, 1), weights
(1 - f, f) per axis, periodic wrap; the weight derivative uses the same split
(-1, +1), i.e. the right-sided derivative at a node.
"""
import numpy as np


def _corners():
    return [(dx, dy, dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)]


def cic_split(x):
    """Base node index and fractional offset per particle and axis."""
    x = np.asarray(x, dtype=np.float64)
    i0 = np.floor(x)
    f = x - i0
    return i0.astype(np.int64), f


def _corner_weights(f, corner):
    """1-d weights (1 - f, f) chosen by the corner offsets, per axis."""
    w = np.ones(f.shape[0])
    parts = []
    for ax in range(3):
        wa = f[:, ax] if corner[ax] else 1.0 - f[:, ax]
        parts.append(wa)
        w = w * wa
    return w, parts


def _flat_index(i0, corner, shape):
    idx = [(i0[:, ax] + corner[ax]) % shape[ax] for ax in range(3)]
    return (idx[0] * shape[1] + idx[1]) * shape[2] + idx[2]


def paint(x, shape, values=None):
    """Scatter: rho(c) = sum_n v_n W(c, x_n) on a periodic mesh of `shape`.
    `values` defaults to unit mass."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    v = np.ones(n) if values is None else np.asarray(values, dtype=np.float64)
    i0, f = cic_split(x)
    size = shape[0] * shape[1] * shape[2]
    rho = np.zeros(size)
    for c in _corners():
        w, _ = _corner_weights(f, c)
        rho += np.bincount(_flat_index(i0, c, shape), weights=w * v, minlength=size)
    return rho.reshape(shape)


def readout(x, field):
    """Gather: out_n = sum_c W(c, x_n) field(c) with the paint's weights."""
    x = np.asarray(x, dtype=np.float64)
    shape = field.shape
    flat = field.ravel()
    i0, f = cic_split(x)
    out = np.zeros(x.shape[0])
    for c in _corners():
        w, _ = _corner_weights(f, c)
        out += w * flat[_flat_index(i0, c, shape)]
    return out


def readout_grad(x, field):
    """out_{n,k} = sum_c d/dx_k W(c, x_n) field(c); derivative of the CIC
    weights with the split of cic_split (right-sided at a node)."""
    x = np.asarray(x, dtype=np.float64)
    shape = field.shape
    flat = field.ravel()
    i0, f = cic_split(x)
    out = np.zeros((x.shape[0], 3))
    for c in _corners():
        _, parts = _corner_weights(f, c)
        vals = flat[_flat_index(i0, c, shape)]
        for k in range(3):
            dk = 1.0 if c[k] else -1.0
            others = np.ones(x.shape[0])
            for ax in range(3):
                if ax != k:
                    others = others * parts[ax]
            out[:, k] += dk * others * vals
    return out


def wavenumbers(shape):
    """k_j grids (cell units) on the rfftn half-spectrum and the Nyquist masks."""
    kx = 2 * np.pi * np.fft.fftfreq(shape[0])
    ky = 2 * np.pi * np.fft.fftfreq(shape[1])
    kz = 2 * np.pi * np.fft.rfftfreq(shape[2])
    KX, KY, KZ = np.meshgrid(kx, ky, kz, indexing="ij")
    nyq = []
    for ax, K in enumerate((KX, KY, KZ)):
        m = np.zeros(K.shape, dtype=bool)
        if shape[ax] % 2 == 0:
            sl = [slice(None)] * 3
            sl[ax] = shape[ax] // 2
            m[tuple(sl)] = True
        nyq.append(m)
    return (KX, KY, KZ), nyq


def gradient_kernels(shape, coef):
    """T_j(k) = i k_j coef / k^2 (the Fourier multiplier of -grad phi~ from
    delta, coef = 1.5 Omega_m), zero at k = 0 and on the Nyquist plane of j."""
    (KX, KY, KZ), nyq = wavenumbers(shape)
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    inv = np.zeros_like(k2)
    nz = k2 > 0
    inv[nz] = 1.0 / k2[nz]
    out = []
    for j, K in enumerate((KX, KY, KZ)):
        T = 1j * K * coef * inv
        T[nyq[j]] = 0.0
        out.append(T)
    return out


def poisson_gradient(delta_k, shape, coef):
    """g_j(k) = T_j(k) delta(k) for j = 0, 1, 2 (Sec. 2.2)."""
    return [T * delta_k for T in gradient_kernels(shape, coef)]


def density_contrast(x, shape, n_particles):
    """delta = rho / rho_bar - 1 with unit particle mass, rho_bar = N_p / N_c."""
    rho = paint(x, shape)
    ncell = shape[0] * shape[1] * shape[2]
    return rho * (ncell / n_particles) - 1.0


def force_fields(x, shape, n_particles, coef):
    """The three mesh components of -grad phi~ for particles at x."""
    delta = density_contrast(x, shape, n_particles)
    dk = np.fft.rfftn(delta)
    return [np.fft.irfftn(g, s=shape, axes=(0, 1, 2)) for g in poisson_gradient(dk, shape, coef)]


def force(x, shape, n_particles, coef):
    """Accelerations a_n = -grad phi~(x_n), shape (n, 3)."""
    g = force_fields(x, shape, n_particles, coef)
    return np.stack([readout(x, gj) for gj in g], axis=1)


def force_vjp(x, abar, shape, n_particles, coef):
    """VJP of the force map x -> a(x; coef) with cotangent abar (n, 3).

    Returns (xbar (n, 3), coef_bar, a):
      a_{m,j} = sum_c W(c, x_m) g_j(c),  g_j = G_j delta,  G_j = irfft T_j rfft,
      delta = (N_c / N_p) rho - 1,  rho = sum_m W(., x_m).
    Chain rule:
      gbar_j(c)  = sum_m abar_{m,j} W(c, x_m)                   (paint of abar_j)
      rhobar     = (N_c/N_p) sum_j G_j^T gbar_j,   G_j^T = irfft conj(T_j) rfft
      xbar_{n,k} = sum_c d_k W(c, x_n) [ sum_j abar_{n,j} g_j(c) + rhobar(c) ]
      coef_bar   = sum_{n,j} abar_{n,j} a_{n,j} / coef  (a is linear in coef)
    """
    x = np.asarray(x, dtype=np.float64)
    abar = np.asarray(abar, dtype=np.float64)
    ncell = shape[0] * shape[1] * shape[2]
    T = gradient_kernels(shape, coef)
    delta = density_contrast(x, shape, n_particles)
    dk = np.fft.rfftn(delta)
    g = [np.fft.irfftn(Tj * dk, s=shape, axes=(0, 1, 2)) for Tj in T]
    a = np.stack([readout(x, gj) for gj in g], axis=1)
    gbar = [paint(x, shape, abar[:, j]) for j in range(3)]
    acc = np.zeros(dk.shape, dtype=complex)
    for j in range(3):
        acc += np.conj(T[j]) * np.fft.rfftn(gbar[j])
    rhobar = np.fft.irfftn(acc, s=shape, axes=(0, 1, 2)) * (ncell / n_particles)
    xbar = readout_grad(x, rhobar)
    for j in range(3):
        # sum_c d_k W(c, x_n) abar_{n,j} g_j(c)
        xbar += abar[:, j:j + 1] * readout_grad(x, g[j])
    coef_bar = float(np.sum(abar * a)) / coef
    return xbar, coef_bar, a


def lattice_positions(ptcl_shape, r, offset=0.0):
    """Lagrangian positions q = (i, j, k) * r + offset (cell units), particles
    in row-major lattice order (Sec. 2.1: particles start on a Cartesian grid).
    `r` is the lattice spacing in mesh cells (scalar or per axis)."""
    r = np.broadcast_to(np.asarray(r, dtype=np.float64), (3,))
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in ptcl_shape], indexing="ij")
    return np.stack([g.ravel() * r[ax] + offset for ax, g in enumerate(grids)], axis=1)
