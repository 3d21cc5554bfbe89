"""Final-snapshot density objective and power-spectrum estimator -- plain
FP64 reference.

Test infrastructure only (see oracle/__init__.py).

Paper passages followed: eq. O (objective on the observed state) and the
gradient test of Sec. 4.2, which uses the mean squared error between two
final CIC density fields on the simulation mesh at a = 1, one of them held
fixed as the target.

Reading: J = (1/N_c) sum_c (delta(c) - delta_t(c))^2 with
delta = rho N_c / N_p - 1; dJ/drho = 2 (delta - delta_t) / N_p; dJ/dp_n = 0.
"""
import numpy as np

from . import pm


def density_mse(x, target, n_particles):
    """(J, dJ/dx) for particles at x (n, 3) against the target contrast."""
    shape = target.shape
    delta = pm.density_contrast(x, shape, n_particles)
    diff = delta - target
    J = float(np.mean(diff * diff))
    mbar = 2.0 * diff / n_particles
    return J, pm.readout_grad(x, mbar)


def power_spectrum(delta, box):
    """Shell-averaged P(k) of a real field delta on a cubic mesh.

    P(k_b) = mean over modes with |k| in [(b - 1/2) k_f, (b + 1/2) k_f) of
    |delta(k) V / N_c|^2 / V, k_f = 2 pi / L; half-spectrum modes carry weight
    2 except on the kz = 0 and Nyquist planes.  No window deconvolution.
    Returns (k_centres, P, mode_counts) for bins b = 1 .. N/2.
    """
    n = delta.shape[0]
    V = box ** 3
    ncell = delta.size
    dk = np.fft.rfftn(delta) * (V / ncell)
    kf = 2 * np.pi / box
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    w = np.full(KZ.shape, 2.0)
    w[..., 0] = 1.0
    if n % 2 == 0:
        w[..., -1] = 1.0
    b = np.floor(kmag + 0.5).astype(int)
    nb = n // 2
    p = np.abs(dk) ** 2 / V
    sel = (b >= 1) & (b <= nb)
    cnt = np.bincount(b[sel], weights=w[sel], minlength=nb + 1)[1:]
    ps = np.bincount(b[sel], weights=(w * p)[sel], minlength=nb + 1)[1:]
    ks = np.bincount(b[sel], weights=(w * kmag)[sel], minlength=nb + 1)[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        return ks / cnt * kf, ps / cnt, cnt
