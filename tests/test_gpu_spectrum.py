"""GPU parity of the power-spectrum estimator (pm_power_spectrum) against
the oracle's objective.power_spectrum, which the CPU tests pin to a
brute-force sum over the full complex spectrum, to single Fourier modes and
to Parseval's identity.  P is defined through <delta(k) delta(k')> = V P(k)
(Sec. 2.1, eq. Plin).

Tolerances: the shell counts are integers and must match exactly; the shell
mean |k| does not depend on the field and differs only by the order of its
FP64 sum over up to ~1e5 modes (1e-12); P follows the oracle to rounding in
FP64 mode (1e-11 per shell, the same summation-order bound) and to the
float32 FFT's rounding in FP32 mode (2e-5 per shell, relative to that
shell's value).
"""
import numpy as np
import pytest
import torch

from oracle import objective as oobj
from paper_2211_09815_amd import inputs
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def _plan(n, box, mdt):
    from paper_2211_09815_amd.api import Plan
    return Plan(n, 2, box=box, mesh_dtype=mdt, state_dtype=torch.float64)


def _field(n, seed):
    """A field with power at every scale: white noise plus two plane waves
    (one on the Nyquist plane of z) and a smooth large-scale component."""
    g = np.stack(np.meshgrid(*[np.arange(n, dtype=float)] * 3, indexing="ij"))
    x = inputs.normal((n, n, n), seed)
    x += 3.0 * np.cos(2 * np.pi * (g[0] + 2 * g[1]) / n + 0.3)
    x += 0.5 * np.cos(np.pi * g[2] + 0.2)
    x += 2.0 * np.sin(2 * np.pi * g[1] / n) * np.cos(2 * np.pi * g[2] / n)
    return x


def _compare(n, box, mdt, seed, tol):
    plan = _plan(n, box, mdt)
    x = _field(n, seed)
    if mdt == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    k, P, cnt = (host(t) for t in plan.power_spectrum(dev(x, mdt)))
    k_ref, P_ref, c_ref = oobj.power_spectrum(x, box)
    np.testing.assert_array_equal(cnt, c_ref)
    np.testing.assert_allclose(k, k_ref, rtol=1e-12)
    np.testing.assert_allclose(P, P_ref, rtol=tol)
    return plan, x


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64, 128])
@pytest.mark.parametrize("mdt,tol", [(torch.float64, 1e-11), (torch.float32, 2e-5)])
def test_power_spectrum_vs_oracle(n, mdt, tol):
    announce("power spectrum n=%d %s" % (n, mdt))
    _compare(n, 3.0 * n, mdt, 70 + n, tol)


def test_power_spectrum_full_size_fp32():
    # the 512^3 FP32 mesh of the single-force and 512^3 benchmark shapes
    announce("power spectrum n=512 fp32")
    _compare(512, 512.0, torch.float32, 71, 2e-5)


@pytest.mark.parametrize("mdt", [torch.float32, torch.float64])
def test_power_spectrum_of_a_spectrum_and_reproducible(mdt):
    announce("power spectrum from a half spectrum %s" % mdt)
    n, box = 32, 100.0
    plan = _plan(n, box, mdt)
    x = dev(_field(n, 72), mdt)
    dk = plan.fft_r2c(x)[0]
    a = [host(t) for t in plan.power_spectrum(dk, spectrum=True)]
    b = [host(t) for t in plan.power_spectrum(dk, spectrum=True)]
    c = [host(t) for t in plan.power_spectrum(x)]
    for u, v, w in zip(a, b, c):
        np.testing.assert_array_equal(u, v)      # fixed-order reduction: bitwise
        np.testing.assert_array_equal(u, w)


def test_power_spectrum_rejects_non_cubic():
    from paper_2211_09815_amd import _lib
    from paper_2211_09815_amd.api import Plan
    announce("power spectrum argument errors")
    plan = Plan((16, 16, 32), 2, box=(16.0, 16.0, 32.0), mesh_dtype=torch.float64)
    with pytest.raises(_lib.PmError) as e:
        plan.power_spectrum(torch.zeros((16, 16, 32), dtype=torch.float64, device="cuda"))
    assert e.value.code == _lib.PM_EUNSUPPORTED
    plan = Plan(16, 2, box=(16.0, 16.0, 20.0), mesh_dtype=torch.float64)
    with pytest.raises(_lib.PmError) as e:
        plan.power_spectrum(torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda"))
    assert e.value.code == _lib.PM_EUNSUPPORTED
