"""The allocation-free power spectrum (pm_power_spectrum_noalloc) against
the plan-based pm_power_spectrum, through the C-ABI: the two share their
kernels and reduction order, so their outputs must be bitwise equal.  Two
calls in a row on one GPU, the second with a smaller mesh, check that the
static scratch left by the first call does not leak into the second; the
limits are refused on the host before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2211_09815_amd import _lib, inputs
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def _noalloc(n, box, mdt, dk):
    L = _lib.lib()
    out = [torch.full((n // 2,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
    code = _lib.PM_F64 if mdt == torch.float64 else _lib.PM_F32
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.pm_power_spectrum_noalloc(n, box, code, ctypes.c_void_p(dk.data_ptr()),
                                     *[ctypes.c_void_p(t.data_ptr()) for t in out], stream)
    _lib.check(rc)
    return out


def test_noalloc_power_spectrum_matches_plan_entry_point():
    from oracle import objective as oobj
    from paper_2211_09815_amd.api import Plan
    for n, box, mdt, seed in ((128, 300.0, torch.float32, 90), (64, 200.0, torch.float64, 91),
                              (16, 40.0, torch.float32, 92)):
        announce("noalloc power spectrum n=%d %s" % (n, mdt))
        plan = Plan(n, 2, box=box, mesh_dtype=mdt, state_dtype=torch.float64)
        x = inputs.normal((n, n, n), seed)
        dk = plan.fft_r2c(dev(x, mdt))[0]
        ref = [host(t) for t in plan.power_spectrum(dk, spectrum=True)]
        got = [host(t) for t in _noalloc(n, box, mdt, dk)]
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)
        # and the estimator itself, against the oracle
        xs = x.astype(np.float32).astype(np.float64) if mdt == torch.float32 else x
        k_ref, P_ref, c_ref = oobj.power_spectrum(xs, box)
        np.testing.assert_array_equal(got[2], c_ref)
        np.testing.assert_allclose(got[1], P_ref, rtol=2e-5 if mdt == torch.float32 else 1e-11)


def test_noalloc_power_spectrum_refuses_bad_sizes():
    announce("noalloc power spectrum argument errors")
    L = _lib.lib()
    buf = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert L.pm_power_spectrum_noalloc(2048, 1.0, _lib.PM_F32, p, p, p, p, None) == _lib.PM_ESHAPE
    assert b"scratch" in L.pm_last_error(None)
    assert L.pm_power_spectrum_noalloc(12, 1.0, _lib.PM_F32, p, p, p, p, None) == _lib.PM_ESHAPE
    assert L.pm_power_spectrum_noalloc(16, 0.0, _lib.PM_F32, p, p, p, p, None) == _lib.PM_EINVAL
    assert L.pm_power_spectrum_noalloc(16, 1.0, 5, p, p, p, p, None) == _lib.PM_EINVAL
    assert L.pm_power_spectrum_noalloc(16, 1.0, _lib.PM_F32, None, p, p, p, None) == _lib.PM_EINVAL
