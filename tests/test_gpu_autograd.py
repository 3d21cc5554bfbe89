"""The torch.autograd wrappers force / force_vjp and the Simulate function:
gradients through them are the library's own discrete VJPs, checked against
the FP64 oracle's force VJP (Sec. 3.6), against a central difference in
Omega_m (the force is linear in it) and against the direct pm_force_vjp call.
"""
import numpy as np
import pytest
import torch

from oracle import pm as opm
from paper_2211_09815_amd import inputs
from gpu_util import announce, aos, dev, host, rel_l2, soa

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mdt,tol", [(torch.float64, 1e-11), (torch.float32, 2e-5)])
def test_force_autograd_vs_oracle(mdt, tol):
    import paper_2211_09815_amd as pmx
    from paper_2211_09815_amd.api import Plan
    announce("autograd force %s" % mdt)
    mesh, ptcl = (32, 32, 32), (16, 16, 16)
    plan = Plan(mesh, ptcl, mesh_dtype=mdt, state_dtype=torch.float64)
    q = opm.lattice_positions(ptcl, 2.0)
    s = inputs.normal(q.shape, 80, 1.2)
    w = inputs.normal(q.shape, 81)
    disp = dev(soa(s), torch.float64).requires_grad_(True)
    om = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    acc = pmx.force(disp, om, plan)
    loss = (acc.double() * dev(soa(w), torch.float64)).sum()
    loss.backward()
    xb_ref, cb_ref, a_ref = opm.force_vjp(q + s, w, mesh, len(q), 1.5 * 0.3)
    assert rel_l2(aos(host(acc)), a_ref) < tol
    assert rel_l2(aos(host(disp.grad)), xb_ref) < tol
    assert float(om.grad) == pytest.approx(1.5 * cb_ref, rel=tol)
    # the functional form returns the same numbers
    xb, ob = pmx.force_vjp(disp.detach(), dev(soa(w), mdt), 0.3, plan)
    np.testing.assert_array_equal(host(xb), host(disp.grad).astype(host(xb).dtype))
    # the FP64 per-tile partials behind omega_m_bar follow the order of the
    # particles within a tile, which the binning's atomics set: equal to rounding
    assert float(ob.cpu()) == pytest.approx(float(om.grad), rel=1e-13)


def test_force_autograd_omega_m_central_difference():
    import paper_2211_09815_amd as pmx
    from paper_2211_09815_amd.api import Plan
    announce("autograd force d/dOmega_m")
    mesh, ptcl = (16, 16, 16), (8, 8, 8)
    plan = Plan(mesh, ptcl, mesh_dtype=torch.float64, state_dtype=torch.float64)
    q = opm.lattice_positions(ptcl, 2.0)
    disp = dev(soa(inputs.normal(q.shape, 82, 0.8)), torch.float64)
    w = dev(soa(inputs.normal(q.shape, 83)), torch.float64)
    om = torch.tensor(0.27, dtype=torch.float64, requires_grad=True)
    (pmx.force(disp, om, plan) * w).sum().backward()
    h = 1e-4
    fp = float((pmx.force(disp, 0.27 + h, plan) * w).sum())
    fm = float((pmx.force(disp, 0.27 - h, plan) * w).sum())
    assert float(om.grad) == pytest.approx((fp - fm) / (2 * h), rel=1e-10)
