"""GPU parity of the paint, readout and force VJP at the degenerate inputs of
the CIC tile scheme (Sec. 2.2, eq. cic), against the FP64 oracle:

- every particle of the lattice in one mesh cell: one tile holds them all, so
  the paint and the gather walk many particle chunks and the fixed-point
  bound of the tile (count times the largest weight) is at its largest, while
  every other tile is empty;
- a single particle;
- positions exactly on mesh nodes, on the last cell's upper edge, below zero
  and beyond the box (the periodic wrap of the base node).

Tolerances are those of the main parity tests: the mesh type's rounding.
"""
import numpy as np
import pytest
import torch

from oracle import pm as opm
from paper_2211_09815_amd import inputs
from gpu_util import announce, aos, dev, host, rel_l2, soa

pytestmark = pytest.mark.gpu

MDTS = [(torch.float32, 2e-7), (torch.float64, 1e-13)]


def _plan(mesh, ptcl, mdt):
    from paper_2211_09815_amd.api import Plan
    return Plan(mesh, ptcl, mesh_dtype=mdt, state_dtype=torch.float64)


def _lattice(mesh, ptcl):
    return opm.lattice_positions(ptcl, [mesh[a] / ptcl[a] for a in range(3)])


def _paint_and_readout(plan, mesh, q, s, mdt, tol, weights=None):
    s_dev = dev(soa(s), torch.float64)
    rho = host(plan.paint(s_dev))[0]
    assert rel_l2(rho, opm.paint(q + s, mesh)) < tol
    assert abs(rho.sum() - len(q)) < (1e-3 if mdt == torch.float32 else 1e-9) * max(len(q), 1)
    if weights is not None:
        w = host(plan.paint(s_dev, dev(weights, mdt)))
        for c in range(weights.shape[0]):
            assert rel_l2(w[c], opm.paint(q + s, mesh, weights[c])) < tol
    fields = inputs.normal((3,) + tuple(mesh), 71)
    got = host(plan.readout(s_dev, dev(fields, mdt)))
    for c in range(3):
        assert rel_l2(got[c], opm.readout(q + s, fields[c])) < tol


@pytest.mark.parametrize("mdt,tol", MDTS)
def test_all_particles_in_one_cell(mdt, tol):
    announce("edges: 4096 particles in one cell %s" % mdt)
    mesh, ptcl = (32, 32, 32), (16, 16, 16)
    plan = _plan(mesh, ptcl, mdt)
    q = _lattice(mesh, ptcl)
    u = np.random.default_rng(72).random(q.shape)
    s = (np.array([5.0, 7.0, 9.0]) + u) - q
    w = inputs.normal((3, len(q)), 73)
    _paint_and_readout(plan, mesh, q, s, mdt, tol, weights=w)
    # the force VJP walks the crowded tile with four channels (FP64: the
    # clustered force is small against the mesh field, so only there is the
    # oracle comparison at rounding level meaningful)
    if mdt == torch.float64:
        abar = inputs.normal((len(q), 3), 74)
        xbar, _, acc = plan.force_vjp(dev(soa(s), torch.float64), dev(soa(abar), mdt), 0.3)
        xb_ref, _, a_ref = opm.force_vjp(q + s, abar, mesh, len(q), 0.45)
        assert rel_l2(aos(host(xbar)), xb_ref) < 1e-10
        assert rel_l2(aos(host(acc)), a_ref) < 1e-10


@pytest.mark.parametrize("mdt,tol", MDTS)
def test_single_particle(mdt, tol):
    announce("edges: one particle %s" % mdt)
    mesh, ptcl = (16, 16, 16), (1, 1, 1)
    plan = _plan(mesh, ptcl, mdt)
    q = _lattice(mesh, ptcl)
    s = np.array([[3.3, 7.9, 12.25]])
    _paint_and_readout(plan, mesh, q, s, mdt, tol, weights=np.array([[0.7], [-1.3], [2.0]]))


@pytest.mark.parametrize("mdt,tol", MDTS)
def test_positions_on_nodes_edges_and_outside_the_box(mdt, tol):
    announce("edges: nodes, edges, wrapped positions %s" % mdt)
    mesh, ptcl = (16, 16, 16), (4, 4, 4)
    plan = _plan(mesh, ptcl, mdt)
    q = _lattice(mesh, ptcl)
    # target positions per axis: nodes, the upper edge from below, below
    # zero and beyond the box, cycled over the 64 particles and 3 axes
    targets = np.array([0.0, 15.0, 8.0, 16.0 - 2.0 ** -40, -0.5, -16.25, 16.0, 31.75, 4.5, 1.0 - 2.0 ** -52,
                        -1e-13, 47.0])
    x = np.stack([np.roll(targets, a)[np.arange(len(q)) % len(targets)] for a in range(3)], axis=1)
    s = x - q
    _paint_and_readout(plan, mesh, q, s, mdt, tol, weights=inputs.normal((3, len(q)), 75))
