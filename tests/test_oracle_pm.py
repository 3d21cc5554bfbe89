"""Pins of the oracle's CIC paint/readout, Poisson gradient, force and force
VJP (no GPU)."""
import itertools

import numpy as np
import pytest

from oracle import pm
from paper_2211_09815_amd import inputs


def test_rfftn_convention_brute_force_dft():
    # the oracle's FFT is numpy's: unnormalised forward, exp(-i k.x), 1/N inverse
    n = (4, 6, 8)
    f = inputs.normal(n, 11)
    F = np.fft.rfftn(f)
    grid = np.stack(np.meshgrid(*[np.arange(m) for m in n], indexing="ij"), -1)
    for m in [(0, 0, 0), (1, 2, 3), (3, 5, 4), (2, 0, 1)]:
        phase = sum(2 * np.pi * m[ax] * grid[..., ax] / n[ax] for ax in range(3))
        ref = np.sum(f * np.exp(-1j * phase))
        assert abs(F[m] - ref) < 1e-12 * np.sum(np.abs(f))
    np.testing.assert_allclose(np.fft.irfftn(F, s=n), f, atol=1e-13)


def _brute_cic(x, shape):
    """eq. cic evaluated directly at every node with minimum-image distances."""
    rho = np.zeros(shape)
    for c in itertools.product(*[range(m) for m in shape]):
        w = np.ones(len(x))
        for ax in range(3):
            d = (x[:, ax] - c[ax]) % shape[ax]
            d = np.minimum(d, shape[ax] - d)
            w = w * np.maximum(1.0 - d, 0.0)
        rho[c] = w.sum()
    return rho


def test_paint_matches_brute_force_cic():
    shape = (4, 5, 6)
    x = inputs.uniform((7, 3), 5, -3.0, 9.0)
    np.testing.assert_allclose(pm.paint(x, shape), _brute_cic(x, shape), atol=1e-13)


def test_paint_mass_conservation_and_node_particles():
    shape = (8, 8, 8)
    x = inputs.uniform((100, 3), 6, -20.0, 20.0)
    assert pm.paint(x, shape).sum() == pytest.approx(100.0, rel=1e-14)
    # a particle exactly on a node puts all its mass there
    rho = pm.paint(np.array([[3.0, 4.0, 5.0]]), shape)
    assert rho[3, 4, 5] == 1.0 and rho.sum() == 1.0


def test_paint_readout_adjoint():
    shape = (8, 6, 10)
    x = inputs.uniform((50, 3), 7, 0.0, 12.0)
    v = inputs.normal(50, 8)
    m = inputs.normal(shape, 9)
    lhs = np.sum(pm.paint(x, shape, v) * m)
    rhs = np.sum(v * pm.readout(x, m))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_readout_constant_and_linear():
    shape = (8, 8, 8)
    x = inputs.uniform((40, 3), 10, 0.0, 7.0)   # away from the wrap
    np.testing.assert_allclose(pm.readout(x, np.full(shape, 2.5)), 2.5, rtol=1e-14)
    # trilinear interpolation reproduces a linear field exactly inside the box
    lin = np.fromfunction(lambda i, j, k: 0.5 * i - 0.25 * j + 2 * k, shape)
    np.testing.assert_allclose(pm.readout(x, lin), 0.5 * x[:, 0] - 0.25 * x[:, 1] + 2 * x[:, 2], rtol=1e-12)


def test_readout_grad_matches_finite_difference():
    shape = (8, 8, 8)
    x = inputs.uniform((30, 3), 12, 0.0, 8.0)
    m = inputs.normal(shape, 13)
    g = pm.readout_grad(x, m)
    h = 1e-7
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (pm.readout(x + e, m) - pm.readout(x - e, m)) / (2 * h)
        np.testing.assert_allclose(g[:, k], fd, rtol=1e-6, atol=1e-8)


def test_poisson_gradient_single_mode():
    # delta = cos(k.x) -> -grad phi~ = -coef k sin(k.x) / k^2 (Sec. 2.2)
    shape = (16, 16, 16)
    coef = 0.45
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1).astype(float)
    for m in [(1, 0, 0), (2, 3, 1), (0, 5, 7), (7, 7, 7)]:
        kv = np.array([2 * np.pi * m[ax] / shape[ax] for ax in range(3)])
        phase = idx @ kv
        delta = np.cos(phase)
        gk = pm.poisson_gradient(np.fft.rfftn(delta), shape, coef)
        k2 = kv @ kv
        for j in range(3):
            g = np.fft.irfftn(gk[j], s=shape)
            np.testing.assert_allclose(g, -coef * kv[j] * np.sin(phase) / k2, atol=1e-13)


def test_gradient_operator_anti_self_adjoint():
    shape = (8, 8, 8)
    u = inputs.normal(shape, 14)
    v = inputs.normal(shape, 15)
    for T in pm.gradient_kernels(shape, 1.0):
        Gu = np.fft.irfftn(T * np.fft.rfftn(u), s=shape)
        Gv = np.fft.irfftn(T * np.fft.rfftn(v), s=shape)
        assert np.sum(Gu * v) == pytest.approx(-np.sum(u * Gv), abs=1e-12)


def test_force_momentum_conservation_and_self_force():
    shape = (16, 16, 16)
    x = inputs.uniform((300, 3), 16, 0.0, 16.0)
    a = pm.force(x, shape, 300, 0.45)
    assert np.abs(a.sum(0)).max() < 1e-12 * np.abs(a).sum()
    # a single particle feels no force from itself, wherever it is
    for p in inputs.uniform((5, 3), 17, 0.0, 16.0):
        a1 = pm.force(p[None, :], shape, 1, 0.45)
        assert np.abs(a1).max() < 1e-11


def test_force_pair_attracts_and_is_antisymmetric():
    shape = (32, 32, 32)
    x = np.array([[10.3, 16.2, 15.9], [14.3, 16.2, 15.9]])
    a = pm.force(x, shape, 2, 0.45)
    np.testing.assert_allclose(a[0], -a[1], atol=1e-12)
    assert a[0, 0] > 0 and a[1, 0] < 0          # attraction along x
    # far from the mesh scale it approaches Newtonian 1/r^2 (loose, periodic)
    a_near = pm.force(np.array([[10.0, 16, 16], [14.0, 16, 16]]), shape, 2, 0.45)[0, 0]
    a_far = pm.force(np.array([[10.0, 16, 16], [18.0, 16, 16]]), shape, 2, 0.45)[0, 0]
    assert 2.0 < a_near / a_far < 6.0


def test_force_vjp_finite_difference_and_dot_product():
    shape = (16, 16, 16)
    q = pm.lattice_positions((8, 8, 8), 2.0)
    x = q + inputs.normal(q.shape, 18, 0.7)
    npart = len(x)
    abar = inputs.normal(x.shape, 19)
    coef = 0.45
    xbar, coef_bar, a = pm.force_vjp(x, abar, shape, npart, coef)
    np.testing.assert_allclose(a, pm.force(x, shape, npart, coef), rtol=1e-14, atol=1e-14)
    h = 1e-6
    for seed in (20, 21, 22):
        v = inputs.normal(x.shape, seed)
        fp = np.sum(abar * pm.force(x + h * v, shape, npart, coef))
        fm = np.sum(abar * pm.force(x - h * v, shape, npart, coef))
        assert np.sum(xbar * v) == pytest.approx((fp - fm) / (2 * h), rel=1e-7)
    fp = np.sum(abar * pm.force(x, shape, npart, coef * (1 + 1e-6)))
    fm = np.sum(abar * pm.force(x, shape, npart, coef * (1 - 1e-6)))
    assert coef_bar == pytest.approx((fp - fm) / (2e-6 * coef), rel=1e-8)
