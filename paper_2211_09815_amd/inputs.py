"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module only draws random numbers; it holds none of the method's
arithmetic.  Both the GPU path and the CPU oracle receive the arrays it makes.

Seeds used throughout: 0 = the simulated run's white noise, 1 = the target
run's white noise, 2 = choice of finite-difference probes, 3 = random
cotangents / displacements of the single-force benchmark.
"""
import numpy as np

SEED_RUN = 0
SEED_TARGET = 1
SEED_PROBES = 2
SEED_COTANGENT = 3


def white_noise(n, seed, dtype=np.float64, chunk=1 << 24):
    """omega(q) ~ N(0, 1) i.i.d. on an n^3 lattice, C order (i, j, k).

    Drawn in float64 from numpy's default generator in chunks of `chunk`
    values and cast to `dtype`, so every dtype sees the same stream."""
    rng = np.random.default_rng(seed)
    total = n ** 3
    out = np.empty(total, dtype=dtype)
    for start in range(0, total, chunk):
        stop = min(total, start + chunk)
        out[start:stop] = rng.standard_normal(stop - start)
    return out.reshape(n, n, n)


def normal(shape, seed, scale=1.0, dtype=np.float64):
    """Gaussian array of `shape` (e.g. cotangents or test displacements)."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(shape)).astype(dtype)


def uniform(shape, seed, low=0.0, high=1.0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=shape).astype(dtype)


def probe_indices(n_total, count, seed=SEED_PROBES):
    """`count` distinct flat indices in [0, n_total) for finite-difference probes."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=count, replace=False))
