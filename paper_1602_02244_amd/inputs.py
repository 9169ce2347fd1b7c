"""Seeded synthetic inputs for the FMM workloads.

This module only draws random numbers; it holds none of the method's
arithmetic.  Every generator works in FP64 and rounds the coordinates once to
FP32, so that the GPU library (FP32 inputs) and any FP64 checker see exactly
the same values.

Distributions:
  * ``uniform_cube``  -- x ~ U[0,1)^3, charges ~ U[-1,1]
  * ``sphere_surface``-- x = g/|g| with g ~ N(0, I_3), charges ~ N(0,1)
  * ``plummer``       -- radius r = (u^(-2/3) - 1)^(-1/2), u ~ U(0,1) (scale
    radius 1), rejected when r > 10; isotropic direction; charges in (0,1]
    as 1 - U[0,1)
"""
import numpy as np

WORKLOADS = {
    # name: (n, distribution, p, ncrit, theta)
    "uniform-4k": (4096, "cube", 6, 64, 0.4),
    "uniform-1M": (1 << 20, "cube", 10, 64, 0.4),
    "sphere-4M": (1 << 22, "sphere", 8, 128, 0.4),
    "plummer-1M": (1 << 20, "plummer", 10, 64, 0.4),
    "uniform-16M": (1 << 24, "cube", 12, 64, 0.4),
}
SEEDS = {"uniform-4k": 1001, "uniform-1M": 1002, "sphere-4M": 1003, "plummer-1M": 1004, "uniform-16M": 1005}


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def uniform_cube(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return _f32(x), _f32(q)


def sphere_surface(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    x = g / np.linalg.norm(g, axis=1, keepdims=True)
    q = rng.standard_normal(n)
    return _f32(x), _f32(q)


def plummer(n, seed, rmax=10.0):
    rng = np.random.default_rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = int((n - out.shape[0]) * 1.05) + 16
        u = rng.random(m)
        u = u[u > 0]
        r = (u ** (-2.0 / 3.0) - 1.0) ** -0.5
        r = r[r <= rmax]
        g = rng.standard_normal((r.shape[0], 3))
        d = g / np.linalg.norm(g, axis=1, keepdims=True)
        out = np.concatenate([out, d * r[:, None]])
    x = out[:n]
    q = 1.0 - rng.random(n)
    return _f32(x), _f32(q)


def make(dist, n, seed):
    if dist == "cube":
        return uniform_cube(n, seed)
    if dist == "sphere":
        return sphere_surface(n, seed)
    if dist == "plummer":
        return plummer(n, seed)
    raise ValueError(dist)


def workload(name, n=None):
    """Points (float32 [n,3]) and charges (float32 [n]) of a named workload.
    ``n`` overrides the size (same distribution and seed)."""
    n0, dist, p, ncrit, theta = WORKLOADS[name]
    return make(dist, n if n is not None else n0, SEEDS[name])


def adjoint_weights(n, seed=3000):
    """Loss weights w ~ N(0,1) for L = sum_i w_i phi_i."""
    return _f32(np.random.default_rng(seed).standard_normal(n))


def fd_coordinates(n, count=64, seed=2000):
    """(index, axis) pairs for finite-difference checks."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, count), rng.integers(0, 3, count)


def sample_targets(n, count=1000, seed=4000):
    """Distinct target indices for sampled checks."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)
