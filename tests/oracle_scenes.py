"""Small scenes for the oracle's own tests (test helper, not a test module)."""
import numpy as np

import workloads as W


def tiny_cantilever(nx=3, ny=2, nz=2, youngs=None):
    sc = W.cantilever(nx, ny, nz, steps=3)
    if youngs is not None:
        sc.youngs = np.asarray(youngs, dtype=np.float64)
    return sc


def tiny_free(nx=2, ny=2, nz=2, gravity=(0.0, 0.0, -9.81)):
    sc = W.cantilever(nx, ny, nz, steps=3)
    sc.fixed_nodes = np.zeros((0, 3), np.int32)
    sc.gravity = gravity
    return sc


def tiny_robot(steps=3, dx=0.05):
    """Legs + slab with muscles, penalty ground and friction, feet below ground.

    A coarser voxel (5 cm) keeps the PD contraction factor near 0.9 so that the
    oracle's plain iterations converge in a few hundred steps.
    """
    sc = W.legged_body(8, 6, 4, steps=steps, leg_height=2)
    sc.dx = dx
    sc.origin = (0.0, 0.0, -0.03 * dx)
    return sc


def perturbed_state(model, scale=2e-3, seed=0):
    rng = np.random.default_rng(seed)
    x = model.X + scale * rng.standard_normal(3 * model.N)
    x[model.fixed] = model.X[model.fixed]
    v = 0.05 * rng.standard_normal(3 * model.N)
    v[model.fixed] = 0.0
    return x, v
