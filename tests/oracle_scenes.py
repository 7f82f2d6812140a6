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


def landing_block(nx=3, ny=3, nz=2, lift=1e-4, youngs=1e5, muscles=False):
    """A free block just above a complementarity ground (no penalty), its
    bottom layer the contact candidates, falling onto it at 0.1 m/s with some
    sideways motion: every bottom node meets the plane inside the first step
    (t = lift / 0.1 < h).  Returns (scene, candidates, x0, v0)."""
    sc = W.cantilever(nx, ny, nz, steps=3)
    sc.fixed_nodes = np.zeros((0, 3), np.int32)
    sc.youngs = np.full(sc.n_elements, youngs)
    sc.h = 5e-3
    sc.origin = (0.0, 0.0, lift)
    if muscles:
        sc.muscle_k = 2.0 * youngs / (2.0 * 1.45)
    nodes = W.present_nodes(sc.cells)
    cand = np.nonzero(nodes[:, 2] == 0)[0].astype(np.int64)
    X = (np.asarray(sc.origin)[None, :] + sc.dx * nodes).reshape(-1)
    rng = np.random.default_rng(5)
    v = np.tile([0.05, 0.02, -0.1], len(nodes)) + 0.01 * rng.standard_normal(3 * len(nodes))
    return sc, cand, X, v
