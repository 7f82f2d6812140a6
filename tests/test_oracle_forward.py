"""Forward PD step of the oracle: invariants, special cases and Newton."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import model as om, forward as of
from oracle_scenes import tiny_free, tiny_cantilever, tiny_robot, perturbed_state
import workloads as W


def test_rest_state_stationary():
    # Dirichlet beam at rest without gravity
    sc = tiny_cantilever()
    sc.gravity = (0.0, 0.0, 0.0)
    m = om.Model(sc)
    x, v = m.X.copy(), np.zeros(3 * m.N)
    for _ in range(3):
        x, v, info = of.pd_step(m, x, v)
    assert np.abs(x - m.X).max() < 1e-15 and np.abs(v).max() < 1e-12
    # free body in a rigidly rotated, translated rest pose
    sc = tiny_free(gravity=(0.0, 0.0, 0.0))
    m = om.Model(sc)
    Q = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    x0 = (m.X.reshape(-1, 3) @ Q.T + np.array([0.1, 0.2, 0.3])).reshape(-1)
    x1, v1, _ = of.pd_step(m, x0, np.zeros_like(x0))
    assert np.abs(x1 - x0).max() < 1e-13


def test_free_fall_is_exact():
    sc = tiny_free()
    m = om.Model(sc)
    v0 = np.tile([0.3, -0.1, 0.2], m.N)
    x1, v1, info = of.pd_step(m, m.X, v0)
    expect = m.X + m.h * v0 + m.h ** 2 * np.tile(sc.gravity, m.N)
    assert np.abs(x1 - expect).max() < 1e-14
    assert info["iters"] == 0


def test_centre_of_mass_of_every_iterate():
    sc = tiny_free(3, 2, 2)
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, scale=3e-3)
    y = m.y_of(x0, v0)
    x, info = of.pd_solve(m, y, max_iter=15, fixed_iters=True, history=True)
    com_y = (m.Mdiag * y).reshape(-1, 3).sum(0)
    for xk in info["history"][1:]:
        com = (m.Mdiag * xk).reshape(-1, 3).sum(0)
        assert np.abs(com - com_y).max() < 1e-15 * 10


def test_fixed_iteration_count():
    m = om.Model(tiny_cantilever())
    x, v, info = of.pd_step(m, m.X, np.zeros(3 * m.N), max_iter=7, fixed_iters=True)
    assert info["iters"] == 7


def _static_equilibrium(m):
    """Newton on E(x) - (M g)^T x with Dirichlet DoFs at rest (independent of PD)."""
    f = m.free
    x = m.X.copy()
    fg = m.Mdiag * m.gravity
    for _ in range(30):
        gradE = m.grad_g(x, x) - fg
        if np.linalg.norm(gradE[f]) < 1e-13 * np.linalg.norm(fg[f]):
            break
        HE = (m.hessian(x) - np.diag(m.Mdiag / m.h ** 2))[f][:, f] if False else None
        H = m.hessian(x)[f][:, f].toarray() - np.diag(m.Mdiag[f] / m.h ** 2)
        x[f] -= np.linalg.solve(H, gradE[f])
    return x


def test_static_equilibrium_is_fixed_point():
    m = om.Model(tiny_cantilever(4, 2, 2))
    xs = _static_equilibrium(m)
    assert np.abs(xs - m.X).max() > 1e-6      # it sags
    x1, v1, info = of.pd_step(m, xs, np.zeros(3 * m.N), max_iter=5000, tol=1e-13)
    assert np.linalg.norm(x1 - xs) <= 1e-9 * np.linalg.norm(xs - m.X)


def test_pd_converged_matches_newton_c1():
    m = om.Model(W.config("c1"))
    x0, v0 = m.X.copy(), np.zeros(3 * m.N)
    x1, v1, info = of.pd_step(m, x0, v0, max_iter=5000, tol=1e-14)
    xn, ninfo = of.newton_solve(m, info["y"])
    assert np.linalg.norm(xn - x1) <= 1e-12 * np.linalg.norm(x1)
    assert np.linalg.norm(xn - x1) <= 1e-9 * np.linalg.norm(x1 - x0)


def test_pd_converged_matches_newton_robot():
    sc = tiny_robot()
    m = om.Model(sc)
    act = np.random.default_rng(0).uniform(0, 1, size=m.E)
    x0, v0 = m.X.copy(), np.zeros(3 * m.N)
    v0[0::3] = 0.05
    x1, v1, info = of.pd_step(m, x0, v0, act, max_iter=20000, tol=1e-14)
    xn, ninfo = of.newton_solve(m, info["y"], act)
    assert np.linalg.norm(xn - x1) <= 1e-9 * np.linalg.norm(x1 - x0)
