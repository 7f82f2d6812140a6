"""Adjoint solvers of the oracle against each other, closed forms and the forward map."""
import numpy as np

from oracle import model as om, forward as of, adjoint as oa
from oracle_scenes import tiny_free, tiny_cantilever, tiny_robot, perturbed_state
import workloads as W


def _after_one_step(sc, act=None, seed=0):
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, seed=seed)
    x1, v1, info = of.pd_step(m, x0, v0, act, max_iter=20000, tol=1e-14)
    return m, x0, v0, x1, info


def test_three_solvers_agree():
    rob = tiny_robot()
    for sc, act in ((W.config("c1"), None),
                    (rob, np.random.default_rng(1).uniform(0, 1, rob.n_elements))):
        m, x0, v0, x1, _ = _after_one_step(sc, act)
        rhs = np.random.default_rng(2).standard_normal(m.free.sum())
        z1, _ = oa.adjoint_direct(m, x1, act, rhs)
        z2, i2 = oa.adjoint_fixed_point(m, x1, act, rhs, tol=1e-13)
        z3, i3 = oa.adjoint_pcg(m, x1, act, rhs, tol=1e-13)
        n = np.linalg.norm(z1)
        assert np.linalg.norm(z2 - z1) <= 1e-11 * n
        assert np.linalg.norm(z3 - z1) <= 1e-11 * n
        assert i3["iters"] < i2["iters"]


def test_centre_of_mass_loss_closed_form():
    sc = tiny_free(3, 2, 2)
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, scale=3e-3)
    x1, _ = of.newton_solve(m, m.y_of(x0, v0))
    t = np.array([0.3, -1.2, 0.7])
    Mtot = m.m.sum()
    dLdx = (m.Mdiag * np.tile(t, m.N)) / Mtot          # L = t . COM(x)
    z_expect = np.tile(m.h ** 2 * t / Mtot, m.N)
    z, _ = oa.adjoint_direct(m, x1, None, dLdx)
    assert np.abs(z - z_expect).max() <= 1e-12 * np.abs(z_expect).max()
    z2, info = oa.adjoint_fixed_point(m, x1, None, dLdx, tol=1e-12)
    assert info["iters"] == 1


def test_dot_product_against_forward_directional_derivative():
    sc = tiny_cantilever(3, 2, 2, youngs=10 ** np.linspace(5, 6.5, 12))
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, seed=4)
    y = m.y_of(x0, v0)
    x1, _ = of.newton_solve(m, y)
    rng = np.random.default_rng(5)
    gbar = rng.standard_normal(3 * m.N)
    dy = rng.standard_normal(3 * m.N) * 1e-3
    eps = 1e-4
    xp, _ = of.newton_solve(m, y + eps * dy, x0=x1)
    xm, _ = of.newton_solve(m, y - eps * dy, x0=x1)
    jvp = (xp - xm) / (2 * eps)
    z, _ = oa.adjoint_direct(m, x1, None, gbar[m.free])
    zf = np.zeros(3 * m.N)
    zf[m.free] = z
    dLdy = m.Mdiag * zf / m.h ** 2
    assert abs(gbar @ jvp - dLdy @ dy) <= 1e-7 * abs(gbar @ jvp)


def test_spectral_radius_and_fixed_point_rate():
    m = om.Model(W.config("c1"))
    x1, v1, _ = of.pd_step(m, m.X, np.zeros(3 * m.N), max_iter=5000, tol=1e-14)
    rho = oa.spectral_radius(m, x1)
    assert 0.0 < rho < 1.0
    rhs = np.random.default_rng(6).standard_normal(m.free.sum())
    z, info = oa.adjoint_fixed_point(m, x1, None, rhs, tol=1e-8)
    # iterations needed for a 1e-8 reduction are of the order log(1e-8)/log(rho)
    assert info["iters"] <= 3 * np.log(1e-8) / np.log(rho) + 10
