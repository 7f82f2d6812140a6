"""The oracle's linear solves: dense LU, sparse LU and conjugate gradients agree
on the same Hessian systems, and the Newton and adjoint solutions do not
depend on which of them is used."""
import numpy as np

import workloads as W
from oracle import adjoint as oa, forward as of, linsolve, model as om
from oracle_scenes import perturbed_state


def _deformed(scene, seed=0):
    m = om.Model(scene)
    x0, v0 = perturbed_state(m, seed=seed)
    x1, _ = of.newton_solve(m, m.y_of(x0, v0))
    return m, x0, v0, x1


def test_three_branches_agree_on_a_hessian_system():
    sc = W.cantilever(6, 3, 3, youngs="loguniform", seed=4)
    m, _, _, x1 = _deformed(sc)
    H = m.hessian(x1)[m.free][:, m.free]
    b = np.random.default_rng(1).standard_normal(H.shape[0])
    zd, i0 = linsolve.solve(H, b)
    zl, i1 = linsolve.solve(H, b, dense_max=0)
    zc, i2 = linsolve.solve(H, b, dense_max=0, lu_max=0)
    assert (i0["method"], i1["method"], i2["method"]) == ("dense", "lu", "cg")
    assert i2["rel_res"] <= 2e-13          # the recursive residual meets 1e-13
    n = np.linalg.norm(zd)
    assert np.linalg.norm(zl - zd) <= 1e-12 * n
    assert np.linalg.norm(zc - zd) <= 1e-10 * n
    # the residual reported is the true one
    assert abs(np.linalg.norm(H @ zc - b) / np.linalg.norm(b) - i2["rel_res"]) <= 1e-15


def test_newton_and_adjoint_independent_of_the_solver(monkeypatch):
    sc = W.cantilever(6, 3, 3, youngs="loguniform", seed=4)
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, seed=2)
    y = m.y_of(x0, v0)
    xa, _ = of.newton_solve(m, y)
    rhs = np.random.default_rng(3).standard_normal(m.free.sum())
    za, _ = oa.adjoint_direct(m, xa, None, rhs)
    monkeypatch.setattr(linsolve, "DENSE_MAX", 0)
    monkeypatch.setattr(linsolve, "LU_MAX", 0)
    xb, info = of.newton_solve(m, y)
    zb, zi = oa.adjoint_direct(m, xa, None, rhs)
    assert zi["method"] == "cg" and zi["rel_res"] <= 2e-13
    assert np.linalg.norm(xb - xa) <= 1e-10 * np.linalg.norm(xa - x0)
    assert np.linalg.norm(zb - za) <= 1e-10 * np.linalg.norm(za)
    # A^{-1} by CG (the PD step of Newton's safeguard) equals the factor's solve
    r = np.random.default_rng(5).standard_normal(m.free.sum())
    s_lu = m.solve_A(r)
    s_cg = linsolve.solve(m.A_ff, r, dense_max=0, lu_max=0)[0]
    assert np.linalg.norm(s_cg - s_lu) <= 1e-10 * np.linalg.norm(s_lu)
