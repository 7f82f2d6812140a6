"""Pins of the oracle's global step with a contact set (Sec. Contact, Alg. 4)."""
import numpy as np
import pytest

import workloads as W
from oracle import contact as oc, model as om
from parity_helpers import robot_scene


def _model(name):
    return om.Model(robot_scene() if name == "robot" else W.config(name))


def _unconstrained(m, nodes):
    mask = m.free.copy()
    mask[(3 * np.asarray(nodes)[:, None] + np.arange(3)).reshape(-1)] = False
    return mask


@pytest.mark.parametrize("name", ["c1", "robot"])
@pytest.mark.parametrize("c", [0, 1, 5, 20])
def test_woodbury_steps_equal_reduced_solve(name, c):
    """Alg. 4 (Woodbury identity on the factor of A) and a direct LU of the
    reduced matrix give the same x."""
    m = _model(name)
    rng = np.random.default_rng(10 + c)
    nodes = rng.choice(np.nonzero(m.free[0::3])[0], c, replace=False)
    xs = rng.standard_normal(3 * c)
    b = rng.standard_normal(3 * m.N)
    x1 = oc.reduced_solve(m, nodes, xs, b)
    x2 = oc.woodbury_solve(m, nodes, xs, b)
    k = _unconstrained(m, nodes)
    assert np.linalg.norm((x1 - x2)[k]) <= 1e-12 * np.linalg.norm(x1[k])
    cd = (3 * nodes[:, None] + np.arange(3)).reshape(-1)
    assert np.array_equal(x1[cd], xs) and np.array_equal(x2[cd], xs)
    assert np.all(x1[m.fixed] == 0.0) and np.all(x2[m.fixed] == 0.0)


def test_empty_set_is_the_plain_global_step():
    m = _model("c1")
    b = np.random.default_rng(3).standard_normal(3 * m.N)
    x = oc.reduced_solve(m, np.zeros(0, np.int64), np.zeros(0), b)
    assert np.allclose(x[m.free], m.solve_A(b[m.free]), rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("name", ["c1", "robot"])
def test_prescribing_the_free_solution_returns_it(name):
    """x = A^{-1} b restricted to C, with the coupling A_{C̄×C} x_C moved into the
    right-hand side (as Alg. 3 forms b), leaves the solution unchanged."""
    m = _model(name)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(3 * m.N)
    x = np.zeros(3 * m.N)
    x[m.free] = m.solve_A(b[m.free])
    nodes = rng.choice(np.nonzero(m.free[0::3])[0], 9, replace=False)
    cd = (3 * nodes[:, None] + np.arange(3)).reshape(-1)
    xc = np.zeros(3 * m.N)
    xc[cd] = x[cd]
    b2 = b - m.A @ xc
    for solve in (oc.reduced_solve, oc.woodbury_solve):
        y = solve(m, nodes, x[cd], b2)
        assert np.linalg.norm(y - x) <= 1e-11 * np.linalg.norm(x)


def test_contact_nodes_must_be_free():
    m = _model("c1")
    fixed_node = int(np.nonzero(m.fixed[0::3])[0][0])
    with pytest.raises(ValueError):
        oc.reduced_solve(m, np.array([fixed_node]), np.zeros(3), np.zeros(3 * m.N))
