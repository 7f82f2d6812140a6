"""Whole-rollout gradients of the oracle against central finite differences."""
import numpy as np

from oracle import model as om, rollout as orr
from oracle_scenes import tiny_cantilever, tiny_robot, perturbed_state
import workloads as W

PD = {"max_iter": 20000, "tol": 1e-14}


def test_gradients_initial_state_and_youngs():
    E0 = 10 ** np.linspace(5, 7, 12)
    sc = tiny_cantilever(3, 2, 2, youngs=E0)
    sc.steps = 3
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, seed=8)
    cx = W.loss_vector(m.N, 0)
    L, g = orr.loss_and_grad(m, x0, v0, None, cx, pd_kw=PD)
    rng = np.random.default_rng(9)
    d = rng.standard_normal(3 * m.N)
    d[m.fixed] = 0.0
    for key, eps in (("x0", 1e-6), ("v0", 1e-4)):
        def f(t, key=key):
            xx = x0 + (t * d if key == "x0" else 0)
            vv = v0 + (t * d if key == "v0" else 0)
            return orr.rollout_loss(sc, xx, vv, None, cx, pd_kw=PD)
        fd = orr.central_difference(f, 0.0, 1.0, eps)
        assert abs(fd - g[key] @ d) <= 2e-5 * abs(fd)
    for e in (0, 7):
        dlog = np.zeros(m.E)
        dlog[e] = 1.0
        f = lambda t: orr.rollout_loss(sc, x0, v0, None, cx, youngs=E0 * np.exp(t * dlog), pd_kw=PD)
        fd = orr.central_difference(f, 0.0, 1.0, 1e-5)
        an = g["youngs"][e] * E0[e]
        assert abs(fd - an) <= 2e-4 * abs(an) + 1e-9 * np.abs(g["youngs"] * E0).max()


def test_gradients_actuation_friction_contact():
    sc = tiny_robot(steps=3)
    m = om.Model(sc)
    acts = W.actuation_sequence(3, m.E, seed=0)
    x0 = m.X.copy()
    v0 = np.zeros(3 * m.N)
    v0[0::3] = 0.1
    v0[1::3] = -0.05
    cx = W.loss_vector(m.N, 1)
    L, g = orr.loss_and_grad(m, x0, v0, acts, cx, pd_kw=PD)
    rng = np.random.default_rng(10)
    d = rng.standard_normal(acts.shape)
    f = lambda t: orr.rollout_loss(sc, x0, v0, acts + t * d, cx, pd_kw=PD)
    fd = orr.central_difference(f, 0.0, 1.0, 1e-5)
    assert abs(fd - np.sum(g["act"] * d)) <= 1e-4 * abs(fd)
    dv = rng.standard_normal(3 * m.N)
    f = lambda t: orr.rollout_loss(sc, x0, v0 + t * dv, acts, cx, pd_kw=PD)
    fd = orr.central_difference(f, 0.0, 1.0, 1e-5)
    assert abs(fd - g["v0"] @ dv) <= 1e-4 * abs(fd)
    dx = rng.standard_normal(3 * m.N)
    f = lambda t: orr.rollout_loss(sc, x0 + t * dx, v0, acts, cx, pd_kw=PD)
    fd = orr.central_difference(f, 0.0, 1.0, 1e-6)
    assert abs(fd - g["x0"] @ dx) <= 1e-4 * abs(fd)
