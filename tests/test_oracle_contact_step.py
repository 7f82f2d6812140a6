"""Pins of the oracle's time step with complementarity contact (Sec. Contact:
Alg. 3 forward, Alg. 5 and the chain rule through x* backward)."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import contact as oc, forward as of, model as om
from oracle_scenes import landing_block


def _complementarity(m, x, v, xn, cand, info, tol=1e-9, pulled=()):
    """eq:lcp and eq:tic_1 at the result: grad g = 0 off C, x_C on the plane
    with r_N >= 0 there (except the nodes in `pulled`), every other candidate
    above it."""
    r = info["r"]
    C = set(int(j) for j in info["C"])
    keep = m.free.copy()
    for j in C:
        keep[3 * j:3 * j + 3] = False
    scale = np.linalg.norm(m.Mdiag * m.y_of(x, v) / m.h ** 2)
    assert np.linalg.norm(r[keep]) <= tol * scale
    for j in cand:
        j = int(j)
        if j in C:
            assert xn[3 * j + 2] == 0.0
            assert r[3 * j + 2] >= 0.0 or j in pulled
        else:
            assert xn[3 * j + 2] >= 0.0


def test_landing_block_satisfies_the_contact_conditions():
    sc, cand, x, v = landing_block()
    m = om.Model(sc)
    xn, vn, info = oc.forward_step_contact(m, x, v, cand)
    assert len(info["C"]) > 0
    _complementarity(m, x, v, xn, cand, info)
    assert np.allclose(vn, (xn - x) / m.h, rtol=0, atol=1e-15)


def test_ray_targets_lie_on_the_ray_and_the_plane():
    """RAY nodes end where x_j + t v_j meets z = 0; STATIC ones keep x and y."""
    sc, cand, x, v = landing_block()
    m = om.Model(sc)
    xn, _, info = oc.forward_step_contact(m, x, v, cand)
    assert np.any(info["kind"] == oc.RAY)
    for j, k in zip(cand, info["kind"]):
        d, vj = xn[3 * j:3 * j + 3] - x[3 * j:3 * j + 3], v[3 * j:3 * j + 3]
        if k == oc.RAY:
            t = -x[3 * j + 2] / vj[2]
            assert 0.0 <= t <= m.h
            assert np.allclose(d, t * vj, rtol=0, atol=1e-15)
        elif k == oc.STATIC:
            assert d[0] == 0.0 and d[1] == 0.0


def test_a_node_resting_on_the_plane_is_in_contact():
    """The ray of a node at z = 0 that does not move along z meets the plane
    at t = 0: it is detected, with its own position as target; one moving up
    is not, and one above the plane at rest is not."""
    sc, cand, x, v = landing_block(1, 1, 1, lift=0.0)
    m = om.Model(sc)
    x, v = x.copy(), v.copy()
    b = [int(j) for j in cand]
    v[3 * b[0] + 2] = 0.0
    v[3 * b[1] + 2] = 0.01
    x[3 * b[2] + 2] = 1e-3
    v[3 * b[2] + 2] = 0.0
    t = oc.collision_targets(m, x, v, cand)
    assert b[0] in t and t[b[0]][1] == oc.STATIC and np.array_equal(t[b[0]][0], x[3 * b[0]:3 * b[0] + 3])
    assert b[1] not in t and b[2] not in t
    assert b[3] in t and t[b[3]][1] == oc.RAY                 # z = 0, moving down: t = 0
    assert np.array_equal(t[b[3]][0], x[3 * b[3]:3 * b[3] + 3])


def test_no_contact_is_the_plain_implicit_step():
    """High above the plane no candidate is detected or added: the step is
    the implicit-Euler step of Alg. 1 (oracle Newton on g)."""
    sc, cand, x, v = landing_block(lift=0.05)
    m = om.Model(sc)
    xn, _, info = oc.forward_step_contact(m, x, v, cand)
    assert len(info["C"]) == 0 and info["sets"] == 1
    ref = of.newton_solve(m, m.y_of(x, v))
    ref = ref[0] if isinstance(ref, tuple) else ref
    assert np.linalg.norm(xn - ref) <= 1e-12 * np.linalg.norm(ref)


def test_a_node_leaves_the_set_at_most_once():
    """The muscle-driven landing cycles without the rule (node 12: pulled off
    its ray target, below the plane once free, pulled at its start-of-step
    target); with it the loop ends, nothing penetrates and only that node
    pulls."""
    sc, cand, x, v = landing_block(muscles=True)
    m = om.Model(sc)
    act = np.random.default_rng(7).uniform(0.0, 1.0, sc.n_elements)
    xn, _, info = oc.forward_step_contact(m, x, v, cand, act)
    assert info["sets"] < 2 * len(cand) + 1
    r = info["r"]
    pulled = [int(j) for j in info["C"] if r[3 * j + 2] < 0.0]
    assert pulled == [12] and info["kind"][list(cand).index(12)] == oc.STATIC
    _complementarity(m, x, v, xn, cand, info, pulled=pulled)


def test_active_set_equals_the_brute_force_complementarity_solution():
    """Every subset S of the candidates of a one-cell cube: reduce with
    x_S = x*, keep S if eq:lcp holds.  The active-set loop lands on the one
    subset that does."""
    sc, cand, x, v = landing_block(1, 1, 1, lift=-1e-4)
    v = v.copy()
    v[2::3] = np.linspace(-0.05, 0.03, len(v[2::3]))     # some nodes rise
    m = om.Model(sc)
    xn, _, info = oc.forward_step_contact(m, x, v, cand)
    y = m.y_of(x, v)
    valid = []
    for bits in itertools.product((0, 1), repeat=len(cand)):
        S = [int(j) for j, b in zip(cand, bits) if b]
        keep = oc._set_dofs(m, S)
        x0 = y.copy()
        for j in S:
            x0[3 * j:3 * j + 3] = (x[3 * j], x[3 * j + 1], 0.0)
        xs = oc._reduced_newton(m, y, None, keep, x0)
        r = m.grad_g(xs, y, None)
        if all(r[3 * j + 2] >= 0.0 for j in S) and all(xs[3 * j + 2] >= 0.0 for j in cand if int(j) not in S):
            valid.append((S, xs))
    assert len(valid) == 1
    S, xs = valid[0]
    assert sorted(S) == list(info["C"])
    assert np.linalg.norm(xn - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("muscles", [False, True])
def test_contact_backward_matches_central_differences(muscles):
    """dL/dx, dL/dv, dL/dE and dL/dact of L = c . x_{i+1} + d . v_{i+1}
    against central differences of the forward step (the set C does not
    change under the perturbations)."""
    sc, cand, x, v = landing_block(muscles=muscles)
    rng = np.random.default_rng(7)
    m = om.Model(sc)
    act = rng.uniform(0.0, 1.0, sc.n_elements) if muscles else None
    xn, vn, info = oc.forward_step_contact(m, x, v, cand, act)
    cx, cv = rng.standard_normal(3 * m.N), rng.standard_normal(3 * m.N)
    gx, gv, gE, gact, _ = oc.backward_step_contact(m, x, v, act, xn, cand, info["kind"], cx, cv)

    def loss(mm, xx, vv, aa):
        a, b, inf = oc.forward_step_contact(mm, xx, vv, cand, aa)
        assert np.array_equal(inf["kind"], info["kind"])
        return cx @ a + cv @ b

    dx, dv = rng.standard_normal(3 * m.N), rng.standard_normal(3 * m.N)
    ex, ev = 1e-7, 1e-6
    fd = (loss(m, x + ex * dx, v, act) - loss(m, x - ex * dx, v, act)) / (2 * ex)
    assert abs(fd - gx @ dx) <= 1e-5 * abs(gx @ dx)
    fd = (loss(m, x, v + ev * dv, act) - loss(m, x, v - ev * dv, act)) / (2 * ev)
    assert abs(fd - gv @ dv) <= 1e-5 * abs(gv @ dv)
    dE = rng.standard_normal(sc.n_elements)
    eE = 1e-4 * sc.youngs[0]

    def with_youngs(Y):
        s2 = landing_block(muscles=muscles)[0]
        s2.youngs = Y
        return om.Model(s2)
    fd = (loss(with_youngs(sc.youngs + eE * dE), x, v, act)
          - loss(with_youngs(sc.youngs - eE * dE), x, v, act)) / (2 * eE)
    assert abs(fd - gE @ dE) <= 1e-4 * abs(gE @ dE)
    if muscles:
        da = rng.standard_normal(sc.n_elements)
        ea = 1e-5
        fd = (loss(m, x, v, act + ea * da) - loss(m, x, v, act - ea * da)) / (2 * ea)
        assert abs(fd - gact @ da) <= 1e-4 * abs(gact @ da)


def test_contact_backward_without_contact_is_the_plain_adjoint():
    from oracle import adjoint as adj
    sc, cand, x, v = landing_block(lift=0.05)
    m = om.Model(sc)
    xn, _, info = oc.forward_step_contact(m, x, v, cand)
    rng = np.random.default_rng(8)
    cx, cv = rng.standard_normal(3 * m.N), rng.standard_normal(3 * m.N)
    a = oc.backward_step_contact(m, x, v, None, xn, cand, info["kind"], cx, cv)
    b = adj.backward_step(m, x, v, None, xn, cx, cv)
    for p, q in zip(a[:3], b[:3]):
        assert np.linalg.norm(p - q) <= 1e-12 * np.linalg.norm(q)


def test_sphere_scene_matches_the_paper_sizes():
    """Rolling sphere (Sec. Evaluation): 552 elements, 2469 DoFs, 72 candidate
    contact nodes, h = 5 ms, 100 frames."""
    sc = W.config("sphere")
    assert sc.n_elements == 552
    assert 3 * len(W.present_nodes(sc.cells)) == 2469
    assert len(W.candidate_nodes(sc)) == 72
    assert sc.h == 5e-3 and sc.steps == 100 and sc.contact_k == 0.0
