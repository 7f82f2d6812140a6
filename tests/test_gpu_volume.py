"""The volume-preserving term (supplemental Sec. Energy Definitions) on the
GPU through the C ABI against the oracle: the gradient of g and the Hessian
product (the projection onto det D = 1 and its derivative from eq:vol_kkt),
the global step with the stiffer A, converged forward steps, adjoint steps
and parameter gradients, rollouts through autograd, the mixed path, and a
state with an inverted Gauss point (there D is the closest rotation)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as oa, forward as of, rollout as orr
from parity_helpers import elem_dev, pair, rel, robot_scene, soa, to_dev

pytestmark = pytest.mark.gpu


def cantilever_vol():
    sc = W.cantilever(5, 3, 3, youngs="loguniform", steps=3, seed=4)
    sc.volume_scale = 1.0
    return sc


def robot_vol():
    sc = robot_scene(steps=3)
    sc.volume_scale = 0.5
    return sc


def c2_vol():
    sc = W.config("c2")
    sc.volume_scale = 1.0
    return sc


SCENES = {"cantilever": cantilever_vol, "robot": robot_vol, "c2": c2_vol}
TIGHT = dict(fwd_solver="newton_pcg", fwd_max_iter=100000, fwd_rel_tol=1e-13, bwd_max_iter=100000,
             bwd_rel_tol=1e-13, check_every=64)


def _perturbed(o, scale=2e-3, seed=0):
    rng = np.random.default_rng(seed)
    x = o.X + scale * rng.standard_normal(3 * o.N)
    x[o.fixed] = o.X[o.fixed]
    v = 0.05 * rng.standard_normal(3 * o.N)
    v[o.fixed] = 0.0
    return x, v


def _act(o, seed):
    return None if o.Gm is None else np.random.default_rng(seed).uniform(0, 1, o.E)


@pytest.mark.parametrize("name", list(SCENES))
def test_gradient_hessian_and_solve(name):
    sc = SCENES[name]()
    g, o = pair(sc)
    assert o.wv is not None and g.info["fused_blocks"] == 0
    x, v = _perturbed(o, seed=2)
    y = o.y_of(x, v)
    act = _act(o, 3)
    a_dev = None if act is None else elem_dev(act)
    r = soa(g.gradient(to_dev(x, o.N), to_dev(y, o.N), a_dev))
    ref = o.grad_g(x, y, act)
    ref[o.fixed] = 0.0
    assert rel(r, ref) <= 1e-11
    p = np.random.default_rng(4).standard_normal(3 * o.N)
    p[o.fixed] = 0.0
    hp = soa(g.hessian_apply(to_dev(x, o.N), to_dev(p, o.N), a_dev))
    ref = o.hessian(x, act) @ p
    ref[o.fixed] = 0.0
    print(name, "grad", rel(r, o.grad_g(x, y, act) * ~o.fixed), "hess", rel(hp, ref), flush=True)
    assert rel(hp, ref) <= 1e-11
    b = np.random.default_rng(5).standard_normal(3 * o.N)
    xs = soa(g.apply_inverse(to_dev(b, o.N)))
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    assert rel(xs, ref) <= 1e-12
    g.close()


def test_inverted_gauss_point():
    """One element squashed through itself: its Gauss points have det F < 0,
    where the projection is the closest rotation; gradient and Hessian
    product still match the oracle."""
    sc = cantilever_vol()
    g, o = pair(sc)
    x, v = _perturbed(o, seed=6)
    e = o.E - 1
    nodes = o.mesh.conn[e]
    top = nodes[4:]                       # local nodes with d_z = 1
    for n in top:
        x[3 * n + 2] -= 1.6 * o.dx       # below the bottom face
    F = o.deformation_gradients(x)
    assert np.any(np.linalg.det(F[8 * e:8 * e + 8]) < 0)
    y = o.y_of(x, v)
    r = soa(g.gradient(to_dev(x, o.N), to_dev(y, o.N)))
    ref = o.grad_g(x, y)
    ref[o.fixed] = 0.0
    assert rel(r, ref) <= 1e-11
    p = np.random.default_rng(7).standard_normal(3 * o.N)
    p[o.fixed] = 0.0
    hp = soa(g.hessian_apply(to_dev(x, o.N), to_dev(p, o.N)))
    ref = o.hessian(x) @ p
    ref[o.fixed] = 0.0
    assert rel(hp, ref) <= 1e-10
    g.close()


@pytest.mark.parametrize("name", ["cantilever", "robot"])
def test_forward_and_backward_step(name):
    sc = SCENES[name]()
    g, o = pair(sc, **TIGHT)
    x, v = _perturbed(o, seed=8)
    act = _act(o, 9)
    a_dev = None if act is None else elem_dev(act)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev)
    print(name, "forward", st, flush=True)
    assert st["converged"] == 1
    xr, _ = of.newton_solve(o, o.y_of(x, v), act)
    assert np.linalg.norm(soa(xn) - xr) <= 1e-9 * np.linalg.norm(xr - x)
    rng = np.random.default_rng(10)
    gxn, gvn = rng.standard_normal(3 * o.N), rng.standard_normal(3 * o.N)
    gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gx, gv, ga, bst = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev, to_dev(xr, o.N),
                                      to_dev(gxn, o.N), to_dev(gvn, o.N), g_youngs=gE,
                                      want_act=act is not None)
    print(name, "backward", bst, flush=True)
    assert bst["converged"] == 1
    rx, rv, rE, ra, _ = oa.backward_step(o, x, v, act, xr, gxn, gvn, solver="direct")
    assert rel(soa(gx), rx) <= 1e-8
    assert rel(soa(gv), rv) <= 1e-8
    assert rel(gE.cpu().numpy(), rE) <= 1e-8
    if act is not None:
        assert rel(ga.cpu().numpy(), ra) <= 1e-8
    g.close()


def test_rollout_gradients_through_autograd():
    from paper_2101_05917_amd.autograd import rollout
    sc = cantilever_vol()
    g, o = pair(sc, **TIGHT)
    x0, v0 = _perturbed(o, seed=11)
    cx = W.loss_vector(o.N, 0)
    x = to_dev(x0, o.N).requires_grad_(True)
    v = to_dev(v0, o.N).requires_grad_(True)
    E = elem_dev(sc.youngs).requires_grad_(True)
    xT, _ = rollout(g, x, v, sc.steps, None, E, checkpoint_every=2)
    L = (to_dev(cx, o.N) * xT).sum()
    L.backward()
    Lo, ref = orr.loss_and_grad(o, x0, v0, None, cx, pd_kw={"max_iter": 20000, "tol": 1e-14})
    assert abs(L.item() - Lo) <= 1e-12 * abs(Lo)
    assert rel(soa(x.grad), ref["x0"]) <= 1e-8
    assert rel(soa(v.grad), ref["v0"]) <= 1e-8
    assert rel(E.grad.cpu().numpy(), ref["youngs"]) <= 1e-8
    g.close()


def test_mixed_precision():
    sc = robot_vol()
    g, o = pair(sc, precision="mixed", **dict(TIGHT, fwd_rel_tol=1e-12, bwd_rel_tol=1e-12))
    x, v = _perturbed(o, seed=12)
    act = _act(o, 13)
    a_dev = elem_dev(act)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev)
    xr, _ = of.newton_solve(o, o.y_of(x, v), act)
    err = np.linalg.norm(soa(xn) - xr) / np.linalg.norm(xr - x)
    gxn = np.random.default_rng(14).standard_normal(3 * o.N)
    gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gx, gv, ga, _ = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev, to_dev(xr, o.N), to_dev(gxn, o.N),
                                    to_dev(np.zeros(3 * o.N), o.N), g_youngs=gE)
    rx, rv, rE, _, _ = oa.backward_step(o, x, v, act, xr, gxn, np.zeros(3 * o.N), solver="direct")
    print("mixed", err, rel(soa(gx), rx), rel(gE.cpu().numpy(), rE), flush=True)
    assert err <= 1e-5
    assert rel(soa(gx), rx) <= 1e-6
    assert rel(gE.cpu().numpy(), rE) <= 1e-6
    g.close()
