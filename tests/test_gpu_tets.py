"""Linear tetrahedra on the GPU through the C ABI against the oracle (the
tetrahedral scenes of Sec. Evaluation): rotations, grad g and the Hessian
product per element kind, the global solve with the ordering of the node
graph, converged forward steps (Alg. 1 and Newton), adjoint steps with dL/dE,
rollout gradients through autograd, the mixed path, and the full-size ball
(every entry of grad g, the global-step residual)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as oa, forward as of, projections as op, rollout as orr
from parity_helpers import elem_dev, pair, rel, soa, to_dev

pytestmark = pytest.mark.gpu

TIGHT = dict(fwd_solver="newton_pcg", fwd_max_iter=100000, fwd_rel_tol=1e-13, bwd_max_iter=100000,
             bwd_rel_tol=1e-13, check_every=64)


def beam():
    return W.tet_cantilever(5, 3, 3, jitter=0.15, youngs="loguniform", seed=2, steps=3)


def ball():
    return W.tet_ball(radius=3.0, steps=3)


SCENES = {"beam": beam, "ball": ball}


def _perturbed(o, scale=2e-3, seed=0):
    rng = np.random.default_rng(seed)
    x = o.X + scale * rng.standard_normal(3 * o.N)
    x[o.fixed] = o.X[o.fixed]
    v = 0.05 * rng.standard_normal(3 * o.N)
    v[o.fixed] = 0.0
    return x, v


@pytest.mark.parametrize("name", list(SCENES))
def test_local_quantities_and_solve(name):
    sc = SCENES[name]()
    g, o = pair(sc)
    assert g.info["qp_per_element"] == 1 and g.info["fused_blocks"] == 0
    assert g.n_nodes == o.N and g.n_elements == o.E
    assert np.array_equal(soa(g.rest_positions()), o.X)
    x, v = _perturbed(o, seed=1)
    if len(o.contact_nodes):
        x[3 * o.contact_nodes + 2] -= 1e-3
    R = g.rotations(to_dev(x, o.N)).cpu().numpy().T.reshape(-1, 3, 3)
    Rr = op.closest_rotation(o.deformation_gradients(x))
    assert np.abs(R - Rr).max() <= 1e-12
    y = o.y_of(x, v)
    r = soa(g.gradient(to_dev(x, o.N), to_dev(y, o.N)))
    ref = o.grad_g(x, y)
    ref[o.fixed] = 0.0
    print(name, "grad", rel(r, ref), flush=True)
    assert rel(r, ref) <= 1e-11
    p = np.random.default_rng(2).standard_normal(3 * o.N)
    p[o.fixed] = 0.0
    hp = soa(g.hessian_apply(to_dev(x, o.N), to_dev(p, o.N)))
    ref = o.hessian(x) @ p
    ref[o.fixed] = 0.0
    assert rel(hp, ref) <= 1e-11
    b = np.random.default_rng(3).standard_normal(3 * o.N)
    xs = soa(g.apply_inverse(to_dev(b, o.N)))
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    assert rel(xs, ref) <= 1e-12
    g.close()


@pytest.mark.parametrize("solver", ["pd", "newton_pcg"])
@pytest.mark.parametrize("name", list(SCENES))
def test_forward_and_backward_step(name, solver):
    sc = SCENES[name]()
    g, o = pair(sc, **dict(TIGHT, fwd_solver=solver))
    x, v = _perturbed(o, seed=4)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N))
    print(name, solver, "forward", st, flush=True)
    assert st["converged"] == 1
    xr, _ = of.newton_solve(o, o.y_of(x, v))
    assert np.linalg.norm(soa(xn) - xr) <= 1e-9 * np.linalg.norm(xr - x)
    assert np.linalg.norm(soa(vn) - (xr - x) / o.h) <= 1e-9 * np.linalg.norm((xr - x) / o.h)
    rng = np.random.default_rng(5)
    gxn, gvn = rng.standard_normal(3 * o.N), rng.standard_normal(3 * o.N)
    gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gx, gv, _, bst = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), None, to_dev(xr, o.N), to_dev(gxn, o.N),
                                     to_dev(gvn, o.N), g_youngs=gE)
    assert bst["converged"] == 1
    rx, rv, rE, _, _ = oa.backward_step(o, x, v, None, xr, gxn, gvn, solver="direct")
    assert rel(soa(gx), rx) <= 1e-8
    assert rel(soa(gv), rv) <= 1e-8
    assert rel(gE.cpu().numpy(), rE) <= 1e-8
    g.close()


def test_rollout_gradients_through_autograd():
    from paper_2101_05917_amd.autograd import rollout
    sc = beam()
    g, o = pair(sc, **TIGHT)
    x0, v0 = _perturbed(o, seed=6)
    cx = W.loss_vector(o.N, 0)
    x = to_dev(x0, o.N).requires_grad_(True)
    v = to_dev(v0, o.N).requires_grad_(True)
    E = elem_dev(sc.youngs).requires_grad_(True)
    xT, _ = rollout(g, x, v, sc.steps, None, E, checkpoint_every=2)
    L = (to_dev(cx, o.N) * xT).sum()
    L.backward()
    Lo, ref = orr.loss_and_grad(o, x0, v0, None, cx, newton=True)
    assert abs(L.item() - Lo) <= 1e-12 * abs(Lo)
    assert rel(soa(x.grad), ref["x0"]) <= 1e-8
    assert rel(soa(v.grad), ref["v0"]) <= 1e-8
    assert rel(E.grad.cpu().numpy(), ref["youngs"]) <= 1e-8
    g.close()


def test_mixed_precision():
    sc = ball()
    g, o = pair(sc, precision="mixed", **dict(TIGHT, fwd_rel_tol=1e-12, bwd_rel_tol=1e-12))
    x, v = _perturbed(o, seed=7)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N))
    xr, _ = of.newton_solve(o, o.y_of(x, v))
    err = np.linalg.norm(soa(xn) - xr) / np.linalg.norm(xr - x)
    gxn = np.random.default_rng(8).standard_normal(3 * o.N)
    gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gx, gv, _, _ = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), None, to_dev(xr, o.N), to_dev(gxn, o.N),
                                   to_dev(np.zeros(3 * o.N), o.N), g_youngs=gE)
    rx, rv, rE, _, _ = oa.backward_step(o, x, v, None, xr, gxn, np.zeros(3 * o.N), solver="direct")
    print("mixed", err, rel(soa(gx), rx), rel(gE.cpu().numpy(), rE), flush=True)
    assert err <= 1e-5
    assert rel(soa(gx), rx) <= 1e-6
    assert rel(gE.cpu().numpy(), rE) <= 1e-6
    g.close()


def test_full_size_ball():
    """The 25,344-tetrahedron ball (15,699 DoFs) at its drop state and after a
    few steps: every entry of grad g against the oracle, and the global step's
    residual A x - b from the oracle's assembled A."""
    sc = W.tet_ball()
    g, o = pair(sc, fwd_solver="newton_pcg", fwd_rel_tol=1e-10, fwd_max_iter=100000)
    assert g.info["n_levels"] > 3
    X = g.rest_positions()
    x, v = X.clone(), torch.zeros_like(X)
    for _ in range(6):
        x, v, st = g.forward_step(x, v)
        assert st["converged"] == 1
    xh, vh = soa(x), soa(v)
    y = o.y_of(xh, vh)
    r = soa(g.gradient(x, to_dev(y, o.N)))
    ref = o.grad_g(xh, y)
    ref[o.fixed] = 0.0
    scale = np.abs(o.Mdiag * y / o.h ** 2).max()
    assert np.abs(r - ref).max() <= 1e-12 * scale
    b = np.random.default_rng(9).standard_normal(3 * o.N)
    xs = soa(g.apply_inverse(to_dev(b, o.N)))
    res = o.A_ff @ xs[o.free] - b[o.free]
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b[o.free])
    g.close()
