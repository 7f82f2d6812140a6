"""Deflated adjoint conjugate gradients (dpd_options.deflation): the search
directions kept H-orthogonal to Ritz vectors of A^{-1} dA's largest
eigenvalues, built by Lanczos on the factor's solve and the Hessian product.
The adjoint solution is the same linear system's (against the oracle's direct
adjoint, eq:adjoint), in fewer iterations; rollouts give the same gradients
as without deflation within the solver tolerance."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as oa, forward as of
from parity_helpers import pair, rel, robot_scene, soa, to_dev, elem_dev

pytestmark = pytest.mark.gpu

TIGHT = dict(fwd_solver="newton_pcg", fwd_max_iter=100000, fwd_rel_tol=1e-13, bwd_max_iter=100000,
             bwd_rel_tol=1e-12, check_every=16, fused_cg=0)


def block():
    return W.dropped_block(12, 8, 6, steps=3, drop=0.001)


def robot():
    return robot_scene(steps=3)


SCENES = {"block": block, "robot": robot, "tet_ball": lambda: W.tet_ball(radius=3.0, steps=3)}


def _state(o, seed):
    rng = np.random.default_rng(seed)
    x = o.X + 1e-3 * rng.standard_normal(3 * o.N)
    x[o.fixed] = o.X[o.fixed]
    v = 0.05 * rng.standard_normal(3 * o.N)
    v[o.fixed] = 0.0
    return x, v


@pytest.mark.parametrize("k", [4, 8, 16])
@pytest.mark.parametrize("name", list(SCENES))
def test_deflated_backward_step_matches_direct_adjoint(name, k):
    sc = SCENES[name]()
    g0, o = pair(sc, **TIGHT)
    gd, _ = pair(sc, **TIGHT, deflation=k, deflation_refresh=1)
    assert g0.info["fused_blocks"] == 0
    x, v = _state(o, 1)
    act = None if o.Gm is None else np.random.default_rng(2).uniform(0, 1, o.E)
    a_dev = None if act is None else elem_dev(act)
    xr, _ = of.newton_solve(o, o.y_of(x, v), act)
    rng = np.random.default_rng(3)
    gxn, gvn = rng.standard_normal(3 * o.N), rng.standard_normal(3 * o.N)
    rx, rv, rE, _, _ = oa.backward_step(o, x, v, act, xr, gxn, gvn, solver="direct")
    out = {}
    for tag, g in (("plain", g0), ("deflated", gd)):
        gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
        gx, gv, _, st = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev, to_dev(xr, o.N), to_dev(gxn, o.N),
                                        to_dev(gvn, o.N), g_youngs=gE)
        assert st["converged"] == 1
        out[tag] = (soa(gx), soa(gv), gE.cpu().numpy(), st["bwd_iters"])
        assert rel(out[tag][0], rx) <= 1e-9
        assert rel(out[tag][1], rv) <= 1e-9
        assert rel(out[tag][2], rE) <= 1e-9
    print(name, k, "iterations plain", out["plain"][3], "deflated", out["deflated"][3], flush=True)
    assert out["deflated"][3] < out["plain"][3]
    g0.close()
    gd.close()


def test_deflated_rollout_gradients():
    """A 6-step rollout of the landing block with deflation refreshed every 2
    steps against the same rollout without it (graphs on, as in the bench)."""
    from paper_2101_05917_amd.autograd import rollout
    sc = W.dropped_block(12, 8, 6, steps=6, drop=0.001)
    res = {}
    for tag, extra in (("plain", {}), ("deflated", {"deflation": 8, "deflation_refresh": 2})):
        from paper_2101_05917_amd.mesh import Mesh
        g = Mesh.from_scene(sc, **dict(TIGHT, bwd_rel_tol=1e-11), **extra)
        X = g.rest_positions()
        x = X.clone().requires_grad_(True)
        v = torch.zeros_like(X).requires_grad_(True)
        c = torch.from_numpy(np.ascontiguousarray(W.loss_vector(g.n_nodes, 0).reshape(-1, 3).T)).cuda()
        xT, _ = rollout(g, x, v, sc.steps, None, None, checkpoint_every=1)
        (c * xT).sum().backward()
        res[tag] = (soa(x.grad), soa(v.grad))
        g.close()
    assert rel(res["deflated"][0], res["plain"][0]) <= 1e-9
    assert rel(res["deflated"][1], res["plain"][1]) <= 1e-9
