"""Whole rollouts of the benchmark workloads on the GPU against the oracle's
stored references (tests/golden/*_rollout_reference.npz, written by
make_rollout_reference.py from the oracle alone: Newton to round-off forward,
the adjoint system solved directly), and central finite differences of the
cantilever's loss in log E.

Bars: gradients within 1e-6 relative of the oracle's at the solver options
bench.py times; at tight tolerances positions within 1e-9
(displacement-relative) and gradients within 1e-8; the mixed path's
positions within 1e-5.
"""
import os

import numpy as np
import pytest
import torch

import bench
import workloads as W
from parity_helpers import rel, soa, elem_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TIGHT = dict(fwd_solver="newton_pcg", fwd_rel_tol=1e-13, fwd_max_iter=200000, bwd_rel_tol=1e-13,
             bwd_max_iter=200000, check_every=32)


def _reference(config):
    return np.load(os.path.join(GOLDEN, f"{config}_rollout_reference.npz"))


def _run(config, options, steps=None):
    """bench.py's rollout of a workload with the given mesh options.
    Returns (scene, x_T, gx, gv, gE, g_act) as node-major numpy arrays."""
    from paper_2101_05917_amd.mesh import Mesh
    sc = W.config(config)
    T = steps or sc.steps
    mesh = Mesh.from_scene(sc, **options)
    X = mesh.rest_positions()
    N = mesh.n_nodes
    c = W.loss_vector(N, sc.loss_seed)
    c_dev = torch.from_numpy(np.ascontiguousarray(c.reshape(N, 3).T)).to(X.device)
    acts = None
    if sc.muscle_k > 0:
        acts = elem_dev(W.actuation_sequence(T, mesh.n_elements, seed=sc.act_seed))
    K = 20 if config == "c3" else 1
    xT, gx, gv, gE, g_act, fi, bi = bench.rollout(mesh, X, c_dev, T, torch, acts, K)
    print(config, "forward iterations per step", fi / T, "adjoint", bi / T, flush=True)
    out = (sc, soa(xT), soa(gx), soa(gv), gE.cpu().numpy(), None if g_act is None else g_act.cpu().numpy())
    mesh.close()
    return out


def _errors(ref, X, xT, gx, gv, gE, g_act):
    e = {"x_T": float(np.linalg.norm(xT - ref["x_T"]) / np.linalg.norm(ref["x_T"] - X)),
         "g_x0": rel(gx, ref["g_x0"]), "g_v0": rel(gv, ref["g_v0"]), "g_youngs": rel(gE, ref["g_youngs"])}
    if g_act is not None:
        e["g_act"] = rel(g_act, ref["g_act"])
    print("errors vs oracle", e, flush=True)
    return e


def _rest(sc):
    if getattr(sc, "tets", None) is not None:
        return np.asarray(sc.X, dtype=np.float64).reshape(-1)
    from oracle import discretization as od
    return od.VoxelMesh(sc.cells, sc.dx, sc.origin).X.reshape(-1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_rollout_at_bench_options(precision):
    """The 16x8x8 cantilever's 100-step rollout with bench.py's options."""
    args = bench.parse(["--config", "c2", "--precision", precision])
    sc, xT, gx, gv, gE, ga = _run("c2", bench.solver_options(args))
    ref = _reference("c2")
    assert int(ref["steps"]) == sc.steps
    e = _errors(ref, _rest(sc), xT, gx, gv, gE, ga)
    assert e["x_T"] <= 1e-5
    for k in ("g_x0", "g_v0", "g_youngs"):
        assert e[k] <= 1e-6, (k, e[k])


def test_c2_rollout_tight():
    """The same rollout solved to round-off: positions within 1e-9 of the
    oracle's, gradients within 1e-8."""
    sc, xT, gx, gv, gE, ga = _run("c2", TIGHT)
    e = _errors(_reference("c2"), _rest(sc), xT, gx, gv, gE, ga)
    assert e["x_T"] <= 1e-9
    for k in ("g_x0", "g_v0", "g_youngs"):
        assert e[k] <= 1e-8, (k, e[k])


def test_c3_rollout_at_bench_options():
    """The legged body's 200-step rollout (ground contact, friction, muscles)
    with bench.py's options and a checkpoint every 20 steps."""
    args = bench.parse(["--config", "c3"])
    sc, xT, gx, gv, gE, ga = _run("c3", bench.solver_options(args))
    ref = _reference("c3")
    assert int(ref["steps"]) == sc.steps
    e = _errors(ref, _rest(sc), xT, gx, gv, gE, ga)
    assert e["x_T"] <= 1e-6
    for k in ("g_x0", "g_v0", "g_youngs", "g_act"):
        assert e[k] <= 1e-6, (k, e[k])


def test_c2_finite_differences_in_log_youngs():
    """Central differences (eps 1e-6) of the GPU's own 100-step loss in log E
    on 16 random elements (seed 1) and along one random direction, against
    the GPU adjoint's dL/dlog E = E dL/dE, all states solved to round-off."""
    from paper_2101_05917_amd.mesh import Mesh
    sc = W.config("c2")
    mesh = Mesh.from_scene(sc, **TIGHT)
    X = mesh.rest_positions()
    N = mesh.n_nodes
    c = W.loss_vector(N, sc.loss_seed)
    c_dev = torch.from_numpy(np.ascontiguousarray(c.reshape(N, 3).T)).to(X.device)
    _, _, _, gE, _, _, _ = bench.rollout(mesh, X, c_dev, sc.steps, torch)
    glog = gE.cpu().numpy() * sc.youngs
    E0 = sc.youngs.copy()

    def loss(E):
        mesh.set_youngs(E)
        x, v = X.clone(), torch.zeros_like(X)
        for _ in range(sc.steps):
            x, v, _ = mesh.forward_step(x, v)
        return float((c_dev * x).sum())

    eps = 1e-6
    rng = np.random.default_rng(1)
    elems = rng.choice(len(E0), 16, replace=False)
    d = rng.standard_normal(len(E0))
    d /= np.linalg.norm(d)
    scale = np.abs(glog).max()
    worst = 0.0
    for e in elems:
        u = np.zeros(len(E0))
        u[e] = 1.0
        fd = (loss(E0 * np.exp(eps * u)) - loss(E0 * np.exp(-eps * u))) / (2 * eps)
        worst = max(worst, abs(fd - glog[e]) / scale)
    fd = (loss(E0 * np.exp(eps * d)) - loss(E0 * np.exp(-eps * d))) / (2 * eps)
    an = glog @ d
    mesh.close()
    # a unit direction's derivative is of order |dL/dlog E| / sqrt(E): its
    # error is measured against the gradient's norm
    print("largest element error / max |dL/dlog E|", worst, "direction", fd, an,
          "error / |dL/dlog E|", abs(fd - an) / np.linalg.norm(glog), flush=True)
    assert worst <= 1e-5
    assert abs(fd - an) <= 1e-5 * np.linalg.norm(glog)


def test_c5_prefix_rollout_at_bench_options():
    """The 64x32x32 block's first 30 steps (free fall, landing on the penalty
    ground, compression) with bench.py's options, against the oracle's
    reference of that prefix: gradients within 1e-6."""
    args = bench.parse(["--config", "c5"])
    ref = _reference("c5")
    T = int(ref["steps"])
    sc, xT, gx, gv, gE, ga = _run("c5", bench.solver_options(args), steps=T)
    e = _errors(ref, _rest(sc), xT, gx, gv, gE, ga)
    assert e["x_T"] <= 1e-6
    for k in ("g_x0", "g_v0", "g_youngs"):
        assert e[k] <= 1e-6, (k, e[k])


def test_tet_ball_prefix_rollout_at_bench_options():
    """The tetrahedral ball's first 30 steps (free fall, landing on the
    penalty ground with friction, bounce) with bench.py's options, against the
    oracle's reference of that prefix: gradients within 1e-6."""
    args = bench.parse(["--config", "tet"])
    ref = _reference("tet")
    T = int(ref["steps"])
    sc, xT, gx, gv, gE, ga = _run("tet", bench.solver_options(args), steps=T)
    e = _errors(ref, _rest(sc), xT, gx, gv, gE, ga)
    assert e["x_T"] <= 1e-8
    for k in ("g_x0", "g_v0", "g_youngs"):
        assert e[k] <= 1e-6, (k, e[k])
