"""Warm-started adjoint conjugate gradients (dpd_options.bwd_warm_start): the
backward steps of a rollout start from the previous step's adjoint solution,
from the linear or quadratic extrapolation of the previous two or three, or
from the Galerkin (H-norm best) combination of the previous five.  The adjoint system and
its stopping test (relative to the right-hand side) are unchanged, so the
rollout gradients equal the cold-started ones to the solver tolerance, with
fewer iterations; the rollouts' gradients against the oracle at the
benchmark's options are checked in test_gpu_rollouts.py."""
import numpy as np
import pytest
import torch

import bench
import workloads as W
from parity_helpers import rel

pytestmark = pytest.mark.gpu


def _rollout(sc, warm, T, fused, tol=1e-10, checkpoint_every=1):
    from paper_2101_05917_amd.mesh import Mesh
    args = bench.parse(["--config", "c5", "--bwd-warm-start", str(warm)])
    opts = bench.solver_options(args)
    opts.update(bwd_rel_tol=tol, fwd_rel_tol=1e-11, fused_cg=fused)
    g = Mesh.from_scene(sc, **opts)
    X = g.rest_positions()
    N = g.n_nodes
    c = W.loss_vector(N, 0)
    c_dev = torch.from_numpy(np.ascontiguousarray(c.reshape(N, 3).T)).to(X.device)
    out = bench.rollout(g, X, c_dev, T, torch, None, checkpoint_every)
    g.close()
    return out


@pytest.mark.parametrize("warm", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("fused", [0, 1])
def test_warm_start_same_gradients_fewer_iterations(fused, warm):
    """fused = 1: the mesh (1,683 nodes) takes the fused dense solver, which
    solves for the correction from the start; 0: the multi-launch solver."""
    sc = W.dropped_block(16, 10, 8, steps=16, drop=0.002)
    T = 16
    xc, gxc, gvc, gEc, _, _, bic = _rollout(sc, 0, T, fused)
    xw, gxw, gvw, gEw, _, _, biw = _rollout(sc, warm, T, fused)
    print("fused", fused, "warm", warm, "adjoint iterations", bic, "->", biw,
          "dx0", rel(gxw.cpu().numpy(), gxc.cpu().numpy()), "dE", rel(gEw.cpu().numpy(), gEc.cpu().numpy()),
          flush=True)
    assert torch.equal(xw, xc)   # the forward pass is untouched
    assert rel(gxw.cpu().numpy(), gxc.cpu().numpy()) <= 1e-8
    assert rel(gvw.cpu().numpy(), gvc.cpu().numpy()) <= 1e-8
    assert rel(gEw.cpu().numpy(), gEc.cpu().numpy()) <= 1e-8
    assert biw < bic


def test_warm_start_with_checkpoint_segments():
    """Checkpointed rollouts recompute each segment's forward states between
    backward steps; the adjoint history is untouched by them."""
    sc = W.dropped_block(16, 10, 8, steps=16, drop=0.002)
    T = 16
    _, gxc, gvc, gEc, _, _, bic = _rollout(sc, 0, T, 0, checkpoint_every=4)
    _, gxw, gvw, gEw, _, _, biw = _rollout(sc, 4, T, 0, checkpoint_every=4)
    print("checkpoint 4: adjoint iterations", bic, "->", biw, flush=True)
    assert rel(gxw.cpu().numpy(), gxc.cpu().numpy()) <= 1e-8
    assert rel(gvw.cpu().numpy(), gvc.cpu().numpy()) <= 1e-8
    assert rel(gEw.cpu().numpy(), gEc.cpu().numpy()) <= 1e-8
    assert biw < bic
