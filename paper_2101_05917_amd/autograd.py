"""torch.autograd wrapper of the PD step and checkpointed rollouts.

Backpropagation through a rollout repeats the single-step adjoint for every
(x, y) pair from the last step back to the first (paper Sec. Background,
backpropagation with implicit time integration).  Each backward call
recomputes the per-Gauss-point rotations at x_{i+1} inside the library, so a
step only has to keep (x_i, v_i, x_{i+1}).  ``checkpoint_every = K > 1``
keeps only every K-th state and recomputes each segment's forward states
during the backward pass.
"""
from __future__ import annotations

from typing import Optional

import torch
from torch.utils.checkpoint import checkpoint

from .mesh import Mesh


class PDStep(torch.autograd.Function):
    """(x_i, v_i, act_i, youngs) -> (x_{i+1}, v_{i+1}) through one PD step."""

    @staticmethod
    def forward(ctx, mesh: Mesh, x, v, act, youngs):
        if youngs is not None:
            # the step runs with these moduli: refactorize A if they changed
            mesh.ensure_youngs(youngs)
        xn, vn, stats = mesh.forward_step(x.contiguous(), v.contiguous(),
                                          None if act is None else act.contiguous())
        ctx.mesh = mesh
        ctx.has_act = act is not None
        ctx.save_for_backward(x, v, act if act is not None else x.new_empty(0), xn)
        ctx.stats = stats
        return xn, vn

    @staticmethod
    def backward(ctx, gxn, gvn):
        mesh = ctx.mesh
        x, v, act, xn = ctx.saved_tensors
        act = act if ctx.has_act else None
        gxn = torch.zeros_like(xn) if gxn is None else gxn.contiguous()
        gvn = torch.zeros_like(xn) if gvn is None else gvn.contiguous()
        g_youngs = None
        if ctx.needs_input_grad[4]:
            g_youngs = torch.zeros(mesh.n_elements, dtype=torch.float64, device=xn.device)
        gx, gv, g_act, _ = mesh.backward_step(x, v, act, xn, gxn, gvn, g_youngs=g_youngs,
                                              want_act=ctx.has_act and ctx.needs_input_grad[3])
        return None, gx, gv, g_act, g_youngs


def pd_step(mesh: Mesh, x, v, act=None, youngs: Optional[torch.Tensor] = None):
    return PDStep.apply(mesh, x, v, act, youngs)


def _segment(mesh, x, v, acts, youngs, t0, t1):
    for t in range(t0, t1):
        a = None if acts is None else acts[t]
        x, v = PDStep.apply(mesh, x, v, a, youngs)
    return x, v


def rollout(mesh: Mesh, x0, v0, steps: int, acts=None, youngs: Optional[torch.Tensor] = None,
            checkpoint_every: int = 1):
    """Run ``steps`` PD steps; differentiable w.r.t. x0, v0, acts and youngs.

    ``youngs`` (float64 [E] on the device, optional) are the per-element
    moduli of the rollout: when they differ from those the mesh was last
    factorized with, the mesh takes them and A is factorized again before the
    first step (the factor is constant within a rollout); dL/dE flows back to
    them.  With checkpoint_every = K > 1 only the
    segment-start states are stored and each segment is recomputed in the
    backward pass.
    """
    x, v = x0, v0
    if checkpoint_every <= 1:
        return _segment(mesh, x, v, acts, youngs, 0, steps)
    t = 0
    while t < steps:
        t1 = min(steps, t + checkpoint_every)
        x, v = checkpoint(_segment, mesh, x, v, acts, youngs, t, t1, use_reentrant=False)
        t = t1
    return x, v
