"""Multi-step rollouts, their gradients and finite differences (oracle).

Backpropagation through a rollout repeats the single-step adjoint for every
pair (x, y) from the last step to the first (Sec. Background, backpropagation
with implicit time integration).  The loss read here is
L = c_x . x_T + c_v . v_T with fixed weight vectors (the paper's random
weighted sum of final positions and velocities, Sec. Evaluation).

Gradients are returned for the initial state (x_0, v_0), the per-element
Young's moduli (summed over steps) and the per-step actuation.
"""
from __future__ import annotations

import numpy as np

from .forward import pd_step, newton_solve
from .adjoint import backward_step
from .model import Model


def initial_state(model):
    return model.X.copy(), np.zeros(3 * model.N)


def forward_rollout(model, x0, v0, acts=None, steps=None, newton=False, **pd_kw):
    """T steps by Alg. 1 (pd_kw: its iteration options), or with newton=True
    by Newton's method on g to round-off (the same implicit-Euler states)."""
    T = model.scene.steps if steps is None else steps
    xs, vs, infos = [x0], [v0], []
    for t in range(T):
        a = None if acts is None else acts[t]
        if newton:
            x, info = newton_solve(model, model.y_of(xs[-1], vs[-1]), a)
            v = (x - xs[-1]) / model.h
        else:
            x, v, info = pd_step(model, xs[-1], vs[-1], a, **pd_kw)
        xs.append(x)
        vs.append(v)
        infos.append(info)
    return xs, vs, infos


def loss_and_grad(model, x0, v0, acts, cx, cv=None, steps=None, *, solver="direct",
                  pd_kw=None, adj_kw=None, newton=False):
    pd_kw = pd_kw or {}
    adj_kw = adj_kw or {}
    xs, vs, finfo = forward_rollout(model, x0, v0, acts, steps, newton=newton, **pd_kw)
    T = len(xs) - 1
    cv = np.zeros_like(cx) if cv is None else cv
    L = float(cx @ xs[-1] + cv @ vs[-1])
    gx, gv = cx.copy(), cv.copy()
    gE = np.zeros(model.E)
    gact = None if acts is None else np.zeros((T, model.E))
    binfo = []
    for t in range(T - 1, -1, -1):
        a = None if acts is None else acts[t]
        gx, gv, ge, ga, info = backward_step(model, xs[t], vs[t], a, xs[t + 1], gx, gv,
                                             solver=solver, **adj_kw)
        gE += ge
        if gact is not None and ga is not None:
            gact[t] = ga
        binfo.append(info)
    return L, {"x0": gx, "v0": gv, "youngs": gE, "act": gact,
               "xs": xs, "vs": vs, "fwd_info": finfo, "bwd_info": binfo}


def rollout_loss(scene, x0, v0, acts, cx, cv=None, youngs=None, steps=None, pd_kw=None, newton=False):
    """Loss only, building a fresh model (for finite differences in E)."""
    model = Model(scene, youngs=youngs)
    xs, vs, _ = forward_rollout(model, x0, v0, acts, steps, newton=newton, **(pd_kw or {}))
    cv = np.zeros_like(cx) if cv is None else cv
    return float(cx @ xs[-1] + cv @ vs[-1])


def central_difference(fun, theta, direction, eps):
    """(f(theta + eps d) - f(theta - eps d)) / (2 eps)."""
    return (fun(theta + eps * direction) - fun(theta - eps * direction)) / (2.0 * eps)
