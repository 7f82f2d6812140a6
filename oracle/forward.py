"""Forward time step: Alg. 1 (local/global PD) and Newton's method (oracle).

``pd_step`` takes the steps of Alg. 1 in the paper's order: y from the
start-of-step state (Sec. Background, eq:time_integration), x = y, then
repeat {local projections; b = M y / h^2 + sum w G^T p; x = A^{-1} b}
(eq:pd_global) with Dirichlet DoFs held at rest and eliminated.  The new
velocity is (x_{i+1} - x_i) / h (eq:implicit_x).

Readings (the paper leaves them open):
* one iteration = one global solve; the residual of x^k is grad g(x^k) =
  A x^k - b(x^k) on free DoFs, formed from the same local pass that builds
  b(x^k); the iterate that passes the test is returned;
* stop when |r^k| <= tol |r^0| or |r^k| <= atol_rel |M y / h^2| (free DoFs),
  or after max_iter solves; ``fixed_iters`` performs exactly max_iter solves;
* x^0 = y with the Dirichlet DoFs set to their rest positions.

``newton_solve`` minimises g (eq:opt) by Newton steps (eq:newton_update2)
with the dense Hessian A - dA and a backtracking line search on g; it is the
cross-check the paper itself uses (Sec. Evaluation, comparisons with other
implicit methods).

Pins: rest state, free fall, centre of mass of every PD iterate of a free
body, static equilibrium, and agreement with Newton on small meshes.
"""
from __future__ import annotations

import numpy as np

from . import linsolve


def _initial_guess(model, y):
    x = y.copy()
    x[model.fixed] = model.X[model.fixed]
    return x


def pd_solve(model, y, act=None, *, max_iter=100, tol=1e-10, atol_rel=1e-12,
             fixed_iters=False, x0=None, history=False):
    """Alg. 1 for a given y.  Returns (x, info)."""
    x = _initial_guess(model, y) if x0 is None else x0.copy()
    free = model.free
    atol = atol_rel * np.linalg.norm((model.Mdiag * y / model.h ** 2)[free])
    hist = []
    r0 = None
    k = 0
    while True:
        b = model.rhs(y, x, act)                                  # local step
        r = (model.A @ x - b)[free]
        nr = float(np.linalg.norm(r))
        if r0 is None:
            r0 = nr
        if history:
            hist.append(x.copy())
        done = k >= max_iter
        if not fixed_iters and (nr <= tol * r0 or nr <= atol):
            done = True
        if done:
            break
        rhs = b[free] - model.A_fc @ x[model.fixed]
        x = x.copy()
        x[free] = model.solve_A(rhs)                              # global step
        k += 1
    info = {"iters": k, "res": nr, "res0": r0, "rel": nr / r0 if r0 > 0 else 0.0}
    if history:
        info["history"] = hist
    return x, info


def pd_step(model, x_i, v_i, act=None, **kw):
    """One implicit-Euler step by Alg. 1.  Returns (x_{i+1}, v_{i+1}, info)."""
    y = model.y_of(x_i, v_i)
    x, info = pd_solve(model, y, act, **kw)
    v = (x - x_i) / model.h
    info["y"] = y
    return x, v, info


def newton_solve(model, y, act=None, *, x0=None, tol_rel=1e-13, max_iter=200):
    """Minimise g(x) for fixed y with Newton steps and backtracking.

    Dense solves up to 1500 free DoFs, sparse LU up to 60 k, conjugate
    gradients to round-off beyond (``linsolve``).  Where the Hessian is
    not positive definite (the muscle energy is not convex) the Newton step
    need not descend; then, and when its line search finds no decrease, the
    step is the plain PD one, -A^{-1} grad g (Alg. 1's update, a descent
    direction since A is SPD), so the iteration stays a descent method on g.

    Stops when |grad g| <= tol_rel |M y / h^2| or, once |grad g| is below
    1e-9 |M y / h^2|, when it has stopped decreasing for three iterations
    (round-off floor reached).
    """
    free = model.free
    x = _initial_guess(model, y) if x0 is None else x0.copy()
    scale = np.linalg.norm((model.Mdiag * y / model.h ** 2)[free])
    its = 0
    best = np.inf
    stall = 0
    for its in range(max_iter):
        gr = model.grad_g(x, y, act)[free]
        ng = np.linalg.norm(gr)
        if ng <= tol_rel * scale:
            break
        if ng < 0.5 * best:
            best, stall = ng, 0
        else:
            stall += 1
            if stall >= 3 and ng <= 1e-9 * scale:
                break
        H = model.hessian(x, act)[free][:, free]
        dx = -linsolve.solve(H, gr)[0]
        g0 = model.g(x, y, act)
        ng0 = np.linalg.norm(gr)
        # the PD step is only formed when the Newton step is not taken
        directions = ([lambda: dx] if gr @ dx < 0 else []) + [lambda: -model.solve_A(gr)]
        for make in directions:
            d = make()
            t = 1.0
            found = False
            for _ in range(30):
                xt = x.copy()
                xt[free] += t * d
                # sufficient decrease of g, or (near round-off, where g no longer
                # resolves the decrease) a smaller gradient
                if model.g(xt, y, act) <= g0 + 1e-4 * t * (gr @ d):
                    found = True
                    break
                if np.linalg.norm(model.grad_g(xt, y, act)[free]) < 0.5 * ng0:
                    found = True
                    break
                t *= 0.5
            if found:
                break
        x = xt
    return x, {"iters": its, "grad": float(np.linalg.norm(model.grad_g(x, y, act)[free]))}
