"""Global step with a contact set (oracle).

Sec. Contact, complementarity-based contact: with a set C of nodes whose
positions are prescribed (x_C = x*), the global step of Alg. 3 solves the
reduced system A_{C̄×C̄} x_{C̄} = b_{C̄} (the rows and columns of C deleted from
A) and sets x_C = x*; Alg. 4 computes the same x from the factor of A by the
Woodbury identity (eq:woodbury) instead of factorizing the reduced matrix.

* ``reduced_solve`` -- the plain definition: the submatrix of A on the free
  DoFs outside C, factorized by sparse LU.
* ``woodbury_solve`` -- Alg. 4's steps in the paper's order and notation:
  B1 = A^{-1} I_{I×C}, B2 = I_{I×C} - B1 A_{C×C}, B3 = (B1, B2),
  B4 = I - V P^T B3 with V P^T read from A (first the rows of A at C with their
  C×C block removed, then the selector of C), a1 = A^{-1} b,
  a2 = (b^T B2, b^T B1), a3 = B4^{-1} a2^T, x = a1 + B3 a3, x_C = x*.

Both work on the free DoFs: Dirichlet DoFs are not unknowns and their output
entries are 0.  C is a list of free node ids; x* is node-major [3 |C|].
Vectors are node-major 3N like the rest of the oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def _free_positions(model, nodes):
    """Positions of the DoFs of `nodes` (x, y, z of each) among the free DoFs."""
    pos = np.cumsum(model.free) - 1
    dofs = (3 * np.asarray(nodes, dtype=np.int64)[:, None] + np.arange(3)[None, :]).reshape(-1)
    if not np.all(model.free[dofs]):
        raise ValueError("contact nodes must be free")
    return pos[dofs]


def reduced_solve(model, nodes, xstar, b):
    """x with x_C = x* and A_{C̄×C̄} x_{C̄} = b_{C̄} (Sec. Contact, reduced global step)."""
    f = model.free
    cpos = _free_positions(model, nodes)
    keep = np.ones(int(f.sum()), dtype=bool)
    keep[cpos] = False
    xf = np.zeros(int(f.sum()))
    A = model.A_ff.tocsc()
    if keep.any():
        xf[keep] = spla.spsolve(A[keep][:, keep].tocsc(), b[f][keep])
    xf[cpos] = np.asarray(xstar, dtype=np.float64)
    x = np.zeros(3 * model.N)
    x[f] = xf
    return x


def woodbury_solve(model, nodes, xstar, b):
    """Alg. 4: the reduced global step from the factor of A (eq:woodbury)."""
    f = model.free
    cpos = _free_positions(model, nodes)
    n, c = int(f.sum()), len(cpos)
    bf = b[f]
    a1 = model.solve_A(bf)                               # A a1 = b
    xf = a1.copy()
    if c:
        A = model.A_ff.tocsr()
        E = np.zeros((n, c))
        E[cpos, np.arange(c)] = 1.0                      # I_{I×C}
        B1 = np.column_stack([model.solve_A(E[:, k]) for k in range(c)])   # A^{-1} I_{I×C}
        A_CC = A[cpos][:, cpos].toarray()
        B2 = E - B1 @ A_CC
        B3 = np.hstack([B1, B2])                         # A^{-1} P U
        A_IC = A[:, cpos].toarray()
        VPt = np.vstack([(A_IC - E @ A_CC).T, E.T])      # V P^T: (P U_R)^T over (P U_L)^T
        B4 = np.eye(2 * c) - VPt @ B3
        a2 = np.concatenate([bf @ B2, bf @ B1])
        a3 = np.linalg.solve(B4, a2)
        xf = a1 + B3 @ a3
        xf[cpos] = np.asarray(xstar, dtype=np.float64)
    x = np.zeros(3 * model.N)
    x[f] = xf
    return x


# ---------------------------------------------------------------- Alg. 3

RAY, STATIC = 1, 2      # how a node of C got its target (see collision_targets)


def collision_targets(model, x, v, candidates):
    """Collision detection against the ground plane z = 0 (phi(x) = x_z).

    A candidate is in contact when the ray x_j + t v_j, 0 <= t <= h, meets the
    plane (z_j + h v_{j,z} <= 0 with v_{j,z} <= 0, the meeting point at t = 0
    included: a node resting on the plane is in contact); its target x*_j is
    the point where it does (Sec. Contact, remarks on friction: the third
    strategy, a sticky surface), x*_j = x_j + t v_j with t = -z_j / v_{j,z}
    when z_j >= 0 and v_{j,z} < 0 (kind RAY).  Reading: a node on the plane
    that does not move along z, or one already below it, meets it at t = 0,
    x*_j = (x_j, y_j, 0) (kind STATIC).
    Returns {node: (x*_j, kind)}."""
    h = model.h
    out = {}
    for j in np.asarray(candidates, dtype=np.int64):
        z, vz = x[3 * j + 2], v[3 * j + 2]
        if z + h * vz <= 0.0 and vz <= 0.0:
            p = x[3 * j:3 * j + 3].copy()
            if z >= 0.0 and vz < 0.0:
                t = -z / vz
                p[0] += t * v[3 * j]
                p[1] += t * v[3 * j + 1]
                kind = RAY
            else:
                kind = STATIC
            p[2] = 0.0
            out[int(j)] = (p, kind)
    return out


def _reduced_newton(model, y, act, keep, x0, tol_rel=1e-13, max_iter=200):
    """Minimise g over the DoFs in `keep` (the others stay at x0): Newton steps
    with backtracking, the plain PD step -A_keep^{-1} grad g when Newton's is
    not a descent direction or its line search fails (as in forward.newton_solve)."""
    x = x0.copy()
    scale = np.linalg.norm((model.Mdiag * y / model.h ** 2)[keep])
    Ak = model.A.tocsr()[keep][:, keep].tocsc()
    best, stall = np.inf, 0
    for _ in range(max_iter):
        gr = model.grad_g(x, y, act)[keep]
        ng = np.linalg.norm(gr)
        if ng <= tol_rel * scale:
            break
        if ng < 0.5 * best:
            best, stall = ng, 0
        else:
            stall += 1
            if stall >= 3 and ng <= 1e-9 * scale:
                break
        H = model.hessian(x, act).tocsr()[keep][:, keep].tocsc()
        dx = -spla.spsolve(H, gr)
        g0 = model.g(x, y, act)
        directions = [dx, -spla.spsolve(Ak, gr)] if gr @ dx < 0 else [-spla.spsolve(Ak, gr)]
        for d in directions:
            t, found = 1.0, False
            for _ in range(30):
                xt = x.copy()
                xt[keep] += t * d
                if model.g(xt, y, act) <= g0 + 1e-4 * t * (gr @ d):
                    found = True
                    break
                if np.linalg.norm(model.grad_g(xt, y, act)[keep]) < 0.5 * ng:
                    found = True
                    break
                t *= 0.5
            if found:
                break
        x = xt
    return x


def _set_dofs(model, nodes):
    keep = model.free.copy()
    for j in nodes:
        keep[3 * j:3 * j + 3] = False
    return keep


def forward_step_contact(model, x, v, candidates, act=None, *, max_sets=None, tol_rel=1e-13):
    """One implicit-Euler step with complementarity contact (Alg. 3).

    Collision detection gives the set C and targets x*; then, until C stops
    changing: solve the reduced implicit-Euler equations (eq:reduced: grad g is
    0 on the free DoFs outside C, x_C = x*), compute the contact forces
    r = M (x - y) / h^2 - f_int(x) = grad g(x) (eq:tic_1), drop the nodes of C
    whose normal force r_z is negative and add the candidates below the plane
    (eq:lcp).  Reading: an added node's target is its start-of-step position
    moved onto the plane (kind STATIC; the sticky surface holds it where it
    touches).  Reading (termination): a node leaves C at most once per step;
    when it is added back it stays, so that the loop ends (after at most
    2 |candidates| + 1 solves) with no candidate below the plane, at the price
    of a pulling force on such a node.  Without the rule the loop can cycle:
    a node pulled off its ray target penetrates once free and is pulled again
    at its start-of-step target.  The inner solve is Newton to round-off; Alg.
    3's PD iterations converge to the same point.
    Returns (x_next, v_next, info): info["kind"] is 0 / RAY / STATIC per
    candidate, info["C"] the set (ascending node ids), info["sets"] the number
    of reduced solves, info["r"] the final grad g (contact forces on C)."""
    h = model.h
    y = model.y_of(x, v)
    cand = np.asarray(candidates, dtype=np.int64)
    if max_sets is None:
        max_sets = 2 * len(cand) + 1
    targets = collision_targets(model, x, v, cand)
    xs = r = None
    left = set()
    for it in range(max_sets):
        keep = _set_dofs(model, targets)
        x0 = y.copy()
        x0[model.fixed] = model.X[model.fixed]
        for j, (p, _) in targets.items():
            x0[3 * j:3 * j + 3] = p
        xs = _reduced_newton(model, y, act, keep, x0, tol_rel=tol_rel)
        r = model.grad_g(xs, y, act)
        drop = [j for j in targets if r[3 * j + 2] < 0.0 and j not in left]
        add = [int(j) for j in cand if int(j) not in targets and xs[3 * j + 2] < 0.0]
        if not drop and not add:
            break
        for j in drop:
            del targets[j]
            left.add(j)
        for j in add:
            p = x[3 * j:3 * j + 3].copy()
            p[2] = 0.0
            targets[j] = (p, STATIC)
    kind = np.array([targets[int(j)][1] if int(j) in targets else 0 for j in cand], dtype=np.int32)
    return xs, (xs - x) / h, {"C": np.array(sorted(targets), dtype=np.int64), "sets": it + 1,
                              "kind": kind, "r": r}


# ---------------------------------------------------------------- Alg. 5

def target_vjp(model, x, v, candidates, kind, gstar):
    """(dL/dx, dL/dv) through the targets x*_j given dL/dx*_j (node-major 3N,
    read at the nodes of C).  RAY: x*_j = (x + t v_x, y + t v_y, 0) with
    t = -z / v_z; STATIC: x*_j = (x, y, 0)."""
    gx = np.zeros(3 * model.N)
    gv = np.zeros(3 * model.N)
    for j, k in zip(np.asarray(candidates, dtype=np.int64), kind):
        if not k:
            continue
        a, b = gstar[3 * j], gstar[3 * j + 1]
        gx[3 * j] += a
        gx[3 * j + 1] += b
        if k == RAY:
            z, vx, vy, vz = x[3 * j + 2], v[3 * j], v[3 * j + 1], v[3 * j + 2]
            t = -z / vz
            s = vx * a + vy * b
            gv[3 * j] += t * a
            gv[3 * j + 1] += t * b
            gx[3 * j + 2] += -s / vz                      # dt/dz = -1/v_z
            gv[3 * j + 2] += s * z / vz ** 2              # dt/dv_z = z/v_z^2
    return gx, gv


def backward_step_contact(model, x, v, act, x_next, candidates, kind, gx_next, gv_next):
    """Map (dL/dx_{i+1}, dL/dv_{i+1}) to (dL/dx_i, dL/dv_i, dL/dE, dL/dact)
    through a step with contact set C (Alg. 5 and the dependencies it skips).

    z solves (grad^2 g)_{C̄×C̄} z = (dL/dx)_{C̄} (the reduced adjoint system) on
    the free DoFs outside C, here by a direct sparse solve; z = 0 on C.  Then
    dL/dy = M z / h^2 (eq:chain_rule; y_C does not reach x), the targets carry
    dL/dx* = (dL/dx)_C - (grad^2 g z)_C (x_{C̄} depends on x* through the
    coupling block), and y = x_i + h v_i + h^2 g, v_{i+1} = (x_{i+1} - x_i)/h
    finish the chain rule.  Parameter gradients are -z^T d(grad g)/dtheta as
    without contact (x* does not depend on them)."""
    h = model.h
    cand = np.asarray(candidates, dtype=np.int64)
    C = [int(j) for j, k in zip(cand, kind) if k]
    keep = _set_dofs(model, C)
    xbar = gx_next + gv_next / h
    H = model.hessian(x_next, act).tocsr()
    z = np.zeros(3 * model.N)
    if keep.any():
        z[keep] = spla.spsolve(H[keep][:, keep].tocsc(), xbar[keep])
    dLdy = model.Mdiag * z / h ** 2
    gx = dLdy - gv_next / h
    gv = h * dLdy
    if model.friction_mu > 0.0:
        w = h ** 2 * dLdy / model.Mdiag
        fx, fv = model.friction_vjp(x, v, w)
        gx = gx + fx
        gv = gv + fv
    gstar = xbar - H @ z
    tx, tv = target_vjp(model, x, v, cand, kind, gstar)
    gx = gx + tx
    gv = gv + tv
    gE = model.youngs_gradient(x_next, z)
    gact = None
    if model.Gm is not None:
        Gmz = (model.Gm @ z).reshape(model.Q, 3)
        n = model.fiber_directions(x_next, act)
        gact = (model.wm * np.sum(Gmz * n, axis=1)).reshape(model.E, 8).sum(axis=1)
    return gx, gv, gE, gact, {"z": z}
