"""Backward time step: the adjoint system and its solvers (oracle).

Sec. Background (backpropagation with implicit time integration): with
grad g(x) = 0 tying x to y, dL/dy = z^T M / h^2 (eq:chain_rule) where z solves
(A - dA) z = (dL/dx)^T (eq:adjoint, eq:hessian, eq:matrix_split).

* ``adjoint_direct`` -- the plain definition: assemble A - dA and solve it
  (sparse LU; on the largest meshes, CG to round-off, ``linsolve``).
* ``adjoint_fixed_point`` -- Alg. 2: z = 0, then z = A^{-1}(dA z + dL/dx)
  (eq:iteration); convergence iff the spectral radius of A^{-1} dA is below 1
  (eq:sp_radius).  Stopping reading: |dL/dx - (A - dA) z| <= tol |dL/dx|.
* ``adjoint_pcg`` -- the quasi-Newton acceleration (Sec. Differentiable
  Projective Dynamics, further acceleration), read as conjugate gradients on
  the quadratic s(z) with A^{-1} as the fixed inverse-Hessian approximation
  (BFGS with exact line search on a quadratic builds the same iterates).

``backward_step`` then applies the chain rule through
y = x_i + h v_i + h^2 M^{-1} (M g + f_fric(x_i, v_i)) and v_{i+1} = (x_{i+1} - x_i)/h,
and returns the parameter gradients that follow from the implicit-function
theorem, dL/dtheta = -z^T d(grad g)/dtheta (the paper skips their derivation):

* dL/dE_e = -V_q / (1 + nu) * sum_{q in e} <G_q z, F_q - R_q>;
* dL/dr_e = sum_{q in e} w_m <G_m,q z, f_q / |f_q|>.

Pins: the three solvers agree; closed-form adjoint of a centre-of-mass loss on
a free body; a dot-product test against a directional derivative of the
forward map; central finite differences of whole rollouts.
"""
from __future__ import annotations

import numpy as np

from . import linsolve


def _free_blocks(model, x_next, act):
    H = model.hessian(x_next, act)
    f = model.free
    return H[f][:, f].tocsc()


def adjoint_direct(model, x_next, act, xbar_free):
    """Sparse LU of A - dA on free DoFs; beyond the LU size, conjugate
    gradients to round-off (``linsolve``; the residual is in the info)."""
    H = _free_blocks(model, x_next, act)
    z, info = linsolve.solve(H, xbar_free, dense_max=0)
    return z, {"iters": info.get("iters", 0), "method": info["method"], "rel_res": info["rel_res"]}


def adjoint_fixed_point(model, x_next, act, xbar_free, *, tol=1e-12, max_iter=20000):
    f = model.free
    dA = model.delta_A(x_next, act)[f][:, f].tocsr()
    H = (model.A[f][:, f] - dA).tocsr()
    z = np.zeros_like(xbar_free)
    nb = np.linalg.norm(xbar_free)
    k = 0
    rel = 1.0 if nb > 0 else 0.0
    while k < max_iter and rel > tol:
        z = model.solve_A(dA @ z + xbar_free)
        k += 1
        rel = np.linalg.norm(xbar_free - H @ z) / nb
    return z, {"iters": k, "rel": rel}


def adjoint_pcg(model, x_next, act, xbar_free, *, tol=1e-12, max_iter=5000):
    f = model.free
    H = model.hessian(x_next, act)[f][:, f].tocsr()
    z = np.zeros_like(xbar_free)
    r = xbar_free.copy()
    nb = np.linalg.norm(xbar_free)
    if nb == 0:
        return z, {"iters": 0, "rel": 0.0}
    s = model.solve_A(r)
    p = s.copy()
    rs = r @ s
    k = 0
    rel = 1.0
    while k < max_iter:
        q = H @ p
        curv = p @ q
        if curv <= 0:
            raise FloatingPointError("non-positive curvature")
        alpha = rs / curv
        z = z + alpha * p
        r = r - alpha * q
        k += 1
        rel = np.linalg.norm(r) / nb
        if rel <= tol:
            break
        s = model.solve_A(r)
        rs_new = r @ s
        p = s + (rs_new / rs) * p
        rs = rs_new
    return z, {"iters": k, "rel": rel}


SOLVERS = {"direct": adjoint_direct, "fixed_point": adjoint_fixed_point, "pcg": adjoint_pcg}


def backward_step(model, x_i, v_i, act, x_next, gx_next, gv_next, *, solver="direct", **kw):
    """Map (dL/dx_{i+1}, dL/dv_{i+1}) to (dL/dx_i, dL/dv_i, dL/dE, dL/dact)."""
    h = model.h
    f = model.free
    xbar = gx_next + gv_next / h
    z_free, info = SOLVERS[solver](model, x_next, act, xbar[f], **kw)
    z = np.zeros(3 * model.N)
    z[f] = z_free
    dLdy = model.Mdiag * z / h ** 2                       # zero on fixed DoFs
    gx = dLdy - gv_next / h
    gv = h * dLdy
    if model.friction_mu > 0.0:
        w = h ** 2 * dLdy / model.Mdiag                   # dL/df_fric
        fx, fv = model.friction_vjp(x_i, v_i, w)
        gx = gx + fx
        gv = gv + fv
    # parameter gradients
    gE = model.youngs_gradient(x_next, z)
    gact = None
    if model.Gm is not None:
        Gmz = (model.Gm @ z).reshape(model.Q, 3)
        n = model.fiber_directions(x_next, act)
        gact = (model.wm * np.sum(Gmz * n, axis=1)).reshape(model.E, 8).sum(axis=1)
    info["z"] = z
    return gx, gv, gE, gact, info


def spectral_radius(model, x_next, act=None):
    """max |eig(A^{-1} dA)| on free DoFs (dense; small meshes only)."""
    f = model.free
    A = model.A[f][:, f].toarray()
    dA = model.delta_A(x_next, act)[f][:, f].toarray()
    return float(np.max(np.abs(np.linalg.eigvals(np.linalg.solve(A, dA)))))
