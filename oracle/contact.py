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
