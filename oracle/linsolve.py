"""Sparse symmetric solves of the oracle (test infrastructure only).

The oracle solves two kinds of systems with the Hessian A - dA of g: Newton's
step (eq:newton_update2) and the adjoint system (eq:adjoint).  Both are plain
linear solves; how they are solved does not change what is computed, only
the rounding.  Three library routines are used, by size:

* up to ``DENSE_MAX`` unknowns: numpy's dense LU;
* up to ``LU_MAX`` unknowns: scipy's sparse LU (SuperLU);
* beyond: scipy's conjugate gradients with a diagonal (Jacobi) preconditioner,
  to a relative residual of ``CG_RTOL``.  The 212 k-unknown block is beyond
  what sparse LU factorizes in reasonable time and memory here (its 3D fill),
  while the symmetric Hessian of the benchmark scenes is positive definite,
  so CG reaches round-off in a few hundred iterations.  The returned solution
  is only as exact as its residual; callers that need it check the residual
  (``info["rel_res"]``).

Pins: every branch agrees with the others on the same system (forced by the
size thresholds in the tests), and the CG branch's residual is checked.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DENSE_MAX = 1500
LU_MAX = 60000
CG_RTOL = 1e-13
CG_MAXITER = 50000


def solve(H, b, *, dense_max=None, lu_max=None, rtol=CG_RTOL):
    """x with H x = b for a sparse symmetric H.  Returns (x, info).  The size
    thresholds default to the module's ``DENSE_MAX`` and ``LU_MAX``."""
    n = H.shape[0]
    dense_max = DENSE_MAX if dense_max is None else dense_max
    lu_max = LU_MAX if lu_max is None else lu_max
    if n <= dense_max:
        return np.linalg.solve(H.toarray(), b), {"method": "dense", "rel_res": None}
    if n <= lu_max:
        return spla.spsolve(sp.csc_matrix(H), b), {"method": "lu", "rel_res": None}
    H = sp.csr_matrix(H)
    d = H.diagonal()
    if np.any(d <= 0):
        raise FloatingPointError("non-positive diagonal: CG needs a positive definite matrix")
    prec = spla.LinearOperator(H.shape, matvec=lambda r: r / d, dtype=np.float64)
    count = [0]

    def cb(_):
        count[0] += 1

    x, code = spla.cg(H, b, rtol=rtol, atol=0.0, maxiter=CG_MAXITER, M=prec, callback=cb)
    nb = np.linalg.norm(b)
    rel = float(np.linalg.norm(H @ x - b) / nb) if nb > 0 else 0.0
    return x, {"method": "cg", "iters": count[0], "rel_res": rel, "code": int(code)}
