"""FP64 CPU oracle for the implicit-Euler Projective Dynamics step and its adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
run this package; only the tests, the smoke entry point and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library: it builds its
own mesh numbering, shape functions, operators and matrices, and solves with
scipy's sparse LU.

Everything is written out plainly, with explicit sparse operators in the
3n-dimensional node-major layout the paper uses (x in R^{3n}, Sec. Background):

* discretization -- voxel hex mesh, trilinear shape-function gradients at the
  2x2x2 Gauss points, deformation-gradient operators G, lumped mass.
* projections   -- closest rotation (polar factor via SVD), its derivative,
  muscle-fibre and ground-contact projections.
* model         -- energies, A = M/h^2 + sum w G^T G (eq:pd_global), the
  gradient of g (eq:opt) and its Hessian A - dA (eq:matrix_split).
* forward       -- Alg. 1 (local/global PD) and a Newton solver (eq:newton_update2).
* adjoint       -- eq:adjoint solved directly, by Alg. 2 and by A-preconditioned CG,
  plus the chain rule of eq:chain_rule and parameter gradients.
* contact       -- the global step with a prescribed contact set (Sec. Contact):
  the reduced system solved directly, and by Alg. 4's Woodbury steps.
* rollout       -- multi-step forward/backward and central finite differences.

Parity status of each function is stated in its module header; pins live in
``tests/test_oracle_*.py``.
"""
from . import discretization, projections, linsolve, model, forward, adjoint, contact, rollout  # noqa: F401
