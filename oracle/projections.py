"""Local-step projections and their derivatives (oracle; test infrastructure only).

* Corotated term: the projection of F onto SO(3) is the rotation closest to F,
  obtained from the polar decomposition (supplemental Sec. Energy Definitions,
  background elasticity).  Reading: F = U diag(s) V^T with s descending and
  R = U diag(1, 1, det(U V^T)) V^T, which is the closest proper rotation also
  when det F <= 0.
* Its derivative, which the paper defers to prior work: differentiate F = R S
  with S = R^T F symmetric.  With dR = R [w]_x one gets
  (tr(S) I - S) w = axial(R^T dF - dF^T R).
* Muscle fibre (supplemental, muscle fibers): F m is projected onto the sphere
  of radius r; derivative (r/|f|)(I - n n^T).  Reading of the garbled printed
  energy: E = (w/2)(|F m| - r)^2, i.e. the distance to that sphere.
* Penalty ground (Sec. Penalty-Based Contact): a node is projected onto the
  half-space of non-negative height, p = (x1, x2, max(x3, 0)); derivative
  diag(1, 1, [x3 >= 0]) (height exactly 0 counts as not in contact).

Pins: scipy.linalg.polar, R(QF) = Q R(F), SPD F gives R = I, the F = I closed
form dR[dF] = skew(dF), symmetry of dR/dF, central differences of the SVD
projection.
"""
from __future__ import annotations

import numpy as np


def closest_rotation(F: np.ndarray) -> np.ndarray:
    """R[..., 3, 3] = argmin over SO(3) of |F - R|_F, via numpy's SVD."""
    U, s, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U @ Vt))
    d = np.where(d == 0, 1.0, d)
    D = np.zeros(F.shape)
    D[..., 0, 0] = 1.0
    D[..., 1, 1] = 1.0
    D[..., 2, 2] = d
    return U @ D @ Vt


def axial(K: np.ndarray) -> np.ndarray:
    """Vector k with [k]_x = skew part convention: k = (K21, K02, K10)."""
    return np.stack([K[..., 2, 1], K[..., 0, 2], K[..., 1, 0]], axis=-1)


def cross_matrix(w: np.ndarray) -> np.ndarray:
    """[w]_x so that [w]_x v = w x v."""
    Z = np.zeros(w.shape[:-1] + (3, 3))
    Z[..., 0, 1] = -w[..., 2]
    Z[..., 0, 2] = w[..., 1]
    Z[..., 1, 0] = w[..., 2]
    Z[..., 1, 2] = -w[..., 0]
    Z[..., 2, 0] = -w[..., 1]
    Z[..., 2, 1] = w[..., 0]
    return Z


def rotation_differential(F: np.ndarray, R: np.ndarray, dF: np.ndarray) -> np.ndarray:
    """dR[dF] for the closest rotation R of F (batched over leading axes)."""
    S = np.swapaxes(R, -1, -2) @ F
    trS = np.trace(S, axis1=-2, axis2=-1)
    K = trS[..., None, None] * np.eye(3) - S
    RtdF = np.swapaxes(R, -1, -2) @ dF
    rhs = axial(RtdF - np.swapaxes(RtdF, -1, -2))
    w = np.linalg.solve(K, rhs[..., None])[..., 0]
    return R @ cross_matrix(w)


def rotation_jacobian(F: np.ndarray) -> np.ndarray:
    """J[..., 9, 9] with J[(i,j),(k,l)] = dR_ij / dF_kl (row-major flattening)."""
    R = closest_rotation(F)
    J = np.zeros(F.shape[:-2] + (9, 9))
    for kl in range(9):
        E = np.zeros(F.shape)
        E[..., kl // 3, kl % 3] = 1.0
        J[..., :, kl] = rotation_differential(F, R, E).reshape(F.shape[:-2] + (9,))
    return J


def sphere_projection(f: np.ndarray, r: np.ndarray, fiber: np.ndarray) -> np.ndarray:
    """p = r f/|f| (p = r m where f = 0)."""
    nrm = np.linalg.norm(f, axis=-1)
    out = np.empty_like(f)
    nz = nrm > 0
    out[nz] = (r[nz] / nrm[nz])[:, None] * f[nz]
    out[~nz] = r[~nz][:, None] * np.asarray(fiber)[None, :]
    return out


def sphere_jacobian(f: np.ndarray, r: np.ndarray) -> np.ndarray:
    """dp/df = (r/|f|)(I - n n^T), n = f/|f| (zero where f = 0)."""
    nrm = np.linalg.norm(f, axis=-1)
    J = np.zeros(f.shape[:-1] + (3, 3))
    nz = nrm > 0
    n = f[nz] / nrm[nz][:, None]
    J[nz] = (r[nz] / nrm[nz])[:, None, None] * (np.eye(3)[None] - n[:, :, None] * n[:, None, :])
    return J


def ground_projection(xc: np.ndarray) -> np.ndarray:
    """p = (x1, x2, max(x3, 0)) per contact candidate node."""
    p = xc.copy()
    p[:, 2] = np.maximum(xc[:, 2], 0.0)
    return p


def ground_jacobian(xc: np.ndarray) -> np.ndarray:
    """diag(1, 1, [x3 >= 0]) per node, as [C, 3] diagonals."""
    d = np.ones_like(xc)
    d[:, 2] = (xc[:, 2] >= 0.0).astype(np.float64)
    return d
