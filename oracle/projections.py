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


# ---------------------------------------------------------------- volume preservation
#
# Supplemental Sec. Energy Definitions, volume-preserving term: E = (w/2)|F - D|^2
# with D the projection of F onto {det D = 1}.  With F = U diag(s) V^T,
# D = U diag(s + d*) V^T where d* minimises |d|^2 subject to prod(s_i + d_i) = 1;
# d* and the Lagrange multiplier satisfy the KKT conditions
#   d + lam grad c(d) = 0,   c(d) = prod(s_i + d_i) - 1 = 0,
# and their differential (eq:vol_kkt) gives dd*/ds.  Readings:
# * the signed SVD (U, V proper rotations, s_3 carrying the sign of det F), as
#   for the closest rotation;
# * the KKT conditions are solved by Newton's method from d = 0, lam = 0 (its
#   Jacobian is eq:vol_kkt's matrix), until the update stops changing d;
# * where det F <= 0 (an inverted Gauss point) the constraint cannot be met on
#   the branch continuous with s; there D is the closest rotation U V^T and
#   dD/dF is dR/dF (so that the energy stays defined);
# * dD/dF for the isotropic map F -> U diag(D_i(s)) V^T: with A = U^T dF V,
#   (U^T dD V)_ii = sum_k dD_i/ds_k A_kk and, for i != j,
#   (U^T dD V)_ij = (D_i - D_j)/(s_i - s_j) (A_ij + A_ji)/2
#                 + (D_i + D_j)/(s_i + s_j) (A_ij - A_ji)/2,
#   the first ratio taken as its limit dD_i/ds_i - dD_i/ds_j where s_i = s_j.

def signed_svd(F: np.ndarray):
    """F = U diag(s) V^T with det U = det V = +1; s_3 < 0 where det F < 0."""
    U, s, Vt = np.linalg.svd(F)
    U, s, Vt = U.copy(), s.copy(), Vt.copy()
    nu = np.linalg.det(U) < 0
    U[nu, :, 2] *= -1.0
    s[nu, 2] *= -1.0
    nv = np.linalg.det(Vt) < 0
    Vt[nv, 2, :] *= -1.0
    s[nv, 2] *= -1.0
    return U, s, Vt


def _kkt_parts(s, d):
    """c(d), grad c(d) and the Hessian of c at s + d (batched)."""
    D = s + d
    c = np.prod(D, axis=-1) - 1.0
    g = np.stack([D[..., 1] * D[..., 2], D[..., 0] * D[..., 2], D[..., 0] * D[..., 1]], axis=-1)
    H = np.zeros(D.shape + (3,))
    H[..., 0, 1] = H[..., 1, 0] = D[..., 2]
    H[..., 0, 2] = H[..., 2, 0] = D[..., 1]
    H[..., 1, 2] = H[..., 2, 1] = D[..., 0]
    return c, g, H


def volume_kkt(s: np.ndarray, max_iter: int = 60):
    """(d*, lam*) for singular values s [..., 3] with prod(s) > 0: Newton's
    method on the KKT conditions from d = 0, lam = 0."""
    d = np.zeros_like(s)
    lam = np.zeros(s.shape[:-1])
    for _ in range(max_iter):
        c, g, H = _kkt_parts(s, d)
        r = np.concatenate([d + lam[..., None] * g, c[..., None]], axis=-1)
        J = np.zeros(s.shape[:-1] + (4, 4))
        J[..., :3, :3] = np.eye(3) + lam[..., None, None] * H
        J[..., :3, 3] = g
        J[..., 3, :3] = g
        step = np.linalg.solve(J, -r[..., None])[..., 0]
        d = d + step[..., :3]
        lam = lam + step[..., 3]
        if np.all(np.abs(step[..., :3]) <= 1e-16 * (1.0 + np.abs(s))):
            break
    return d, lam


def volume_projection(F: np.ndarray) -> np.ndarray:
    """D[..., 3, 3], the projection of F onto {det D = 1} (rotation where det F <= 0)."""
    U, s, Vt = signed_svd(F)
    ok = s[..., 2] > 0
    Dd = np.ones_like(s)
    if np.any(ok):
        d, _ = volume_kkt(s[ok])
        Dd[ok] = s[ok] + d
    return U @ (Dd[..., :, None] * Vt)


def volume_diag_jacobian(s: np.ndarray) -> np.ndarray:
    """dD_i/ds_j [..., 3, 3] from eq:vol_kkt with one-hot ds."""
    d, lam = volume_kkt(s)
    c, g, H = _kkt_parts(s, d)
    K = np.zeros(s.shape[:-1] + (4, 4))
    K[..., :3, :3] = np.eye(3) + lam[..., None, None] * H
    K[..., :3, 3] = g
    K[..., 3, :3] = g
    out = np.zeros(s.shape + (3,))
    for j in range(3):
        e = np.zeros(s.shape)
        e[..., j] = 1.0
        rhs = np.concatenate([-lam[..., None] * (H @ e[..., None])[..., 0], -(g * e).sum(-1, keepdims=True)],
                             axis=-1)
        sol = np.linalg.solve(K, rhs[..., None])[..., 0]
        out[..., :, j] = e + sol[..., :3]          # dD_i/ds_j = delta_ij + dd*_i/ds_j
    return out, s + d


def volume_differential(F: np.ndarray, dF: np.ndarray) -> np.ndarray:
    """dD[dF] for the volume projection (batched over leading axes)."""
    U, s, Vt = signed_svd(F)
    V = np.swapaxes(Vt, -1, -2)
    A = np.swapaxes(U, -1, -2) @ dF @ V
    ok = s[..., 2] > 0
    out = np.zeros(F.shape)
    if np.any(~ok):
        R = U[~ok] @ Vt[~ok]
        out[~ok] = rotation_differential(F[~ok], R, dF[~ok])
    if np.any(ok):
        G, Dd = volume_diag_jacobian(s[ok])
        a = A[ok]
        sk = s[ok]
        B = np.zeros(a.shape)
        for i in range(3):
            B[:, i, i] = (G[:, i, :] * np.diagonal(a, axis1=1, axis2=2)).sum(-1)
            for j in range(3):
                if i == j:
                    continue
                ds = sk[:, i] - sk[:, j]
                close = np.abs(ds) <= 1e-9 * (np.abs(sk[:, i]) + np.abs(sk[:, j]))
                ratio = np.where(close, G[:, i, i] - G[:, i, j], (Dd[:, i] - Dd[:, j]) / np.where(close, 1.0, ds))
                skew = (Dd[:, i] + Dd[:, j]) / (sk[:, i] + sk[:, j])
                B[:, i, j] = ratio * 0.5 * (a[:, i, j] + a[:, j, i]) + skew * 0.5 * (a[:, i, j] - a[:, j, i])
        out[ok] = U[ok] @ B @ Vt[ok]
    return out


def volume_jacobian(F: np.ndarray) -> np.ndarray:
    """J[..., 9, 9] with J[(i,j),(k,l)] = dD_ij / dF_kl (row-major flattening)."""
    J = np.zeros(F.shape[:-2] + (9, 9))
    for kl in range(9):
        E = np.zeros(F.shape)
        E[..., kl // 3, kl % 3] = 1.0
        J[..., :, kl] = volume_differential(F, E).reshape(F.shape[:-2] + (9,))
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
