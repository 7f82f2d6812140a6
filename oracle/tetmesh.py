"""Linear-tetrahedron FEM discretization (oracle; test infrastructure only).

The paper's method is stated for any finite-element mesh whose energies act
through an operator G_c mapping nodal positions to deformation gradients
(Sec. Background, Projective Dynamics paragraph); its tetrahedral scenes
(Sec. Evaluation) use linear tetrahedra.  On a linear tetrahedron the
deformation gradient is constant: with the rest edge matrix
D_m = [X_1 - X_0, X_2 - X_0, X_3 - X_0] and the deformed one D_s,
F = D_s D_m^{-1}, so G_e is a constant 9 x 12 matrix and each element is one
"quadrature point" of weight V_e = |det D_m| / 6.  Readings used here:

* mass lumped as rho V_e / 4 to each corner of each tetrahedron;
* the corotated weight 2 mu_e V_e per element (the voxel reading with V_q
  replaced by the element volume).

Pins (tests/test_oracle_tets.py): F = I at rest and F = A for every element
under any affine map x = A X + t; sum of volumes = the meshed solid's volume;
the tetrahedral and the hexahedral energies agree on affine deformations of a
voxel-aligned mesh; mass per node in closed form on a single tetrahedron.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class TetMesh:
    """Nodes, connectivity and rest positions of a tetrahedral mesh."""

    def __init__(self, X, tets):
        X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
        tets = np.asarray(tets, dtype=np.int64).reshape(-1, 4)
        if tets.min() < 0 or tets.max() >= len(X):
            raise ValueError("tetrahedron corner out of range")
        self.X = X.copy()                                               # [N, 3]
        self.conn = tets.copy()                                         # [E, 4]
        Dm = (X[tets[:, 1:]] - X[tets[:, :1]]).transpose(0, 2, 1)       # [E, 3, 3], columns = edges
        det = np.linalg.det(Dm)
        if np.any(np.abs(det) <= 1e-300):
            raise ValueError("degenerate tetrahedron")
        self.Dm_inv = np.linalg.inv(Dm)                                 # [E, 3, 3]
        self.volumes = np.abs(det) / 6.0                                # [E]

    @property
    def n_nodes(self) -> int:
        return self.X.shape[0]

    @property
    def n_elements(self) -> int:
        return self.conn.shape[0]

    def shape_gradients(self) -> np.ndarray:
        """dN_a/dX per element: [E, 4, 3] (rows a = 0..3 of the element's corners).

        N_1..N_3 are the barycentric coordinates D_m^{-1}(X - X_0), so their
        gradients are the rows of D_m^{-1}; N_0 = 1 - N_1 - N_2 - N_3."""
        B = np.zeros((self.n_elements, 4, 3))
        B[:, 1:, :] = self.Dm_inv
        B[:, 0, :] = -self.Dm_inv.sum(axis=1)
        return B


def deformation_operator(mesh: TetMesh) -> sp.csr_matrix:
    """G (9E x 3N): row 9e + 3i + j holds F_ij of element e = sum_a x_{a,i} dN_a/dX_j."""
    E = mesh.n_elements
    B = mesh.shape_gradients()
    rows, cols, vals = [], [], []
    for i in range(3):
        for j in range(3):
            for a in range(4):
                rows.append(9 * np.arange(E) + 3 * i + j)
                cols.append(3 * mesh.conn[:, a] + i)
                vals.append(B[:, a, j])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(9 * E, 3 * mesh.n_nodes))


def lumped_mass(mesh: TetMesh, rho: float) -> np.ndarray:
    """m_j = sum over the tetrahedra at node j of rho V_e / 4."""
    m = np.zeros(mesh.n_nodes)
    np.add.at(m, mesh.conn.reshape(-1), np.repeat(rho * mesh.volumes / 4.0, 4))
    return m
