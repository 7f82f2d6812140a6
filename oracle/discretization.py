"""Hex-voxel FEM discretization (oracle; test infrastructure only).

The paper defines each elastic energy on finite elements through an operator
G_c that maps nodal positions to deformation gradients (Sec. Background,
Projective Dynamics paragraph) and integrates the energy density with Gaussian
quadrature (supplemental Sec. Energy Definitions, background elasticity).  The
lumped mass matrix is introduced with the implicit integrator
(Sec. Background, eq:implicit_v).  Readings used here:

* trilinear (Q1) cubic voxels of edge dx, local node a = dx + 2 dy + 4 dz;
* 2x2x2 Gauss points at +-1/sqrt(3) with volume weight dx^3/8 each;
* mass lumped as rho dx^3 / 8 to each corner of each voxel.

Pins: mesh counts printed in the paper (tests/golden/mesh_counts.json), the
rest state giving F = I, partition of unity of the gradients, and exact
rigid-motion reproduction F(QX + t) = Q.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

GAUSS = 1.0 / np.sqrt(3.0)


class VoxelMesh:
    """Nodes, connectivity and rest positions of a set of cubic voxels."""

    def __init__(self, cells, dx: float, origin=(0.0, 0.0, 0.0)):
        cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
        if len(np.unique(cells, axis=0)) != len(cells):
            raise ValueError("duplicate voxels")
        offs = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.int64)
        corners = cells[:, None, :] + offs[None, :, :]                  # [E, 8, 3]
        flat = corners.reshape(-1, 3)
        # lexicographic order with i fastest: sort rows of (k, j, i)
        uniq, inv = np.unique(flat[:, ::-1], axis=0, return_inverse=True)
        self.cells = cells
        self.node_ijk = uniq[:, ::-1].copy()                             # [N, 3]
        self.conn = inv.reshape(-1, 8)                                   # [E, 8]
        self.dx = float(dx)
        self.origin = np.asarray(origin, dtype=np.float64)
        self.X = self.origin[None, :] + self.dx * self.node_ijk.astype(np.float64)   # [N, 3]

    @property
    def n_nodes(self) -> int:
        return self.node_ijk.shape[0]

    @property
    def n_elements(self) -> int:
        return self.conn.shape[0]

    def node_index(self, ijk) -> np.ndarray:
        """Public index of each grid node in ``ijk`` (must be present)."""
        lut = {tuple(v): n for n, v in enumerate(self.node_ijk.tolist())}
        return np.array([lut[tuple(v)] for v in np.asarray(ijk).reshape(-1, 3).tolist()],
                        dtype=np.int64)


def gauss_points() -> np.ndarray:
    """[8, 3] reference coordinates; q = qx + 2 qy + 4 qz, bit 0 -> -1/sqrt(3)."""
    return np.array([[(-GAUSS, GAUSS)[(q >> k) & 1] for k in range(3)] for q in range(8)])


def shape_gradients(dx: float) -> np.ndarray:
    """B[q, j, a] = dN_a/dX_j at Gauss point q for a cubic voxel of edge dx.

    N_a(xi) = 1/8 prod_k (1 + s_ak xi_k) with s_ak = +-1, and X = X0 + dx (xi + 1)/2,
    so dN_a/dX_j = (2/dx) dN_a/dxi_j.
    """
    B = np.zeros((8, 3, 8))
    xi = gauss_points()
    for q in range(8):
        for a in range(8):
            s = np.array([2 * ((a >> k) & 1) - 1 for k in range(3)], dtype=np.float64)
            for j in range(3):
                val = 0.125 * s[j]
                for k in range(3):
                    if k != j:
                        val *= 1.0 + s[k] * xi[q, k]
                B[q, j, a] = val * 2.0 / dx
    return B


def deformation_operator(mesh: VoxelMesh) -> sp.csr_matrix:
    """G (9Q x 3N): row 9(8e+q) + 3i + j holds F_q[i, j] = sum_a x_a[i] dN_a/dX_j."""
    B = shape_gradients(mesh.dx)
    E = mesh.n_elements
    e, q, i, j, a = np.meshgrid(np.arange(E), np.arange(8), np.arange(3), np.arange(3),
                                np.arange(8), indexing="ij")
    rows = 9 * (8 * e + q) + 3 * i + j
    cols = 3 * mesh.conn[e, a] + i
    vals = B[q, j, a]
    return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(9 * 8 * E, 3 * mesh.n_nodes))


def fiber_operator(mesh: VoxelMesh, fiber) -> sp.csr_matrix:
    """G_m (3Q x 3N): row 3(8e+q) + i holds (F_q m)[i] = sum_a x_a[i] (grad N_a . m)."""
    m = np.asarray(fiber, dtype=np.float64)
    Bm = np.einsum("qja,j->qa", shape_gradients(mesh.dx), m)          # [8, 8]
    E = mesh.n_elements
    e, q, i, a = np.meshgrid(np.arange(E), np.arange(8), np.arange(3), np.arange(8),
                             indexing="ij")
    rows = 3 * (8 * e + q) + i
    cols = 3 * mesh.conn[e, a] + i
    vals = Bm[q, a]
    return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(3 * 8 * E, 3 * mesh.n_nodes))


def selector(n_nodes: int, nodes) -> sp.csr_matrix:
    """S (3C x 3N) picking the 3 coordinates of each listed node."""
    nodes = np.asarray(nodes, dtype=np.int64)
    C = len(nodes)
    rows = np.arange(3 * C)
    cols = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
    return sp.csr_matrix((np.ones(3 * C), (rows, cols)), shape=(3 * C, 3 * n_nodes))


def lumped_mass(mesh: VoxelMesh, rho: float) -> np.ndarray:
    """m[N]: rho dx^3 / 8 from every voxel touching the node."""
    m = np.zeros(mesh.n_nodes)
    np.add.at(m, mesh.conn.ravel(), rho * mesh.dx ** 3 / 8.0)
    return m
