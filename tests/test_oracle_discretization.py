"""Pins of the oracle's discretization against printed counts and closed forms."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import discretization as disc
from oracle import model as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mesh_counts.json")


@pytest.mark.parametrize("key", ["cantilever", "routing_tendon"])
def test_printed_mesh_counts(key):
    g = json.load(open(GOLDEN))[key]
    sc = W.cantilever(*g["cells"])
    mesh = disc.VoxelMesh(sc.cells, sc.dx)
    assert mesh.n_elements == g["elements"]
    assert 3 * mesh.n_nodes == g["dofs"]
    if "dirichlet_dofs" in g:
        assert 3 * len(sc.fixed_nodes) == g["dirichlet_dofs"]


def test_node_order_lexicographic():
    mesh = disc.VoxelMesh(W.box_cells(3, 2, 2), 0.01)
    ijk = mesh.node_ijk
    key = ijk[:, 0] + 100 * ijk[:, 1] + 10000 * ijk[:, 2]
    assert np.all(np.diff(key) > 0)
    # every element's local node a sits at cell + (a&1, a>>1&1, a>>2&1)
    for e in range(mesh.n_elements):
        for a in range(8):
            off = np.array([a & 1, (a >> 1) & 1, (a >> 2) & 1])
            assert np.array_equal(ijk[mesh.conn[e, a]], mesh.cells[e] + off)


def _shape_fn(a, xi):
    s = np.array([2 * ((a >> k) & 1) - 1 for k in range(3)])
    return np.prod(1 + s * xi) / 8.0


def test_shape_gradients_central_difference():
    dx = 0.02
    B = disc.shape_gradients(dx)
    xi_q = disc.gauss_points()
    eps = 1e-6
    for q in range(8):
        for a in range(8):
            for j in range(3):
                d = np.zeros(3)
                d[j] = eps
                fd = (_shape_fn(a, xi_q[q] + d) - _shape_fn(a, xi_q[q] - d)) / (2 * eps) * 2.0 / dx
                assert abs(fd - B[q, j, a]) < 1e-7 * 2.0 / dx


def test_partition_of_unity_and_linear_reproduction():
    dx = 0.01
    B = disc.shape_gradients(dx)
    assert np.abs(B.sum(axis=2)).max() < 1e-12
    corners = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)]) * dx
    # sum_a X_a (x) grad N_a = I for every Gauss point
    for q in range(8):
        F = corners.T @ B[q].T
        assert np.allclose(F, np.eye(3), atol=1e-14)


def test_rest_state_and_rigid_motion_give_F():
    sc = W.cantilever(3, 2, 2)
    m = om.Model(sc)
    F = m.deformation_gradients(m.X)
    assert np.abs(F - np.eye(3)).max() < 1e-13
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    t = rng.standard_normal(3)
    x = (m.X.reshape(-1, 3) @ Q.T + t).reshape(-1)
    F = m.deformation_gradients(x)
    assert np.abs(F - Q[None]).max() < 1e-12


def test_mass_and_matrix_invariants():
    sc = W.legged_body(8, 6, 5, steps=1, leg_height=2)
    m = om.Model(sc)
    assert np.isclose(m.m.sum(), sc.rho * sc.dx ** 3 * m.E, rtol=1e-14)
    A = m.A
    assert abs(A - A.T).max() < 1e-9 * abs(A).max()
    # rows of A applied to a uniform translation: M/h^2 (+k on contact nodes)
    for c in range(3):
        ones = np.zeros(3 * m.N)
        ones[c::3] = 1.0
        expect = m.Mdiag / m.h ** 2
        expect = expect + m.contact_k * (m.Sc.T @ (m.Sc @ ones))
        got = A @ ones
        assert np.abs(got - expect * ones).max() < 1e-9 * abs(A).max()
    assert len(m.contact_nodes) > 0


def test_lumped_mass_per_node_closed_form_on_a_box():
    """On a full nx x ny x nz box every node collects rho dx^3 / 8 from each
    voxel it touches: 1 voxel at a corner, 2 on an edge, 4 on a face and 8
    inside, i.e. prod over the axes of (1 on the box boundary, else 2)."""
    nx, ny, nz, dx, rho = 4, 3, 5, 0.02, 1.3e3
    mesh = disc.VoxelMesh(W.box_cells(nx, ny, nz), dx)
    m = disc.lumped_mass(mesh, rho)
    unit = rho * dx ** 3 / 8.0
    for n, (i, j, k) in enumerate(mesh.node_ijk.tolist()):
        count = 1
        for c, top in ((i, nx), (j, ny), (k, nz)):
            count *= 1 if c in (0, top) else 2
        assert m[n] == pytest.approx(count * unit, rel=1e-14), (i, j, k)
    kinds = {1: 8, 2: 4 * (nx - 1 + ny - 1 + nz - 1), 8: (nx - 1) * (ny - 1) * (nz - 1)}
    for count, expect in kinds.items():
        assert int(np.sum(np.isclose(m, count * unit, rtol=1e-12))) == expect


def test_lumped_mass_per_node_irregular_voxels_brute_force():
    """An irregular voxel set (the legged body): each node's mass is rho dx^3 / 8
    times the number of voxels having it as one of their 8 corners, counted by
    testing every voxel against every node."""
    sc = W.legged_body(8, 6, 4, steps=1, leg_height=2)
    mesh = disc.VoxelMesh(sc.cells, sc.dx)
    m = disc.lumped_mass(mesh, sc.rho)
    cells = np.asarray(sc.cells, dtype=np.int64)
    for n, p in enumerate(mesh.node_ijk):
        d = p[None, :] - cells
        touching = int(np.sum(np.all((d == 0) | (d == 1), axis=1)))
        assert m[n] == pytest.approx(touching * sc.rho * sc.dx ** 3 / 8.0, rel=1e-14)
