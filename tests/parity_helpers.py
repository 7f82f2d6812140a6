"""Shared helpers of the GPU parity tests (test helper, not a test module)."""
import numpy as np
import torch

import workloads as W
from oracle import model as om


def soa(t):
    """[3, N] device tensor -> node-major 3N numpy vector."""
    return t.detach().cpu().numpy().T.reshape(-1).copy()


def to_dev(v_aos, n_nodes, device="cuda:0"):
    """node-major 3N numpy vector -> contiguous [3, N] float64 device tensor."""
    return torch.from_numpy(np.ascontiguousarray(v_aos.reshape(n_nodes, 3).T)).to(device)


def elem_dev(a, device="cuda:0"):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64))).to(device)


def pair(scene, **iteration):
    """(GPU mesh, oracle model) of one scene."""
    from paper_2101_05917_amd.mesh import Mesh
    g = Mesh.from_scene(scene, **iteration)
    o = om.Model(scene)
    return g, o


def rel(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    n = np.linalg.norm(np.asarray(b))
    return d / n if n > 0 else d


def robot_scene(steps=3, dx=0.05):
    sc = W.legged_body(8, 6, 4, steps=steps, leg_height=2)
    sc.dx = dx
    sc.origin = (0.0, 0.0, -0.03 * dx)
    return sc


def ragged_scene():
    """An irregular voxel set: 45 cells (not a multiple of the 32-element tile)."""
    cells = W.box_cells(5, 3, 3)
    keep = np.ones(len(cells), bool)
    keep[[4, 13, 22, 31, 40, 44]] = False
    cells = cells[keep][:41]
    sc = W.cantilever(5, 3, 3, youngs="loguniform", seed=3)
    sc.cells = cells
    sc.youngs = sc.youngs[: len(cells)]
    sc.fixed_nodes = W.present_nodes(cells)[W.present_nodes(cells)[:, 0] == 0]
    return sc
