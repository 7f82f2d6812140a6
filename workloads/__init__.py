"""Seeded synthetic workloads for the implicit-Euler PD step and its adjoint.

This module holds scene descriptions and seeded random draws only: voxel
masks, material fields, boundary-node lists, actuation sequences, loss
vectors and request traces.  It performs none of the method's arithmetic
(no shape functions, no masses, no projections, no solves), so the CPU
oracle and the HIP path can both read it without sharing any of the method.

The paper's meshes (cantilever, quadruped, contact scenes; Sec. Evaluation
and Applications) are not available, so voxel boxes of the stated sizes and
shapes stand in for them.  Every array is drawn from
``numpy.random.default_rng(seed)``.

Conventions
-----------
* A scene is a set of cubic voxels with integer corner coordinates
  ``(i, j, k)``; a node exists wherever a voxel corner exists.  Public node
  order is lexicographic over present grid nodes with ``i`` fastest, then
  ``j``, then ``k``.
* The rest position of grid node ``(i, j, k)`` is ``origin + dx * (i, j, k)``;
  ``z`` is up and gravity points along ``-z`` (the paper puts gravity along
  the negative z axis in its supplemental experiment details).
* Loss vectors are node-major (x0, y0, z0, x1, ...) over all nodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np

__all__ = [
    "Scene",
    "box_cells",
    "cantilever",
    "legged_body",
    "dropped_block",
    "rolling_sphere",
    "candidate_nodes",
    "initial_velocity",
    "served_requests",
    "loss_vector",
    "actuation_sequence",
    "present_nodes",
    "TetScene",
    "tet_body",
    "tet_cantilever",
    "tet_ball",
    "config",
    "CONFIG_NAMES",
]


@dataclass
class Scene:
    """One simulated body and its physical constants (SI units)."""

    name: str
    cells: np.ndarray                 # [E, 3] int32 voxel indices
    youngs: np.ndarray                # [E] float64, Pa
    fixed_nodes: np.ndarray           # [F, 3] int32 grid coordinates held at rest
    dx: float = 0.01                  # voxel edge, m
    rho: float = 1e3                  # density, kg/m^3
    nu: float = 0.45                  # Poisson ratio
    h: float = 0.01                   # time step, s
    gravity: tuple = (0.0, 0.0, -9.81)
    origin: tuple = (0.0, 0.0, 0.0)
    contact_k: float = 0.0            # ground penalty stiffness, N/m (0 = off)
    friction_mu: float = 0.0          # Coulomb coefficient of the explicit friction
    friction_eps: float = 1e-3        # velocity regulariser of the friction, m/s
    muscle_k: float = 0.0             # fibre stiffness per unit volume, Pa (0 = off)
    volume_scale: float = 0.0         # weight of the volume-preserving term in units of
                                      # Lame's lambda per unit volume (0 = off)
    fiber: tuple = (1.0, 0.0, 0.0)    # unit fibre direction
    steps: int = 10
    loss_seed: int = 0
    act_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(self.cells.shape[0])

    def physics(self) -> dict:
        d = asdict(self)
        for key in ("cells", "youngs", "fixed_nodes", "extra", "name"):
            d.pop(key)
        return d


def box_cells(nx: int, ny: int, nz: int) -> np.ndarray:
    """All voxels of an nx x ny x nz box, in lexicographic order (i fastest)."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int32)


def present_nodes(cells: np.ndarray) -> np.ndarray:
    """Grid coordinates of all voxel corners, unique, lexicographic (i fastest).

    This is set bookkeeping on integer coordinates (which corners exist), not
    part of the discretisation.
    """
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    corners = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=np.int64)
    allc = (cells[:, None, :] + corners[None, :, :]).reshape(-1, 3)
    uniq = np.unique(allc[:, ::-1], axis=0)
    return uniq[:, ::-1].astype(np.int32)


def _face_nodes(cells: np.ndarray, axis: int, value: int) -> np.ndarray:
    nodes = present_nodes(cells)
    return nodes[nodes[:, axis] == value]


def cantilever(nx: int, ny: int, nz: int, *, youngs="const", steps: int = 10,
               seed: int = 0, name: Optional[str] = None) -> Scene:
    """Hex beam along +x with the x = 0 face held (the paper's Cantilever layout).

    ``youngs="const"`` gives E = 1e6 Pa everywhere; ``"loguniform"`` draws
    log10(E_e) ~ U(5, 7) per element from ``default_rng(seed)``.
    """
    cells = box_cells(nx, ny, nz)
    E = cells.shape[0]
    if youngs == "const":
        ym = np.full(E, 1e6)
    elif youngs == "loguniform":
        ym = 10.0 ** np.random.default_rng(seed).uniform(5.0, 7.0, size=E)
    else:
        ym = np.asarray(youngs, dtype=np.float64).reshape(E)
    return Scene(name=name or f"cantilever_{nx}x{ny}x{nz}", cells=cells, youngs=ym,
                 fixed_nodes=_face_nodes(cells, 0, 0), steps=steps)


def legged_body(nx: int = 20, ny: int = 10, nz: int = 6, *, steps: int = 200,
                leg_height: int = 3) -> Scene:
    """Quadruped-like voxel body: a slab on four corner legs, feet on z = 0.

    A cell (i, j, k) is present iff k >= leg_height, or it lies in one of the
    four corner leg columns (i < 4 or i >= nx - 4) and (j < 3 or j >= ny - 3).
    Muscles run along +x in every element; the feet touch a penalty ground.
    """
    allc = box_cells(nx, ny, nz)
    i, j, k = allc[:, 0], allc[:, 1], allc[:, 2]
    leg = ((i < 4) | (i >= nx - 4)) & ((j < 3) | (j >= ny - 3))
    cells = allc[(k >= leg_height) | leg]
    E = cells.shape[0]
    nu = 0.45
    mu = 1e6 / (2.0 * (1.0 + nu))
    return Scene(name=f"legged_{nx}x{ny}x{nz}", cells=cells, youngs=np.full(E, 1e6),
                 fixed_nodes=np.zeros((0, 3), np.int32), h=5e-3, steps=steps,
                 contact_k=1e4, friction_mu=0.5, muscle_k=2.0 * mu)


def dropped_block(nx: int = 64, ny: int = 32, nz: int = 32, *, steps: int = 200,
                  drop: float = 0.02) -> Scene:
    """Free hex block released ``drop`` metres above a frictionless penalty ground."""
    cells = box_cells(nx, ny, nz)
    E = cells.shape[0]
    return Scene(name=f"block_{nx}x{ny}x{nz}", cells=cells, youngs=np.full(E, 1e6),
                 fixed_nodes=np.zeros((0, 3), np.int32), origin=(0.0, 0.0, drop),
                 steps=steps, contact_k=1e4)


def rolling_sphere(radius: float = 5.0, n: int = 10, *, steps: int = 100, youngs: float = 1e5,
                   speed: float = 0.05, n_candidates: int = 72) -> Scene:
    """Voxelised sphere rolling on the ground, the stand-in for the paper's
    Rolling sphere (Sec. Evaluation: 552 elements, 2469 DoFs, h = 5 ms, 100
    frames, at most 72 contact nodes).

    Cells of an n^3 grid whose centres lie within ``radius`` voxels of the
    grid centre (552 cells and 823 nodes for the defaults).  The bottom node
    layer rests on z = 0 with no penalty ground (``contact_k = 0``): contact is
    the complementarity kind, on ``extra["candidates_ijk"]``, the
    ``n_candidates`` surface nodes lowest in z (ties broken by the distance to
    the vertical axis, then lexicographically).  The initial motion is a rigid
    roll along +x, ``extra["velocity"]`` with spin ``speed / R`` about +y.
    """
    allc = box_cells(n, n, n)
    c = allc + 0.5 - n / 2.0
    cells = allc[(c ** 2).sum(axis=1) <= radius * radius]
    nodes = present_nodes(cells)
    count = {}
    for cl in cells:
        for a in range(8):
            key = (int(cl[0]) + (a & 1), int(cl[1]) + ((a >> 1) & 1), int(cl[2]) + ((a >> 2) & 1))
            count[key] = count.get(key, 0) + 1
    surface = np.array([count[tuple(int(t) for t in p)] < 8 for p in nodes])
    sn = nodes[surface].astype(np.int64)
    d2 = (2 * sn[:, 0] - n) ** 2 + (2 * sn[:, 1] - n) ** 2
    order = np.lexsort((sn[:, 0], sn[:, 1], d2, sn[:, 2]))
    cand = sn[order[:n_candidates]]
    cand = cand[np.lexsort((cand[:, 0], cand[:, 1], cand[:, 2]))]
    dx = 0.01
    R = radius * dx
    return Scene(name=f"sphere_{len(cells)}", cells=cells, youngs=np.full(len(cells), youngs),
                 fixed_nodes=np.zeros((0, 3), np.int32), dx=dx, h=5e-3, steps=steps,
                 extra={"candidates_ijk": cand.astype(np.int32),
                        "velocity": (speed, 0.0, 0.0), "spin": (0.0, speed / R, 0.0),
                        "center": (n / 2.0 * dx, n / 2.0 * dx, n / 2.0 * dx)})


@dataclass
class TetScene:
    """A body meshed by linear tetrahedra and its physical constants (SI units)."""

    name: str
    X: np.ndarray                     # [N, 3] float64 rest positions, m
    tets: np.ndarray                  # [E, 4] int32 node ids, positively oriented
    youngs: np.ndarray                # [E] float64, Pa
    fixed_nodes: np.ndarray           # [F] int32 node ids held at rest
    rho: float = 1e3
    nu: float = 0.45
    h: float = 0.01
    gravity: tuple = (0.0, 0.0, -9.81)
    contact_k: float = 0.0            # ground penalty on the nodes of minimal rest height
    friction_mu: float = 0.0
    friction_eps: float = 1e-3
    muscle_k: float = 0.0             # not available on tetrahedra (kept 0)
    volume_scale: float = 0.0         # not available on tetrahedra (kept 0)
    fiber: tuple = (1.0, 0.0, 0.0)
    steps: int = 10
    loss_seed: int = 0
    act_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    def physics(self) -> dict:
        d = asdict(self)
        for key in ("X", "tets", "youngs", "fixed_nodes", "extra", "name"):
            d.pop(key)
        return d


# the six tetrahedra of a cube along its main diagonal (one per order in which
# the path from corner 000 to 111 visits the axes); faces shared by
# neighbouring cubes are split along the same diagonal, so the mesh conforms
_KUHN_AXES = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def tet_body(cells: np.ndarray, *, dx: float = 0.01, origin=(0.0, 0.0, 0.0), jitter: float = 0.0,
             pinned=None, seed: int = 0) -> tuple:
    """Nodes and tetrahedra of a voxel set, each voxel split into six.

    Nodes are the voxel corners in lexicographic order (i fastest), at
    ``origin + dx * ijk``; with ``jitter`` > 0 every node not on the set's
    bounding-box faces (and not in ``pinned``) moves by U(-jitter, jitter) * dx
    per coordinate (``default_rng(seed)``), which makes the mesh irregular.
    Returns (X [N, 3], tets [E, 4], ijk [N, 3]); corners ordered so that every
    tetrahedron has positive volume."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    ijk = present_nodes(cells).astype(np.int64)
    index = {tuple(int(t) for t in p): i for i, p in enumerate(ijk)}
    tets = []
    for c in cells:
        for ax in _KUHN_AXES:
            p = np.array(c)
            path = [index[tuple(int(t) for t in p)]]
            for a in ax:
                p = p.copy()
                p[a] += 1
                path.append(index[tuple(int(t) for t in p)])
            tets.append(path)
    tets = np.array(tets, dtype=np.int64)

    def signed_volumes(P):
        e1, e2, e3 = (P[tets[:, k]] - P[tets[:, 0]] for k in (1, 2, 3))
        return np.einsum("ij,ij->i", np.cross(e1, e2), e3)

    X = np.asarray(origin, dtype=np.float64)[None, :] + dx * ijk.astype(np.float64)
    flip = signed_volumes(X) < 0
    tets[flip, 1], tets[flip, 2] = tets[flip, 2].copy(), tets[flip, 1].copy()
    if jitter > 0.0:
        lo, hi = ijk.min(axis=0), ijk.max(axis=0)
        inner = np.all((ijk > lo) & (ijk < hi), axis=1)
        if pinned is not None:
            inner[np.asarray(pinned, dtype=np.int64)] = False
        rng = np.random.default_rng(seed)
        X[inner] += dx * rng.uniform(-jitter, jitter, size=(int(inner.sum()), 3))
        if np.any(signed_volumes(X) <= 0):
            raise ValueError("jitter too large: a tetrahedron inverted")
    return X, tets.astype(np.int32), ijk.astype(np.int32)


def tet_cantilever(nx: int, ny: int, nz: int, *, youngs="const", jitter: float = 0.15, steps: int = 10,
                   seed: int = 0, name: Optional[str] = None) -> TetScene:
    """Tetrahedral beam along +x (six tetrahedra per cell of an nx x ny x nz
    box, interior nodes jittered) with its x = 0 face held."""
    X, tets, ijk = tet_body(box_cells(nx, ny, nz), jitter=jitter, seed=seed)
    E = len(tets)
    if youngs == "const":
        ym = np.full(E, 1e6)
    elif youngs == "loguniform":
        ym = 10.0 ** np.random.default_rng(seed).uniform(5.0, 7.0, size=E)
    else:
        ym = np.asarray(youngs, dtype=np.float64).reshape(E)
    fixed = np.nonzero(ijk[:, 0] == 0)[0].astype(np.int32)
    return TetScene(name=name or f"tet_cantilever_{nx}x{ny}x{nz}", X=X, tets=tets, youngs=ym,
                    fixed_nodes=fixed, steps=steps)


def tet_ball(radius: float = 10.0, *, jitter: float = 0.15, steps: int = 100, drop: float = 0.01,
             youngs: float = 1e6, seed: int = 0, name: Optional[str] = None) -> TetScene:
    """Free tetrahedral ball dropped ``drop`` metres onto a penalty ground
    (k = 1e4, friction 0.5): the voxels of a 2r-cell grid whose centres lie
    within ``radius`` cells of its centre, six tetrahedra each, nodes off the
    bounding box jittered.  The defaults give 4,224 cells, 25,344 tetrahedra and
    5,233 nodes (15,699 DoFs), near the size of the paper's tetrahedral duck (Sec.
    Evaluation, Slope: 24,875 tetrahedra, 16,776 DoFs), whose mesh is not
    available."""
    n = int(np.ceil(2 * radius))
    allc = box_cells(n, n, n)
    c = allc + 0.5 - n / 2.0
    cells = allc[(c ** 2).sum(axis=1) <= radius * radius]
    X, tets, ijk = tet_body(cells, jitter=jitter, origin=(0.0, 0.0, drop), seed=seed)
    zmin = ijk[:, 2].min()
    X[ijk[:, 2] == zmin, 2] = drop
    return TetScene(name=name or f"tet_ball_{len(tets)}", X=X, tets=tets, youngs=np.full(len(tets), youngs),
                    fixed_nodes=np.zeros(0, np.int32), h=5e-3, steps=steps, contact_k=1e4, friction_mu=0.5)


def candidate_nodes(scene: Scene) -> np.ndarray:
    """Public node ids of ``scene.extra["candidates_ijk"]`` (ascending)."""
    nodes = present_nodes(scene.cells)
    index = {tuple(int(t) for t in p): i for i, p in enumerate(nodes)}
    ids = [index[tuple(int(t) for t in p)] for p in scene.extra["candidates_ijk"]]
    return np.sort(np.asarray(ids, dtype=np.int64))


def initial_velocity(scene: Scene) -> np.ndarray:
    """Node-major 3N rigid velocity v + w x (X - c) at the rest positions, from
    ``extra["velocity"]``, ``extra["spin"]`` and ``extra["center"]`` (zeros
    when the scene has none)."""
    nodes = present_nodes(scene.cells).astype(np.float64)
    X = np.asarray(scene.origin)[None, :] + scene.dx * nodes
    if "velocity" not in scene.extra:
        return np.zeros(X.size)
    v = np.asarray(scene.extra["velocity"], dtype=np.float64)
    w = np.asarray(scene.extra.get("spin", (0.0, 0.0, 0.0)), dtype=np.float64)
    c = np.asarray(scene.extra.get("center", (0.0, 0.0, 0.0)), dtype=np.float64)
    return (v[None, :] + np.cross(w[None, :], X - c[None, :])).reshape(-1)


def loss_vector(n_nodes: int, seed: int = 0) -> np.ndarray:
    """Weights of the loss dot(c, x_T): N(0, 1) draws, node-major over all nodes."""
    return np.random.default_rng(seed).standard_normal(3 * n_nodes)


def actuation_sequence(steps: int, n_elements: int, seed: int = 0) -> np.ndarray:
    """Per-step, per-element muscle actuation u[t, e] ~ U[0, 1]."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(steps, n_elements))


def served_requests(n_requests: int = 64, lo: int = 4, hi: int = 24, steps: int = 50,
                    rate: float = 10.0, seed: int = 0) -> list:
    """Request trace for the rollout server: cube cantilevers of random size.

    Sizes n ~ U{lo..hi} (cubes of n^3 cells), Poisson arrivals with the given
    rate (requests per second; ``inf`` puts every arrival at t = 0).  The loss
    seed of request r is r.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=n_requests)
    if np.isinf(rate):
        arrivals = np.zeros(n_requests)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
        arrivals -= arrivals[0]
    reqs = []
    for r in range(n_requests):
        n = int(sizes[r])
        sc = cantilever(n, n, n, steps=steps, name=f"req{r}_{n}^3")
        sc.loss_seed = r
        reqs.append({"id": r, "scene": sc, "arrival": float(arrivals[r])})
    return reqs


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5", "sphere", "tet")


def config(name: str) -> Scene:
    """The five benchmark scenes.

    c1: 4x4x4 cantilever, E = 1e6, 10 steps.
    c2: 16x8x8 cantilever, log-uniform E in [1e5, 1e7], 100 steps.
    c3: legged 20x10x6 body, muscles, penalty ground + friction, h = 5 ms, 200 steps.
    c5: 64x32x32 block dropped 2 cm onto a penalty ground, 200 steps.
    sphere: 552-element sphere rolling on a complementarity ground, 100 steps.
    tet: 25,344-tetrahedron ball dropped 1 cm onto a penalty ground with
         friction, h = 5 ms, 100 steps (a ``TetScene``).
    (c4 is a request trace, see ``served_requests``.)
    """
    if name == "c1":
        return cantilever(4, 4, 4, steps=10, name="c1_cantilever_4x4x4")
    if name == "c2":
        return cantilever(16, 8, 8, youngs="loguniform", steps=100, seed=0,
                          name="c2_cantilever_16x8x8")
    if name == "c3":
        return legged_body()
    if name == "c5":
        return dropped_block()
    if name == "sphere":
        return rolling_sphere()
    if name == "tet":
        return tet_ball(name="tet_ball_25344")
    raise KeyError(name)
