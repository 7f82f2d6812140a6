"""Linear tetrahedra in the oracle (Sec. Background: energies through G_c on
any finite-element mesh; the tetrahedral scenes of Sec. Evaluation): the
constant deformation gradient, volumes and lumped mass, agreement with the
hexahedral discretization on affine deformations, and the method's
invariants and derivatives on tetrahedral scenes (forward step against
Newton's method, gradient and Hessian against central differences, rollout
gradients against central differences)."""
import numpy as np

from oracle import adjoint as oa, forward as of, model as om, rollout as orr, tetmesh as tm
from oracle_scenes import perturbed_state
import workloads as W


def _rotation(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def test_affine_maps_give_their_matrix_in_every_element():
    sc = W.tet_cantilever(4, 3, 2, jitter=0.2, seed=3)
    mesh = tm.TetMesh(sc.X, sc.tets)
    G = tm.deformation_operator(mesh)
    X = sc.X.reshape(-1)
    F0 = (G @ X).reshape(-1, 3, 3)
    assert np.abs(F0 - np.eye(3)).max() <= 1e-12
    rng = np.random.default_rng(0)
    for _ in range(3):
        A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
        t = rng.standard_normal(3)
        x = (sc.X @ A.T + t).reshape(-1)
        F = (G @ x).reshape(-1, 3, 3)
        assert np.abs(F - A[None]).max() <= 1e-12
    Q = _rotation(rng)
    F = (G @ (sc.X @ Q.T).reshape(-1)).reshape(-1, 3, 3)
    assert np.abs(F - Q[None]).max() <= 1e-12


def test_volumes_and_lumped_mass():
    rng = np.random.default_rng(1)
    # one tetrahedron: V = |det D_m| / 6 and a quarter of rho V per corner
    P = rng.standard_normal((4, 3))
    mesh = tm.TetMesh(P, [[0, 1, 2, 3]])
    V = abs(np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], axis=1))) / 6.0
    assert abs(mesh.volumes[0] - V) <= 1e-15 * V
    assert np.allclose(tm.lumped_mass(mesh, 7.0), 7.0 * V / 4.0, rtol=1e-15)
    # a jittered box: the volumes tile the box exactly, the mass is rho times it
    sc = W.tet_cantilever(5, 3, 2, jitter=0.2, seed=4)
    mesh = tm.TetMesh(sc.X, sc.tets)
    assert abs(mesh.volumes.sum() - 30 * 0.01 ** 3) <= 1e-12 * 30 * 0.01 ** 3
    assert np.all(mesh.volumes > 0)
    assert abs(tm.lumped_mass(mesh, 1e3).sum() - 1e3 * 30 * 0.01 ** 3) <= 1e-12
    # shape gradients sum to zero (partition of unity)
    assert np.abs(mesh.shape_gradients().sum(axis=1)).max() <= 1e-9


def test_affine_energy_equals_the_hexahedral_one():
    """On an affine deformation every element of either mesh sees F = A, so the
    corotated energies of the voxel beam (8 Gauss points per cell) and of its
    tetrahedral split (one point per tetrahedron, jittered nodes) are equal."""
    hx = W.cantilever(4, 2, 2)
    tt = W.tet_cantilever(4, 2, 2, jitter=0.2, seed=5)
    mh, mt = om.Model(hx), om.Model(tt)
    rng = np.random.default_rng(6)
    for _ in range(3):
        A = _rotation(rng) @ (np.eye(3) + 0.2 * rng.standard_normal((3, 3)))
        t = rng.standard_normal(3)
        eh = mh.elastic_energy((mh.X.reshape(-1, 3) @ A.T + t).reshape(-1))
        et = mt.elastic_energy((mt.X.reshape(-1, 3) @ A.T + t).reshape(-1))
        assert eh > 0
        assert abs(eh - et) <= 1e-12 * eh


def test_matrix_row_sums_and_symmetry():
    sc = W.tet_ball(radius=3.0, steps=3)
    m = om.Model(sc)
    A = m.A.toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    t = np.tile([0.3, -0.2, 0.5], m.N)
    k = np.zeros(3 * m.N)
    k[3 * m.contact_nodes + 0] = k[3 * m.contact_nodes + 1] = k[3 * m.contact_nodes + 2] = m.contact_k
    assert np.allclose(A @ t, (m.Mdiag / m.h ** 2 + k) * t, rtol=1e-12, atol=1e-9 * np.abs(A).max())
    assert len(m.contact_nodes) > 0


def test_gradient_and_hessian_against_central_differences():
    sc = W.tet_ball(radius=2.5, steps=3)
    m = om.Model(sc)
    x, v = perturbed_state(m, seed=7)
    x[3 * m.contact_nodes + 2] -= 1e-3            # some ground contacts active
    y = m.y_of(x, v)
    gr = m.grad_g(x, y)
    H = m.hessian(x)
    rng = np.random.default_rng(8)
    eps = 1e-7
    for _ in range(4):
        d = rng.standard_normal(3 * m.N)
        fd = (m.g(x + eps * d, y) - m.g(x - eps * d, y)) / (2 * eps)
        assert abs(fd - gr @ d) <= 1e-6 * (abs(gr @ d) + 1e-3 * np.linalg.norm(gr) * np.linalg.norm(d))
        fd = (m.grad_g(x + eps * d, y) - m.grad_g(x - eps * d, y)) / (2 * eps)
        assert np.linalg.norm(fd - H @ d) <= 1e-6 * np.linalg.norm(H @ d)


def test_pd_step_reaches_newtons_state():
    sc = W.tet_cantilever(4, 2, 2, jitter=0.15, youngs="loguniform", seed=9, steps=3)
    m = om.Model(sc)
    x0, v0 = m.X.copy(), np.zeros(3 * m.N)
    x1, v1, info = of.pd_step(m, x0, v0, max_iter=20000, tol=1e-14)
    xn, _ = of.newton_solve(m, info["y"])
    assert np.linalg.norm(xn - x1) <= 1e-9 * np.linalg.norm(x1 - x0)
    # the rest state of a body without gravity stays put
    sc0 = W.tet_cantilever(3, 2, 2, jitter=0.15, seed=10)
    sc0.gravity = (0.0, 0.0, 0.0)
    m0 = om.Model(sc0)
    x, v, _ = of.pd_step(m0, m0.X.copy(), np.zeros(3 * m0.N), max_iter=10, tol=1e-14)
    assert np.abs(x - m0.X).max() <= 1e-15 and np.abs(v).max() <= 1e-13


def test_adjoint_solvers_agree():
    sc = W.tet_ball(radius=2.5, steps=3)
    m = om.Model(sc)
    x, v = perturbed_state(m, seed=11)
    xr, _ = of.newton_solve(m, m.y_of(x, v))
    rng = np.random.default_rng(12)
    gxn, gvn = rng.standard_normal(3 * m.N), rng.standard_normal(3 * m.N)
    direct = oa.backward_step(m, x, v, None, xr, gxn, gvn, solver="direct")
    cg = oa.backward_step(m, x, v, None, xr, gxn, gvn, solver="pcg")
    for a, b in zip(direct[:3], cg[:3]):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(a)


def test_rollout_gradients_against_central_differences():
    sc = W.tet_cantilever(3, 2, 2, jitter=0.15, youngs="loguniform", seed=13, steps=3)
    E0 = sc.youngs.copy()
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, seed=14)
    cx = W.loss_vector(m.N, 0)
    L, g = orr.loss_and_grad(m, x0, v0, None, cx, newton=True)
    rng = np.random.default_rng(15)
    d = rng.standard_normal(3 * m.N)
    d[m.fixed] = 0.0
    fd = orr.central_difference(lambda t: orr.rollout_loss(sc, x0 + t * d, v0, None, cx, newton=True), 0.0,
                                1.0, 1e-6)
    assert abs(fd - g["x0"] @ d) <= 1e-6 * abs(fd)
    # a velocity moves the positions by h times as much: a larger step keeps
    # the difference above the solver's round-off
    fd = orr.central_difference(lambda t: orr.rollout_loss(sc, x0, v0 + t * d, None, cx, newton=True), 0.0,
                                1.0, 1e-4)
    assert abs(fd - g["v0"] @ d) <= 1e-6 * abs(fd)
    # log E of the three most sensitive elements and of element 0
    gl = g["youngs"] * E0
    for e in list(np.argsort(-np.abs(gl))[:3]) + [0]:
        dlog = np.zeros(m.E)
        dlog[e] = 1.0
        f = lambda t: orr.rollout_loss(sc, x0, v0, None, cx, youngs=E0 * np.exp(t * dlog), newton=True)  # noqa: E731
        fd = orr.central_difference(f, 0.0, 1.0, 1e-4)
        assert abs(fd - gl[e]) <= 1e-6 * abs(gl[e]) + 1e-6 * np.abs(gl).max()
