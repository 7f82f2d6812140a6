"""The volume-preserving term of the oracle (supplemental Sec. Energy
Definitions): the projection onto det D = 1 against the constrained problem
solved by a general optimizer and by brute force, its closed forms and
symmetries, its derivative (eq:vol_kkt plus the rotations of the SVD) against
central differences, and the energy's gradient, Hessian and rollout gradients
against central differences."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import model as om, projections as op, rollout as orr
from oracle_scenes import perturbed_state, tiny_cantilever
import workloads as W


def _rotation(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def test_projection_has_unit_determinant_and_symmetries():
    rng = np.random.default_rng(0)
    F = np.eye(3)[None] + 0.25 * rng.standard_normal((300, 3, 3))
    F = F[np.linalg.det(F) > 0.05]
    D = op.volume_projection(F)
    assert np.abs(np.linalg.det(D) - 1.0).max() <= 1e-13
    # D(Q1 F Q2) = Q1 D(F) Q2 for rotations Q1, Q2
    Q1, Q2 = _rotation(rng), _rotation(rng)
    D2 = op.volume_projection(Q1[None] @ F @ Q2[None])
    assert np.abs(D2 - Q1[None] @ D @ Q2[None]).max() <= 1e-12


def test_projection_closed_forms():
    rng = np.random.default_rng(1)
    Q = _rotation(rng)
    # a scaled rotation projects to the rotation (uniform stretches below 2,
    # where the isotropic point is the minimiser)
    for s in (0.6, 0.95, 1.3, 1.9):
        assert np.abs(op.volume_projection((s * Q)[None])[0] - Q).max() <= 1e-12
    # a matrix of unit determinant is its own projection
    F = Q @ np.diag([1.7, 0.8, 1.0 / (1.7 * 0.8)]) @ _rotation(rng)
    assert np.abs(op.volume_projection(F[None])[0] - F).max() <= 1e-14


def test_projection_is_the_closest_unit_determinant_matrix():
    """Against a general constrained optimizer over all 3x3 matrices (SLSQP on
    min |D - F|^2 s.t. det D = 1), and the reduced problem against a fine
    brute-force search over the surface prod(D_i) = 1."""
    rng = np.random.default_rng(2)
    for _ in range(5):
        F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
        if np.linalg.det(F) < 0.2:
            continue
        res = minimize(lambda v: np.sum((v - F.ravel()) ** 2), F.ravel() / np.cbrt(np.linalg.det(F)),
                       constraints=[{"type": "eq", "fun": lambda v: np.linalg.det(v.reshape(3, 3)) - 1.0}],
                       method="SLSQP", options={"ftol": 1e-15, "maxiter": 500})
        D = op.volume_projection(F[None])[0]
        assert np.sum((D - F) ** 2) <= res.fun + 1e-12
        assert np.abs(D - res.x.reshape(3, 3)).max() <= 1e-5
    for _ in range(4):
        s = np.sort(rng.uniform(0.6, 1.6, 3))[::-1]
        d, lam = op.volume_kkt(s[None])
        best = np.inf
        a = np.linspace(-0.8, 0.8, 801)
        A, B = np.meshgrid(a, a, indexing="ij")
        Dd = np.stack([np.exp(A), np.exp(B), np.exp(-A - B)], axis=-1)
        dist = np.sum((Dd - s) ** 2, axis=-1)
        i = np.unravel_index(np.argmin(dist), dist.shape)
        best = dist[i]
        assert np.sum(d[0] ** 2) <= best + 1e-12
        assert np.abs((s + d[0]) - Dd[i]).max() <= 2e-3          # the grid's resolution
        # the KKT conditions hold
        D = s + d[0]
        grad_c = np.array([D[1] * D[2], D[0] * D[2], D[0] * D[1]])
        assert np.abs(d[0] + lam[0] * grad_c).max() <= 1e-14
        assert abs(np.prod(D) - 1.0) <= 1e-14


@pytest.mark.parametrize("case", ["generic", "repeated", "inverted"])
def test_projection_derivative_against_central_differences(case):
    rng = np.random.default_rng(3)
    Q1, Q2 = _rotation(rng), _rotation(rng)
    if case == "generic":
        F = np.eye(3)[None] + 0.2 * rng.standard_normal((40, 3, 3))
        F = F[np.linalg.det(F) > 0.2]
    elif case == "repeated":      # two equal singular values: the limit form of the ratio
        F = (Q1 @ np.diag([1.1, 1.1, 0.85]) @ Q2)[None]
    else:                         # det F < 0: the closest rotation and its derivative
        F = (Q1 @ np.diag([1.2, 0.9, -0.3]) @ Q2)[None]
    eps = 1e-6
    for _ in range(3):
        dF = rng.standard_normal(F.shape)
        fd = (op.volume_projection(F + eps * dF) - op.volume_projection(F - eps * dF)) / (2 * eps)
        an = op.volume_differential(F, dF)
        assert np.abs(fd - an).max() <= 1e-7 * max(1.0, np.abs(an).max())
    if case == "inverted":
        R = op.closest_rotation(F)
        assert np.abs(op.volume_projection(F) - R).max() <= 1e-14


def _volume_scene():
    sc = tiny_cantilever(3, 2, 2, youngs=10 ** np.linspace(5, 6.5, 12))
    sc.volume_scale = 1.0
    return sc


def test_energy_gradient_and_hessian_with_volume_term():
    sc = _volume_scene()
    m = om.Model(sc)
    assert m.wv is not None
    x, v = perturbed_state(m, seed=4)
    y = m.y_of(x, v)
    gr = m.grad_g(x, y)
    rng = np.random.default_rng(5)
    eps = 1e-7
    for _ in range(4):
        d = rng.standard_normal(3 * m.N)
        fd = (m.g(x + eps * d, y) - m.g(x - eps * d, y)) / (2 * eps)
        assert abs(fd - gr @ d) <= 1e-6 * (abs(gr @ d) + np.linalg.norm(gr) * np.linalg.norm(d) * 1e-3)
    H = m.hessian(x)
    for _ in range(4):
        d = rng.standard_normal(3 * m.N)
        fd = (m.grad_g(x + eps * d, y) - m.grad_g(x - eps * d, y)) / (2 * eps)
        assert np.linalg.norm(fd - H @ d) <= 1e-6 * np.linalg.norm(H @ d)
    # the volume term adds a Kronecker term w_v G^T G: A stays symmetric and
    # translations still see only the mass
    A = m.A.toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    t = np.tile([0.3, -0.2, 0.5], m.N)
    assert np.allclose(A @ t, m.Mdiag * t / m.h ** 2, rtol=1e-10, atol=1e-9 * np.abs(A).max())


def test_rollout_gradients_with_volume_term():
    sc = _volume_scene()
    sc.steps = 3
    E0 = sc.youngs.copy()
    m = om.Model(sc)
    x0, v0 = perturbed_state(m, seed=6)
    cx = W.loss_vector(m.N, 0)
    # forward steps by Newton's method to round-off (Alg. 1 converges slowly with
    # the stiffer volume term; the states are the same)
    L, g = orr.loss_and_grad(m, x0, v0, None, cx, newton=True)
    rng = np.random.default_rng(7)
    d = rng.standard_normal(3 * m.N)
    d[m.fixed] = 0.0
    fd = orr.central_difference(lambda t: orr.rollout_loss(sc, x0 + t * d, v0, None, cx, newton=True), 0.0, 1.0,
                                1e-6)
    assert abs(fd - g["x0"] @ d) <= 2e-5 * abs(fd)
    for e in (0, 7):
        dlog = np.zeros(m.E)
        dlog[e] = 1.0
        f = lambda t: orr.rollout_loss(sc, x0, v0, None, cx, youngs=E0 * np.exp(t * dlog), newton=True)  # noqa: E731
        fd = orr.central_difference(f, 0.0, 1.0, 1e-5)
        an = g["youngs"][e] * E0[e]
        assert abs(fd - an) <= 2e-4 * abs(an) + 1e-9 * np.abs(g["youngs"] * E0).max()
