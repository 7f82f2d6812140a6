"""Pins of the oracle's projections against library routines and closed forms."""
import numpy as np
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import projections as P


def _rand_F(rng, n, det_sign=1):
    F = np.eye(3)[None] + 0.4 * rng.standard_normal((n, 3, 3))
    d = np.linalg.det(F)
    flip = np.sign(d) != det_sign
    F[flip, :, 0] *= -1
    return F


def test_polar_matches_scipy():
    rng = np.random.default_rng(0)
    F = _rand_F(rng, 200)
    R = P.closest_rotation(F)
    for k in range(len(F)):
        U, _ = scipy.linalg.polar(F[k])
        assert np.abs(R[k] - U).max() < 1e-13


def test_rotation_properties_including_inverted():
    rng = np.random.default_rng(1)
    for sgn in (1, -1):
        F = _rand_F(rng, 100, sgn)
        R = P.closest_rotation(F)
        RtR = np.swapaxes(R, 1, 2) @ R
        assert np.abs(RtR - np.eye(3)).max() < 1e-13
        assert np.abs(np.linalg.det(R) - 1).max() < 1e-13


def test_closest_rotation_is_optimal_for_inverted_F():
    # brute force: no sampled rotation is closer to F than R (det F < 0 reading)
    rng = np.random.default_rng(2)
    F = _rand_F(rng, 20, -1)
    R = P.closest_rotation(F)
    samples = Rotation.random(20000, random_state=3).as_matrix()
    for k in range(len(F)):
        best = np.linalg.norm(F[k] - R[k])
        d = np.linalg.norm(F[k][None] - samples, axis=(1, 2))
        assert d.min() >= best - 1e-12
        # local refinement around R cannot improve either
        for _ in range(50):
            w = 1e-3 * rng.standard_normal(3)
            Rp = R[k] @ Rotation.from_rotvec(w).as_matrix()
            assert np.linalg.norm(F[k] - Rp) >= best - 1e-14


def test_rotation_equivariance_and_spd():
    rng = np.random.default_rng(4)
    F = _rand_F(rng, 50)
    Q = Rotation.random(50, random_state=5).as_matrix()
    assert np.abs(P.closest_rotation(Q @ F) - Q @ P.closest_rotation(F)).max() < 1e-12
    A = rng.standard_normal((50, 3, 3))
    S = np.swapaxes(A, 1, 2) @ A + 0.1 * np.eye(3)
    assert np.abs(P.closest_rotation(S) - np.eye(3)).max() < 1e-12


def test_rotation_differential_identity_closed_form():
    rng = np.random.default_rng(6)
    dF = rng.standard_normal((30, 3, 3))
    I = np.broadcast_to(np.eye(3), dF.shape).copy()
    dR = P.rotation_differential(I, I, dF)
    assert np.abs(dR - 0.5 * (dF - np.swapaxes(dF, 1, 2))).max() < 1e-14


def test_rotation_differential_finite_difference_and_symmetry():
    rng = np.random.default_rng(7)
    F = _rand_F(rng, 40)
    R = P.closest_rotation(F)
    dF = rng.standard_normal(F.shape)
    eps = 1e-6
    fd = (P.closest_rotation(F + eps * dF) - P.closest_rotation(F - eps * dF)) / (2 * eps)
    an = P.rotation_differential(F, R, dF)
    assert np.abs(fd - an).max() < 1e-7
    B = rng.standard_normal(F.shape)
    lhs = np.sum(B * P.rotation_differential(F, R, dF), axis=(1, 2))
    rhs = np.sum(dF * P.rotation_differential(F, R, B), axis=(1, 2))
    assert np.abs(lhs - rhs).max() < 1e-12
    # positive semidefinite for det F > 0
    J = P.rotation_jacobian(F)
    ev = np.linalg.eigvalsh(0.5 * (J + np.swapaxes(J, 1, 2)))
    assert ev.min() > -1e-12


def test_sphere_and_ground_projections():
    rng = np.random.default_rng(8)
    f = rng.standard_normal((30, 3))
    r = rng.uniform(0, 1, 30)
    p = P.sphere_projection(f, r, np.array([1.0, 0, 0]))
    assert np.allclose(np.linalg.norm(p, axis=1), r)
    assert np.allclose(np.cross(p, f), 0, atol=1e-14)
    eps = 1e-7
    J = P.sphere_jacobian(f, r)
    for c in range(3):
        d = np.zeros(3)
        d[c] = eps
        fd = (P.sphere_projection(f + d, r, np.array([1.0, 0, 0]))
              - P.sphere_projection(f - d, r, np.array([1.0, 0, 0]))) / (2 * eps)
        assert np.abs(fd - J[:, :, c]).max() < 1e-6
    xc = rng.standard_normal((20, 3))
    g = P.ground_projection(xc)
    assert np.all(g[:, 2] >= 0) and np.array_equal(g[:, :2], xc[:, :2])
    assert np.array_equal(P.ground_jacobian(xc)[:, 2], (xc[:, 2] >= 0).astype(float))
