"""grad g and the Hessian split of the oracle, against central differences of g."""
import numpy as np

from oracle import model as om
from oracle_scenes import tiny_robot, tiny_cantilever, perturbed_state


def _check_grad_and_hessian(sc, act=None, seed=0):
    m = om.Model(sc)
    x, v = perturbed_state(m, seed=seed)
    # keep contact heights away from the kink at z = 0
    for j in m.contact_nodes:
        if abs(x[3 * j + 2]) < 2e-4:
            x[3 * j + 2] -= 5e-4
    y = m.y_of(x, v)
    gr = m.grad_g(x, y, act)
    rng = np.random.default_rng(seed + 1)
    eps = 1e-7
    for _ in range(4):
        d = rng.standard_normal(3 * m.N)
        fd = (m.g(x + eps * d, y, act) - m.g(x - eps * d, y, act)) / (2 * eps)
        assert abs(fd - gr @ d) <= 1e-6 * (abs(gr @ d) + np.linalg.norm(gr) * np.linalg.norm(d) * 1e-3)
    H = m.hessian(x, act)
    for _ in range(4):
        d = rng.standard_normal(3 * m.N)
        fd = (m.grad_g(x + eps * d, y, act) - m.grad_g(x - eps * d, y, act)) / (2 * eps)
        assert np.linalg.norm(fd - H @ d) <= 1e-6 * np.linalg.norm(H @ d)
    return m


def test_grad_and_hessian_corotated_dirichlet():
    _check_grad_and_hessian(tiny_cantilever(youngs=10 ** np.linspace(5, 7, 12)))


def test_grad_and_hessian_muscle_contact():
    sc = tiny_robot()
    act = np.random.default_rng(3).uniform(0, 1, size=sc.n_elements)
    m = _check_grad_and_hessian(sc, act=act)
    assert len(m.contact_nodes) > 0 and m.Gm is not None
