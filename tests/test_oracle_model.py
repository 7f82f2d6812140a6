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


def _contact_scene(mu, k=None):
    sc = tiny_robot()
    sc.friction_mu = mu
    if k is not None:
        sc.contact_k = k
    return sc


def _penalty_normal_force(with_ground, without_ground, x, j, eps=1e-9):
    """Upward force of the ground penalty on node j, -dE_ground/dz_j, by central
    differences of the energy difference between the scene with and without
    the ground term (independent of the friction code)."""
    d = np.zeros(3 * with_ground.N)
    d[3 * j + 2] = eps
    e = lambda xx: with_ground.elastic_energy(xx) - without_ground.elastic_energy(xx)  # noqa: E731
    return -(e(x + d) - e(x - d)) / (2 * eps)


def test_friction_force_opposes_tangential_velocity_and_obeys_coulomb_bound():
    """Regularised Coulomb friction on the ground-contact nodes: horizontal,
    antiparallel to the horizontal velocity, its magnitude never above mu times
    the penalty's normal force, reaching that bound when |v_t| >> eps and
    vanishing with v_t, off contact (z >= 0) and for mu = 0."""
    mu = 0.5
    m = om.Model(_contact_scene(mu))
    bare = om.Model(_contact_scene(mu, k=0.0))
    rng = np.random.default_rng(11)
    x, v = perturbed_state(m, seed=4)
    cn = m.contact_nodes
    x[3 * cn + 2] = -rng.uniform(1e-4, 1e-3, size=len(cn))        # in contact ...
    x[3 * cn[:3] + 2] = np.array([0.0, 1e-4, 3e-3])               # ... but three
    v[3 * cn] = rng.standard_normal(len(cn))
    v[3 * cn + 1] = rng.standard_normal(len(cn))
    f = m.friction_force(x, v)
    other = np.setdiff1d(np.arange(m.N), cn)
    assert np.all(f[3 * other] == 0) and np.all(f[3 * other + 1] == 0)
    assert np.all(f[2::3] == 0)                                   # no normal component
    for j in cn:
        ft = f[3 * j:3 * j + 2]
        vt = v[3 * j:3 * j + 2]
        fn = _penalty_normal_force(m, bare, x, j)
        if x[3 * j + 2] >= 0:
            assert abs(fn) <= 1e-6 and np.all(ft == 0), j
            continue
        assert fn > 0
        cross = ft[0] * vt[1] - ft[1] * vt[0]
        assert abs(cross) <= 1e-12 * np.linalg.norm(ft) * np.linalg.norm(vt)   # parallel ...
        assert ft @ vt < 0                                                      # ... and opposed
        assert np.linalg.norm(ft) <= mu * fn * (1 + 1e-5)
    # the Coulomb limit |f_t| -> mu f_n when |v_t| >> eps, and |f_t| -> 0 with v_t
    j = cn[5]
    fn = _penalty_normal_force(m, bare, x, j)
    for speed, lo, hi in ((1e3 * m.friction_eps, 1 - 1e-5, 1 + 1e-5), (1e-6 * m.friction_eps, 0, 2e-6)):
        vv = v.copy()
        vv[3 * j:3 * j + 2] = speed * np.array([0.6, -0.8])
        ratio = np.linalg.norm(m.friction_force(x, vv)[3 * j:3 * j + 2]) / (mu * fn)
        assert lo <= ratio <= hi, (speed, ratio)
    # mu = 0: no friction at all
    m0 = om.Model(_contact_scene(0.0))
    assert np.all(m0.friction_force(x, v) == 0)

def test_friction_force_vjp_matches_central_differences():
    """(w^T df/dx, w^T df/dv) of the explicit friction against central
    differences of the friction force itself."""
    m = om.Model(_contact_scene(0.5))
    x, v = perturbed_state(m, seed=7)
    cn = m.contact_nodes
    x[3 * cn + 2] = -np.random.default_rng(2).uniform(2e-4, 1e-3, size=len(cn))
    w = np.random.default_rng(3).standard_normal(3 * m.N)
    gx, gv = m.friction_vjp(x, v, w)
    eps = 1e-8
    for d_seed in range(3):
        d = np.random.default_rng(20 + d_seed).standard_normal(3 * m.N) * 1e-2
        fdx = (m.friction_force(x + eps * d, v) - m.friction_force(x - eps * d, v)) @ w / (2 * eps)
        fdv = (m.friction_force(x, v + eps * d) - m.friction_force(x, v - eps * d)) @ w / (2 * eps)
        assert abs(fdx - gx @ d) <= 1e-6 * (abs(fdx) + 1e-12)
        assert abs(fdv - gv @ d) <= 1e-6 * (abs(fdv) + 1e-12)
