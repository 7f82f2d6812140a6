"""Global step with a contact set (Sec. Contact, Alg. 4) through the C ABI,
against the oracle's reduced solve."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import contact as oc, model as om
from paper_2101_05917_amd import _lib as L
from parity_helpers import pair, rel, robot_scene, soa, to_dev

pytestmark = pytest.mark.gpu


def _candidates(o, rng, n):
    if len(o.contact_nodes):
        return np.asarray(o.contact_nodes, dtype=np.int64)
    return np.sort(rng.choice(np.nonzero(o.free[0::3])[0], n, replace=False))


def _check(g, o, cand, active, rng):
    c = len(active)
    nodes = cand[active]
    xs = rng.standard_normal(3 * c)                      # node-major [c][3]
    b = rng.standard_normal(3 * o.N)
    xs_dev = torch.from_numpy(np.ascontiguousarray(xs.reshape(c, 3).T)).to("cuda:0")
    x = soa(g.contact_solve(active, xs_dev, to_dev(b, o.N)))
    ref = oc.reduced_solve(o, nodes, xs, b)
    keep = o.free.copy()
    cd = (3 * nodes[:, None] + np.arange(3)).reshape(-1)
    keep[cd] = False
    print("c", c, "rel", rel(x[keep], ref[keep]), flush=True)
    assert rel(x[keep], ref[keep]) <= 1e-10
    assert np.array_equal(x[cd], xs)
    assert np.all(x[o.fixed] == 0.0)


@pytest.mark.parametrize("name", ["c1", "robot", "c3"])
def test_contact_solve_matches_reduced_solve(name):
    sc = robot_scene() if name == "robot" else W.config(name)
    g, o = pair(sc)
    rng = np.random.default_rng(71)
    cand = _candidates(o, rng, 40)
    g.contact_prepare(cand)
    n = len(cand)
    sizes = [0, 1, 7, min(n, 120)]
    if n > 33:
        sizes.append(33)
    for c in sizes:                                      # several calls on one handle
        _check(g, o, cand, np.sort(rng.choice(n, c, replace=False)).astype(np.int32), rng)


def test_contact_solve_argument_errors():
    sc = W.config("c1")
    g, o = pair(sc)
    rng = np.random.default_rng(72)
    cand = _candidates(o, rng, 30)
    b = to_dev(np.zeros(3 * o.N), o.N)
    with pytest.raises(L.DiffPDError):
        g.contact_solve([0], torch.zeros(3, 1, dtype=torch.float64, device="cuda:0"), b)  # not prepared
    fixed_node = int(np.nonzero(o.fixed[0::3])[0][0])
    with pytest.raises(L.DiffPDError):
        g.contact_prepare([fixed_node])
    with pytest.raises(L.DiffPDError):
        g.contact_prepare([int(cand[0]), int(cand[0])])
    g.contact_prepare(cand[:5])
    g.contact_prepare(cand)                              # replaces the candidate list
    xs = torch.zeros(3, 2, dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.DiffPDError):
        g.contact_solve([3, 3], xs, b)                   # repeated index
    with pytest.raises(L.DiffPDError):
        g.contact_solve([0, len(cand)], xs, b)           # out of range
    # the handle stays usable after rejected calls
    _check(g, o, cand, np.array([1, 4], np.int32), rng)
    # a new factor discards the cached columns
    g.set_youngs(np.asarray(sc.youngs, dtype=np.float64) * 1.1)   # refactorizes
    with pytest.raises(L.DiffPDError):
        g.contact_solve([1, 4], xs, b)


def test_contact_solve_reuses_the_set_factor():
    """Same set with new right-hand sides (the cached inverse), another set,
    then the first set again: every result matches the oracle."""
    sc = robot_scene()
    g, o = pair(sc)
    rng = np.random.default_rng(74)
    cand = _candidates(o, rng, 40)
    g.contact_prepare(cand)
    s1 = np.sort(rng.choice(len(cand), 17, replace=False)).astype(np.int32)
    s2 = np.sort(rng.choice(len(cand), 9, replace=False)).astype(np.int32)
    for act in (s1, s1, s2, s1, s1):
        _check(g, o, cand, act, rng)


def test_contact_solve_full_size_block():
    """The 64x32x32 dropped block, its 2145 ground-contact candidates and 120
    of them active: the oracle's assembled A (no factorization) finds the
    reduced system solved and x_C = x*."""
    from paper_2101_05917_amd.mesh import Mesh
    sc = W.config("c5")
    g = Mesh.from_scene(sc)
    o = om.Model(sc)
    cand = np.asarray(o.contact_nodes, dtype=np.int64)
    g.contact_prepare(cand)
    rng = np.random.default_rng(73)
    active = np.sort(rng.choice(len(cand), 120, replace=False)).astype(np.int32)
    nodes = cand[active]
    xs = rng.standard_normal(3 * 120) * 1e-3
    b = rng.standard_normal(3 * o.N)
    xs_dev = torch.from_numpy(np.ascontiguousarray(xs.reshape(120, 3).T)).to("cuda:0")
    x = soa(g.contact_solve(active, xs_dev, to_dev(b, o.N)))
    cd = (3 * nodes[:, None] + np.arange(3)).reshape(-1)
    keep = o.free.copy()
    keep[cd] = False
    assert np.array_equal(x[cd], xs)
    A = o.A.tocsr()
    res = A[keep][:, keep] @ x[keep] - b[keep]
    print("residual", np.linalg.norm(res) / np.linalg.norm(b[keep]), flush=True)
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(b[keep])
