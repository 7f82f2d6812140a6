"""The multifrontal Cholesky factorization on the device (dense fronts, FP64
MFMA updates) against the host factorization and the oracle: the global
step's solve A^{-1} b (eq:pd_global; Sec. Background: the factorization of A
is computed once and reused) on meshes whose fronts span one tile, several
tiles and ragged tails, every dissection leaf size, a single dense supernode,
linear tetrahedra, muscles and contact candidates, the 64x32x32 block, the
FP32 copies of the mixed path, and a refactorization after new moduli."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import model as om
from parity_helpers import pair, ragged_scene, rel, robot_scene, soa, to_dev

pytestmark = pytest.mark.gpu

SCENES = {
    "ragged_41": ragged_scene,
    "cantilever_16x8x8": lambda: W.cantilever(16, 8, 8, youngs="loguniform", seed=1, steps=2),
    "legged_8x6x4": robot_scene,
    "block_20x12x10": lambda: W.dropped_block(20, 12, 10, steps=2),
    "tet_ball_r4": lambda: W.tet_ball(radius=4.0, steps=2),
}


def _solve_pair(sc, **opts):
    """(device-factor mesh, host-factor mesh, oracle) of one scene."""
    from paper_2101_05917_amd.mesh import Mesh
    gd = Mesh.from_scene(sc, factor_on_host=0, **opts)
    gh = Mesh.from_scene(sc, factor_on_host=1, **opts)
    return gd, gh, om.Model(sc)


def _rhs(o, seed):
    b = np.random.default_rng(seed).standard_normal(3 * o.N)
    b[o.fixed] = 0.0
    return b


@pytest.mark.parametrize("leaf", [64, 256, 0])
@pytest.mark.parametrize("name", list(SCENES))
def test_device_factor_solves_like_host_and_oracle(name, leaf):
    sc = SCENES[name]()
    gd, gh, o = _solve_pair(sc, leaf_nodes=leaf)
    assert gd.info["n_supernodes"] == gh.info["n_supernodes"]
    assert gd.info["factor_us"] > 0
    b = _rhs(o, 11)
    xd = soa(gd.apply_inverse(to_dev(b, o.N)))
    xh = soa(gh.apply_inverse(to_dev(b, o.N)))
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    print(name, leaf, gd.info["n_supernodes"], gd.info["leaf_nodes"], "dev-host", rel(xd, xh), "dev-oracle",
          rel(xd, ref), "us", gd.info["factor_us"], gh.info["factor_us"], flush=True)
    assert rel(xd, xh) <= 1e-12
    assert rel(xd, ref) <= 1e-12
    assert np.all(xd[o.fixed] == 0.0)
    gd.close()
    gh.close()


def test_single_dense_supernode():
    """All free nodes in one supernode (the dense-inverse meshes): one front,
    many block columns, no extend-add."""
    sc = W.cantilever(10, 6, 6, youngs="loguniform", seed=4, steps=2)
    gd, gh, o = _solve_pair(sc, leaf_nodes=100000, fused_cg=0)
    assert gd.info["n_supernodes"] == 1
    b = _rhs(o, 12)
    xd = soa(gd.apply_inverse(to_dev(b, o.N)))
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    assert rel(xd, ref) <= 1e-12
    gd.close()
    gh.close()


def test_full_size_block():
    """The 64x32x32 block (70,785 nodes, 212 k DoFs): the device factor's solve
    against the host factor's and the residual A x - b from the oracle's A."""
    sc = W.config("c5")
    gd, gh, o = _solve_pair(sc)
    b = _rhs(o, 13)
    xd = soa(gd.apply_inverse(to_dev(b, o.N)))
    xh = soa(gh.apply_inverse(to_dev(b, o.N)))
    res = o.A_ff @ xd[o.free] - b[o.free]
    print("c5 dev-host", rel(xd, xh), "residual", np.linalg.norm(res) / np.linalg.norm(b[o.free]),
          "factor ms device", gd.info["factor_us"] / 1e3, "host", gh.info["factor_us"] / 1e3, flush=True)
    assert rel(xd, xh) <= 1e-12
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b[o.free])
    gd.close()
    gh.close()


def test_fp32_copies_and_refactorization():
    """The mixed path's FP32 panels (converted on the device) solve to FP32
    accuracy; new moduli and a refactorization give the new A's solve."""
    sc = W.cantilever(16, 8, 8, youngs="loguniform", seed=5, steps=2)
    g, o = pair(sc, precision="mixed")
    b = _rhs(o, 14)
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    x32 = soa(g.apply_inverse(to_dev(b, o.N), precision="mixed"))
    assert rel(x32, ref) <= 1e-5
    new = 10.0 ** np.random.default_rng(6).uniform(5.0, 7.0, size=len(sc.youngs))
    g.set_youngs(new)
    sc.youngs = new
    o2 = om.Model(sc)
    ref2 = np.zeros(3 * o.N)
    ref2[o2.free] = o2.solve_A(b[o2.free])
    assert rel(ref2, ref) > 1e-3
    x = soa(g.apply_inverse(to_dev(b, o.N)))
    assert rel(x, ref2) <= 1e-12
    x32 = soa(g.apply_inverse(to_dev(b, o.N), precision="mixed"))
    assert rel(x32, ref2) <= 1e-5
    g.close()
