"""GPU path (through the C ABI) against the FP64 oracle, element by element."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import forward as of, adjoint as oa, projections as op
from parity_helpers import soa, to_dev, elem_dev, pair, rel, robot_scene, ragged_scene

pytestmark = pytest.mark.gpu

SCENES = {
    "c1": lambda: W.config("c1"),
    "c2": lambda: W.config("c2"),
    "robot": robot_scene,
    "ragged": ragged_scene,
}


def converged_state(o, x, v, act=None):
    """The implicit-Euler solution for the start state: Newton on g to round-off."""
    xr, info = of.newton_solve(o, o.y_of(x, v), act)
    return xr


def _perturbed(o, scale=2e-3, seed=0):
    rng = np.random.default_rng(seed)
    x = o.X + scale * rng.standard_normal(3 * o.N)
    x[o.fixed] = o.X[o.fixed]
    v = 0.05 * rng.standard_normal(3 * o.N)
    v[o.fixed] = 0.0
    return x, v


@pytest.mark.parametrize("name", list(SCENES))
def test_mesh_numbering_and_rest_positions(name):
    sc = SCENES[name]()
    g, o = pair(sc)
    print(name, g.info, flush=True)
    assert np.array_equal(g.node_ijk(), o.mesh.node_ijk)
    assert np.abs(soa(g.rest_positions()) - o.X).max() == 0.0
    if len(o.contact_nodes):
        assert np.array_equal(np.sort(g.contact_nodes()), o.contact_nodes)


@pytest.mark.parametrize("name", list(SCENES))
def test_apply_inverse(name):
    sc = SCENES[name]()
    g, o = pair(sc)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(3 * o.N)
    x = soa(g.apply_inverse(to_dev(b, o.N)))
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    assert rel(x, ref) <= 1e-12
    assert np.all(x[o.fixed] == 0.0)


@pytest.mark.parametrize("name", ["c1", "robot", "ragged"])
def test_rotations(name):
    sc = SCENES[name]()
    g, o = pair(sc)
    x, _ = _perturbed(o, scale=3e-3)
    R = g.rotations(to_dev(x, o.N)).cpu().numpy()          # [9, Q]
    Rref = op.closest_rotation(o.deformation_gradients(x)).reshape(o.Q, 9).T
    assert np.abs(R - Rref).max() <= 1e-13


@pytest.mark.parametrize("name", list(SCENES))
def test_gradient_and_hessian(name):
    sc = SCENES[name]()
    g, o = pair(sc)
    x, v = _perturbed(o, seed=2)
    y = o.y_of(x, v)
    act = None
    if o.Gm is not None:
        act = np.random.default_rng(3).uniform(0, 1, o.E)
    a_dev = None if act is None else elem_dev(act)
    r = soa(g.gradient(to_dev(x, o.N), to_dev(y, o.N), a_dev))
    ref = o.grad_g(x, y, act)
    ref[o.fixed] = 0.0
    assert rel(r, ref) <= 1e-11
    p = np.random.default_rng(4).standard_normal(3 * o.N)
    p[o.fixed] = 0.0
    hp = soa(g.hessian_apply(to_dev(x, o.N), to_dev(p, o.N), a_dev))
    ref = o.hessian(x, act) @ p
    ref[o.fixed] = 0.0
    assert rel(hp, ref) <= 1e-11


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_forward_fixed_iterations(name):
    """Same algorithm, same number of global solves (100)."""
    sc = SCENES[name]()
    g, o = pair(sc, fwd_max_iter=100, fwd_fixed_iters=1)
    x, v = _perturbed(o, seed=5)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N))
    assert st["fwd_iters"] == 100
    xr, vr, info = of.pd_step(o, x, v, max_iter=100, fixed_iters=True)
    assert info["iters"] == 100
    assert rel(soa(xn), xr) <= 1e-12
    assert np.linalg.norm(soa(xn) - xr) <= 1e-9 * np.linalg.norm(xr - x)
    assert rel(soa(vn), vr) <= 1e-9


@pytest.mark.parametrize("solver", ["pd", "newton_pcg"])
@pytest.mark.parametrize("name", ["c1", "c2", "robot"])
def test_forward_converged(name, solver):
    sc = SCENES[name]()
    g, o = pair(sc, fwd_solver=solver, fwd_max_iter=100000, fwd_rel_tol=1e-13, check_every=64)
    x, v = o.X.copy(), np.zeros(3 * o.N)
    act = None
    if o.Gm is not None:
        act = np.random.default_rng(6).uniform(0, 1, o.E)
        v[0::3] = 0.05
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N),
                                None if act is None else elem_dev(act))
    print(name, st, flush=True)
    assert st["converged"] == 1
    xr = converged_state(o, x, v, act)
    assert np.linalg.norm(soa(xn) - xr) <= 1e-9 * np.linalg.norm(xr - x)


@pytest.mark.parametrize("solver", ["pcg", "fixed_point"])
@pytest.mark.parametrize("name", ["c1", "robot", "ragged"])
def test_backward_step(name, solver):
    sc = SCENES[name]()
    g, o = pair(sc, bwd_solver=solver, bwd_max_iter=100000, bwd_rel_tol=1e-13, check_every=64)
    x, v = _perturbed(o, seed=7)
    act = None if o.Gm is None else np.random.default_rng(8).uniform(0, 1, o.E)
    a_dev = None if act is None else elem_dev(act)
    xr = converged_state(o, x, v, act)
    rng = np.random.default_rng(9)
    gxn, gvn = rng.standard_normal(3 * o.N), rng.standard_normal(3 * o.N)
    gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gx, gv, ga, st = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev, to_dev(xr, o.N),
                                     to_dev(gxn, o.N), to_dev(gvn, o.N), g_youngs=gE,
                                     want_act=act is not None)
    print(name, solver, st, flush=True)
    assert st["converged"] == 1
    rx, rv, rE, ra, _ = oa.backward_step(o, x, v, act, xr, gxn, gvn, solver="direct")
    assert rel(soa(gx), rx) <= 1e-8
    assert rel(soa(gv), rv) <= 1e-8
    assert rel(gE.cpu().numpy(), rE) <= 1e-8
    if act is not None:
        assert rel(ga.cpu().numpy(), ra) <= 1e-8


@pytest.mark.parametrize("name", ["c2", "robot"])
def test_mixed_precision_forward_and_backward(name):
    """FP32 panels inside FP64 residual corrections: same converged state."""
    sc = SCENES[name]()
    g, o = pair(sc, precision="mixed", fwd_solver="newton_pcg", fwd_max_iter=100000,
                fwd_rel_tol=1e-12, bwd_rel_tol=1e-12, bwd_max_iter=100000, check_every=32)
    x, v = _perturbed(o, seed=11)
    act = None if o.Gm is None else np.random.default_rng(12).uniform(0, 1, o.E)
    a_dev = None if act is None else elem_dev(act)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev)
    print(name, "mixed fwd", st, flush=True)
    xr = converged_state(o, x, v, act)
    err_x = np.linalg.norm(soa(xn) - xr) / np.linalg.norm(xr - x)
    assert err_x <= 1e-5
    gxn = np.random.default_rng(13).standard_normal(3 * o.N)
    gE = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gx, gv, ga, bst = g.backward_step(to_dev(x, o.N), to_dev(v, o.N), a_dev, to_dev(xr, o.N),
                                      to_dev(gxn, o.N), to_dev(np.zeros(3 * o.N), o.N), g_youngs=gE)
    print(name, "mixed bwd", bst, flush=True)
    rx, rv, rE, ra, _ = oa.backward_step(o, x, v, act, xr, gxn, np.zeros(3 * o.N), solver="direct")
    assert rel(soa(gx), rx) <= 1e-6
    assert rel(gE.cpu().numpy(), rE) <= 1e-6
    # mixed-precision solve alone: FP32 panels, error at single-precision level
    b = np.random.default_rng(14).standard_normal(3 * o.N)
    xs = soa(g.apply_inverse(to_dev(b, o.N), precision="mixed"))
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    assert 1e-12 < rel(xs, ref) <= 1e-4


def test_rest_state_converges_immediately():
    """Zero residual at x^0: the stopping test's absolute floor ends the step."""
    sc = W.config("c1")
    sc.gravity = (0.0, 0.0, 0.0)
    g, o = pair(sc, fwd_solver="newton_pcg")
    X = g.rest_positions()
    xn, vn, st = g.forward_step(X, torch.zeros_like(X))
    assert st["converged"] == 1 and st["fwd_iters"] == 0
    assert torch.equal(xn, X) and float(vn.abs().max()) == 0.0


def test_single_voxel_free_fall_is_exact():
    sc = W.dropped_block(1, 1, 1, steps=1)
    sc.contact_k = 0.0
    g, o = pair(sc)
    X = g.rest_positions()
    v = torch.zeros_like(X)
    v[0] = 0.3
    xn, vn, st = g.forward_step(X, v)
    expect = X.clone()
    expect[0] += 0.01 * 0.3
    expect[2] += 1e-4 * -9.81
    assert float((xn - expect).abs().max()) <= 1e-15


@pytest.mark.parametrize("name", ["c1", "robot"])
def test_graph_replay_equals_direct_launches(name):
    """Captured conjugate-gradient iterations give bitwise the result of direct
    launches, over many replays with eager work and syncs in between."""
    sc = SCENES[name]()
    g1, o = pair(sc, fwd_solver="newton_pcg", use_graphs=1, fused_cg=0, fwd_rel_tol=1e-12,
                 bwd_rel_tol=1e-12, fwd_max_iter=100000, bwd_max_iter=100000)
    g0, _ = pair(sc, fwd_solver="newton_pcg", use_graphs=0, fused_cg=0, fwd_rel_tol=1e-12,
                 bwd_rel_tol=1e-12, fwd_max_iter=100000, bwd_max_iter=100000)
    act = None if o.Gm is None else elem_dev(np.random.default_rng(3).uniform(0, 1, o.E))
    for seed in range(3):
        x, v = _perturbed(o, seed=20 + seed)
        xd, vd = to_dev(x, o.N), to_dev(v, o.N)
        a1 = g1.forward_step(xd, vd, act)
        a0 = g0.forward_step(xd, vd, act)
        assert torch.equal(a1[0], a0[0]) and a1[2]["fwd_iters"] == a0[2]["fwd_iters"]
        gxn = to_dev(np.random.default_rng(seed).standard_normal(3 * o.N), o.N)
        b1 = g1.backward_step(xd, vd, act, a1[0], gxn, torch.zeros_like(gxn))
        b0 = g0.backward_step(xd, vd, act, a0[0], gxn, torch.zeros_like(gxn))
        assert torch.equal(b1[0], b0[0]) and torch.equal(b1[1], b0[1])
        torch.cuda.synchronize()


def wide_beam():
    """2016 free nodes: the largest dense size, where r and q no longer fit in
    LDS next to the element tile and go through device memory."""
    return W.cantilever(14, 11, 11, youngs="loguniform", seed=5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["c1", "c2", "robot", "ragged", "wide"])
def test_fused_dense_cg_matches_multilaunch_and_oracle(name, precision):
    """The one-launch dense solver and the level-scheduled multi-launch solver
    run the same preconditioned iteration: same converged states, both at the
    oracle's, and the same iteration counts up to rounding."""
    sc = wide_beam() if name == "wide" else SCENES[name]()
    kw = dict(precision=precision, fwd_solver="newton_pcg", fwd_rel_tol=1e-12, bwd_rel_tol=1e-12,
              fwd_max_iter=100000, bwd_max_iter=100000, check_every=16)
    g1, o = pair(sc, fused_cg=1, **kw)
    g0, _ = pair(sc, fused_cg=0, **kw)
    print(name, precision, g1.info, flush=True)
    assert g1.info["fused_blocks"] > 0 and g0.info["fused_blocks"] == 0
    x, v = _perturbed(o, seed=31)
    act = None if o.Gm is None else np.random.default_rng(32).uniform(0, 1, o.E)
    a_dev = None if act is None else elem_dev(act)
    xd, vd = to_dev(x, o.N), to_dev(v, o.N)
    x1, _, s1 = g1.forward_step(xd, vd, a_dev)
    x0, _, s0 = g0.forward_step(xd, vd, a_dev)
    print("fwd", s1, s0, flush=True)
    assert s1["converged"] == 1 and s0["converged"] == 1
    xr = converged_state(o, x, v, act)
    tol_x = 1e-9 if precision == "fp64" else 1e-5
    for xn in (x1, x0):
        assert np.linalg.norm(soa(xn) - xr) <= tol_x * np.linalg.norm(xr - x)
    rng = np.random.default_rng(33)
    gxn, gvn = rng.standard_normal(3 * o.N), rng.standard_normal(3 * o.N)
    gE1 = torch.zeros(o.E, dtype=torch.float64, device="cuda:0")
    gE0 = torch.zeros_like(gE1)
    xrd = to_dev(xr, o.N)
    b1 = g1.backward_step(xd, vd, a_dev, xrd, to_dev(gxn, o.N), to_dev(gvn, o.N), g_youngs=gE1,
                          want_act=act is not None)
    b0 = g0.backward_step(xd, vd, a_dev, xrd, to_dev(gxn, o.N), to_dev(gvn, o.N), g_youngs=gE0,
                          want_act=act is not None)
    print("bwd", b1[3], b0[3], flush=True)
    assert b1[3]["converged"] == 1 and b0[3]["converged"] == 1
    assert abs(b1[3]["bwd_iters"] - b0[3]["bwd_iters"]) <= 2
    rx, rv, rE, ra, _ = oa.backward_step(o, x, v, act, xr, gxn, gvn, solver="direct")
    tol_g = 1e-8 if precision == "fp64" else 1e-6
    for gx, gE in ((b1[0], gE1), (b0[0], gE0)):
        assert rel(soa(gx), rx) <= tol_g
        assert rel(gE.cpu().numpy(), rE) <= tol_g
    assert rel(soa(b1[0]), soa(b0[0])) <= (1e-10 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("name", ["c1", "robot"])
def test_fused_dense_cg_iteration_cap(name):
    """With the iteration cap reached, both solvers stop after exactly that many
    updates, report no convergence and agree on the partial solution."""
    sc = SCENES[name]()
    kw = dict(bwd_rel_tol=1e-14, bwd_max_iter=3, check_every=1)
    g1, o = pair(sc, fused_cg=1, **kw)
    g0, _ = pair(sc, fused_cg=0, **kw)
    assert g1.info["fused_blocks"] > 0
    x, v = _perturbed(o, seed=41)
    act = None if o.Gm is None else elem_dev(np.random.default_rng(42).uniform(0, 1, o.E))
    xd, vd = to_dev(x, o.N), to_dev(v, o.N)
    gxn = to_dev(np.random.default_rng(43).standard_normal(3 * o.N), o.N)
    zero = torch.zeros_like(gxn)
    r1 = g1.backward_step(xd, vd, act, xd, gxn, zero)
    r0 = g0.backward_step(xd, vd, act, xd, gxn, zero)
    print(r1[3], r0[3], flush=True)
    assert r1[3]["bwd_iters"] == 3 and r0[3]["bwd_iters"] == 3
    assert r1[3]["converged"] == 0 and r0[3]["converged"] == 0
    assert rel(soa(r1[0]), soa(r0[0])) <= 1e-11


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_dense_cg_lds_placements_agree_bitwise(precision):
    """Where the vectors and the rows of A^{-1} are read from (LDS or device
    memory) does not change the arithmetic: all four placements give the
    same bits."""
    sc = SCENES["robot"]()
    kw = dict(precision=precision, fwd_solver="newton_pcg", fwd_rel_tol=1e-10, bwd_rel_tol=1e-10,
              fwd_max_iter=100000, bwd_max_iter=100000)
    o = None
    out = []
    for mode in range(4):
        g, o = pair(sc, fused_cg=2 + mode, **kw)
        lds = g.info["fused_lds"] >> (2 if precision == "mixed" else 0) & 3
        print(mode, g.info["fused_blocks"], lds, flush=True)
        assert g.info["fused_blocks"] > 0 and lds == mode
        x, v = _perturbed(o, seed=51)
        act = elem_dev(np.random.default_rng(52).uniform(0, 1, o.E))
        xd, vd = to_dev(x, o.N), to_dev(v, o.N)
        xn, _, st = g.forward_step(xd, vd, act)
        gxn = to_dev(np.random.default_rng(53).standard_normal(3 * o.N), o.N)
        gx, gv, _, bst = g.backward_step(xd, vd, act, xn, gxn, torch.zeros_like(gxn))
        out.append((xn, gx, st["fwd_iters"], bst["bwd_iters"]))
    for xn, gx, fi, bi in out[1:]:
        assert torch.equal(xn, out[0][0]) and torch.equal(gx, out[0][1])
        assert fi == out[0][2] and bi == out[0][3]


@pytest.mark.parametrize("name", ["c1", "robot"])
def test_mixed_local_step_rotations(name):
    """Mixed precision: FP32 q-method rotations polished by one FP64 Newton step
    agree with the oracle's SVD polar decomposition to FP64 round-off."""
    sc = SCENES[name]()
    g, o = pair(sc, precision="mixed")
    x, _ = _perturbed(o, scale=3e-3, seed=61)
    R = g.rotations(to_dev(x, o.N)).cpu().numpy()          # [9, Q]
    Rref = op.closest_rotation(o.deformation_gradients(x)).reshape(o.Q, 9).T
    err = np.abs(R - Rref).max()
    print(name, err, flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("name", ["c1", "robot"])
def test_forward_newton_eisenstat_walker(name):
    """Adaptive inner tolerances (Eisenstat-Walker forcing terms) reach the same
    converged implicit-Euler state."""
    sc = SCENES[name]()
    g, o = pair(sc, fwd_solver="newton_pcg", fwd_inner_tol=-0.1, fwd_max_iter=100000,
                fwd_rel_tol=1e-13, check_every=64)
    x, v = _perturbed(o, seed=71)
    act = None if o.Gm is None else np.random.default_rng(72).uniform(0, 1, o.E)
    xn, vn, st = g.forward_step(to_dev(x, o.N), to_dev(v, o.N), None if act is None else elem_dev(act))
    print(name, st, flush=True)
    assert st["converged"] == 1
    xr = converged_state(o, x, v, act)
    assert np.linalg.norm(soa(xn) - xr) <= 1e-9 * np.linalg.norm(xr - x)


@pytest.mark.parametrize("fused", [0, 1])
def test_profiling_leaves_results_unchanged_and_times_every_class(fused):
    """Kernel timing (device clocks in the kernels, events around solves)
    changes no result bit, and every class that ran reports a plausible
    per-launch duration and nonzero algorithmic bytes."""
    sc = wide_beam()
    kw = dict(fwd_solver="newton_pcg", fused_cg=fused, fwd_rel_tol=1e-10, bwd_rel_tol=1e-10,
              fwd_max_iter=100000, bwd_max_iter=100000)
    g, o = pair(sc, **kw)
    x, v = _perturbed(o, seed=41)
    xd, vd = to_dev(x, o.N), to_dev(v, o.N)
    gxn = to_dev(np.random.default_rng(41).standard_normal(3 * o.N), o.N)
    ref_f = g.forward_step(xd, vd, None)
    ref_b = g.backward_step(xd, vd, None, ref_f[0], gxn, torch.zeros_like(gxn))
    classes = ["sweep_fwd", "sweep_fwd_wide", "sweep_bwd", "sweep_bwd_narrow", "elem_hvp", "elem_forces",
               "solve", "cg_dense"]
    ran = {}
    for cls in classes:
        g.profile_start(cls)
        f = g.forward_step(xd, vd, None)
        b = g.backward_step(xd, vd, None, f[0], gxn, torch.zeros_like(gxn))
        prof = g.profile_read()
        print(cls, prof, flush=True)
        assert torch.equal(f[0], ref_f[0]) and torch.equal(b[0], ref_b[0]) and torch.equal(b[1], ref_b[1])
        if prof["launches"]:
            us = 1e3 * prof["total_ms"] / prof["launches"]
            assert 0.2 < us < 1e5, (cls, us)
            assert prof["bytes"] > 0
        ran[cls] = prof["launches"]
    assert ran["elem_forces"] > 0 and ran["elem_hvp"] + ran["cg_dense"] > 0
    if fused:
        assert ran["cg_dense"] > 0
    else:
        assert ran["solve"] > 0
        assert sum(ran[c] for c in classes if c.startswith("sweep")) > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_inverted_elements_rotations_and_gradient(precision):
    """Strongly perturbed state with many inverted Gauss points (det F <= 0):
    the closest proper rotation (the Newton polar iteration hands over to the
    q-method there) and grad g agree with the oracle's SVD-based projection."""
    sc = W.config("c1")
    g, o = pair(sc, precision=precision)
    rng = np.random.default_rng(61)
    x = o.X + 0.6 * sc.dx * rng.standard_normal(3 * o.N)
    F = o.deformation_gradients(x)
    det = np.linalg.det(F)
    print("inverted", int((det <= 0).sum()), "of", o.Q, flush=True)
    assert (det <= 0).sum() >= o.Q // 10
    R = g.rotations(to_dev(x, o.N)).cpu().numpy()
    Rref = op.closest_rotation(F).reshape(o.Q, 9).T
    # compare where the projection is well conditioned: the two singular
    # values that decide it (the two smallest when det F <= 0) are apart
    s = np.linalg.svd(F, compute_uv=False)
    gap = np.where(det > 0, s[:, 1] + s[:, 2], s[:, 1] - s[:, 2]) / s[:, 0]
    ok = gap > 1e-2
    assert ok.sum() >= o.Q // 2
    assert np.abs(R - Rref)[:, ok].max() <= 1e-10
    Rq = R.T.reshape(-1, 3, 3)                      # every Gauss point: a proper rotation
    assert np.abs(Rq @ Rq.transpose(0, 2, 1) - np.eye(3)).max() <= 1e-12
    assert np.abs(np.linalg.det(Rq) - 1.0).max() <= 1e-12
    v = np.zeros(3 * o.N)
    y = o.y_of(x, v)
    r = soa(g.gradient(to_dev(x, o.N), to_dev(y, o.N)))
    ref = o.grad_g(x, y)
    ref[o.fixed] = 0.0
    print("gradient rel", rel(r, ref), flush=True)
    assert rel(r, ref) <= 1e-6


@pytest.mark.parametrize("name", ["c1", "robot"])
def test_spectral_radius_matches_oracle(name):
    """Lanczos estimate of rho(A^{-1} dA) from the library's solve and Hessian
    product against the oracle's dense eigenvalues (eq:sp_radius)."""
    sc = SCENES[name]()
    g, o = pair(sc)
    x, v = _perturbed(o, seed=3)
    act = np.random.default_rng(2).uniform(0, 1, o.E) if o.muscle_k > 0 else None
    xr = converged_state(o, x, v, act)
    rho = g.spectral_radius(to_dev(xr, o.N), None if act is None else elem_dev(act), steps=60)
    ref = oa.spectral_radius(o, xr, act)
    print(name, "rho", rho, "oracle", ref, flush=True)
    assert abs(rho - ref) <= 1e-8 * ref
