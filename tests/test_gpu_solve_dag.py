"""The single-launch solve (both triangular sweeps in one launch, tasks
waiting on the tasks they depend on) against the per-level launches: the
same arithmetic, so the same bits, solve after solve (its counters are reset
by the launch itself); in whole time steps (conjugate-gradient iterations
replayed as HIP graphs) the same bits as well; and against the oracle."""
import numpy as np
import pytest
import torch

import bench
import workloads as W
from parity_helpers import soa, to_dev, pair, rel, robot_scene, ragged_scene

pytestmark = pytest.mark.gpu

SCENES = {
    "c1": lambda: W.config("c1"),
    "robot": robot_scene,
    "ragged": ragged_scene,
    "c2": lambda: W.config("c2"),
    "block_16x8x8": lambda: W.dropped_block(16, 8, 8, steps=1),
    "block_64x32x32": lambda: W.config("c5"),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_single_launch_solve_equals_level_launches(name):
    sc = SCENES[name]()
    g, o = pair(sc, precision="mixed", sweep_launch=0)
    print(name, "entries", g.info["solve_entries"], "workgroups", g.info["solve_workgroups"], flush=True)
    assert g.info["solve_workgroups"] > 0
    rng = np.random.default_rng(5)
    for precision in ("fp64", "mixed"):
        bs = [to_dev(rng.standard_normal(3 * o.N), o.N) for _ in range(3)]
        g.set_options(sweep_launch=0)
        ref = [g.apply_inverse(b, precision=precision) for b in bs]
        g.set_options(sweep_launch=1)
        for rep in range(2):
            got = [g.apply_inverse(b, precision=precision) for b in bs]
            torch.cuda.synchronize()
            for a, r in zip(got, ref):
                assert torch.equal(a, r), (precision, rep)
        if precision == "fp64" and o.N * 3 < 60000:
            b = soa(bs[0])
            x = np.zeros(3 * o.N)
            x[o.free] = o.solve_A(b[o.free])
            assert rel(soa(got[0]), x) <= 1e-12
    g.close()


def test_single_launch_solve_in_time_steps():
    """Three forward and backward steps of the 64x32x32 block with bench.py's
    options (conjugate-gradient iterations as HIP graphs): both solve forms
    give the same states and gradients bit for bit."""
    from paper_2101_05917_amd.mesh import Mesh
    sc = W.config("c5")
    args = bench.parse(["--config", "c5"])
    res = {}
    for form in (0, 1):
        g = Mesh.from_scene(sc, **bench.solver_options(args), sweep_launch=form)
        X = g.rest_positions()
        N = g.n_nodes
        c = torch.from_numpy(np.ascontiguousarray(W.loss_vector(N, 0).reshape(N, 3).T)).to(X.device)
        xT, gx, gv, gE, _, fi, bi = bench.rollout(g, X, c, 8, torch)
        print("form", form, "iterations", fi, bi, flush=True)
        res[form] = (xT, gx, gv, gE)
        g.close()
    for a, b in zip(res[0], res[1]):
        assert torch.equal(a, b)
