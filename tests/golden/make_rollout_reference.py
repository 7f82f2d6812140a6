"""Write the oracle's reference rollout gradient of a benchmark scene.

Calls only the oracle: each forward step is solved to round-off by Newton's
method on g (the implicit-Euler solution, eq:time_integration), each backward
step by a direct solve of the adjoint system (eq:adjoint).  The loss is
dot(c, x_T) with c ~ N(0, 1) (seed 0), node-major.

A scene with complementarity-contact candidates (the rolling sphere) starts
from its rigid initial velocity and steps with the oracle's Alg. 3 (Newton to
round-off on each reduced system) and its adjoint (Alg. 5, direct reduced
solve); its loss also weighs the final velocity, dot(c, x_T) + dot(d, v_T)
with d ~ N(0, 1) (seed 1), and the contact kinds of every step are stored.

With fewer steps than the scene's, the file holds the reference of that
prefix of the rollout (the 64x32x32 block: the first 30 steps, through the
landing; about an hour and a half on 8 host cores, where each Newton step and
each adjoint solve runs conjugate gradients on the assembled Hessian to
round-off, ``oracle.linsolve``; the tetrahedral ball: the first 30 of 100
steps, landing at step 8 and bouncing, about 16 minutes).

Newton stops at |grad g| <= tol |M y / h^2| (default 1e-13).  On the block,
whose 212 k DoFs put the round-off floor of grad g near 3e-12 of that scale,
the reference uses tol 1e-11 (position error about 1e-9 m; without it every
step runs Newton into the floor, about six minutes a step), and so does the
tetrahedral ball (its contact steps stall Newton near the floor).

usage: python tests/golden/make_rollout_reference.py c2 [steps] [newton_tol]
       (c5 30 1e-11 and tet 30 1e-11 for the stored prefixes)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import model as om, forward as of, adjoint as oa, contact as oc  # noqa: E402


def contact_reference(name, sc, steps):
    m = om.Model(sc)
    cand = W.candidate_nodes(sc)
    x, v = m.X.copy(), W.initial_velocity(sc)
    xs, vs, kinds = [x], [v], []
    t0 = time.time()
    for t in range(steps):
        x, v, info = oc.forward_step_contact(m, x, v, cand)
        xs.append(x)
        vs.append(v)
        kinds.append(info["kind"])
        print(f"forward {t} sets {info['sets']} contact {int((info['kind'] > 0).sum())} "
              f"{time.time() - t0:.0f}s", flush=True)
    c = W.loss_vector(m.N, sc.loss_seed)
    d = W.loss_vector(m.N, sc.loss_seed + 1)
    gx, gv = c.copy(), d.copy()
    gE = np.zeros(m.E)
    for t in range(steps - 1, -1, -1):
        gx, gv, ge, _, _ = oc.backward_step_contact(m, xs[t], vs[t], None, xs[t + 1], cand, kinds[t], gx, gv)
        gE += ge
    out = os.path.join(HERE, f"{name}_rollout_reference.npz")
    np.savez_compressed(out, steps=steps, loss=float(c @ xs[-1] + d @ vs[-1]), x_T=xs[-1], g_x0=gx, g_v0=gv,
                        g_youngs=gE, kinds=np.array(kinds, dtype=np.int8))
    print("wrote", out, f"{time.time() - t0:.0f}s")


def main():
    name = sys.argv[1]
    sc = W.config(name)
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else sc.steps
    newton_tol = float(sys.argv[3]) if len(sys.argv) > 3 else 1e-13
    if "candidates_ijk" in sc.extra:
        return contact_reference(name, sc, steps)
    m = om.Model(sc)
    x, v = m.X.copy(), np.zeros(3 * m.N)
    xs, vs = [x], [v]
    # muscle actuation per step and element, the benchmark's seeded sequence
    acts = W.actuation_sequence(steps, m.E, seed=sc.act_seed) if sc.muscle_k > 0 else None
    t0 = time.time()
    for t in range(steps):
        a = None if acts is None else acts[t]
        xn, info = of.newton_solve(m, m.y_of(x, v), a, tol_rel=newton_tol)
        vn = (xn - x) / m.h
        xs.append(xn)
        vs.append(vn)
        x, v = xn, vn
        print(f"forward {t} newton iters {info['iters']} |grad| {info['grad']:.2e} "
              f"{time.time() - t0:.0f}s", flush=True)
    c = W.loss_vector(m.N, sc.loss_seed)
    gx, gv = c.copy(), np.zeros(3 * m.N)
    gE = np.zeros(m.E)
    g_act = None if acts is None else np.zeros_like(acts)
    for t in range(steps - 1, -1, -1):
        a = None if acts is None else acts[t]
        gx, gv, ge, ga, info = oa.backward_step(m, xs[t], vs[t], a, xs[t + 1], gx, gv, solver="direct")
        gE += ge
        print(f"backward {t} {info['method']} rel res {info['rel_res']} {time.time() - t0:.0f}s", flush=True)
        if g_act is not None:
            g_act[t] = ga
    out = os.path.join(HERE, f"{name}_rollout_reference.npz")
    extra = {} if g_act is None else {"g_act": g_act}
    np.savez_compressed(out, steps=steps, loss=float(c @ xs[-1]), x_T=xs[-1], g_x0=gx, g_v0=gv,
                        g_youngs=gE, newton_tol=newton_tol, **extra)
    print("wrote", out, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
