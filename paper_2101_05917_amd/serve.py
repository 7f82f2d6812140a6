"""Python front of the rollout server (dpd_server_* in the C ABI).

Each request is a whole differentiable rollout of a voxel body; the server
keeps several of them resident on the GPU (each with its own factor and
states), admits queued requests as slots and HBM budget free up, and returns
the loss c . x_T with its gradients w.r.t. x0, v0 and the Young's moduli.
With ``batched`` (the default) the conjugate-gradient iterations of all
resident requests share their launches (the batch engine of the library);
without it each request iterates on its own stream.  Marshalling only:
everything runs inside libdiffpd.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib as L
from .mesh import make_options


STATES = {0: "queued", 1: "running", 2: "done", 3: "failed"}

# Servers still open at interpreter exit are drained and destroyed by an exit
# hook (their worker threads joined) before the HIP runtime shuts down.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_servers():
    for s in list(_LIVE):
        try:
            s.close()
        except Exception:
            pass


@dataclass
class RolloutResult:
    ticket: int
    state: str
    status: int
    loss: float
    t_submit: float
    t_admit: float
    t_done: float
    n_nodes: int
    n_elements: int
    footprint_bytes: int
    fwd_iters: int
    bwd_iters: int
    g_x0: Optional[np.ndarray] = None   # [3, N]
    g_v0: Optional[np.ndarray] = None
    g_youngs: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class Server:
    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, batched: bool = True):
        import torch  # the device must be initialised in this process first
        torch.cuda.init()
        self.lib = L.load()
        h = C.c_void_p()
        L.check(self.lib.dpd_server_create(int(hbm_budget_bytes), int(max_slots), 1 if batched else 0,
                                           C.byref(h)))
        self.batched = bool(batched)
        self.handle = h
        self._sizes = {}
        _LIVE.add(self)

    def submit(self, scene, loss_x: np.ndarray, steps: Optional[int] = None, **iteration) -> int:
        """Queue a rollout of ``scene``; ``loss_x`` node-major 3N weights of c . x_T."""
        import workloads as W
        cells = np.ascontiguousarray(np.asarray(scene.cells, np.int32).reshape(-1, 3))
        youngs = np.ascontiguousarray(np.asarray(scene.youngs, np.float64))
        fixed = np.ascontiguousarray(np.asarray(scene.fixed_nodes, np.int32).reshape(-1, 3))
        N = len(W.present_nodes(cells))
        c = np.ascontiguousarray(np.asarray(loss_x, np.float64).reshape(N, 3).T)
        q = L.Request()
        q.cells_ijk = cells.ctypes.data_as(L._I32)
        q.n_cells = len(cells)
        q.youngs = youngs.ctypes.data_as(L._D)
        q.fixed_ijk = fixed.ctypes.data_as(L._I32) if len(fixed) else None
        q.n_fixed = len(fixed)
        q.loss_x = c.ctypes.data_as(L._D)
        q.n_nodes = N
        q.steps = int(steps or scene.steps)
        q.opt = make_options(scene.physics(), **iteration)
        t = C.c_int64()
        L.check(self.lib.dpd_server_submit(self.handle, C.byref(q), C.byref(t)))
        self._sizes[t.value] = (N, len(cells))
        return t.value

    def poll(self, ticket: int, gradients: bool = True) -> RolloutResult:
        N, E = self._sizes[ticket]
        r = L.Result()
        gx = np.zeros((3, N)) if gradients else None
        gv = np.zeros((3, N)) if gradients else None
        gE = np.zeros(E) if gradients else None
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        L.check(self.lib.dpd_server_poll(self.handle, ticket, C.byref(r), ptr(gx), ptr(gv), ptr(gE)))
        done = r.state == 2
        return RolloutResult(ticket, STATES[r.state], r.status, r.loss, r.t_submit, r.t_admit,
                             r.t_done, r.n_nodes, r.n_elements, r.footprint_bytes, r.fwd_iters,
                             r.bwd_iters, gx if done else None, gv if done else None,
                             gE if done else None)

    def drain(self):
        L.check(self.lib.dpd_server_drain(self.handle))

    def stats(self):
        pb, pa = C.c_int64(), C.c_int32()
        L.check(self.lib.dpd_server_stats(self.handle, C.byref(pb), C.byref(pa)))
        return {"peak_bytes": pb.value, "peak_active": pa.value}

    def batch_stats(self):
        b = L.BatchStats()
        L.check(self.lib.dpd_server_batch_stats(self.handle, C.byref(b)))
        return {"iterations": b.iterations, "slot_iterations": b.slot_iterations, "launches": b.launches,
                "solves": b.solves, "peak_slots": b.peak_slots,
                "mean_slots": b.slot_iterations / b.iterations if b.iterations else 0.0}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.dpd_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
