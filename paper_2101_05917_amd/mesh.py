"""Python handle of a simulated voxel body on the GPU.

Thin marshalling over the C ABI: tensors provide device memory and the
current HIP stream; every computation happens in libdiffpd's kernels.
State tensors are float64 with shape [3, N] (SoA, public node order).
"""
from __future__ import annotations

import atexit
import ctypes as C
import warnings
import weakref
from typing import Optional

import numpy as np
import torch

from . import _lib as L

PHYSICS_KEYS = ("dx", "rho", "nu", "h", "contact_k", "friction_mu", "friction_eps", "muscle_k", "volume_scale")


def make_options(physics: Optional[dict] = None, **iteration) -> L.Options:
    lib = L.load()
    o = L.Options()
    L.check(lib.dpd_default_options(C.byref(o)))
    physics = physics or {}
    for k in PHYSICS_KEYS:
        if k in physics:
            setattr(o, k, float(physics[k]))
    for k in ("gravity", "origin", "fiber"):
        if k in physics:
            arr = getattr(o, k)
            for i, val in enumerate(physics[k]):
                arr[i] = float(val)
    for k, val in iteration.items():
        if k == "precision" and isinstance(val, str):
            val = {"fp64": L.DPD_FP64, "mixed": L.DPD_MIXED}[val]
        if k == "bwd_solver" and isinstance(val, str):
            val = {"fixed_point": L.DPD_BWD_FIXED_POINT, "pcg": L.DPD_BWD_PCG}[val]
        if k == "fwd_solver" and isinstance(val, str):
            val = {"pd": L.DPD_FWD_PD, "newton_pcg": L.DPD_FWD_NEWTON_PCG}[val]
        setattr(o, k, val)
    return o


# Handles still open when the interpreter exits are destroyed by an exit hook,
# after the device has finished its work, rather than from __del__ during
# interpreter teardown (when the HIP runtime may already be shutting down).
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_meshes():
    meshes = list(_LIVE)
    if not meshes:
        return
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for m in meshes:
        try:
            m.close()
        except Exception:
            pass


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Mesh:
    """A voxel body (or, through ``from_tets``, a tetrahedral one): mesh,
    factor and workspaces live in the library handle."""

    def __init__(self, cells, youngs, fixed_nodes=None, physics: Optional[dict] = None,
                 device="cuda:0", factorize=True, tets=None, **iteration):
        self.lib = L.load()
        self.device = torch.device(device)
        youngs = np.ascontiguousarray(np.asarray(youngs, dtype=np.float64).reshape(-1))
        self.options = make_options(physics, **iteration)
        self.physics = dict(physics or {})
        h = C.c_void_p()
        if tets is None:
            cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
            fixed = (np.zeros((0, 3), np.int32) if fixed_nodes is None
                     else np.ascontiguousarray(np.asarray(fixed_nodes, dtype=np.int32).reshape(-1, 3)))
            with torch.cuda.device(self.device):
                L.check(self.lib.dpd_create_mesh(
                    cells.ctypes.data_as(L._I32), cells.shape[0],
                    youngs.ctypes.data_as(L._D),
                    fixed.ctypes.data_as(L._I32) if len(fixed) else None, fixed.shape[0],
                    C.byref(self.options), C.byref(h)))
        else:
            # cells holds the rest positions [N, 3] of a tetrahedral mesh
            X = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 3))
            T = np.ascontiguousarray(np.asarray(tets, dtype=np.int32).reshape(-1, 4))
            fixed = (np.zeros(0, np.int32) if fixed_nodes is None
                     else np.ascontiguousarray(np.asarray(fixed_nodes, dtype=np.int32).reshape(-1)))
            with torch.cuda.device(self.device):
                L.check(self.lib.dpd_create_tet_mesh(
                    X.ctypes.data_as(L._D), X.shape[0], T.ctypes.data_as(L._I32), T.shape[0],
                    youngs.ctypes.data_as(L._D),
                    fixed.ctypes.data_as(L._I32) if len(fixed) else None, fixed.shape[0],
                    C.byref(self.options), C.byref(h)))
        self.handle = h
        _LIVE.add(self)
        self._read_info()
        self.n_nodes = self.info["n_nodes"]
        self.n_elements = self.info["n_elements"]
        self.youngs = youngs.copy()
        self._youngs_dev = None      # device copy of the factorized moduli (on first use)
        self._youngs_seen = None     # (weakref, _version) of the last tensor found equal
        if factorize:
            self.factorize()

    @classmethod
    def from_scene(cls, scene, device="cuda:0", **iteration):
        if getattr(scene, "tets", None) is not None:
            return cls.from_tets(scene.X, scene.tets, scene.youngs, scene.fixed_nodes, scene.physics(),
                                 device=device, **iteration)
        return cls(scene.cells, scene.youngs, scene.fixed_nodes, scene.physics(), device=device,
                   **iteration)

    @classmethod
    def from_tets(cls, X, tets, youngs, fixed_nodes=None, physics: Optional[dict] = None, device="cuda:0",
                  factorize=True, **iteration):
        """Linear tetrahedra: rest positions X [N, 3], corners tets [E, 4],
        moduli [E], fixed node ids (dpd_create_tet_mesh)."""
        return cls(X, youngs, fixed_nodes, physics, device=device, factorize=factorize, tets=tets, **iteration)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.dpd_destroy_mesh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ setup
    def _read_info(self):
        info = L.MeshInfo()
        L.check(self.lib.dpd_get_info(self.handle, C.byref(info)), self.handle)
        self.info = {k: getattr(info, k) for k, _ in info._fields_}

    def factorize(self):
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_factorize(self.handle, _stream(self.device)), self.handle)
        self._read_info()

    def set_options(self, **iteration):
        for k, val in iteration.items():
            if k == "precision" and isinstance(val, str):
                val = {"fp64": L.DPD_FP64, "mixed": L.DPD_MIXED}[val]
            if k == "bwd_solver" and isinstance(val, str):
                val = {"fixed_point": L.DPD_BWD_FIXED_POINT, "pcg": L.DPD_BWD_PCG}[val]
            if k == "fwd_solver" and isinstance(val, str):
                val = {"pd": L.DPD_FWD_PD, "newton_pcg": L.DPD_FWD_NEWTON_PCG}[val]
            setattr(self.options, k, val)
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_set_options(self.handle, C.byref(self.options)), self.handle)

    def set_youngs(self, youngs, refactorize=True):
        ym = np.ascontiguousarray(np.asarray(youngs, dtype=np.float64).reshape(-1))
        L.check(self.lib.dpd_set_youngs(self.handle, ym.ctypes.data_as(C.c_void_p), 0, None),
                self.handle)
        self.youngs = ym.copy()
        self._youngs_dev = None
        self._youngs_seen = None
        if refactorize:
            self.factorize()

    def ensure_youngs(self, youngs: torch.Tensor) -> bool:
        """Make the factor match ``youngs`` (float64 [E] on the device): when its
        values differ from the moduli the mesh was factorized with, they replace
        them (dpd_set_youngs) and A is factorized again.  A tensor already found
        equal and not modified in place since (the same live tensor object with
        the same version counter) is not compared again; a tensor allocated
        later at the same address is a different object and is compared.
        Returns True if it refactorized."""
        seen = self._youngs_seen
        if seen is not None and seen[0]() is youngs and seen[1] == youngs._version:
            return False
        t = youngs.detach()
        self._check_elem(t)
        if self._youngs_dev is None:
            self._youngs_dev = torch.from_numpy(self.youngs).to(self.device)
        changed = not torch.equal(t, self._youngs_dev)
        if changed:
            with torch.cuda.device(self.device):
                L.check(self.lib.dpd_set_youngs(self.handle, _ptr(t), 1, _stream(self.device)),
                        self.handle)
                self.factorize()
            self._youngs_dev = t.clone()
            self.youngs = self._youngs_dev.cpu().numpy().copy()
        self._youngs_seen = (weakref.ref(youngs), youngs._version)
        return changed

    def node_ijk(self) -> np.ndarray:
        out = np.zeros((self.n_nodes, 3), np.int32)
        L.check(self.lib.dpd_node_ijk(self.handle, out.ctypes.data_as(L._I32)), self.handle)
        return out

    def rest_positions(self) -> torch.Tensor:
        out = np.zeros((3, self.n_nodes), np.float64)
        L.check(self.lib.dpd_rest_positions(self.handle, out.ctypes.data_as(L._D)), self.handle)
        return torch.from_numpy(out).to(self.device)

    def contact_nodes(self) -> np.ndarray:
        out = np.zeros(max(1, self.info["n_contact"]), np.int32)
        L.check(self.lib.dpd_contact_nodes(self.handle, out.ctypes.data_as(L._I32)), self.handle)
        return out[: self.info["n_contact"]]

    def zeros_state(self) -> torch.Tensor:
        return torch.zeros(3, self.n_nodes, dtype=torch.float64, device=self.device)

    def _check_state(self, *ts):
        for t in ts:
            if t is None:
                continue
            if (t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous()
                    or tuple(t.shape) != (3, self.n_nodes)):
                raise ValueError(f"expected contiguous float64 [3, {self.n_nodes}] on {self.device}")

    def _check_elem(self, t):
        if t is None:
            return
        if (t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous()
                or t.numel() != self.n_elements):
            raise ValueError(f"expected contiguous float64 [{self.n_elements}] on {self.device}")

    # ------------------------------------------------------------------ steps
    def forward_step(self, x, v, act=None, out=None, strict=False):
        """One implicit-Euler PD step.  Returns (x_next, v_next, stats dict)."""
        self._check_state(x, v)
        self._check_elem(act)
        xn, vn = out if out is not None else (torch.empty_like(x), torch.empty_like(v))
        st = L.Stats()
        with torch.cuda.device(self.device):
            code = L.check(self.lib.dpd_forward_step(self.handle, _stream(self.device), _ptr(x),
                                                     _ptr(v), _ptr(act), _ptr(xn), _ptr(vn),
                                                     C.byref(st)), self.handle)
        stats = st.as_dict()
        if code == L.DPD_NOT_CONVERGED:
            if strict:
                raise L.DiffPDError(code, f"forward step not converged: {stats}")
            warnings.warn(f"forward PD step not converged: {stats}", RuntimeWarning, stacklevel=2)
        return xn, vn, stats

    def backward_step(self, x, v, act, x_next, gx_next, gv_next, g_youngs=None, want_act=False,
                      strict=False):
        """Adjoint of one step.  Returns (gx, gv, g_act or None, stats dict).

        ``g_youngs`` (float64 [E] on the device) is accumulated in place."""
        self._check_state(x, v, x_next, gx_next, gv_next)
        self._check_elem(act)
        self._check_elem(g_youngs)
        gx = torch.empty_like(gx_next)
        gv = torch.empty_like(gv_next)
        g_act = (torch.empty(self.n_elements, dtype=torch.float64, device=self.device)
                 if want_act else None)
        st = L.Stats()
        with torch.cuda.device(self.device):
            code = L.check(self.lib.dpd_backward_step(
                self.handle, _stream(self.device), _ptr(x), _ptr(v), _ptr(act), _ptr(x_next),
                _ptr(gx_next), _ptr(gv_next), _ptr(gx), _ptr(gv), _ptr(g_youngs), _ptr(g_act),
                C.byref(st)), self.handle)
        stats = st.as_dict()
        if code == L.DPD_NOT_CONVERGED:
            if strict:
                raise L.DiffPDError(code, f"adjoint not converged: {stats}")
            warnings.warn(f"adjoint iteration not converged: {stats}", RuntimeWarning, stacklevel=2)
        return gx, gv, g_act, stats

    # ------------------------------------------------------------------ building blocks
    def apply_inverse(self, b, precision="fp64"):
        self._check_state(b)
        out = torch.empty_like(b)
        prec = {"fp64": L.DPD_FP64, "mixed": L.DPD_MIXED}[precision]
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_apply_inverse(self.handle, _stream(self.device), prec, _ptr(b),
                                               _ptr(out)), self.handle)
        return out

    def gradient(self, x, y, act=None):
        self._check_state(x, y)
        out = torch.empty_like(x)
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_gradient(self.handle, _stream(self.device), _ptr(x), _ptr(y),
                                          _ptr(act), _ptr(out)), self.handle)
        return out

    def gradient_noalloc(self, x, y, act=None, out=None):
        """grad g(x) through dpd_gradient_noalloc (no device allocation in the
        library; at most 16384 elements).  ``out`` may be given preallocated."""
        self._check_state(x, y)
        self._check_elem(act)
        if out is None:
            out = torch.empty_like(x)
        self._check_state(out)
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_gradient_noalloc(self.handle, _stream(self.device), _ptr(x), _ptr(y),
                                                  _ptr(act), _ptr(out)), self.handle)
        return out

    def hessian_apply(self, x, p, act=None):
        self._check_state(x, p)
        out = torch.empty_like(p)
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_hessian_apply(self.handle, _stream(self.device), _ptr(x),
                                               _ptr(act), _ptr(p), _ptr(out)), self.handle)
        return out

    def spectral_radius(self, x, act=None, steps=40, seed=0):
        """Largest eigenvalue of A^{-1} dA at state x (the contraction factor of
        the adjoint fixed-point iteration, eq:sp_radius), by Lanczos on the
        similar operator dA A^{-1} = I - H A^{-1}, which is self-adjoint in the
        inner product <u, v> = u^T A^{-1} v.  Each step is one solve with the
        factor (dpd_apply_inverse) and one Hessian product (dpd_hessian_apply);
        the vectors are reorthogonalized in full.  Returns the Ritz values'
        maximum (eigenvalues of A^{-1} dA are real and, without negative
        curvature, in [0, 1))."""
        self._check_state(x)
        g = torch.Generator(device="cpu").manual_seed(seed)
        u = torch.randn((3, self.n_nodes), generator=g, dtype=torch.float64).to(self.device)
        s = self.apply_inverse(u)
        u = u * (s.abs() > 0)                   # free rows only
        s = self.apply_inverse(u)
        beta = float(torch.sqrt((u * s).sum()))
        Q, S = [u / beta], [s / beta]
        alphas, betas = [], []
        for j in range(steps):
            w = Q[j] - self.hessian_apply(x, S[j], act)
            a = float((w * S[j]).sum())
            alphas.append(a)
            for qi, si in zip(Q, S):             # full reorthogonalization (A^{-1} inner product)
                w = w - float((w * si).sum()) * qi
            sw = self.apply_inverse(w)
            b = float((w * sw).sum())
            if b <= 1e-28 or j == steps - 1:
                break
            b = b ** 0.5
            betas.append(b)
            Q.append(w / b)
            S.append(sw / b)
        T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) + np.diag(betas[:len(alphas) - 1], -1)
        return float(np.linalg.eigvalsh(T).max())

    def rotations(self, x):
        self._check_state(x)
        out = torch.empty(9, self.info["qp_per_element"] * self.n_elements, dtype=torch.float64,
                          device=self.device)
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_rotations(self.handle, _stream(self.device), _ptr(x), _ptr(out)),
                    self.handle)
        return out

    # ------------------------------------------------------------------ contact global step
    def contact_prepare(self, nodes):
        """Cache A^{-1} e_j for the candidate nodes (public ids), see dpd_contact_prepare."""
        arr = np.ascontiguousarray(np.asarray(nodes, dtype=np.int32))
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_contact_prepare(self.handle, _stream(self.device),
                                                 arr.ctypes.data_as(C.c_void_p), int(arr.size)), self.handle)
        self._contact_count = int(arr.size)

    def contact_solve(self, active, xstar, b):
        """x with x_C = x* and A_{C̄×C̄} x_{C̄} = b_{C̄}; active: indices into the
        candidate list; xstar: [3, c] float64 on the device (dpd_contact_solve)."""
        self._check_state(b)
        arr = np.ascontiguousarray(np.asarray(active, dtype=np.int32))
        c = int(arr.size)
        if c and (xstar is None or tuple(xstar.shape) != (3, c) or xstar.dtype != torch.float64
                  or xstar.device != self.device or not xstar.is_contiguous()):
            raise ValueError(f"xstar must be a contiguous float64 [3, {c}] tensor on {self.device}")
        out = torch.empty_like(b)
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_contact_solve(self.handle, _stream(self.device),
                                               arr.ctypes.data_as(C.c_void_p) if c else None, c,
                                               _ptr(xstar) if c else None, _ptr(b), _ptr(out)), self.handle)
        return out

    def contact_forward_step(self, x, v, act=None, out=None, strict=False):
        """One implicit-Euler step with complementarity contact on the prepared
        candidates (Alg. 3, dpd_contact_forward_step).  Returns (x_next,
        v_next, kind, stats): kind is the int32 numpy array of 0 / 1 (ray
        target) / 2 (static target) per candidate."""
        self._check_state(x, v)
        self._check_elem(act)
        xn, vn = out if out is not None else (torch.empty_like(x), torch.empty_like(v))
        kind = np.zeros(self._n_candidates(), dtype=np.int32)
        st = L.Stats()
        with torch.cuda.device(self.device):
            code = L.check(self.lib.dpd_contact_forward_step(
                self.handle, _stream(self.device), _ptr(x), _ptr(v), _ptr(act), _ptr(xn), _ptr(vn),
                kind.ctypes.data_as(C.c_void_p), C.byref(st)), self.handle)
        stats = st.as_dict()
        if code == L.DPD_NOT_CONVERGED:
            if strict:
                raise L.DiffPDError(code, f"contact forward step not converged: {stats}")
            warnings.warn(f"contact forward step not converged: {stats}", RuntimeWarning, stacklevel=2)
        return xn, vn, kind, stats

    def contact_backward_step(self, x, v, act, x_next, kind, gx_next, gv_next, g_youngs=None,
                              want_act=False, strict=False):
        """Adjoint of a step with contact (Alg. 5, dpd_contact_backward_step).
        Returns (gx, gv, g_act or None, stats); ``g_youngs`` is accumulated."""
        self._check_state(x, v, x_next, gx_next, gv_next)
        self._check_elem(act)
        self._check_elem(g_youngs)
        k = np.ascontiguousarray(np.asarray(kind, dtype=np.int32))
        if k.size != self._n_candidates():
            raise ValueError(f"kind must hold {self._n_candidates()} entries")
        gx = torch.empty_like(gx_next)
        gv = torch.empty_like(gv_next)
        g_act = (torch.empty(self.n_elements, dtype=torch.float64, device=self.device)
                 if want_act else None)
        st = L.Stats()
        with torch.cuda.device(self.device):
            code = L.check(self.lib.dpd_contact_backward_step(
                self.handle, _stream(self.device), _ptr(x), _ptr(v), _ptr(act), _ptr(x_next),
                k.ctypes.data_as(C.c_void_p), _ptr(gx_next), _ptr(gv_next), _ptr(gx), _ptr(gv),
                _ptr(g_youngs), _ptr(g_act), C.byref(st)), self.handle)
        stats = st.as_dict()
        if code == L.DPD_NOT_CONVERGED:
            if strict:
                raise L.DiffPDError(code, f"contact adjoint not converged: {stats}")
            warnings.warn(f"contact adjoint not converged: {stats}", RuntimeWarning, stacklevel=2)
        return gx, gv, g_act, stats

    def _n_candidates(self) -> int:
        n = getattr(self, "_contact_count", 0)
        if not n:
            raise L.DiffPDError(-5, "no contact candidates (call contact_prepare)")
        return n

    # ------------------------------------------------------------------ timing
    def profile_start(self, kernel_class: str):
        """Time the launches of one kernel class (device clock or events, see dpd_profile_start)."""
        L.check(self.lib.dpd_profile_start(self.handle, L.DPD_PROF[kernel_class]), self.handle)

    def profile_read(self) -> dict:
        out = L.KernelProfile()
        with torch.cuda.device(self.device):
            L.check(self.lib.dpd_profile_read(self.handle, _stream(self.device), C.byref(out)),
                    self.handle)
        return {k: getattr(out, k) for k, _ in out._fields_}
