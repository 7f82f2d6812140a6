"""Scene model: energies, the PD matrix A, grad g and the Hessian split (oracle).

Follows Sec. Background and Sec. Differentiable Projective Dynamics:

* g(x) = (x - y)^T M (x - y) / (2 h^2) + E(x)                       (eq:opt)
* E = sum_c (w_c / 2) |G_c x - p_c|^2 with p_c the projection         (eq:pd_energy_single)
* A = M / h^2 + sum_c w_c G_c^T G_c                                  (eq:pd_global)
* b(x) = M y / h^2 + sum_c w_c G_c^T p_c(x)                          (eq:pd_global, Alg. 1)
* grad g(x) = A x - b(x) (envelope theorem)                          (eq:energy_grad)
* Hessian = A - dA, dA = sum_c w_c G_c^T dp_c/dx                     (eq:matrix_split)

Energies (readings): corotated w_q = 2 mu V_q with mu = E / (2 (1 + nu)) and
V_q = dx^3 / 8 per Gauss point (on a tetrahedral scene one point per element
with V_q = the element's volume, oracle/tetmesh.py); muscle w_m = k_m V_q per Gauss point along a
fixed fibre, actuation r_e per element; ground penalty (k / 2) min(z, 0)^2 on
the nodes of minimal rest height; gravity f = M g; explicit friction
(Sec. Penalty-Based Contact) added to the external force:
f_t = -mu k max(0, -z) v_t / sqrt(|v_t|^2 + eps^2), v_t the horizontal velocity,
evaluated at the start-of-step state.

Dirichlet nodes are held at their rest positions and eliminated (free DoFs
only in every solve).  Vectors are node-major 3N arrays.

Pins: symmetric A with row sums m/h^2 (+k on contact nodes); grad g against
central differences of g; the Hessian against central differences of grad g.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretization as disc
from . import linsolve
from . import projections as proj
from . import tetmesh as tm


def _block_diag(blocks: np.ndarray) -> sp.csr_matrix:
    """Block-diagonal sparse matrix from a stack of dense [n, b, b] blocks."""
    n, b, _ = blocks.shape
    q, i, j = np.meshgrid(np.arange(n), np.arange(b), np.arange(b), indexing="ij")
    return sp.csr_matrix((blocks.ravel(), ((b * q + i).ravel(), (b * q + j).ravel())),
                         shape=(n * b, n * b))


class Model:
    def __init__(self, scene, youngs=None):
        self.scene = scene
        self.tets = getattr(scene, "tets", None) is not None
        if self.tets:
            # linear tetrahedra: one deformation gradient per element, weight V_e
            self.mesh = tm.TetMesh(scene.X, scene.tets)
            mesh = self.mesh
            self.qpe = 1
            self.Vq = mesh.volumes.copy()                                 # [Q]
            self.m = tm.lumped_mass(mesh, scene.rho)
            self.G = tm.deformation_operator(mesh)
            if float(scene.muscle_k) > 0.0 or float(getattr(scene, "volume_scale", 0.0)) > 0.0:
                raise ValueError("tetrahedral scenes: corotated term, ground contact and gravity only")
        else:
            self.mesh = disc.VoxelMesh(scene.cells, scene.dx, scene.origin)
            mesh = self.mesh
            self.qpe = 8
            self.dx = float(scene.dx)
            self.Vq = self.dx ** 3 / 8.0
            self.m = disc.lumped_mass(mesh, scene.rho)
            self.G = disc.deformation_operator(mesh)
        N, E = mesh.n_nodes, mesh.n_elements
        self.N, self.E, self.Q = N, E, self.qpe * E
        self.h = float(scene.h)
        self.nu = float(scene.nu)
        self.Mdiag = np.repeat(self.m, 3)
        self.X = mesh.X.reshape(-1).copy()
        self.gravity = np.tile(np.asarray(scene.gravity, dtype=np.float64), N)
        self.youngs = np.asarray(scene.youngs if youngs is None else youngs, dtype=np.float64).copy()
        mu = self.youngs / (2.0 * (1.0 + self.nu))
        self.wq = np.repeat(2.0 * mu, self.qpe) * self.Vq              # [Q]

        if self.tets:
            fixed_nodes = np.asarray(scene.fixed_nodes, dtype=np.int64).reshape(-1)
        else:
            fixed_nodes = (mesh.node_index(scene.fixed_nodes) if len(scene.fixed_nodes)
                           else np.zeros(0, np.int64))
        fixed = np.zeros(3 * N, dtype=bool)
        for n in fixed_nodes:
            fixed[3 * n:3 * n + 3] = True
        self.fixed = fixed
        self.free = ~fixed
        self.fixed_nodes = fixed_nodes

        self.contact_k = float(scene.contact_k)
        if self.contact_k > 0.0:
            # the nodes of minimal rest height
            if self.tets:
                z = mesh.X[:, 2]
                self.contact_nodes = np.nonzero(z <= z.min() + 1e-12 * max(1.0, abs(z.min())))[0]
            else:
                zmin = mesh.node_ijk[:, 2].min()
                self.contact_nodes = np.nonzero(mesh.node_ijk[:, 2] == zmin)[0]
        else:
            self.contact_nodes = np.zeros(0, np.int64)
        self.Sc = disc.selector(N, self.contact_nodes)
        self.friction_mu = float(scene.friction_mu)
        self.friction_eps = float(scene.friction_eps)

        # volume-preserving term (supplemental Sec. Energy Definitions): reading,
        # w_v = volume_scale * lambda * V_q per Gauss point with Lame's
        # lambda = E nu / ((1 + nu)(1 - 2 nu)); off when volume_scale = 0
        self.volume_scale = float(getattr(scene, "volume_scale", 0.0))
        if self.volume_scale > 0.0:
            lam_per_E = self.nu / ((1.0 + self.nu) * (1.0 - 2.0 * self.nu))
            self.dwv_dE = self.volume_scale * lam_per_E * self.Vq
            self.wv = np.repeat(self.dwv_dE * self.youngs, 8)            # [Q]
        else:
            self.dwv_dE = 0.0
            self.wv = None

        self.muscle_k = float(scene.muscle_k)
        self.fiber = np.asarray(scene.fiber, dtype=np.float64)
        if self.muscle_k > 0.0:
            self.Gm = disc.fiber_operator(mesh, self.fiber)
            self.wm = np.full(self.Q, self.muscle_k * self.Vq)
        else:
            self.Gm = None
            self.wm = None

    # The PD matrix and its factorization are built on first use, so that the
    # local quantities (deformation gradients, projections, grad g) of a large
    # mesh can be evaluated without factorizing A.
    @functools.cached_property
    def A(self) -> sp.csr_matrix:
        """A = M/h^2 + sum_c w_c G_c^T G_c (eq:pd_global), assembled explicitly."""
        A = sp.diags(self.Mdiag / self.h ** 2)
        A = A + self.G.T @ sp.diags(np.repeat(self.wq, 9)) @ self.G
        if self.wv is not None:
            A = A + self.G.T @ sp.diags(np.repeat(self.wv, 9)) @ self.G
        if self.Gm is not None:
            A = A + self.Gm.T @ sp.diags(np.repeat(self.wm, 3)) @ self.Gm
        if len(self.contact_nodes):
            A = A + self.contact_k * (self.Sc.T @ self.Sc)
        return sp.csr_matrix(A)

    @functools.cached_property
    def A_ff(self) -> sp.csc_matrix:
        return sp.csc_matrix(self.A[self.free][:, self.free])

    @functools.cached_property
    def A_fc(self) -> sp.csr_matrix:
        return sp.csr_matrix(self.A[self.free][:, self.fixed])

    @functools.cached_property
    def _lu(self):
        return spla.splu(self.A_ff)

    # ---------------------------------------------------------------- helpers
    def solve_A(self, rhs_free: np.ndarray) -> np.ndarray:
        """A_ff^{-1} rhs on free DoFs (factor computed once, Sec. Background);
        beyond the sparse-LU size, conjugate gradients to round-off."""
        if self.A_ff.shape[0] > linsolve.LU_MAX:
            return linsolve.solve(self.A_ff, rhs_free, dense_max=0)[0]
        return self._lu.solve(rhs_free)

    def act_per_qp(self, act):
        if act is None:
            return np.ones(self.Q)
        return np.repeat(np.asarray(act, dtype=np.float64), 8)

    def deformation_gradients(self, x):
        return (self.G @ x).reshape(self.Q, 3, 3)

    # ---------------------------------------------------------------- external
    def friction_force(self, x, v):
        f = np.zeros(3 * self.N)
        if self.friction_mu == 0.0 or not len(self.contact_nodes):
            return f
        for j in self.contact_nodes:
            z = x[3 * j + 2]
            fn = self.contact_k * max(0.0, -z)
            vt = v[3 * j:3 * j + 2]
            s = np.sqrt(vt @ vt + self.friction_eps ** 2)
            f[3 * j:3 * j + 2] = -self.friction_mu * fn * vt / s
        return f

    def friction_vjp(self, x, v, w):
        """(w^T df/dx, w^T df/dv) of the explicit friction force."""
        gx = np.zeros(3 * self.N)
        gv = np.zeros(3 * self.N)
        if self.friction_mu == 0.0 or not len(self.contact_nodes):
            return gx, gv
        mu, k, eps = self.friction_mu, self.contact_k, self.friction_eps
        for j in self.contact_nodes:
            z = x[3 * j + 2]
            fn = k * max(0.0, -z)
            dfn_dz = -k if z < 0.0 else 0.0
            vt = v[3 * j:3 * j + 2]
            s = np.sqrt(vt @ vt + eps ** 2)
            wt = w[3 * j:3 * j + 2]
            gx[3 * j + 2] += wt @ (-mu * dfn_dz * vt / s)
            J = -mu * fn * (np.eye(2) / s - np.outer(vt, vt) / s ** 3)
            gv[3 * j:3 * j + 2] += J.T @ wt
        return gx, gv

    def y_of(self, x, v):
        """y = x + h v + h^2 M^{-1} f_ext (Sec. Background, eq:time_integration)."""
        fext = self.Mdiag * self.gravity + self.friction_force(x, v)
        return x + self.h * v + self.h ** 2 * fext / self.Mdiag

    # ---------------------------------------------------------------- energy
    def elastic_energy(self, x, act=None):
        F = self.deformation_gradients(x)
        R = proj.closest_rotation(F)
        e = 0.5 * np.sum(self.wq * np.sum((F - R) ** 2, axis=(1, 2)))
        if self.wv is not None:
            e += 0.5 * np.sum(self.wv * np.sum((F - proj.volume_projection(F)) ** 2, axis=(1, 2)))
        if self.Gm is not None:
            f = (self.Gm @ x).reshape(self.Q, 3)
            r = self.act_per_qp(act)
            e += 0.5 * np.sum(self.wm * (np.linalg.norm(f, axis=1) - r) ** 2)
        if len(self.contact_nodes):
            z = x[3 * self.contact_nodes + 2]
            e += 0.5 * self.contact_k * np.sum(np.minimum(z, 0.0) ** 2)
        return e

    def g(self, x, y, act=None):
        d = x - y
        return 0.5 * d @ (self.Mdiag * d) / self.h ** 2 + self.elastic_energy(x, act)

    # ---------------------------------------------------------------- PD parts
    def rhs(self, y, x, act=None):
        """b(x) = M y / h^2 + sum w G^T p(x), all 3N rows."""
        F = self.deformation_gradients(x)
        R = proj.closest_rotation(F)
        b = self.Mdiag * y / self.h ** 2 + self.G.T @ (np.repeat(self.wq, 9) * R.reshape(-1))
        if self.wv is not None:
            b = b + self.G.T @ (np.repeat(self.wv, 9) * proj.volume_projection(F).reshape(-1))
        if self.Gm is not None:
            f = (self.Gm @ x).reshape(self.Q, 3)
            p = proj.sphere_projection(f, self.act_per_qp(act), self.fiber)
            b = b + self.Gm.T @ (np.repeat(self.wm, 3) * p.reshape(-1))
        if len(self.contact_nodes):
            xc = (self.Sc @ x).reshape(-1, 3)
            b = b + self.contact_k * (self.Sc.T @ proj.ground_projection(xc).reshape(-1))
        return b

    def grad_g(self, x, y, act=None):
        """grad g = A x - b(x) on all 3N rows."""
        return self.A @ x - self.rhs(y, x, act)

    def delta_A(self, x, act=None) -> sp.csr_matrix:
        """dA = sum_c w_c G_c^T (dp_c/dx) (eq:matrix_split), assembled explicitly."""
        F = self.deformation_gradients(x)
        J = proj.rotation_jacobian(F) * self.wq[:, None, None]
        if self.wv is not None:
            J = J + proj.volume_jacobian(F) * self.wv[:, None, None]
        blk = _block_diag(J)
        dA = self.G.T @ blk @ self.G
        if self.Gm is not None:
            f = (self.Gm @ x).reshape(self.Q, 3)
            Jm = proj.sphere_jacobian(f, self.act_per_qp(act)) * self.wm[:, None, None]
            dA = dA + self.Gm.T @ _block_diag(Jm) @ self.Gm
        if len(self.contact_nodes):
            xc = (self.Sc @ x).reshape(-1, 3)
            d = proj.ground_jacobian(xc).reshape(-1)
            dA = dA + self.contact_k * (self.Sc.T @ sp.diags(d) @ self.Sc)
        return sp.csr_matrix(dA)

    def hessian(self, x, act=None) -> sp.csr_matrix:
        """Hessian of g: A - dA (eq:matrix_split)."""
        return sp.csr_matrix(self.A - self.delta_A(x, act))

    # ---------------------------------------------------------------- params
    def youngs_force_derivative(self, x):
        """Per qp: d(grad g)/dw_q contracted later; returns (F - R) [Q, 3, 3]."""
        F = self.deformation_gradients(x)
        return F - proj.closest_rotation(F)

    def volume_youngs_derivative(self, x):
        """Per qp: (F - D) [Q, 3, 3]; d(grad g)/dE_e through the volume weight is
        sum_q G_q^T (F - D) dw_v/dE (zero when the term is off)."""
        F = self.deformation_gradients(x)
        return F - proj.volume_projection(F)

    def youngs_gradient(self, x_next, z):
        """dL/dE_e = -z^T d(grad g)/dE_e at the step's solution (both terms)."""
        Gz = (self.G @ z).reshape(self.Q, 3, 3)
        per_q = np.sum(Gz * self.youngs_force_derivative(x_next), axis=(1, 2)) * self.Vq / (1.0 + self.nu)
        if self.wv is not None:
            per_q = per_q + np.sum(Gz * self.volume_youngs_derivative(x_next), axis=(1, 2)) * self.dwv_dE
        return -per_q.reshape(self.E, self.qpe).sum(axis=1)

    def fiber_directions(self, x, act=None):
        """dp/dr per muscle qp: f/|f| (the fibre m where f = 0)."""
        f = (self.Gm @ x).reshape(self.Q, 3)
        nrm = np.linalg.norm(f, axis=1)
        n = np.tile(self.fiber, (self.Q, 1))
        nz = nrm > 0
        n[nz] = f[nz] / nrm[nz][:, None]
        return n
