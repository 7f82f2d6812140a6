/*
 * diffpd.h -- C ABI of the MI355X (gfx950) implementation of the implicit-Euler
 * Projective Dynamics time step on hexahedral voxel meshes and its adjoint
 * (Du et al., "DiffPD: Differentiable Projective Dynamics").
 *
 * Every entry point returns a dpd_status; nothing throws across the ABI.
 * Arguments are plain host or device pointers and sizes.  A "stream" argument
 * is a hipStream_t passed as void* (NULL = the default stream).
 *
 * Layouts
 *   - State vectors (x, v, gradients) are device arrays of doubles in SoA
 *     layout [3][N]: x[c * N + n] is coordinate c of node n.
 *   - Node order ("public order") is lexicographic over present grid nodes,
 *     i fastest, then j, then k.  Node (i, j, k) rests at
 *     origin + dx * (i, j, k).
 *   - Element e is the voxel cells_ijk[3e .. 3e+2]; per-element arrays
 *     (Young's moduli, actuation, their gradients) follow that order.
 *
 * Ownership
 *   - The mesh handle owns all internal device memory (connectivity, the
 *     factor, workspaces, per-quadrature-point caches).
 *   - The caller owns every state and gradient buffer; they must stay valid
 *     until the work enqueued on the stream completes.
 *   - One handle is used by at most one stream at a time (its workspaces are
 *     shared by all calls on it).  Distinct handles are independent.
 *
 * Errors
 *   - Negative codes are hard errors: outputs are undefined; the handle stays
 *     usable unless the code is DPD_EHIP.  dpd_last_error() gives a message.
 *   - DPD_NOT_CONVERGED is soft: outputs hold the last iterate; see stats.
 */
#ifndef DIFFPD_H
#define DIFFPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dpd_mesh dpd_mesh;

typedef enum {
  DPD_OK = 0,
  DPD_NOT_CONVERGED = 1,   /* iteration cap reached; outputs = last iterate          */
  DPD_EINVAL = -1,         /* invalid argument or mesh description                     */
  DPD_ENOTSPD = -2,        /* non-positive pivot while factorizing A                   */
  DPD_ENOMEM = -3,         /* device or host allocation failed                         */
  DPD_EHIP = -4,           /* a HIP runtime call failed                                 */
  DPD_ESTATE = -5,         /* call not valid in the handle's state (e.g. no factor)    */
  DPD_ENONFINITE = -6,     /* NaN or Inf met in a residual                             */
  DPD_ECURVATURE = -7      /* adjoint CG met non-positive curvature and no fallback    */
} dpd_status;

/* Precision of the iteration.  DPD_MIXED: FP32 triangular sweeps (and dense
 * A^{-1}) applied to FP64 residuals in correction form, and closest rotations
 * computed in FP32 and refined in FP64 (Newton steps of the polar iteration on
 * the FP32 factor, then one step of the rotation-derivative algebra against
 * F), accurate to FP64 round-off; factorization, residuals, corrections and
 * reductions stay FP64 (the fixed point is unchanged).                      */
enum { DPD_FP64 = 0, DPD_MIXED = 1 };
/* Adjoint solver.                                                          */
enum { DPD_BWD_FIXED_POINT = 0, DPD_BWD_PCG = 1 };
/* Forward solver: Alg. 1 (local/global PD), or Newton steps whose linear
 * systems (A - dA) d = -grad g are solved by conjugate gradients
 * preconditioned with the same factor of A.  Both stop on the same test and
 * converge to the same implicit-Euler state.                                */
enum { DPD_FWD_PD = 0, DPD_FWD_NEWTON_PCG = 1 };

typedef struct {
  /* physics (SI units) */
  double dx;               /* voxel edge length, m                               */
  double rho;              /* density, kg/m^3                                    */
  double nu;               /* Poisson ratio, 0 <= nu < 0.5                       */
  double h;                /* time step, s                                       */
  double gravity[3];       /* m/s^2                                              */
  double origin[3];        /* rest position of grid node (0,0,0), m              */
  double contact_k;        /* ground penalty stiffness per node, N/m; 0 = off    */
  double friction_mu;      /* explicit Coulomb friction coefficient; 0 = off     */
  double friction_eps;     /* friction velocity regulariser, m/s                 */
  double muscle_k;         /* fibre stiffness per volume, Pa; 0 = no muscles     */
  double fiber[3];         /* unit fibre direction, same for every element       */
  /* forward iteration (Alg. 1) */
  int32_t fwd_max_iter;    /* maximum number of global solves per step           */
  int32_t fwd_fixed_iters; /* 1: perform exactly fwd_max_iter solves              */
  double fwd_rel_tol;      /* stop when |grad g| <= tol |grad g(x^0)|            */
  double fwd_abs_tol_rel;  /* ... or |grad g| <= this * |M y / h^2| (free DoFs)   */
  int32_t fwd_solver;      /* DPD_FWD_PD or DPD_FWD_NEWTON_PCG                     */
  int32_t fwd_inner_max_iter; /* CG iterations per Newton step                    */
  double fwd_inner_tol;    /* CG relative tolerance per Newton step; a negative
                              value -e selects Eisenstat-Walker forcing terms
                              capped at e                                        */
  /* backward iteration (Alg. 2 or CG) */
  int32_t bwd_max_iter;
  int32_t bwd_solver;      /* DPD_BWD_FIXED_POINT or DPD_BWD_PCG                   */
  double bwd_rel_tol;      /* stop when |xbar - H z| <= tol |xbar|               */
  int32_t precision;       /* DPD_FP64 or DPD_MIXED                                */
  int32_t check_every;     /* iterations before the first host convergence check,
                              >= 1 (Alg. 1: every check_every iterations; a
                              multi-launch CG solve sizes its later chunks from
                              the observed convergence rate)                     */
  int32_t use_graphs;      /* 1: run conjugate-gradient iterations as HIP graphs  */
  int32_t fused_cg;        /* 1: meshes of at most 2048 free nodes keep A^{-1}
                              dense and run each conjugate-gradient solve in one
                              cooperative launch (same method and tolerances);
                              0: off; 2 + m: only with LDS placement m (bit 0:
                              r and q, bit 1: the workgroup's rows of A^{-1}),
                              off when m does not fit; read at factorization  */
  int32_t contact_fused;   /* 1: with the dense inverse, the inner loop of a time
                              step with contact (all iterations for one contact
                              set) runs as one cooperative launch; 0: a few
                              launches per iteration (same iteration)           */
  int32_t sweep_launch;    /* global step A^{-1} b through the factor's sweeps:
                              1: both sweeps in one launch whose tasks wait on
                              the tasks they depend on (default); 0: one launch
                              per tree level and sweep.  Same arithmetic, same
                              result bit for bit                                */
  double volume_scale;     /* volume-preserving term (supplemental Sec. Energy
                              Definitions, E = w/2 |F - D|^2, D the projection
                              of F onto det D = 1): weight per Gauss point
                              w = volume_scale * lambda * V_q with Lame's
                              lambda = E nu / ((1 + nu)(1 - 2 nu)); 0 = off.
                              With it on, solves use the factor's sweeps (the
                              fused dense solver and fused contact loops are
                              not used)                                        */
  int32_t leaf_nodes;      /* nested-dissection leaf size of the factor: 0 = chosen
                              by the solve-time estimate among 64, 128, 256, 512
                              (and all free nodes when they fit one block);
                              > 0 forces it.  Read at mesh creation.            */
  int32_t deflation;       /* adjoint CG on the multi-launch path: keep the search
                              directions H-orthogonal to this many (<= 16) Ritz
                              vectors of A^{-1} dA's largest eigenvalues (the
                              modes that make Alg. 2 and its acceleration slow),
                              built by Lanczos on the factor's solve and the
                              Hessian product; 0 = off.  The solution is the
                              same (to the tolerance); only iterations change  */
  int32_t deflation_refresh;  /* backward steps between rebuilds of those vectors
                              (0 = 25); the Hessian's products with them are
                              recomputed every step                            */
  int32_t factor_on_host;  /* 0 (default): dpd_factorize runs the multifrontal
                              Cholesky on the device (dense fronts, FP64 MFMA
                              updates; a transient workspace of sum ld^2 doubles
                              over the supernodes is allocated and freed by the
                              call); 1: on the host (C++ with OpenMP), the
                              panels then uploaded.  Same factor to rounding   */
  int32_t bwd_warm_start;  /* adjoint CG (multi-launch, fused or in the batch
                              engine; not deflated): 1 = start from the
                              previous backward step's solution z (the adjoint
                              of the step after this one), 2 = from the linear
                              extrapolation 2 z_{t+1} - z_{t+2} of the previous
                              two, 3 = from the quadratic one 3 z_{t+1} -
                              3 z_{t+2} + z_{t+3}, 4 = the Galerkin (H-norm best)
                              combination of the last five, Z c with
                              (Z^T H Z) c = Z^T xbar, 5..12 = the same over the
                              last that many; a start is kept only if its
                              residual is smaller than the right-hand side,
                              else zero.  0 (default) = from zero.  Same
                              stopping test (relative to the right-hand side);
                              the handle keeps the last solutions across calls
                              (one extra Hessian product per kept solution and
                              a host round trip with mode 4)                   */
  int32_t pad_opt;
} dpd_options;

typedef struct {
  int32_t fwd_iters;       /* global solves performed in the last forward step   */
  int32_t fwd_outer;       /* Newton steps (DPD_FWD_NEWTON_PCG), else fwd_iters   */
  int32_t bwd_iters;       /* adjoint iterations in the last backward step       */
  int32_t converged;       /* 1 if the last call met its tolerance                */
  int32_t fallbacks;       /* CG -> fixed-point fallbacks in the last backward    */
  int32_t inverted_qps;    /* quadrature points with det F <= 0, summed over the
                              local passes of the last forward step              */
  double fwd_rel_res;      /* final |grad g| / |grad g(x^0)|                      */
  double bwd_rel_res;      /* final |xbar - H z| / |xbar|                          */
  double ms_total;         /* wall time of the call when stats were requested     */
} dpd_stats;

typedef struct {
  int64_t n_nodes, n_elements, n_free, n_fixed, n_contact;
  int64_t n_supernodes, n_levels;
  int64_t factor_nnz;      /* stored entries of the factor panels (packed count)  */
  int64_t factor_bytes;    /* device bytes of the FP64 panels (both layouts)      */
  int64_t device_bytes;    /* all device memory owned by the handle               */
  int64_t leaf_nodes;      /* dissection leaf size chosen for the factor          */
  int64_t fused_blocks;    /* workgroups of the fused dense conjugate-gradient
                              launch; 0 when solves use the multi-launch path    */
  int64_t fused_lds;       /* its LDS placement, FP64 | FP32 << 2 (bits as in
                              dpd_options.fused_cg)                              */
  int64_t solve_workgroups;/* workgroups of the single-launch solve; 0 when its
                              plan does not fit (solves use the level launches) */
  int64_t solve_entries;   /* entries of its queue (both sweeps)                 */
  int64_t qp_per_element;  /* 8 (voxels, 2x2x2 Gauss points) or 1 (tetrahedra):
                              per-quadrature-point arrays hold this x n_elements */
  int64_t factor_us;       /* wall time of the last dpd_factorize (microseconds,
                              including the FP32 copies; 0 before the first)    */
  int64_t factor_flops;    /* floating-point operations of the numeric
                              factorization and panel construction: per
                              supernode 2n^3/3 + 2rn^2 + r^2 n (n columns,
                              r rows below)                                      */
} dpd_mesh_info;

/* Default options: dx 0.01, rho 1e3, nu 0.45, h 0.01, gravity (0,0,-9.81),
 * no contact, friction or muscles, fwd PD 100 iterations / 1e-10 / 1e-12
 * (Newton-CG inner loop: 200 iterations / 1e-2),
 * bwd CG 5000 iterations / 1e-10, FP64, check_every 8, HIP graphs on. */
dpd_status dpd_default_options(dpd_options* opt);

/* Build a mesh from voxels (Sec. Background: FEM nodes, lumped mass; supp.
 * Sec. Energy Definitions: energies integrated at Gauss points).
 *   cells_ijk   host, [n_cells][3] int32 voxel indices, unique
 *   youngs      host, [n_cells] Young's moduli in Pa (> 0)
 *   fixed_ijk   host, [n_fixed][3] grid nodes held at rest (Dirichlet), or NULL
 *   opt         host options (copied)
 *   out         receives the handle; NULL on failure
 * Assembles A = M/h^2 + sum_c w_c G_c^T G_c (eq:pd_global) over free nodes,
 * orders it by geometric nested dissection (leaf size chosen by an estimate of
 * the solve time) and performs the symbolic analysis; the numeric
 * factorization is dpd_factorize.  DPD_EINVAL on bad input (duplicate voxels,
 * fixed nodes not on the mesh, nu out of range, ...). */
dpd_status dpd_create_mesh(const int32_t* cells_ijk, int64_t n_cells, const double* youngs,
                           const int32_t* fixed_ijk, int64_t n_fixed,
                           const dpd_options* opt, dpd_mesh** out);

/* Build a mesh of linear tetrahedra (the paper's tetrahedral scenes, Sec.
 * Evaluation; the same energies through a constant deformation gradient per
 * element, F = D_s D_m^{-1}, i.e. G_e a constant 9 x 12 matrix, integrated
 * with weight V_e = |det D_m| / 6; lumped mass rho V_e / 4 per corner).
 *   X            host, [n_nodes][3] rest positions (m); public node order
 *   tets         host, [n_tets][4] corner node ids (either orientation;
 *                degenerate tetrahedra are rejected)
 *   youngs       host, [n_tets] Young's moduli in Pa (> 0)
 *   fixed_nodes  host, [n_fixed] node ids held at rest, or NULL
 *   opt          host options (copied); dx, origin, muscles and the
 *                volume-preserving term do not apply (muscle_k and
 *                volume_scale must be 0); contact_k > 0 puts the ground
 *                penalty on the nodes of minimal rest height
 * Orders A_s by nested dissection of the node graph (median splits of the
 * rest positions, the boundary nodes of one half as separators).  Every step,
 * solve and gradient call accepts the handle; the fused dense solver, the
 * complementarity-contact calls and dpd_node_ijk do not apply (the latter two
 * return DPD_EINVAL).  DPD_EINVAL on bad input. */
dpd_status dpd_create_tet_mesh(const double* X, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                               const double* youngs, const int32_t* fixed_nodes, int64_t n_fixed,
                               const dpd_options* opt, dpd_mesh** out);

/* Waits for the device to finish outstanding work, then frees the handle. */
void dpd_destroy_mesh(dpd_mesh* mesh);

dpd_status dpd_get_info(const dpd_mesh* mesh, dpd_mesh_info* info);

/* Host copies: node grid coordinates [N][3] int32; rest positions [3][N];
 * contact-candidate node indices [n_contact] int32 (nodes of minimal rest
 * height when contact_k > 0). */
dpd_status dpd_node_ijk(const dpd_mesh* mesh, int32_t* ijk_host);
dpd_status dpd_rest_positions(const dpd_mesh* mesh, double* X_host);
dpd_status dpd_contact_nodes(const dpd_mesh* mesh, int32_t* nodes_host);

/* Replace the options used by later step calls (physics fields must not
 * change: dx, rho, nu, h, contact, muscles are fixed at creation; changing
 * them returns DPD_EINVAL).  Iteration controls and precision may change. */
dpd_status dpd_set_options(dpd_mesh* mesh, const dpd_options* opt);

/* Replace the per-element Young's moduli (device or host pointer as flagged,
 * [n_elements] Pa).  Marks the factor stale: the next step needs
 * dpd_factorize again (DPD_ESTATE otherwise). */
dpd_status dpd_set_youngs(dpd_mesh* mesh, const double* youngs, int32_t on_device, void* stream);

/* Numeric Cholesky factorization of A, computed once per material
 * (Sec. Background: the factorization of the constant matrix A can be
 * precomputed).  Builds the FP64 panels of the sweeps (and FP32 copies when
 * precision is DPD_MIXED): on the device by default (multifrontal, level by
 * level, FP64 MFMA on the dense fronts; see dpd_options.factor_on_host).
 * Synchronizes the stream.  DPD_ENOTSPD on a non-positive (or non-finite)
 * pivot, DPD_ENOMEM if the transient front workspace cannot be allocated. */
dpd_status dpd_factorize(dpd_mesh* mesh, void* stream);

/* One implicit-Euler step (eq:time_integration):
 *   y = x + h v + h^2 M^{-1} (M g + f_friction(x, v)); x^0 = y (Dirichlet nodes
 *   at rest); then Alg. 1 (local projections and a global solve with A) or,
 *   with DPD_FWD_NEWTON_PCG, Newton steps on g whose systems are solved by
 *   conjugate gradients preconditioned with A; both stop on the same test.
 *   x, v        device [3][N], read-only
 *   act         device [n_elements] muscle actuation (1 = rest length), or NULL
 *   x_next      device [3][N], overwritten; must not alias x or v
 *   v_next      device [3][N], overwritten: (x_next - x) / h
 *   stats       host or NULL
 * The host reads the iteration state between chunks of enqueued iterations
 * (see check_every; with the fused solver, after batches of Newton steps
 * enqueued ahead of their test) and at the end: the call returns with the
 * step complete on the stream. */
dpd_status dpd_forward_step(dpd_mesh* mesh, void* stream, const double* x, const double* v,
                            const double* act, double* x_next, double* v_next, dpd_stats* stats);

/* Adjoint of one step (eq:adjoint, eq:chain_rule; Alg. 2 or its CG
 * acceleration).  Given dL/dx_next and dL/dv_next, returns dL/dx, dL/dv and
 * parameter gradients.
 *   x, v, act, x_next   as passed to / returned by dpd_forward_step
 *   gx_next, gv_next    device [3][N]
 *   gx, gv              device [3][N], overwritten; must not alias the inputs
 *   g_youngs            device [n_elements], ACCUMULATED (+=), or NULL
 *   g_act               device [n_elements], overwritten, or NULL
 *   stats               host or NULL
 * Returns with the step complete on the stream (the host reads the adjoint
 * iteration's state between chunks of iterations and at the end). */
dpd_status dpd_backward_step(dpd_mesh* mesh, void* stream, const double* x, const double* v,
                             const double* act, const double* x_next, const double* gx_next,
                             const double* gv_next, double* gx, double* gv, double* g_youngs,
                             double* g_act, dpd_stats* stats);

/* Building blocks, exposed for kernel-level tests and custom solvers.  All
 * device [3][N] arrays; fixed-node rows of outputs are zero.
 *   dpd_apply_inverse:  out = A^{-1} b on free nodes (eq:pd_global's matrix)
 *   dpd_gradient:       out = grad g(x) = A x - b(x) for the given y (eq:energy_grad)
 *   dpd_hessian_apply:  out = (A - dA(x)) p (eq:matrix_split)
 *   dpd_rotations:      R_out device [9][8 n_elements]: closest rotation at each
 *                       Gauss point q = 8e + (qx + 2 qy + 4 qz), row-major 3x3
 *                       (tetrahedra: [9][n_elements], one per element) */
dpd_status dpd_apply_inverse(dpd_mesh* mesh, void* stream, int32_t precision, const double* b,
                             double* out);
dpd_status dpd_gradient(dpd_mesh* mesh, void* stream, const double* x, const double* y,
                        const double* act, double* out);
dpd_status dpd_hessian_apply(dpd_mesh* mesh, void* stream, const double* x, const double* act,
                             const double* p, double* out);
dpd_status dpd_rotations(dpd_mesh* mesh, void* stream, const double* x, double* R_out);

/* dpd_gradient for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, but the element forces, the
 * reduction partials and the reduction's state live in one library-owned
 * static device array per GPU (3 MiB plus a few KiB, held until the process
 * ends) instead of the mesh's workspace.  The call allocates nothing.
 *   Limit: meshes of at most 16384 elements; larger ones get DPD_EINVAL and
 *          nothing is launched.
 *   Sharing: every call on one GPU uses that GPU's array; calls that overlap
 *          on one GPU (other streams or threads) race.  Stream-ordered calls
 *          are safe: each call resets the state it needs.
 *   Arguments as dpd_gradient (device [3][N] x, y, out; act device [E] or NULL). */
dpd_status dpd_gradient_noalloc(dpd_mesh* mesh, void* stream, const double* x, const double* y,
                                const double* act, double* out);

/* Global step with a contact set (Sec. Contact, complementarity contact; the
 * low-rank update of Alg. 4): x with x_C = x* and A_{C̄×C̄} x_{C̄} = b_{C̄},
 * from the factor of A.  C is a set of free nodes whose positions are
 * prescribed; b is the right-hand side the contact step forms (the effect of
 * x* through the elements is already in it).
 *
 * dpd_contact_prepare caches A^{-1} e_j for every candidate node j (the
 * paper's precomputed A^{-1} I_{I×C} for the largest contact set: one scalar
 * column per node since A = I_3 (x) A_s; n_cand x N doubles on the device).
 *   nodes_host  host, [n_cand] int32 public ids of free nodes, distinct
 * After dpd_factorize (which discards the cache); calling it again replaces
 * the candidate list.  Synchronizes the stream.  DPD_EINVAL for
 * out-of-range, fixed or repeated nodes.
 *
 * dpd_contact_solve:
 *   set_host    host, [c] int32 indices into the candidate list, distinct,
 *               0 <= c <= 120 (the c x c capacitance matrix is factorized
 *               in one workgroup's LDS); c = 0 is the plain global step
 *   xstar       device, [3][c] prescribed positions of the set's nodes
 *   b           device, [3][N]
 *   x           device, [3][N], overwritten (rows of fixed nodes 0); must
 *               not alias b
 * Computes a1 = A^{-1} b, lam = -((A^{-1})_{C×C})^{-1} (a1)_C (the Woodbury
 * identity in capacitance form: c x c and SPD), x = a1 + the set's columns of
 * A^{-1} times lam, x_C = x*.  The inverse of the c x c matrix depends on
 * the set only (fixed through Alg. 3's inner iterations): it is computed by
 * Cholesky when the set differs from the previous call's, which synchronizes
 * the stream (DPD_ENOTSPD on a non-positive pivot); otherwise the call is
 * asynchronous. */
dpd_status dpd_contact_prepare(dpd_mesh* mesh, void* stream, const int32_t* nodes_host, int32_t n_cand);
dpd_status dpd_contact_solve(dpd_mesh* mesh, void* stream, const int32_t* set_host, int32_t c,
                             const double* xstar, const double* b, double* x);

/* Time step with complementarity contact against the ground plane z = 0
 * (Sec. Contact: eq:lcp, eq:time_integration_with_contact; Alg. 3 forward,
 * Alg. 5 backward), on the candidates of the last dpd_contact_prepare.
 *
 * dpd_contact_forward_step: collision detection (a candidate whose ray
 * x_j + t v_j, 0 <= t <= h, meets the plane gets the meeting point as its
 * target, kind 1; one already below it gets (x_j, y_j, 0), kind 2), then
 * Alg. 3: for the set C of candidates with a target, x = y with x_C = x*,
 * local steps and reduced global steps (each one A^{-1} solve and the
 * low-rank correction of dpd_contact_solve) until |grad g| over the free
 * nodes outside C is within fwd_rel_tol of its first value (or fwd_abs_tol_rel
 * of |M y / h^2|); then the contact forces r = grad g(x) on C update the set:
 * a node with r_z < 0 leaves it (at most once per step, so the loop ends), a
 * candidate below the plane joins it with target (x_j, y_j, 0) of its
 * start-of-step position.  Repeats until the set stays the same.
 *   x, v, act, x_next, v_next   as dpd_forward_step
 *   kind_out    host, [n_cand] int32, overwritten: 0 (not in contact), 1
 *               (ray target), 2 (static target), per candidate; the input
 *               of the backward step
 *   stats       fwd_iters = PD iterations over all sets, fwd_outer = sets
 *               tried, fwd_rel_res = the largest final relative residual
 * Synchronizes the stream (the set decisions are taken on the host from
 * device results).  DPD_ESTATE without candidates, DPD_EINVAL when the set
 * would exceed 120 nodes, DPD_NOT_CONVERGED when a set's PD loop reached
 * fwd_max_iter (the outputs are still written).  The fwd_solver option is not
 * used: the inner loop is Alg. 3's PD iteration; its global steps run in FP64
 * (the local step's rotations follow the precision option).  Where A^{-1} is held
 * dense (fused_cg on, at most 2048 free nodes) the reduced matrix's inverse
 * is formed once per set from it and each reduced global step is one dense
 * product (with contact_fused, the set's whole loop is one cooperative
 * launch); otherwise each is a sweep of the factor plus the low-rank
 * correction.
 *
 * dpd_contact_backward_step: z solves (A - dA)_{C̄×C̄} z = xbar_{C̄} (the
 * reduced adjoint system) by Alg. 5's iteration, each step a reduced global
 * step; dL/dy = M z / h^2; the targets carry dL/dx* = xbar_C - ((A - dA) z)_C
 * back to x and v through their formulas (kind 1: t = -z_j / v_{j,z});
 * parameter gradients as dpd_backward_step.
 *   kind_host   host, [n_cand] int32 from the forward step (values 0..2)
 *   other arguments as dpd_backward_step
 * Alg. 5's fixed-point iteration, FP64; where the fused loop runs (dense
 * inverse, contact_fused) and bwd_solver is DPD_BWD_PCG, its quasi-Newton
 * acceleration instead: conjugate gradients on the same reduced system
 * preconditioned by the reduced inverse, falling back to Alg. 5's iteration
 * from the current z on non-positive curvature (stats->fallbacks = 1).
 * Synchronizes the stream.  DPD_NOT_CONVERGED when bwd_max_iter is reached. */
dpd_status dpd_contact_forward_step(dpd_mesh* mesh, void* stream, const double* x, const double* v,
                                    const double* act, double* x_next, double* v_next, int32_t* kind_out,
                                    dpd_stats* stats);
dpd_status dpd_contact_backward_step(dpd_mesh* mesh, void* stream, const double* x, const double* v,
                                     const double* act, const double* x_next, const int32_t* kind_host,
                                     const double* gx_next, const double* gv_next, double* gx, double* gv,
                                     double* g_youngs, double* g_act, dpd_stats* stats);

/* Kernel timing for roofline measurement.  After dpd_profile_start(mesh, k),
 * launches of kernel class k made by calls on this handle are timed and the
 * algorithmic bytes and flops of each timed launch (what the method must move
 * or compute, from the factor structure and the mesh) are added up;
 * dpd_profile_read synchronizes the stream, returns the totals since the start
 * and stops timing.  Launches that exit at once because their iteration had
 * already converged are not counted.
 *  - Single-kernel classes (sweeps, local steps): every launch outside graph
 *    capture is timed on the device by the constant-rate clock
 *    (hipDeviceAttributeWallClockRate): from the entry of workgroup 0 to the
 *    exit of the last workgroup to finish.  While such a class is profiled,
 *    the conjugate-gradient loop replays one chunk of iterations in every 17
 *    as direct launches (the rest as graphs), so the totals describe those.
 *  - DPD_PROF_SOLVE: one whole A^{-1} b in every 17 is bracketed by events on
 *    the launch stream behind a bounded stream hold.
 *  - DPD_PROF_CG_DENSE: every fused solve, by its own device clock
 *    (workgroup 0 at entry and at exit).
 * Class DPD_PROF_OFF disables timing.  Profiling one handle from several
 * streams at once is not supported. */
enum {
  DPD_PROF_OFF = 0,
  DPD_PROF_SWEEP_FWD = 1,        /* k_sweep_fwd: forward level, blocks of <= 64 columns     */
  DPD_PROF_SWEEP_BWD = 2,        /* k_sweep_bwd: backward level, column tasks               */
  DPD_PROF_ELEM_HVP = 3,         /* k_elem_hvp: adjoint local step                          */
  DPD_PROF_ELEM_FORCES = 4,      /* k_elem_forces: forward local step                       */
  DPD_PROF_SOLVE = 5,            /* a whole A^{-1} b, all of its launches                   */
  DPD_PROF_SWEEP_FWD_WIDE = 6,   /* k_sweep_fwd_wide: forward level, wide blocks            */
  DPD_PROF_SWEEP_BWD_NARROW = 7, /* k_sweep_bwd_narrow: backward level of many small blocks */
  DPD_PROF_CG_DENSE = 8,         /* k_cg_dense: a whole fused conjugate-gradient solve      */
  DPD_PROF_CONTACT_UPDATE = 9,   /* k_contact_update: active-set columns of A^{-1} applied  */
  DPD_PROF_CONTACT_DESCEND = 10, /* k_contact_descend: reduced global step of a contact step */
  DPD_PROF_CONTACT_DENSE = 11,   /* k_contact_dense_step: the same with a dense inverse      */
  DPD_PROF_CONTACT_FUSED = 12,   /* k_contact_fused: a contact set's whole inner loop        */
  DPD_PROF_CONTACT_FUSED_CG = 13,/* k_contact_fused_cg: the contact adjoint's CG loop         */
  DPD_PROF_SOLVE_DAG = 14        /* k_solve_dag: a whole A^{-1} b in one launch (sweep_launch 1) */
};
typedef struct {
  int64_t launches;
  double total_ms;         /* summed durations of the timed launches (device
                              clock; event pairs for DPD_PROF_SOLVE)           */
  double bytes;            /* summed algorithmic bytes                           */
  double flops;            /* summed algorithmic floating-point operations       */
  int64_t iterations;      /* device-side iterations of the timed launches (class
                              DPD_PROF_CG_DENSE), else 0                         */
  double event_ms;         /* summed event-pair durations (DPD_PROF_SOLVE), else 0 */
} dpd_kernel_profile;
dpd_status dpd_profile_start(dpd_mesh* mesh, int32_t kernel_class);
dpd_status dpd_profile_read(dpd_mesh* mesh, void* stream, dpd_kernel_profile* out);

/* ------------------------------------------------------------------------
 * Rollout server with continuous batching.
 *
 * A request is a whole differentiable rollout: build the mesh, factorize A,
 * run T forward steps from rest, evaluate L = c . x_T and run the T adjoint
 * steps back to the initial state.  The server keeps up to max_slots requests
 * resident on the device at once, each with its own factor and states (the
 * factorization is done once per request and kept, Sec. Background).  A
 * queued request is admitted as soon as a slot is free and its device
 * footprint (factor panels, mesh buffers, the T + 1 stored states) fits in
 * what remains of hbm_budget_bytes; requests arriving while others run join
 * as slots and memory free up.
 *
 * batched != 0: the conjugate-gradient solves of all resident requests (the
 * Newton steps of the forward steps and the adjoint systems of Alg. 2's
 * quasi-Newton acceleration, Sec. DiffPD) run together: each iteration is
 * one launch per triangular-sweep level and kernel shape over every
 * request's tasks, then one launch each for the element Hessian product (the
 * adjoint local step), the node gather with the inner products, and the
 * vector update; solves join and leave the batch every few iterations.  The
 * rest of each step (the forward local step and residual, prologue and
 * epilogue kernels) runs on the request's own stream.  Requests take the
 * multi-launch solver (dpd_options.fused_cg is ignored).  Served
 * requests never capture HIP graphs (dpd_options.use_graphs is ignored): a
 * capture under way in one worker would make another worker's synchronous
 * runtime calls fail.
 * batched == 0: each request iterates on its own HIP stream (default
 * priority); kernels of different requests overlap on the device.
 *
 * Either way a request's results do not depend on what else runs, bitwise:
 * every kernel is deterministic and a batched slot runs exactly its own
 * blocks' arithmetic.
 * ------------------------------------------------------------------------ */
typedef struct dpd_server dpd_server;

typedef struct {
  const int32_t* cells_ijk;  /* host [n_cells][3]                             */
  int64_t n_cells;
  const double* youngs;      /* host [n_cells]                                */
  const int32_t* fixed_ijk;  /* host [n_fixed][3] or NULL                     */
  int64_t n_fixed;
  const double* loss_x;      /* host [3][N] weights c of L = c . x_T           */
  int64_t n_nodes;           /* N of the mesh the cells define (checked)      */
  int32_t steps;             /* T >= 1                                         */
  int32_t pad;
  dpd_options opt;           /* physics and solver settings of this request    */
} dpd_request;               /* everything is copied by dpd_server_submit      */

enum { DPD_REQ_QUEUED = 0, DPD_REQ_RUNNING = 1, DPD_REQ_DONE = 2, DPD_REQ_FAILED = 3 };

typedef struct {
  int32_t state;             /* DPD_REQ_*                                      */
  int32_t status;            /* dpd_status of the request (soft or hard)       */
  double loss;               /* c . x_T                                        */
  double t_submit, t_admit, t_done;  /* seconds since dpd_server_create        */
  int64_t n_nodes, n_elements, footprint_bytes;
  int64_t fwd_iters, bwd_iters;      /* summed over the T steps                */
} dpd_result;

/* max_slots >= 1 requests resident at once within hbm_budget_bytes of device
 * memory, on the device current at creation; batched selects the batch engine
 * (above). */
dpd_status dpd_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int32_t batched,
                             dpd_server** out);
/* Queue a request (copied); returns its ticket.  Never blocks on the GPU. */
dpd_status dpd_server_submit(dpd_server* srv, const dpd_request* req, int64_t* ticket);
/* Result of a ticket; the gradient outputs (host, or NULL) are filled once the
 * request is done: g_x0, g_v0 [3][N], g_youngs [n_cells]. */
dpd_status dpd_server_poll(dpd_server* srv, int64_t ticket, dpd_result* out, double* g_x0,
                           double* g_v0, double* g_youngs);
/* Block until every submitted request has finished. */
dpd_status dpd_server_drain(dpd_server* srv);
/* Peak device bytes admitted at once and peak number of resident requests. */
dpd_status dpd_server_stats(dpd_server* srv, int64_t* peak_bytes, int32_t* peak_active);
void dpd_server_destroy(dpd_server* srv);   /* drains first */

typedef struct {
  int64_t iterations;       /* batched conjugate-gradient iterations launched      */
  int64_t slot_iterations;  /* their sum over the solves taking part (occupancy)   */
  int64_t launches;         /* kernel launches made for them                       */
  int64_t solves;           /* solves completed in the batch engine                */
  int32_t peak_slots;       /* most solves in one batch                            */
  int32_t pad;
} dpd_batch_stats;
/* Counters of the batch engine since creation (all zero when batched == 0). */
dpd_status dpd_server_batch_stats(dpd_server* srv, dpd_batch_stats* out);

const char* dpd_status_string(dpd_status s);
const char* dpd_last_error(const dpd_mesh* mesh);   /* thread-local if mesh is NULL */

#ifdef __cplusplus
}
#endif
#endif /* DIFFPD_H */
