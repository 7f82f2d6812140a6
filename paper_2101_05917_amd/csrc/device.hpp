// Device-side data of one mesh and the kernel launchers (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace dpd {

// Scalars the iteration kernels exchange without host round trips.  One per
// handle; reductions finalize into it with a last-block-done pattern.
struct IterState {
  double r0sq, rsq, atolsq, tolsq;   // forward / fixed-point residual norms
  double nb2;                        // |xbar|^2 (adjoint)
  double rs, pq, alpha, beta;        // conjugate-gradient scalars
  double acc;                        // scratch accumulator
  int32_t iter, done, converged, nonfinite, curvature, inverted;
  uint32_t counter;                  // last-block-done ticket
  int32_t max_iter;                  // iteration cap of the conjugate-gradient loop
  int32_t aborted;                   // the fused solver's grid barrier timed out
  int32_t solves;                    // Newton forward: conjugate-gradient iterations so far
  double g_prev, eta;                // Newton forward: previous |grad g| and forcing term
};

// Device-side accumulation of the fused solver's launches while it is being
// profiled: constant-rate clock ticks from workgroup 0's entry to its exit,
// iterations and launches (launches that exit at once are not counted).
struct ProfAcc {
  unsigned long long ticks, iters, launches, pad;
};

struct DevSolve {
  int32_t nf;                 // free nodes
  const int32_t* perm_pub;    // [nf] internal index -> public node id
  const int32_t* rows;        // concatenated R_s (internal)
  const int32_t* cptr;        // [nf + 1]
  const int32_t* cidx;        // positions into U
  const double* panel64;       // column-major panels (backward, narrow forward)
  const float* panel32;
  const double* panelT64;      // row-major copies (wide forward)
  const float* panelT32;
  double* y_int;              // [3][nf]
  double* x_int;              // [3][nf]
  double* U;                  // [u_size][3]
  double* bt;                 // [3][nf] gathered right-hand sides of pre-gathered levels
};

struct DevMesh {
  int32_t N, E, nf;
  int32_t local32;            // 1: FP32 closest rotations polished in FP64 (mixed precision)
  double h, dx, nu, Vq;
  double g[3];
  double contact_k, friction_mu, friction_eps;
  double muscle_k, fiber[3];
  const double* X;            // [3][N]
  const double* mass;         // [N]
  const int32_t* conn;        // [8][E]
  const int32_t* node_inc;    // [8][N], 8e + a or -1
  const uint8_t* fixed;       // [N]
  const uint8_t* contact;     // [N]
  const double* w_e;          // [E] corotated weight per Gauss point, 2 mu_e V_q
  const double* wv_e;         // [E] volume-preserving weight per Gauss point, or null (term off)
  double dwv_dE;              // d(wv_e)/dE_e
  uint8_t* cmask;             // [N] ground contact active at the linearisation point
  // linear tetrahedra (corners = 4; voxels: 8): conn is [4][E]; the node
  // gather runs over the compressed incidence instead of node_inc
  int32_t corners;
  const double* dminv;        // [9][E] D_m^{-1} (row-major entries), tetrahedra
  const double* vol;          // [E] element volumes, tetrahedra
  const int32_t* inc_ptr;     // [N + 1] incidence ranges, tetrahedra (else null)
  const int32_t* inc;         // [4E] entries 4e + a
};

constexpr int kElemsPerBlock = kBlock / 8;

// Dense form of the preconditioned conjugate-gradient solve for meshes with
// few free nodes: A^{-1} kept as an explicit n x n matrix (internal order) and
// the whole iteration in one cooperative launch.  Workgroup b owns the rows
// [b R, b R + R) of every internal-order vector and the hex elements that touch
// them (computed redundantly where workgroups share an element).
constexpr int kDenseMaxRows = 8;                // rows per workgroup (R)
constexpr int kDenseBlock = 512;                // threads per workgroup
constexpr int kDenseElems = kDenseBlock / 8;    // elements evaluated at once, one per 8 lanes
static_assert(8 * kDenseMaxRows <= kDenseElems, "a workgroup's rows touch at most 8 R elements");
constexpr int kDenseBarWords = 64 * 9;          // barrier counters (top, abort, 8 groups)
constexpr int kDenseVecLds = 1;                 // r and q of every row live in each workgroup's LDS
constexpr int kDenseAinvLds = 2;                // the workgroup's rows of A^{-1} live in its LDS
struct DenseCG {
  int32_t n, rows;            // free nodes; rows per workgroup R
  int32_t max_elems;          // largest element list of a workgroup
  int32_t mode64, mode32;     // kDenseVecLds | kDenseAinvLds per precision of A^{-1}
  int32_t pad;
  const int32_t* perm;        // [n] internal row -> public node
  const int32_t* inv;         // [N] public node -> internal row, -1 when fixed
  const double* ainv64;       // [n][n] A^{-1} (symmetric; row j = column j)
  const float* ainv32;
  const int32_t* blk_eoff;    // [G + 1] element-list ranges
  const int32_t* blk_elems;   // concatenated element lists
  const int32_t* row_inc;     // [n][8] list slot * 8 + corner per incidence, -1 padded
  double* r;                  // [2][3][n] residuals r_k (k even, odd)
  double* q;                  // [2][3][n] H p_k (k even, odd)
  double* p;                  // [3][n]
  double* s;                  // [3][n] A^{-1} r_k
  double* w;                  // [2][3][n] H s_k (k even, odd)
  double* z;                  // [3][n] solution
  double* part;               // [2][G][2] per-workgroup partial inner products (k even, odd)
  uint32_t* bar;              // [kDenseBarWords] barrier counters and abort flag
  uint32_t* ready;            // [G] how many s vectors workgroup b has published in this launch
  const int32_t* nbr_off;     // [G + 1] ranges of nbr
  const int32_t* nbr;         // workgroups owning rows at workgroup b's element corners (b excluded)
  const double* nb2_ref;      // set for a warm-started solve: |b|^2 of the stopping test (else |r_0|^2)
};

void launch_hold(hipStream_t s, int periods);

// Element kernels of linear tetrahedra (one lane per element; the element
// launchers above dispatch to them when DevMesh::corners == 4).
void launch_tet_forces(const DevMesh& M, hipStream_t s, const double* x, double* fe, double* R_out, IterState* st);
void launch_tet_adj_cache(const DevMesh& M, hipStream_t s, const double* x, double* cache, IterState* st,
                          const IterState* gate);
void launch_tet_hvp(const DevMesh& M, hipStream_t s, const double* p, const double* cache, double* fe,
                    const IterState* st);
void launch_tet_grad_params(const DevMesh& M, hipStream_t s, const double* xn, const double* z, const double* cache,
                            double* g_youngs, const IterState* gate);

// Deflated conjugate gradients: the adjoint solve's search directions are kept
// H-orthogonal to a space W of k <= kDeflMax vectors (Ritz vectors of the
// preconditioned operator's slowest modes), with E = W^T H W.
constexpr int kDeflMax = 16;
struct DeflState {
  double einv[kDeflMax * kDeflMax];  // E^{-1}, row-major k x k
  double mu[kDeflMax];               // this iteration's projection coefficients E^{-1} (HW)^T s
};
// Chronopoulos-Gear step with deflation: w = H s, gamma = r.s, delta = w.s and
// c = (HW)^T s in one deterministic grid reduction (partials: (k + 2) per
// block); mu = E^{-1} c; alpha = gamma / (delta - beta gamma / alpha_old - mu.c).
void launch_cg_hvp_dots_defl(const DevMesh& M, hipStream_t s, const double* sv, const double* fe, const double* r,
                             double* w, IterState* st, double* partials, const double* HW, int k, DeflState* D);
// p = s + beta p - W mu; q = w + beta q - HW mu; z += alpha p; r -= alpha q; |r|^2.
void launch_cg_step_defl(const DevMesh& M, hipStream_t s, double* z, double* r, double* p, double* q,
                         const double* sv, const double* w, IterState* st, double* partials, const double* W,
                         const double* HW, int k, const DeflState* D);
// out[i] = X_i . y for the cnt vectors X_i = X + i * n (n doubles each), in a
// fixed summation order (per-chunk partials, then one block per i).
void launch_multi_dot(hipStream_t s, const double* X, int cnt, const double* y, int64_t n, double* partials,
                      double* out);
// y += sign * sum_i c[i] X_i (c on the device, cnt <= 64).
void launch_multi_axpy(hipStream_t s, double* y, const double* X, int cnt, const double* c, int64_t n, double sign);

// Dynamic LDS a backward column task may use to stage [y_s; x_R] (3 doubles per
// panel row); longer panels read the vector from memory.
constexpr int64_t kSweepLdsBudget = 60 * 1024;

// One handle's conjugate-gradient solve inside a batched iteration (several
// handles' iterations in the same launches): its mesh, vectors and state, and
// where its blocks start in the batched element and node launches.
struct BatchCgSlot {
  DevMesh M;
  const double* cache;        // per-Gauss-point adjoint cache at the linearisation point
  double* fe;                 // [3][8E] element corner forces
  double* sv;                 // [3][N] s = A^{-1} r
  double* r;                  // [3][N] residual
  double* w;                  // [3][N] H s
  double *z, *p, *q;          // [3][N] solution and direction vectors
  IterState* st;              // the solve's scalars and stopping state
  double* partials;           // per-block partial sums of its reductions
  int32_t elem_block0, node_block0, node_blocks, pad;
};

// One handle's triangular solve inside a batched sweep launch: its factor and
// the right-hand side / solution vectors (public order, [3][N]).  Tasks of a
// batched launch name their slot in SweepTask::pad0 and, on pre-gathered wide
// forward levels, carry pad1 = 1.
struct BatchSolveSlot {
  DevSolve S;
  const double* b;
  double* out;
  const IterState* st;
  int32_t N, pad;
};

// Batched launches.  Forward and backward level launches take the tasks of one
// kernel shape (kind, lanes per row or column, LDS staging) from any number of
// slots; gather entries are (slot, internal column) pairs.
void launch_batch_sweep_fwd(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks, int ntasks,
                            int lds_cols, bool fp32);
void launch_batch_sweep_fwd_wide(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks, int ntasks,
                                 int lpr, int lds_cols, bool fp32);
void launch_batch_sweep_gather(const BatchSolveSlot* slots, hipStream_t s, const int2* cols, int ncols);
void launch_batch_sweep_bwd(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks, int ntasks,
                            int lpr, bool use_lds, int lds_rows, bool fp32);
void launch_batch_sweep_bwd_narrow(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks,
                                   int ntasks, int lds_rows, bool fp32);
// element Hessian product, node gather + inner products, vector update
void launch_batch_cg_iteration_tail(const BatchCgSlot* slots, int nslots, int elem_blocks, int node_blocks,
                                    hipStream_t s);

// Device side of the single-launch solve (DagPlan uploaded).
struct DevDag {
  const DagEntry* q;
  int32_t nq, ns, grid, bwd_region;
  const SweepTask* fwd;
  const SweepTask* bwd;
  const int32_t* gcols;
  const DagSn* sn;
  uint32_t* ctr;
  size_t lds_bytes;
};

// Device-side timing of the launches of one kernel class while it is being
// profiled, by the constant 100 MHz clock of s_memrealtime (the same on every
// XCD): workgroup 0 subtracts its entry time from the total and the last
// workgroup to finish adds its exit time (two additions to one counter, so
// their order does not matter), then counts the launch and its work.
// Launches that exit at once because their iteration has already finished
// stamp nothing.  Launches of one class on one handle run in stream order, so
// one record serves them all.
struct LaunchClock {
  unsigned long long ticks, launches;
  double bytes, flops;          // algorithmic work of the counted launches
  unsigned int arrived, pad;    // workgroups of the launch in flight that have finished
};
struct ClockArg {
  LaunchClock* c;               // null: not timed
  double bytes, flops;          // algorithmic work of this launch
};
extern thread_local ClockArg g_launch_clock;
inline ClockArg take_launch_clock() {
  const ClockArg a = g_launch_clock;
  g_launch_clock = ClockArg{};
  return a;
}

// Launch of a kernel whose last parameter is a ClockArg: the clock set for the
// next launch of its class (by the profiler's scope), else none.
#define DPD_LAUNCH(kernel, grid, block, shmem, stream, ...) \
  hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__, ::dpd::take_launch_clock())

__device__ inline void clock_enter(const ClockArg& ck) {
  if (ck.c && blockIdx.x == 0 && threadIdx.x == 0)
    atomicAdd(&ck.c->ticks, 0ull - (unsigned long long)wall_clock64());
}

// Every thread of the workgroup calls this last (it holds a workgroup barrier).
__device__ inline void clock_exit(const ClockArg& ck) {
  if (!ck.c) return;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const unsigned int n = gridDim.x * gridDim.y * gridDim.z;
  if (atomicAdd(&ck.c->arrived, 1u) != n - 1) return;
  atomicAdd(&ck.c->ticks, (unsigned long long)wall_clock64());
  atomicAdd(&ck.c->launches, 1ull);
  atomicAdd(&ck.c->bytes, ck.bytes);
  atomicAdd(&ck.c->flops, ck.flops);
  atomicExch(&ck.c->arrived, 0u);
}

}  // namespace dpd

namespace dpd {
// kernel launchers (kernels.hip)
void launch_lincomb(hipStream_t s, int64_t n, double* out, double a, const double* x, double b,
                    const double* y);
void launch_fill(hipStream_t s, int64_t n, double* out, double v);
void launch_reset(hipStream_t s, IterState* st, double tolsq, int max_iter);
void launch_prologue(const DevMesh& M, hipStream_t s, const double* x, const double* v, double* y,
                     double* xn, IterState* st, double* partials, double abs_tol_rel);
void launch_elem_forces(const DevMesh& M, hipStream_t s, const double* x, const double* act,
                        double* fe, double* R_out, IterState* st);
void launch_node_residual(const DevMesh& M, hipStream_t s, const double* x, const double* y,
                          const double* fe, double* r, IterState* st, double* partials, int k,
                          int max_iter, int fixed_iters);
void launch_velocity(const DevMesh& M, hipStream_t s, const double* x, const double* xn, double* vn);
void launch_zero_fixed(const DevMesh& M, hipStream_t s, double* v);
// Warm start safeguard on the device: where |r_0|^2 (w[1].nb2) is not below
// |b|^2 (w[0].nb2), z0 := 0 and r := b.
void launch_warm_select(hipStream_t s, int64_t n, double* z0, double* r, const double* b, const IterState* w);
void launch_solve_dag(const DevSolve& S, const DevDag& D, hipStream_t s, bool fp32, const double* b, double* out,
                      int N, double alpha, int accumulate, const IterState* st);
const void* solve_dag_kernel(bool fp32);
void launch_sweep_fwd(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks,
                      int lds_cols, bool fp32, const double* b, int N, const IterState* st);
void launch_sweep_fwd_wide(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks,
                           int lds_cols, bool fp32, const double* b, int N, const int32_t* gather_cols,
                           int n_gather, const IterState* st);
void launch_sweep_bwd_narrow(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks,
                             int lds_rows, bool fp32, double* out, int N, double alpha, int accumulate,
                             const IterState* st);
void launch_sweep_bwd(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks,
                      int lds_rows, bool use_lds, bool fp32, double* out, int N, double alpha,
                      int accumulate, const IterState* st);
void launch_adj_cache(const DevMesh& M, hipStream_t s, const double* x, const double* act,
                      double* cache, IterState* st, const IterState* gate = nullptr);
void launch_newton_inner(hipStream_t s, IterState* outer, IterState* inner, double eta_max, int adaptive,
                         double rel_tol, int inner_max_iter, int max_iter);
void launch_newton_update(hipStream_t s, int64_t n3, IterState* outer, const IterState* inner, double* xn,
                          const double* z);
void launch_elem_hvp(const DevMesh& M, hipStream_t s, const double* p, const double* cache,
                     double* fe, const IterState* st);
void launch_node_hvp(const DevMesh& M, hipStream_t s, const double* p, const double* fe,
                     const double* rhs, double* out, IterState* st, double* partials, int mode, int k,
                     int max_iter);
void launch_dot(const DevMesh& M, hipStream_t s, const double* a, const double* b, IterState* st,
                double* partials, int what);
void launch_cg_hvp_dots(const DevMesh& M, hipStream_t s, const double* sv, const double* fe,
                        const double* r, double* w, IterState* st, double* partials);
void launch_cg_step(const DevMesh& M, hipStream_t s, double* z, double* r, double* p, double* q,
                    const double* sv, const double* w, IterState* st, double* partials);
// gate: when given and its iteration met non-positive curvature, the kernel
// does nothing (the adjoint is finished by the fallback first)
void launch_adj_epilogue(const DevMesh& M, hipStream_t s, const double* x, const double* v,
                         const double* z, const double* gv_next, double* gx, double* gv,
                         const IterState* gate = nullptr);
void launch_grad_params(const DevMesh& M, hipStream_t s, const double* xn, const double* z,
                        const double* cache, double* g_youngs, double* g_act, const IterState* gate = nullptr);
constexpr int kAdjCacheRows = 19;
// With the volume-preserving term the cache also holds, per Gauss point:
// V (rows 19-27), G = dD/ds (28-36), r (37-39), k (40-42), the projected
// singular values (43-45) and 1 where the projection applies (46).
constexpr int kAdjCacheRowsVolume = 47;
constexpr int kVolV = 19, kVolG = 28, kVolR = 37, kVolK = 40, kVolD = 43, kVolOk = 46;
// fused dense solver (cg_dense.hip)
size_t cg_dense_lds_bytes(int n, int rows, int mode, bool fp32);
int cg_dense_max_blocks(int n, int rows, int mode, bool fp32);
hipError_t launch_cg_dense(const DevMesh& M, const DenseCG& D, hipStream_t s, int blocks, bool fp32,
                           const double* cache, const double* rhs, double rhs_scale, int pd_fallback,
                           double* z_out, IterState* st, ProfAcc* prof,
                           const double* nb2_ref = nullptr);
void launch_unit_rhs(hipStream_t s, int N, int n, const int32_t* perm, int j0, double* b);
void launch_collect_rows(hipStream_t s, int N, int n, const int32_t* perm, int j0, const double* x,
                         double* ainv);
void launch_to_fp32(hipStream_t s, int64_t count, const double* in, float* out);
// device factorization (factor_gpu.hip)
void launch_factor_scatter(hipStream_t s, const int64_t* dst, const int32_t* src, const double* aval, int64_t n,
                           double* F);
void launch_factor_identity(hipStream_t s, const FrontDesc* fd, const int32_t* snode_of, int32_t n, double* P);
void launch_factor_op(hipStream_t s, const FactorOp& op, const FrontDesc* fd, const int32_t* ints,
                      const int32_t* relmap, double* F, double* P, int32_t* status);
void launch_factor_transpose(hipStream_t s, const FactorOp& op, const FrontDesc* fd, const int32_t* ints,
                             const double* P, double* out);
}  // namespace dpd
