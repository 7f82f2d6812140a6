// Device-side data of one mesh and the kernel launchers (internal).
#pragma once

#include <hip/hip_ext.h>
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
  uint8_t* cmask;             // [N] ground contact active at the linearisation point
};

constexpr int kElemsPerBlock = kBlock / 8;

// Kernel timing: when start/stop events are set, the next launch made with
// DPD_LAUNCH records them at its own dispatch start and completion
// (hipExtLaunchKernelGGL), so the measured time is the kernel's alone.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool used = false;
};
extern thread_local LaunchEvents g_launch_events;

#define DPD_LAUNCH(kernel, grid, block, shmem, stream, ...)                                        \
  do {                                                                                             \
    if (::dpd::g_launch_events.start) {                                                            \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ::dpd::g_launch_events.start,      \
                            ::dpd::g_launch_events.stop, 0, __VA_ARGS__);                          \
      ::dpd::g_launch_events.start = nullptr;                                                      \
      ::dpd::g_launch_events.used = true;                                                          \
    } else {                                                                                       \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                         \
    }                                                                                              \
  } while (0)


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
                      double* cache, IterState* st);
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
void launch_adj_epilogue(const DevMesh& M, hipStream_t s, const double* x, const double* v,
                         const double* z, const double* gv_next, double* gx, double* gv);
void launch_grad_params(const DevMesh& M, hipStream_t s, const double* xn, const double* z,
                        const double* cache, double* g_youngs, double* g_act);
constexpr int kAdjCacheRows = 19;
}  // namespace dpd
