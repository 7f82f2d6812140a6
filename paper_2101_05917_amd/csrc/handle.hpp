// The library's mesh handle (the opaque dpd_mesh of the C ABI): host mesh,
// factor, plan, device buffers and per-handle solver state.  Shared by the
// step drivers (api.hip) and the batched conjugate-gradient engine
// (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/diffpd.h"
#include "contact.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace dpd {
class Batcher;
}

struct TimedLaunch {
  std::pair<hipEvent_t, hipEvent_t> ev;
  double bytes, flops;
  int st_idx, k;
  bool strict;
};

struct dpd_mesh {
  dpd_options opt{};
  dpd::HostMesh hm;
  dpd::Csr A;
  dpd::Symbolic S;
  dpd::LevelPlan plan;
  dpd::DevMesh dm{};
  dpd::DevSolve ds{};
  bool factored = false;
  bool have_fp32 = false;
  std::string err;
  int64_t device_bytes = 0;
  std::vector<void*> allocs;
  // device buffers
  dpd::SweepTask* d_fwd = nullptr;
  dpd::SweepTask* d_bwd = nullptr;
  int32_t* d_gather = nullptr;
  dpd::DagPlan dag;                                    // single-launch solve (both sweeps)
  dpd::DevDag dd{};
  bool dag_ok = false;                            // plan uploaded and fits the launch limits
  uint32_t* h_dag_aborts = nullptr;               // pinned mirror of its abort count
  double solve_bytes = 0.0, solve_flops = 0.0;   // algorithmic work of one A^{-1} b
  int32_t leaf_max = 0;                           // chosen dissection leaf size
  int64_t method_factor_nnz = 0;                  // packed entries of a sparse factor (64-node leaves)
  uint8_t* cmask = nullptr;                       // [N] contact active at the linearisation point
  hipGraphExec_t cg_exec[2][2][2] = {};           // captured CG iterations [state][fp32][deflated]
  bool graphs_failed = false;                     // a capture failed: direct launches only
  int32_t cg_last[2] = {0, 0};                    // iterations of the last multi-launch solve per state
  // fused dense conjugate gradients (meshes with few free nodes)
  dpd::DenseCG dcg{};
  int dense_blocks = 0;                           // workgroups of its launch; 0: not available
  bool dense_alloc = false;
  double* ainv64 = nullptr;
  float* ainv32 = nullptr;
  bool capturing = false;
  hipStream_t capture_stream = nullptr;
  double* w_e = nullptr;
  double* wv_e = nullptr;                         // volume-preserving weights (null: term off)
  // device factorization: plan (built on first use) and its device copies
  dpd::FactorPlan fplan;
  bool fplan_ready = false;
  dpd::FrontDesc* d_fronts = nullptr;
  int64_t* d_adst = nullptr;
  int32_t* d_asrc = nullptr;
  int32_t* d_relmap = nullptr;
  int32_t* d_fints = nullptr;
  int32_t* d_snode_of = nullptr;
  double* d_aval = nullptr;
  int32_t* d_fstatus = nullptr;
  double factor_ms = 0.0;                         // wall time of the last dpd_factorize
  double* panel64 = nullptr;
  float* panel32 = nullptr;
  double* panelT64 = nullptr;
  float* panelT32 = nullptr;
  double *fe = nullptr, *r = nullptr, *y = nullptr, *partials = nullptr, *cache = nullptr;
  double *z = nullptr, *p = nullptr, *q = nullptr, *s = nullptr, *xbar = nullptr, *cg_r = nullptr;
  double* xbar_w = nullptr;   // H s of the conjugate-gradient iteration
  // the last three backward steps' adjoint solutions, newest first, and the
  // start built from them (dpd_options.bwd_warm_start)
  double* z_hist[3] = {nullptr, nullptr, nullptr};
  double* z_start = nullptr;
  int z_hist_n = 0;           // solutions held (0..3)
  dpd::IterState* warm_st = nullptr;   // [2] |b|^2 and |r_0|^2 of a warm-started fused solve
  // Galerkin start (bwd_warm_start = 4): the last kGalMax solutions in slots of one
  // block, their Hessian products, reduction scratch and the small system
  double* gal_Z = nullptr;             // [kGalMax][3N]
  double* gal_HZ = nullptr;            // [kGalMax][3N]
  double* gal_part = nullptr;          // multi-dot partial sums
  double* gal_dots = nullptr;          // [kGalMax + 1][kGalMax] G columns, then Z^T xbar
  double* gal_coef = nullptr;          // [kGalMax]
  double* h_gal = nullptr;             // pinned host mirror
  int gal_n = 0, gal_next = 0, gal_cap = 0;   // held, next slot, slots in use
  dpd::IterState* st = nullptr;     // [2]: outer iteration, inner conjugate gradients
  dpd::IterState* h_st = nullptr;   // pinned host mirror [2]
  // kernel timing (dpd_profile_start / dpd_profile_read)
  int32_t prof_class = DPD_PROF_OFF;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
  std::vector<TimedLaunch> ev_pending;
  int64_t prof_launches = 0, prof_seen = 0, prof_iters = 0;
  double prof_ms = 0.0, prof_bytes = 0.0, prof_flops = 0.0, prof_event_ms = 0.0;
  double clock_khz = 1.0e5;   // device wall-clock rate (hipDeviceAttributeWallClockRate)
  dpd::ProfAcc* prof_acc = nullptr;  // fused solver's device-side timing (class DPD_PROF_CG_DENSE)
  dpd::LaunchClock* prof_clock = nullptr;  // device-side timing of the single-kernel classes
  // global step with a contact set (dpd_contact_prepare / dpd_contact_solve)
  int32_t contact_n = 0;               // candidates (0: not prepared for the current factor)
  int32_t contact_cap = 0;             // candidates the buffers below hold
  int32_t* contact_cand = nullptr;     // [cap] public ids
  double* contact_B1 = nullptr;        // [cap][N] columns of A_s^{-1}, fixed rows 0
  int32_t* contact_set = nullptr;      // [kContactMaxSet] active set of the cached inverse
  double* contact_Sinv = nullptr;      // [c][c] inverse of (A^{-1})_{C×C} for that set
  double* contact_lam = nullptr;       // [3][kContactMaxSet]
  int32_t* contact_status = nullptr;   // non-positive pivot flag
  std::vector<int32_t> contact_cached; // the set whose inverse is cached (empty: none)
  // time step with contact (dpd_contact_forward_step / dpd_contact_backward_step)
  double* contact_tgt = nullptr;       // [3][cap] target of each candidate
  int32_t* contact_kind = nullptr;     // [cap] 0: free, 1: ray target, 2: static target
  uint8_t* contact_left = nullptr;     // [cap] left the set once in this step
  uint8_t* contact_mask = nullptr;     // [N] Dirichlet nodes and the set's nodes
  // with a dense A^{-1}: (A_{C̄×C̄})^{-1} held dense for the current set
  double* contact_W = nullptr;         // [n][n] internal order, rows and columns of C zero
  double* contact_T = nullptr;         // [n][kContactMaxSet] work
  uint8_t* contact_inc = nullptr;      // [n] internal rows in C
  bool contact_red_ok = false;
  uint32_t* contact_bar = nullptr;     // [kContactBarWords] grid barrier of the fused contact loop
  std::vector<int32_t> contact_red;    // the set W belongs to
  // deflated adjoint conjugate gradients (dpd_options.deflation)
  int32_t defl_k = 0;                  // vectors in W (0: not built)
  int32_t defl_age = 0;                // backward steps since W was built
  int32_t defl_steps = 0;              // Lanczos vectors allocated (m + 1)
  int32_t defl_graph_k = 0;            // vectors the captured deflated iterations use
  bool defl_active = false;            // the current backward solve runs deflated
  double* defl_W = nullptr;            // [kDeflMax][3N]
  double* defl_HW = nullptr;           // [kDeflMax][3N] H W at the current linearisation point
  double* defl_Q = nullptr;            // [m + 1][3N] Lanczos vectors
  double* defl_S = nullptr;            // [m + 1][3N] A^{-1} Q
  double* defl_part = nullptr;         // partial sums of the deflated reductions
  double* defl_dots = nullptr;         // [64] device results of multi-dots
  double* defl_coef = nullptr;         // [64] device coefficients of multi-axpys
  dpd::DeflState* defl_state = nullptr;
  double* h_defl = nullptr;            // pinned host scratch [64 * 64]
  // conjugate-gradient solves of the multi-launch path go through this engine
  // (several handles' iterations in the same launches) when set; not owned
  dpd::Batcher* batcher = nullptr;
};

