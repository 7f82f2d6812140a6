// C ABI of the diffpd library: mesh handles, factorization and the step
// drivers for the forward PD iteration (Alg. 1) and its adjoint (Alg. 2 and
// the conjugate-gradient acceleration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/diffpd.h"
#include "batch.hpp"
#include "contact.hpp"
#include "device.hpp"
#include "handle.hpp"
#include "internal.hpp"

using namespace dpd;

namespace {

thread_local std::string g_last_error;

constexpr double kLaunchSeconds = 4e-6;      // measured time of a small dependent launch
constexpr double kSweepBandwidth = 1.5e12;    // measured effective bytes/s of the sweeps
constexpr int32_t kSepMax = 2048;
constexpr int64_t kProfStride = 17;   // prime: no lock-step with the launch pattern of a solve
constexpr int kHoldPeriodsAround = 40;  // about 130 us of s_sleep ahead of a timed multi-launch solve
constexpr int kGraphIters = 2;   // conjugate-gradient iterations per captured graph
constexpr int kGalMax = 12;      // most stored adjoint solutions of the Galerkin start (buffer capacity)
constexpr int kGalDefault = 5;   // solutions kept with bwd_warm_start = 4
static_assert(kGalMax <= 64, "multi-dot and multi-axpy take at most 64 vectors");
constexpr int kNewtonAhead = 4;  // fused Newton forward: steps enqueued before the first check
constexpr int kNewtonMore = 2;   // ... and per later check

}  // namespace

namespace {

dpd_status fail(dpd_mesh* m, dpd_status code, const std::string& msg) {
  if (m) m->err = msg;
  g_last_error = msg;
  return code;
}

#define HIPCHECK(m, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((m), DPD_EHIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
dpd_status dev_alloc(dpd_mesh* m, T** out, int64_t count) {
  *out = nullptr;
  if (count <= 0) count = 1;
  void* p = nullptr;
  if (hipMalloc(&p, (size_t)count * sizeof(T)) != hipSuccess)
    return fail(m, DPD_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  m->allocs.push_back(p);
  m->device_bytes += count * (int64_t)sizeof(T);
  *out = (T*)p;
  return DPD_OK;
}

template <typename T>
dpd_status upload(dpd_mesh* m, T** out, const std::vector<T>& v) {
  dpd_status s = dev_alloc(m, out, (int64_t)v.size());
  if (s != DPD_OK) return s;
  if (!v.empty()) HIPCHECK(m, hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DPD_OK;
}

// Time one launch of kernel class cls when that class is being profiled.
// Single-kernel classes: every launch outside graph capture carries the
// handle's device-side clock and its algorithmic work (DPD_LAUNCH passes them
// to the kernel, which stamps itself).  A whole solve (several launches): one
// in every kProfStride is bracketed by events behind a bounded stream hold; it
// is tagged with its iteration k and the state (0 outer, 1 inner) that gates
// it, and dropped when harvested if the iteration had converged before it.
// (The fused solver times itself: cg_dense_async.)
struct ProfScope {
  dpd_mesh* m;
  hipStream_t s;
  bool on, clocked = false;
  TimedLaunch t{};
  ProfScope(dpd_mesh* mm, hipStream_t ss, int32_t cls, double bytes, double flops, int st_idx = -1,
            int k = 0, bool strict = true)
      : m(mm), s(ss), on(mm->prof_class == cls && cls != DPD_PROF_OFF && cls != DPD_PROF_CG_DENSE &&
                         !mm->capturing) {
    if (!on) return;
    if (cls != DPD_PROF_SOLVE) {
      on = false;
      if (m->prof_clock) {
        g_launch_clock = ClockArg{m->prof_clock, bytes, flops};
        clocked = true;
      }
      return;
    }
    on = (m->prof_seen++ % kProfStride) == 0;
    if (!on) return;
    if (m->ev_free.empty()) {
      hipEvent_t a = nullptr, b = nullptr;
      // timing-only events: no system-scope fence (cache writeback and
      // invalidate) when they are recorded; they are read after a stream
      // synchronisation
      const unsigned fl = hipEventDisableSystemFence;
      if (hipEventCreateWithFlags(&a, fl) != hipSuccess || hipEventCreateWithFlags(&b, fl) != hipSuccess) {
        on = false;
        return;
      }
      m->ev_free.push_back({a, b});
    }
    t.ev = m->ev_free.back();
    m->ev_free.pop_back();
    t.bytes = bytes;
    t.flops = flops;
    t.st_idx = st_idx;
    t.k = k;
    t.strict = strict;
    // Hold the stream while the solve's launches are enqueued, so the GPU
    // reaches them back to back and the host's enqueue time is not counted.
    launch_hold(s, kHoldPeriodsAround);
    (void)hipEventRecord(t.ev.first, s);
  }
  ~ProfScope() {
    if (clocked) g_launch_clock = ClockArg{};
    if (!on) return;
    (void)hipEventRecord(t.ev.second, s);
    m->ev_pending.push_back(t);
  }
};

// Accumulate the timed launches that did their work (after a stream sync,
// with the iteration states freshly read into h_st).
void prof_harvest(dpd_mesh* m) {
  for (auto& t : m->ev_pending) {
    bool live = true;
    if (t.st_idx >= 0) {
      const IterState& h = m->h_st[t.st_idx];
      live = !h.done || (t.strict ? t.k < h.iter : t.k <= h.iter);
    }
    if (live) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, t.ev.first, t.ev.second) == hipSuccess) {
        m->prof_event_ms += ms;
        m->prof_ms += ms;
      }
      m->prof_launches += 1;
      m->prof_bytes += t.bytes;
      m->prof_flops += t.flops;
    }
    m->ev_free.push_back(t.ev);
  }
  m->ev_pending.clear();
}

// A^{-1} b on free nodes, out[perm] = alpha x (+ out when accumulate).
void solve(dpd_mesh* m, hipStream_t s, bool fp32, const double* b, double* out, double alpha,
           int accumulate, const IterState* st, int k = 0) {
  const int st_idx = st == nullptr ? -1 : (st == m->st ? 0 : 1);
  const double scale = fp32 ? 0.5 : 1.0;
  ProfScope whole(m, s, DPD_PROF_SOLVE, m->solve_bytes * scale, m->solve_flops, st_idx, k);

  if (m->opt.sweep_launch && m->dag_ok) {
    ProfScope ps(m, s, DPD_PROF_SOLVE_DAG, m->solve_bytes * scale, m->solve_flops, st_idx, k);
    launch_solve_dag(m->ds, m->dd, s, fp32, b, out, m->dm.N, alpha, accumulate, st);
    return;
  }
  const LevelPlan& P = m->plan;
  const int32_t L = m->S.n_levels;
  for (int32_t l = 0; l < L; ++l) {
    const int n = P.fwd_off[l + 1] - P.fwd_off[l];
    if (!n) continue;
    ProfScope ps(m, s, P.fwd_wide[l] ? DPD_PROF_SWEEP_FWD_WIDE : DPD_PROF_SWEEP_FWD,
                 P.fwd_bytes[l] * scale, P.fwd_flops[l], st_idx, k);
    if (P.fwd_wide[l])
      launch_sweep_fwd_wide(m->ds, s, m->d_fwd + P.fwd_off[l], n, P.fwd_cols[l], fp32, b, m->dm.N,
                            m->d_gather + P.gather_off[l], P.gather_off[l + 1] - P.gather_off[l], st);
    else
      launch_sweep_fwd(m->ds, s, m->d_fwd + P.fwd_off[l], n, P.fwd_cols[l], fp32, b, m->dm.N, st);
  }
  for (int32_t l = L - 1; l >= 0; --l) {
    const int n = P.bwd_off[l + 1] - P.bwd_off[l];
    const bool lds = (int64_t)3 * P.bwd_rows[l] * (int64_t)sizeof(double) <= kSweepLdsBudget;
    if (!n) continue;
    ProfScope ps(m, s, P.bwd_narrow[l] ? DPD_PROF_SWEEP_BWD_NARROW : DPD_PROF_SWEEP_BWD,
                 P.bwd_bytes[l] * (fp32 ? 0.5 : 1.0), P.bwd_flops[l], st_idx, k);
    if (P.bwd_narrow[l])
      launch_sweep_bwd_narrow(m->ds, s, m->d_bwd + P.bwd_off[l], n, P.bwd_rows[l], fp32, out, m->dm.N,
                              alpha, accumulate, st);
    else
      launch_sweep_bwd(m->ds, s, m->d_bwd + P.bwd_off[l], n, P.bwd_rows[l], lds, fp32, out, m->dm.N,
                       alpha, accumulate, st);
  }
}

dpd_status read_state(dpd_mesh* m, hipStream_t s) {
  HIPCHECK(m, hipMemcpyAsync(m->h_st, m->st, 2 * sizeof(IterState), hipMemcpyDeviceToHost, s));
  if (m->dag_ok)
    HIPCHECK(m, hipMemcpyAsync(m->h_dag_aborts, m->dd.ctr + kDagAborts, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  prof_harvest(m);
  if (m->dag_ok && *m->h_dag_aborts != 0u)
    return fail(m, DPD_EHIP, "single-launch solve: a dependency wait timed out (results invalid)");
  return DPD_OK;
}

// Per-launch algorithmic work of the element kernels: node gather (24 B per
// node), per-Gauss-point cache (15 doubles read by the adjoint kernel),
// element forces written (24 doubles), connectivity and weights.
double elem_hvp_bytes(const dpd_mesh* m) {
  const double E = m->dm.E, N = m->dm.N;
  return 24.0 * N + E * (8 * 15 * 8.0 + 24 * 8.0 + 32.0 + 8.0);
}
double elem_hvp_flops(const dpd_mesh* m) { return 411.0 * 8.0 * m->dm.E; }
double elem_forces_bytes(const dpd_mesh* m) {
  const double E = m->dm.E, N = m->dm.N;
  return 24.0 * N + E * (24 * 8.0 + 32.0 + 8.0);
}

void fill_devmesh(dpd_mesh* m) {
  const dpd_options& o = m->opt;
  DevMesh& d = m->dm;
  d.N = (int32_t)m->hm.n_nodes;
  d.E = (int32_t)m->hm.n_elems;
  d.nf = (int32_t)m->hm.n_free;
  d.local32 = o.precision == DPD_MIXED ? 1 : 0;
  d.h = o.h;
  d.dx = o.dx;
  d.nu = o.nu;
  d.Vq = o.dx * o.dx * o.dx / 8.0;
  for (int k = 0; k < 3; ++k) {
    d.g[k] = o.gravity[k];
    d.fiber[k] = o.fiber[k];
  }
  d.contact_k = o.contact_k;
  d.friction_mu = o.friction_mu;
  d.friction_eps = o.friction_eps;
  d.muscle_k = o.muscle_k;
  d.corners = m->hm.corners;
}

// 2 mu_e V_q per Gauss point (tetrahedra: 2 mu_e V_e per element).
std::vector<double> corotated_weights(const HostMesh& hm, const dpd_options& o) {
  std::vector<double> w(hm.n_elems);
  const double Vq = o.dx * o.dx * o.dx / 8.0;
  for (int64_t e = 0; e < hm.n_elems; ++e)
    w[e] = 2.0 * hm.youngs[e] / (2.0 * (1.0 + o.nu)) * (hm.corners == 4 ? hm.vol[e] : Vq);
  return w;
}

// Volume-preserving weight per Gauss point, volume_scale lambda_e V_q, and its
// derivative in E_e.
double volume_weight_per_youngs(const dpd_options& o) {
  return o.volume_scale * o.nu / ((1.0 + o.nu) * (1.0 - 2.0 * o.nu)) * (o.dx * o.dx * o.dx / 8.0);
}
std::vector<double> volume_weights(const HostMesh& hm, const dpd_options& o) {
  std::vector<double> w(hm.n_elems);
  const double c = volume_weight_per_youngs(o);
  for (int64_t e = 0; e < hm.n_elems; ++e) w[e] = c * hm.youngs[e];
  return w;
}
int cache_rows(const dpd_options& o) { return o.volume_scale > 0.0 ? kAdjCacheRowsVolume : kAdjCacheRows; }

// FP32 copies (column-major and row-major) of the FP64 panels.
// FP32 copies of both panel layouts, converted on the device.
dpd_status make_fp32_panels(dpd_mesh* m, hipStream_t s) {
  if (!m->panel32) {
    dpd_status st = dev_alloc(m, &m->panel32, m->S.panel_size);
    if (st != DPD_OK) return st;
  }
  if (!m->panelT32) {
    dpd_status st = dev_alloc(m, &m->panelT32, m->S.panel_size);
    if (st != DPD_OK) return st;
  }
  launch_to_fp32(s, m->S.panel_size, m->panel64, m->panel32);
  launch_to_fp32(s, m->S.panel_size, m->panelT64, m->panelT32);
  HIPCHECK(m, hipGetLastError());
  HIPCHECK(m, hipStreamSynchronize(s));
  m->ds.panel32 = m->panel32;
  m->ds.panelT32 = m->panelT32;
  m->have_fp32 = true;
  return DPD_OK;
}

// Multifrontal Cholesky on the device (factor_gpu.hip): A's entries scattered
// into zeroed fronts, then the plan's launches level by level, then the
// row-major panel copy.  The fronts live in a workspace allocated for the call.
dpd_status factor_on_device(dpd_mesh* m, hipStream_t s) {
  if (!m->fplan_ready) {
    const std::string e = build_factor_plan(m->S, m->A, m->fplan);
    if (!e.empty()) return fail(m, DPD_EINVAL, "device factorization plan: " + e);
    const FactorPlan& P = m->fplan;
    dpd_status st;
    if ((st = upload(m, &m->d_fronts, P.fronts)) != DPD_OK) return st;
    if ((st = upload(m, &m->d_adst, P.a_dst)) != DPD_OK) return st;
    if ((st = upload(m, &m->d_asrc, P.a_src)) != DPD_OK) return st;
    if ((st = upload(m, &m->d_relmap, P.relmap)) != DPD_OK) return st;
    if ((st = upload(m, &m->d_fints, P.ints)) != DPD_OK) return st;
    if ((st = upload(m, &m->d_snode_of, m->S.snode_of)) != DPD_OK) return st;
    if ((st = dev_alloc(m, &m->d_aval, (int64_t)m->A.val.size())) != DPD_OK) return st;
    if ((st = dev_alloc(m, &m->d_fstatus, 1)) != DPD_OK) return st;
    m->fplan_ready = true;
  }
  const FactorPlan& P = m->fplan;
  HIPCHECK(m, hipMemcpyAsync(m->d_aval, m->A.val.data(), m->A.val.size() * sizeof(double), hipMemcpyHostToDevice,
                             s));
  double* F = nullptr;
  if (hipMalloc(&F, (size_t)std::max<int64_t>(1, P.front_size) * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(m, DPD_ENOMEM,
                "hipMalloc of the factorization workspace (" + std::to_string(P.front_size * 8) + " bytes) failed");
  }
  HIPCHECK(m, hipMemsetAsync(m->d_fstatus, 0, sizeof(int32_t), s));
  launch_fill(s, P.front_size, F, 0.0);
  launch_fill(s, m->S.panel_size, m->panel64, 0.0);
  launch_factor_identity(s, m->d_fronts, m->d_snode_of, m->S.n, m->panel64);
  launch_factor_scatter(s, m->d_adst, m->d_asrc, m->d_aval, (int64_t)P.a_dst.size(), F);
  for (const FactorOp& op : P.ops)
    launch_factor_op(s, op, m->d_fronts, m->d_fints, m->d_relmap, F, m->panel64, m->d_fstatus);
  launch_factor_transpose(s, P.transpose, m->d_fronts, m->d_fints, m->panel64, m->panelT64);
  const hipError_t le = hipGetLastError();
  const hipError_t se = hipStreamSynchronize(s);
  (void)hipFree(F);
  if (le != hipSuccess || se != hipSuccess)
    return fail(m, DPD_EHIP, std::string("device factorization: ") + hipGetErrorString(le != hipSuccess ? le : se));
  int32_t status = 0;
  HIPCHECK(m, hipMemcpy(&status, m->d_fstatus, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (status) return fail(m, DPD_ENOTSPD, "non-positive pivot in the device factorization");
  return DPD_OK;
}

dpd_status check_ready(dpd_mesh* m) {
  if (!m) return fail(nullptr, DPD_EINVAL, "null mesh");
  if (!m->factored) return fail(m, DPD_ESTATE, "mesh is not factorized (call dpd_factorize)");
  return DPD_OK;
}

// FP32 copy of the dense inverse for mixed precision.
dpd_status dense_fp32(dpd_mesh* m, hipStream_t s) {
  if (!m->dense_blocks) return DPD_OK;
  const int64_t n = m->hm.n_free;
  if (!m->ainv32) {
    dpd_status st = dev_alloc(m, &m->ainv32, n * n);
    if (st != DPD_OK) return st;
    m->dcg.ainv32 = m->ainv32;
  }
  launch_to_fp32(s, n * n, m->ainv64, m->ainv32);
  HIPCHECK(m, hipGetLastError());
  HIPCHECK(m, hipStreamSynchronize(s));
  return DPD_OK;
}

// Fused dense conjugate gradients for meshes of at most kSepMax free nodes:
// the workgroup partition (R consecutive internal rows per workgroup, the hex
// elements touching them, the incidence codes of each row in the fixed order
// of the node-incidence table), the iteration vectors, and A^{-1} itself,
// formed column by column by the factor's own sweeps on unit right-hand sides
// (three per solve).  Leaves dense_blocks = 0 when the path is off or the
// launch would not fit on the device.
dpd_status setup_dense(dpd_mesh* m, hipStream_t s) {
  const int n = (int)m->hm.n_free, N = (int)m->hm.n_nodes;
  m->dense_blocks = 0;
  // the fused kernels' element phase carries the corotated, muscle and ground
  // terms only: with the volume-preserving term solves use the sweeps
  if (!m->opt.fused_cg || m->opt.volume_scale > 0.0 || m->hm.corners != 8 || n < 1 || n > kSepMax) return DPD_OK;
  int G = 0;
  if (!m->dense_alloc) {
    int dev = 0, cus = 0;
    HIPCHECK(m, hipGetDevice(&dev));
    HIPCHECK(m, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int R = std::max(2, std::min(kDenseMaxRows, (n + std::max(1, cus) - 1) / std::max(1, cus)));
    G = (n + R - 1) / R;
    const HostMesh& hm = m->hm;
    std::vector<int32_t> perm(n), inv(N, -1);
    for (int i = 0; i < n; ++i) {
      perm[i] = hm.free_nodes[m->S.perm[i]];
      inv[perm[i]] = i;
    }
    std::vector<int32_t> eoff(G + 1, 0), elems, row_inc((size_t)8 * n, -1);
    int max_e = 0;
    for (int b = 0; b < G; ++b) {
      const int j0 = b * R, j1 = std::min(n, j0 + R);
      std::vector<int32_t> list;
      for (int j = j0; j < j1; ++j)
        for (int a = 0; a < 8; ++a) {
          const int32_t code = hm.node_inc[(size_t)a * N + perm[j]];
          if (code >= 0) list.push_back(code / 8);
        }
      std::sort(list.begin(), list.end());
      list.erase(std::unique(list.begin(), list.end()), list.end());
      for (int j = j0; j < j1; ++j)
        for (int a = 0; a < 8; ++a) {
          const int32_t code = hm.node_inc[(size_t)a * N + perm[j]];
          if (code < 0) continue;
          const int slot = (int)(std::lower_bound(list.begin(), list.end(), code / 8) - list.begin());
          row_inc[(size_t)8 * j + a] = slot * 8 + code % 8;
        }
      elems.insert(elems.end(), list.begin(), list.end());
      eoff[b + 1] = (int32_t)elems.size();
      max_e = std::max(max_e, (int)list.size());
    }
    // the workgroups whose rows of s workgroup b reads at its element corners
    std::vector<int32_t> nbr_off(G + 1, 0), nbr;
    for (int b = 0; b < G; ++b) {
      std::vector<int32_t> owners;
      for (int i = eoff[b]; i < eoff[b + 1]; ++i)
        for (int a = 0; a < 8; ++a) {
          const int32_t row = inv[hm.conn[(size_t)8 * elems[i] + a]];
          if (row >= 0 && row / R != b) owners.push_back(row / R);
        }
      std::sort(owners.begin(), owners.end());
      owners.erase(std::unique(owners.begin(), owners.end()), owners.end());
      nbr.insert(nbr.end(), owners.begin(), owners.end());
      nbr_off[b + 1] = (int32_t)nbr.size();
    }
    // What lives in LDS, per precision of A^{-1}, in order of preference: the
    // full r and q and the workgroup's rows of A^{-1}; r and q alone; the rows
    // alone; neither.  The first that fits with one workgroup per CU wins
    // (r and q in LDS remove two device-coherent vector reads per iteration,
    // the rows in LDS only shorten the dense product's load latency).
    // (fused_cg = 2 + m asks for placement m only.)
    int mode[2] = {-1, -1};
    for (int p = 0; p < 2; ++p)
      for (int md : {kDenseVecLds | kDenseAinvLds, kDenseVecLds, kDenseAinvLds, 0})
        if (mode[p] < 0 && (m->opt.fused_cg < 2 || md == m->opt.fused_cg - 2) &&
            cg_dense_max_blocks(n, R, md, p == 1) >= G)
          mode[p] = md;
    if (max_e > kDenseElems || mode[0] < 0 || mode[1] < 0)
      return DPD_OK;  // does not fit as one resident grid: keep the multi-launch path
    DenseCG& d = m->dcg;
    d.n = n;
    d.rows = R;
    d.max_elems = max_e;
    d.mode64 = mode[0];
    d.mode32 = mode[1];
    int32_t *dinv, *deoff, *delems, *drinc, *dnoff, *dnbr;
    double *r, *q, *p, *sv, *w, *z, *part;
    uint32_t *bar, *ready;
    dpd_status st;
    if ((st = upload(m, &dinv, inv)) != DPD_OK || (st = upload(m, &deoff, eoff)) != DPD_OK ||
        (st = upload(m, &delems, elems)) != DPD_OK || (st = upload(m, &drinc, row_inc)) != DPD_OK ||
        (st = upload(m, &dnoff, nbr_off)) != DPD_OK || (st = upload(m, &dnbr, nbr)) != DPD_OK ||
        (st = dev_alloc(m, &r, 6 * (int64_t)n)) != DPD_OK || (st = dev_alloc(m, &q, 6 * (int64_t)n)) != DPD_OK ||
        (st = dev_alloc(m, &p, 3 * (int64_t)n)) != DPD_OK || (st = dev_alloc(m, &sv, 3 * (int64_t)n)) != DPD_OK ||
        (st = dev_alloc(m, &w, 6 * (int64_t)n)) != DPD_OK || (st = dev_alloc(m, &z, 3 * (int64_t)n)) != DPD_OK ||
        (st = dev_alloc(m, &part, 4 * (int64_t)G)) != DPD_OK || (st = dev_alloc(m, &bar, kDenseBarWords)) != DPD_OK ||
        (st = dev_alloc(m, &ready, G)) != DPD_OK || (st = dev_alloc(m, &m->ainv64, (int64_t)n * n)) != DPD_OK)
      return st;
    d.perm = m->ds.perm_pub;
    d.inv = dinv;
    d.blk_eoff = deoff;
    d.blk_elems = delems;
    d.row_inc = drinc;
    d.r = r;
    d.q = q;
    d.p = p;
    d.s = sv;
    d.w = w;
    d.z = z;
    d.part = part;
    d.bar = bar;
    d.ready = ready;
    d.nbr_off = dnoff;
    d.nbr = dnbr;
    d.ainv64 = m->ainv64;
    m->dense_alloc = true;
  }
  G = (n + m->dcg.rows - 1) / m->dcg.rows;
  for (int j0 = 0; j0 < n; j0 += 3) {
    launch_unit_rhs(s, N, n, m->ds.perm_pub, j0, m->r);
    solve(m, s, false, m->r, m->y, 1.0, 0, nullptr);
    launch_collect_rows(s, N, n, m->ds.perm_pub, j0, m->y, m->ainv64);
  }
  HIPCHECK(m, hipGetLastError());
  HIPCHECK(m, hipStreamSynchronize(s));
  m->dense_blocks = G;
  if (m->have_fp32) return dense_fp32(m, s);
  return DPD_OK;
}

}  // namespace

namespace {
dpd_status conjugate_gradient(dpd_mesh* m, hipStream_t s, IterState* st, const double* rhs, bool fp32,
                              int max_it, int check_every, const double* z0 = nullptr);
dpd_status cg_dense_async(dpd_mesh* m, hipStream_t s, IterState* st, const double* rhs, double rhs_scale,
                          bool fp32, bool pd_fallback, const double* nb2_ref = nullptr);
dpd_status check_aborted(dpd_mesh* m, int st_idx);
}  // namespace

extern "C" {

dpd_status dpd_default_options(dpd_options* o) {
  if (!o) return fail(nullptr, DPD_EINVAL, "null options");
  std::memset(o, 0, sizeof(*o));
  o->dx = 0.01;
  o->rho = 1e3;
  o->nu = 0.45;
  o->h = 0.01;
  o->gravity[2] = -9.81;
  o->friction_eps = 1e-3;
  o->fiber[0] = 1.0;
  o->fwd_max_iter = 100;
  o->fwd_fixed_iters = 0;
  o->fwd_rel_tol = 1e-10;
  o->fwd_abs_tol_rel = 1e-12;
  o->fwd_solver = DPD_FWD_PD;
  o->fwd_inner_max_iter = 200;
  o->fwd_inner_tol = 1e-2;
  o->bwd_max_iter = 5000;
  o->bwd_solver = DPD_BWD_PCG;
  o->bwd_rel_tol = 1e-10;
  o->precision = DPD_FP64;
  o->check_every = 8;
  o->use_graphs = 1;
  o->fused_cg = 1;
  o->contact_fused = 1;
  o->sweep_launch = 0;
  return DPD_OK;
}

dpd_status dpd_create_mesh(const int32_t* cells_ijk, int64_t n_cells, const double* youngs,
                           const int32_t* fixed_ijk, int64_t n_fixed, const dpd_options* opt,
                           dpd_mesh** out) {
  dpd_status st = dpd::create_host(cells_ijk, n_cells, youngs, fixed_ijk, n_fixed, opt, out);
  if (st != DPD_OK) return st;
  st = dpd::upload_device(*out);
  if (st != DPD_OK) *out = nullptr;
  return st;
}

dpd_status dpd_create_tet_mesh(const double* X, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                               const double* youngs, const int32_t* fixed_nodes, int64_t n_fixed,
                               const dpd_options* opt, dpd_mesh** out) {
  dpd_status st = dpd::create_tet_host(X, n_nodes, tets, n_tets, youngs, fixed_nodes, n_fixed, opt, out);
  if (st != DPD_OK) return st;
  st = dpd::upload_device(*out);
  if (st != DPD_OK) *out = nullptr;
  return st;
}

}  // extern "C"

namespace dpd {

// Host stage of mesh creation: validation, numbering, A_s, ordering, plan.
dpd_status create_host(const int32_t* cells_ijk, int64_t n_cells, const double* youngs,
                       const int32_t* fixed_ijk, int64_t n_fixed, const dpd_options* opt,
                       dpd_mesh** out) {
  if (!out) return fail(nullptr, DPD_EINVAL, "null output handle");
  *out = nullptr;
  if (!opt) return fail(nullptr, DPD_EINVAL, "null options");
  if (n_fixed > 0 && !fixed_ijk) return fail(nullptr, DPD_EINVAL, "null fixed-node list");
  dpd_mesh* m = new (std::nothrow) dpd_mesh();
  if (!m) return fail(nullptr, DPD_ENOMEM, "host allocation failed");
  m->opt = *opt;
  if (m->opt.check_every < 1) m->opt.check_every = 1;
  std::string e = build_mesh(cells_ijk, n_cells, youngs, fixed_ijk, n_fixed, m->opt, m->hm);
  if (!e.empty()) {
    delete m;
    return fail(nullptr, DPD_EINVAL, e);
  }
  plan_host(m);
  *out = m;
  return DPD_OK;
}

dpd_status create_tet_host(const double* X, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                           const double* youngs, const int32_t* fixed_nodes, int64_t n_fixed, const dpd_options* opt,
                           dpd_mesh** out) {
  if (!out) return fail(nullptr, DPD_EINVAL, "null output handle");
  *out = nullptr;
  if (!opt) return fail(nullptr, DPD_EINVAL, "null options");
  if (n_fixed > 0 && !fixed_nodes) return fail(nullptr, DPD_EINVAL, "null fixed-node list");
  dpd_mesh* m = new (std::nothrow) dpd_mesh();
  if (!m) return fail(nullptr, DPD_ENOMEM, "host allocation failed");
  m->opt = *opt;
  if (m->opt.check_every < 1) m->opt.check_every = 1;
  m->opt.fused_cg = 0;   // the fused dense solver's element phase is the voxel one
  std::string e = build_tet_mesh(X, n_nodes, tets, n_tets, youngs, fixed_nodes, n_fixed, m->opt, m->hm);
  if (!e.empty()) {
    delete m;
    return fail(nullptr, DPD_EINVAL, e);
  }
  plan_host(m);
  *out = m;
  return DPD_OK;
}

// A_s, its ordering (leaf size by the solve-time estimate) and symbolic
// analysis, the sweep plan and the device mesh description.
void plan_host(dpd_mesh* m) {
  assemble_As(m->hm, m->opt, m->A);
  // Partition: among candidate leaf sizes pick the one with the smallest
  // estimated solve time, launches x kLaunchSeconds + factor bytes / kSweepBandwidth.
  // Small meshes end up with few levels (one dense supernode when every free
  // node fits in one block); large meshes keep the deep dissection tree.
  double best = 1e300;
  std::vector<int32_t> leaves = {64, 128, 256, 512};
  if (m->hm.n_free <= kSepMax) leaves.push_back((int32_t)m->hm.n_free);
  if (m->opt.leaf_nodes > 0) leaves = {m->opt.leaf_nodes};
  for (int32_t leaf : leaves) {
    Symbolic S;
    analyse(m->hm, m->A, leaf, kSepMax, S);
    LevelPlan P;
    build_plan(S, P);
    double launches = 0.0;
    for (int32_t l = 0; l < S.n_levels; ++l)
      launches += 2.0 + (P.gather_off[l + 1] > P.gather_off[l] ? 1.0 : 0.0);
    const double est = launches * kLaunchSeconds + 2.0 * 8.0 * (double)S.packed_nnz / kSweepBandwidth;
    if (est < best) {
      best = est;
      m->S = std::move(S);
      m->plan = std::move(P);
      m->leaf_max = leaf;
    }
  }
  // the sparse factor the method would sweep (for the dense path's traffic count)
  if (m->leaf_max == 64) {
    m->method_factor_nnz = m->S.packed_nnz;
  } else {
    Symbolic S;
    analyse(m->hm, m->A, 64, kSepMax, S);
    m->method_factor_nnz = S.packed_nnz;
  }
  fill_devmesh(m);
}

// Device bytes the handle will own once uploaded and factorized.
int64_t footprint_bytes(const dpd_mesh* m) {
  const int64_t N = m->hm.n_nodes, E = m->hm.n_elems, nf = m->hm.n_free;
  const Symbolic& S = m->S;
  int64_t b = 0;
  b += 8 * (3 * N + N + E);                                  // X, mass, weights
  b += 4 * (8 * E + 8 * N + nf) + 2 * N;                     // conn, incidence, perm, flags
  b += (int64_t)S.sn.size() * (3 * 4 + 3 * 8) + 4 * (int64_t)S.rows.size();
  b += 4 * ((int64_t)S.cptr.size() + (int64_t)S.cidx.size());
  b += 16 * (int64_t)(m->plan.fwd.size() + m->plan.bwd.size());
  b += 8 * (9 * nf + 3 * S.u_size + 24 * E + 9 * 3 * N);    // sweep vectors, fe, work vectors
  b += 4 * (int64_t)m->plan.gather_cols.size();
  b += 8 * ((int64_t)cache_rows(m->opt) * 8 * E + 2 * (std::max<int64_t>(N, 8 * E) / kBlock + 16));
  if (m->opt.volume_scale > 0.0) b += 8 * E;                 // volume weights
  b += 2 * 8 * S.panel_size;                                 // FP64 panels, both layouts
  if (m->opt.precision == DPD_MIXED) b += 2 * 4 * S.panel_size;  // FP32 copies
  if (m->opt.fused_cg && m->opt.volume_scale == 0.0 && nf >= 1 && nf <= kSepMax) {  // dense inverse
    b += nf * nf * (m->opt.precision == DPD_MIXED ? 12 : 8);
    b += 8 * 24 * nf + 4 * (9 * nf + N + 8 * E) + 8 * nf;
  }
  return b;
}

// Device stage: allocate and upload everything; frees the handle on failure.
dpd_status upload_device(dpd_mesh* m) {
  const HostMesh& hm = m->hm;
  const int64_t N = hm.n_nodes, E = hm.n_elems, nf = hm.n_free;
  const int K = hm.corners;
  const int64_t Q = K == 4 ? E : 8 * E;   // quadrature points
  std::vector<int32_t> conn_soa(K * E);
  for (int64_t el = 0; el < E; ++el)
    for (int a = 0; a < K; ++a) conn_soa[a * E + el] = hm.conn[K * el + a];
  std::vector<int32_t> perm_pub(nf);
  for (int64_t i = 0; i < nf; ++i) perm_pub[i] = hm.free_nodes[m->S.perm[i]];
  dpd_status st = DPD_OK;
  double *X, *mass;
  int32_t *conn, *inc, *pp, *rows, *cptr, *cidx;
  uint8_t *fixed, *contact;
#define UP(ptr, vec)                       \
  if ((st = upload(m, &ptr, vec)) != DPD_OK) { \
    dpd_destroy_mesh(m);                   \
    return st;                             \
  }
  UP(X, hm.X);
  UP(mass, hm.mass);
  UP(conn, conn_soa);
  inc = nullptr;
  double *dminv = nullptr, *vol = nullptr;
  int32_t *inc_ptr = nullptr, *inc_csr = nullptr;
  if (K == 4) {
    std::vector<double> dminv_soa(9 * E);
    for (int64_t el = 0; el < E; ++el)
      for (int i = 0; i < 9; ++i) dminv_soa[i * E + el] = hm.dminv[9 * el + i];
    UP(dminv, dminv_soa);
    UP(vol, hm.vol);
    UP(inc_ptr, hm.inc_ptr);
    UP(inc_csr, hm.inc);
  } else {
    UP(inc, hm.node_inc);
  }
  UP(fixed, hm.fixed);
  UP(contact, hm.is_contact);
  UP(m->w_e, corotated_weights(hm, m->opt));
  if (m->opt.volume_scale > 0.0) UP(m->wv_e, volume_weights(hm, m->opt));
  UP(pp, perm_pub);
  UP(rows, m->S.rows);
  UP(cptr, m->S.cptr);
  UP(cidx, m->S.cidx);
  UP(m->d_fwd, m->plan.fwd);
  UP(m->d_bwd, m->plan.bwd);
  UP(m->d_gather, m->plan.gather_cols);
  // single-launch solve: its queue, supernode table and counters (zeroed here,
  // then by the last workgroup of each launch); off when its LDS does not fit
  build_dag(m->S, m->plan, kSweepLdsBudget, m->dag);
  if (m->dag.usable && !m->dag.q.empty()) {
    DagEntry* q = nullptr;
    DagSn* sn = nullptr;
    uint32_t* ctr = nullptr;
    UP(q, m->dag.q);
    UP(sn, m->dag.sn);
    if ((st = dev_alloc(m, &ctr, m->dag.counter_words())) != DPD_OK) {
      dpd_destroy_mesh(m);
      return st;
    }
    if (hipMemset(ctr, 0, m->dag.counter_words() * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&m->h_dag_aborts, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
      dpd_destroy_mesh(m);
      return fail(nullptr, DPD_EHIP, "single-launch solve set-up failed");
    }
    *m->h_dag_aborts = 0u;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      dpd_destroy_mesh(m);
      return fail(nullptr, DPD_EHIP, "device query failed");
    }
    // resident workgroups of the FP64 kernel (the FP32 one uses no more resources)
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, solve_dag_kernel(false), kDagThreads,
                                                     m->dag.lds_bytes) != hipSuccess)
      per_cu = 1;
    DevDag& dd = m->dd;
    dd.q = q;
    dd.nq = (int32_t)m->dag.q.size();
    dd.ns = (int32_t)m->dag.sn.size();
    dd.grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(dd.nq, (int64_t)std::max(1, per_cu) * cus));
    dd.bwd_region = m->dag.bwd_region;
    dd.fwd = m->d_fwd;
    dd.bwd = m->d_bwd;
    dd.gcols = m->d_gather;
    dd.sn = sn;
    dd.ctr = ctr;
    dd.lds_bytes = (size_t)m->dag.lds_bytes;
    m->dag_ok = true;
  }
  for (int32_t l = 0; l < m->S.n_levels; ++l) {
    m->solve_bytes += m->plan.fwd_bytes[l] + m->plan.bwd_bytes[l];
    m->solve_flops += m->plan.fwd_flops[l] + m->plan.bwd_flops[l];
  }
#undef UP
  DevMesh& d = m->dm;
  d.X = X;
  d.mass = mass;
  d.conn = conn;
  d.node_inc = inc;
  d.dminv = dminv;
  d.vol = vol;
  d.inc_ptr = inc_ptr;
  d.inc = inc_csr;
  d.fixed = fixed;
  d.contact = contact;
  d.w_e = m->w_e;
  d.wv_e = m->wv_e;
  d.dwv_dE = m->opt.volume_scale > 0.0 ? volume_weight_per_youngs(m->opt) : 0.0;
  DevSolve& ds = m->ds;
  ds.nf = (int32_t)nf;
  ds.perm_pub = pp;
  ds.rows = rows;
  ds.cptr = cptr;
  ds.cidx = cidx;
#define AL(ptr, count)                                   \
  if ((st = dev_alloc(m, &ptr, (count))) != DPD_OK) {    \
    dpd_destroy_mesh(m);                                 \
    return st;                                           \
  }
  AL(ds.y_int, 3 * nf);
  AL(ds.x_int, 3 * nf);
  AL(ds.U, 3 * m->S.u_size);
  AL(ds.bt, 3 * nf);
  AL(m->fe, 3 * K * E);
  AL(m->r, 3 * N);
  AL(m->y, 3 * N);
  AL(m->partials, 2 * (std::max<int64_t>(N, 8 * E) / kBlock + 16));
  AL(m->cache, (int64_t)cache_rows(m->opt) * Q);
  AL(m->z, 3 * N);
  AL(m->p, 3 * N);
  AL(m->q, 3 * N);
  AL(m->s, 3 * N);
  AL(m->xbar, 3 * N);
  AL(m->cg_r, 3 * N);
  AL(m->xbar_w, 3 * N);
  AL(m->cmask, N);
  m->dm.cmask = m->cmask;
  AL(m->st, 2);
#undef AL
  if (hipHostMalloc((void**)&m->h_st, 2 * sizeof(IterState), hipHostMallocDefault) != hipSuccess) {
    dpd_destroy_mesh(m);
    return fail(nullptr, DPD_ENOMEM, "pinned host allocation failed");
  }
  std::memset(m->h_st, 0, 2 * sizeof(IterState));
  // zero the scratch vectors whose fixed-node rows are read
  for (double* v : {m->z, m->p, m->q, m->s, m->xbar, m->r, m->cg_r, m->xbar_w})
    if (hipMemset(v, 0, 3 * N * sizeof(double)) != hipSuccess) {
      dpd_destroy_mesh(m);
      return fail(nullptr, DPD_EHIP, "hipMemset failed");
    }
  if (hipMemset(m->st, 0, 2 * sizeof(IterState)) != hipSuccess) {
    dpd_destroy_mesh(m);
    return fail(nullptr, DPD_EHIP, "hipMemset failed");
  }
  return DPD_OK;
}

}  // namespace dpd

extern "C" {

void dpd_destroy_mesh(dpd_mesh* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  dpd::destroy_synced(m);
}

}  // extern "C"

namespace dpd {

// Free a handle whose streams the caller has already synchronized.
void destroy_synced(dpd_mesh* m) {
  if (!m) return;
  for (auto& plane : m->cg_exec)
    for (auto& row : plane)
      for (auto& ex : row)
        if (ex) (void)hipGraphExecDestroy(ex);
  if (m->h_defl) (void)hipHostFree(m->h_defl);
  if (m->h_gal) (void)hipHostFree(m->h_gal);
  if (m->capture_stream) (void)hipStreamDestroy(m->capture_stream);
  for (void* p : m->allocs) (void)hipFree(p);
  for (auto& e : m->ev_free) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : m->ev_pending) {
    (void)hipEventDestroy(e.ev.first);
    (void)hipEventDestroy(e.ev.second);
  }
  if (m->h_st) (void)hipHostFree(m->h_st);
  if (m->h_dag_aborts) (void)hipHostFree(m->h_dag_aborts);
  delete m;
}

}  // namespace dpd

extern "C" {

dpd_status dpd_get_info(const dpd_mesh* m, dpd_mesh_info* info) {
  if (!m || !info) return fail(nullptr, DPD_EINVAL, "null argument");
  info->n_nodes = m->hm.n_nodes;
  info->n_elements = m->hm.n_elems;
  info->qp_per_element = m->hm.corners == 4 ? 1 : 8;
  double fl = 0.0;
  for (const Supernode& sn : m->S.sn) {
    const double n = sn.ncols, r = sn.nrows;
    fl += 2.0 * n * n * n / 3.0 + 2.0 * r * n * n + r * r * n;
  }
  info->factor_flops = (int64_t)fl;
  info->n_free = m->hm.n_free;
  info->n_fixed = m->hm.n_nodes - m->hm.n_free;
  info->n_contact = (int64_t)m->hm.contact.size();
  info->n_supernodes = (int64_t)m->S.sn.size();
  info->n_levels = m->S.n_levels;
  info->factor_nnz = m->S.packed_nnz;
  info->factor_bytes = 2 * m->S.panel_size * (int64_t)sizeof(double);
  info->factor_us = (int64_t)(m->factor_ms * 1e3);
  info->device_bytes = m->device_bytes;
  info->leaf_nodes = m->leaf_max;
  info->fused_blocks = m->opt.fused_cg ? m->dense_blocks : 0;
  info->fused_lds = info->fused_blocks ? m->dcg.mode64 | (m->dcg.mode32 << 2) : 0;
  info->solve_workgroups = m->dag_ok ? m->dd.grid : 0;
  info->solve_entries = m->dag_ok ? m->dd.nq : 0;
  return DPD_OK;
}

dpd_status dpd_node_ijk(const dpd_mesh* m, int32_t* ijk) {
  if (!m || !ijk) return fail(nullptr, DPD_EINVAL, "null argument");
  if (m->hm.corners != 8) return fail(nullptr, DPD_EINVAL, "a tetrahedral mesh has no grid coordinates");
  std::memcpy(ijk, m->hm.node_ijk.data(), m->hm.node_ijk.size() * sizeof(int32_t));
  return DPD_OK;
}

dpd_status dpd_rest_positions(const dpd_mesh* m, double* X) {
  if (!m || !X) return fail(nullptr, DPD_EINVAL, "null argument");
  std::memcpy(X, m->hm.X.data(), m->hm.X.size() * sizeof(double));
  return DPD_OK;
}

dpd_status dpd_contact_nodes(const dpd_mesh* m, int32_t* nodes) {
  if (!m || (!nodes && !m->hm.contact.empty())) return fail(nullptr, DPD_EINVAL, "null argument");
  if (!m->hm.contact.empty())
    std::memcpy(nodes, m->hm.contact.data(), m->hm.contact.size() * sizeof(int32_t));
  return DPD_OK;
}

dpd_status dpd_set_options(dpd_mesh* m, const dpd_options* o) {
  if (!m || !o) return fail(nullptr, DPD_EINVAL, "null argument");
  const dpd_options& c = m->opt;
  bool same = c.dx == o->dx && c.rho == o->rho && c.nu == o->nu && c.h == o->h &&
              c.contact_k == o->contact_k && c.muscle_k == o->muscle_k &&
              c.friction_mu == o->friction_mu && c.friction_eps == o->friction_eps &&
              c.volume_scale == o->volume_scale;
  for (int k = 0; k < 3; ++k)
    same = same && c.gravity[k] == o->gravity[k] && c.origin[k] == o->origin[k] && c.fiber[k] == o->fiber[k];
  if (!same) return fail(m, DPD_EINVAL, "physics options are fixed at mesh creation");
  const bool need32 = o->precision == DPD_MIXED && !m->have_fp32;
  m->opt = *o;
  if (m->opt.check_every < 1) m->opt.check_every = 1;
  m->dm.local32 = m->opt.precision == DPD_MIXED ? 1 : 0;
  if (need32 && m->factored) {
    dpd_status st = make_fp32_panels(m, nullptr);
    if (st != DPD_OK) return st;
    if ((st = dense_fp32(m, nullptr)) != DPD_OK) return st;
  }
  return DPD_OK;
}

dpd_status dpd_set_youngs(dpd_mesh* m, const double* youngs, int32_t on_device, void* stream) {
  if (!m || !youngs) return fail(nullptr, DPD_EINVAL, "null argument");
  std::vector<double> ym(m->hm.n_elems);
  if (on_device) {
    HIPCHECK(m, hipMemcpyAsync(ym.data(), youngs, ym.size() * sizeof(double), hipMemcpyDeviceToHost,
                               (hipStream_t)stream));
    HIPCHECK(m, hipStreamSynchronize((hipStream_t)stream));
  } else {
    std::memcpy(ym.data(), youngs, ym.size() * sizeof(double));
  }
  for (double v : ym)
    if (!(v > 0) || !std::isfinite(v)) return fail(m, DPD_EINVAL, "Young's moduli must be positive");
  m->hm.youngs = ym;
  std::vector<double> w = corotated_weights(m->hm, m->opt);
  HIPCHECK(m, hipMemcpy(m->w_e, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
  if (m->wv_e) {
    std::vector<double> wv = volume_weights(m->hm, m->opt);
    HIPCHECK(m, hipMemcpy(m->wv_e, wv.data(), wv.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  assemble_As(m->hm, m->opt, m->A);
  m->factored = false;
  return DPD_OK;
}

dpd_status dpd_factorize(dpd_mesh* m, void* stream) {
  if (m) {  // cached columns of A^{-1} for contact belong to the previous factor
    m->contact_n = 0;
    m->contact_cached.clear();
    m->contact_red_ok = false;
    m->factored = false;
  }
  if (!m) return fail(nullptr, DPD_EINVAL, "null mesh");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  if (!m->panel64) {
    dpd_status st = dev_alloc(m, &m->panel64, m->S.panel_size);
    if (st != DPD_OK) return st;
  }
  if (!m->panelT64) {
    dpd_status st = dev_alloc(m, &m->panelT64, m->S.panel_size);
    if (st != DPD_OK) return st;
  }
  if (m->opt.factor_on_host) {
    std::vector<double> panels;
    std::string e;
    if (!factor_panels(m->S, m->A, panels, e)) return fail(m, DPD_ENOTSPD, e);
    HIPCHECK(m, hipMemcpyAsync(m->panel64, panels.data(), panels.size() * sizeof(double),
                               hipMemcpyHostToDevice, s));
    const std::vector<double> pt = transpose_panels<double>(m->S, panels);
    HIPCHECK(m, hipMemcpyAsync(m->panelT64, pt.data(), pt.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHECK(m, hipStreamSynchronize(s));
  } else {
    dpd_status st = factor_on_device(m, s);
    if (st != DPD_OK) return st;
  }
  m->ds.panel64 = m->panel64;
  m->ds.panelT64 = m->panelT64;
  if (m->opt.precision == DPD_MIXED || m->have_fp32) {
    dpd_status st = make_fp32_panels(m, s);
    if (st != DPD_OK) return st;
  }
  HIPCHECK(m, hipStreamSynchronize(s));
  m->factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  {
    dpd_status st = setup_dense(m, s);
    if (st != DPD_OK) return st;
  }
  m->factored = true;
  return DPD_OK;
}

dpd_status dpd_forward_step(dpd_mesh* m, void* stream, const double* x, const double* v,
                            const double* act, double* xn, double* vn, dpd_stats* stats) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!x || !v || !xn || !vn) return fail(m, DPD_EINVAL, "null state pointer");
  if (xn == x || xn == v || vn == x || vn == v || xn == vn)
    return fail(m, DPD_EINVAL, "outputs must not alias inputs");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  const dpd_options& o = m->opt;
  const bool fp32 = o.precision == DPD_MIXED;
  if (fp32 && !m->have_fp32) return fail(m, DPD_ESTATE, "mixed precision needs FP32 panels (refactorize)");
  const int max_it = std::max(0, o.fwd_max_iter);
  launch_reset(s, m->st, o.fwd_rel_tol * o.fwd_rel_tol, std::max(0, o.fwd_max_iter));
  launch_prologue(m->dm, s, x, v, m->y, xn, m->st, m->partials, o.fwd_abs_tol_rel);
  int solves = -1, outer = 0;
  if (o.fwd_solver == DPD_FWD_NEWTON_PCG && !o.fwd_fixed_iters) {
    // Newton on g: (A - dA(x)) d = -grad g(x) by A-preconditioned CG to a
    // relative tolerance; the same stopping test as Alg. 1 on grad g.
    IterState* inner = m->st + 1;
    const int64_t n3 = 3 * (int64_t)m->dm.N;
    const int never = 0x3fffffff;
    solves = 0;
    {
      ProfScope ps(m, s, DPD_PROF_ELEM_FORCES, elem_forces_bytes(m), 0.0);
      launch_elem_forces(m->dm, s, xn, act, m->fe, nullptr, m->st);
    }
    launch_node_residual(m->dm, s, xn, m->y, m->fe, m->r, m->st, m->partials, 0, never, 0);
    // Inner tolerance: fixed, or (fwd_inner_tol < 0) the Eisenstat-Walker
    // forcing terms ("choice 2": eta_k = 0.9 (|g_k| / |g_{k-1}|)^2, safeguarded
    // by 0.9 eta_{k-1}^2 when that exceeds 0.1, capped at |fwd_inner_tol|, and
    // kept above half the outer tolerance relative to |g_k|).
    const bool adaptive = o.fwd_inner_tol < 0.0;
    const double eta_max = std::fabs(o.fwd_inner_tol);
    if (m->dense_blocks > 0 && o.fused_cg) {
      // Fused solver: Newton steps are enqueued ahead of their convergence
      // test (kNewtonAhead, then kNewtonMore at a time) and decide on the
      // device: inner set-up (forcing term, cap), solve (-grad g; the plain
      // PD step after a curvature failure), x += z, next residual; every
      // kernel does nothing once the outer iteration has finished.  One host
      // synchronisation per batch.
      for (int batch = kNewtonAhead;; batch = kNewtonMore) {
        for (int i = 0; i < batch; ++i, ++outer) {
          launch_adj_cache(m->dm, s, xn, act, m->cache, nullptr, m->st);
          launch_newton_inner(s, m->st, inner, eta_max, adaptive ? 1 : 0, o.fwd_rel_tol, o.fwd_inner_max_iter,
                              max_it);
          if ((rc = cg_dense_async(m, s, inner, m->r, -1.0, fp32, true)) != DPD_OK) return rc;
          launch_newton_update(s, n3, m->st, inner, xn, m->z);
          {
            ProfScope ps(m, s, DPD_PROF_ELEM_FORCES, elem_forces_bytes(m), 0.0);
            launch_elem_forces(m->dm, s, xn, act, m->fe, nullptr, m->st);
          }
          launch_node_residual(m->dm, s, xn, m->y, m->fe, m->r, m->st, m->partials, outer + 1, never, 0);
        }
        if ((rc = read_state(m, s)) != DPD_OK) return rc;
        if ((rc = check_aborted(m, 1)) != DPD_OK) return rc;
        if (m->h_st[0].done) break;
      }
      solves = m->h_st[0].solves;
      outer = m->h_st[0].iter;
    } else {
      double eta = eta_max, g_prev = -1.0;
      for (outer = 0;; ++outer) {
        if ((rc = read_state(m, s)) != DPD_OK) return rc;
        if (m->h_st[0].done || solves >= max_it) break;
        if (adaptive) {
          const double gk = std::sqrt(m->h_st[0].rsq);
          if (g_prev > 0.0 && gk > 0.0) {
            double e = 0.9 * (gk / g_prev) * (gk / g_prev);
            const double safe = 0.9 * eta * eta;
            if (safe > 0.1) e = std::max(e, safe);
            const double floor = 0.5 * o.fwd_rel_tol * std::sqrt(m->h_st[0].r0sq) / gk;
            eta = std::min(eta_max, std::max(e, floor));
          }
          g_prev = gk;
        }
        launch_adj_cache(m->dm, s, xn, act, m->cache, nullptr);
        const int inner_max = std::max(1, std::min(o.fwd_inner_max_iter, max_it - solves));
        launch_reset(s, inner, eta * eta, inner_max);
        launch_lincomb(s, n3, m->xbar, -1.0, m->r, 0.0, nullptr);
        // the solve returns with the host mirror of its final state current
        if ((rc = conjugate_gradient(m, s, inner, m->xbar, fp32, inner_max, o.check_every)) !=
            DPD_OK)
          return rc;
        solves += std::max(1, m->h_st[1].iter);
        if (m->h_st[1].curvature) {
          // not a descent direction: take one plain PD step instead
          solve(m, s, fp32, m->r, xn, -1.0, 1, nullptr);
        } else {
          launch_lincomb(s, n3, xn, 1.0, xn, 1.0, m->z);
        }
        {
          ProfScope ps(m, s, DPD_PROF_ELEM_FORCES, elem_forces_bytes(m), 0.0);
          launch_elem_forces(m->dm, s, xn, act, m->fe, nullptr, m->st);
        }
        launch_node_residual(m->dm, s, xn, m->y, m->fe, m->r, m->st, m->partials, outer + 1, never, 0);
      }
    }
  }
  for (int k = 0; solves < 0; ++k) {
    {
      ProfScope ps(m, s, DPD_PROF_ELEM_FORCES, elem_forces_bytes(m), 0.0, 0, k, false);
      launch_elem_forces(m->dm, s, xn, act, m->fe, nullptr, m->st);
    }
    launch_node_residual(m->dm, s, xn, m->y, m->fe, m->r, m->st, m->partials, k, max_it,
                         o.fwd_fixed_iters);
    if (k >= max_it) break;
    solve(m, s, fp32, m->r, xn, -1.0, 1, m->st, k);
    if (!o.fwd_fixed_iters && (k + 1) % o.check_every == 0) {
      if ((rc = read_state(m, s)) != DPD_OK) return rc;
      if (m->h_st->done) break;
    }
  }
  launch_velocity(m->dm, s, x, xn, vn);
  HIPCHECK(m, hipGetLastError());
  if ((rc = read_state(m, s)) != DPD_OK) return rc;
  const IterState& h = *m->h_st;
  if (stats) {
    stats->fwd_iters = solves < 0 ? h.iter : solves;
    stats->fwd_outer = solves < 0 ? h.iter : outer;
    stats->converged = h.converged;
    stats->inverted_qps = h.inverted;
    stats->fwd_rel_res = h.r0sq > 0 ? std::sqrt(h.rsq / h.r0sq) : 0.0;
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (h.nonfinite) return fail(m, DPD_ENONFINITE, "non-finite residual in the forward iteration");
  if (!o.fwd_fixed_iters && !h.converged) return DPD_NOT_CONVERGED;
  return DPD_OK;
}

namespace {

// Alg. 2 in correction form: z <- z - A^{-1}((A - dA) z - xbar), from the current z.
dpd_status fixed_point(dpd_mesh* m, hipStream_t s, const double* xn, bool fp32, int max_it) {
  dpd_status rc;
  const dpd_options& o = m->opt;
  for (int k = 0;; ++k) {
    {
      ProfScope ps(m, s, DPD_PROF_ELEM_HVP, elem_hvp_bytes(m), elem_hvp_flops(m), 0, k, false);
      launch_elem_hvp(m->dm, s, m->z, m->cache, m->fe, m->st);
    }
    launch_node_hvp(m->dm, s, m->z, m->fe, m->xbar, m->r, m->st, m->partials, 1, k, max_it);
    if (k >= max_it) break;
    solve(m, s, fp32, m->r, m->z, -1.0, 1, m->st, k);
    if ((k + 1) % o.check_every == 0) {
      if ((rc = read_state(m, s)) != DPD_OK) return rc;
      if (m->h_st->done) break;
    }
  }
  return DPD_OK;
}

// Conjugate gradients on (A - dA(xk)) z = rhs preconditioned by A^{-1}, from
// z = 0, with its scalars in *st (stopping test |r| <= sqrt(st->tolsq) |rhs|).
// Uses m->cg_r, p, q, s as work vectors; the cached rotations must be at xk.
// One conjugate-gradient iteration (Chronopoulos-Gear): s = M^{-1} r, w = H s,
// the fused inner products, then the vector updates.  Every argument is a
// buffer of the handle, so the sequence can be captured once and replayed.
void cg_iteration(dpd_mesh* m, hipStream_t s, IterState* st, bool fp32, int k) {
  const int st_idx = st == m->st ? 0 : 1;
  const bool defl = st == m->st && m->defl_active;
  solve(m, s, fp32, m->cg_r, m->s, 1.0, 0, st, k);
  {
    ProfScope ps(m, s, DPD_PROF_ELEM_HVP, elem_hvp_bytes(m), elem_hvp_flops(m), st_idx, k);
    launch_elem_hvp(m->dm, s, m->s, m->cache, m->fe, st);
  }
  if (defl) {
    launch_cg_hvp_dots_defl(m->dm, s, m->s, m->fe, m->cg_r, m->xbar_w, st, m->defl_part, m->defl_HW, m->defl_k,
                            m->defl_state);
    launch_cg_step_defl(m->dm, s, m->z, m->cg_r, m->p, m->q, m->s, m->xbar_w, st, m->partials, m->defl_W,
                        m->defl_HW, m->defl_k, m->defl_state);
    return;
  }
  launch_cg_hvp_dots(m->dm, s, m->s, m->fe, m->cg_r, m->xbar_w, st, m->partials);
  launch_cg_step(m->dm, s, m->z, m->cg_r, m->p, m->q, m->s, m->xbar_w, st, m->partials);
}

// Graph of kGraphIters iterations on state st (captured on first use).
hipGraphExec_t cg_graph(dpd_mesh* m, hipStream_t s, IterState* st, bool fp32) {
  const bool defl = st == m->st && m->defl_active;
  hipGraphExec_t& ex = m->cg_exec[st == m->st ? 0 : 1][fp32 ? 1 : 0][defl ? 1 : 0];
  if (ex && defl && m->defl_graph_k != m->defl_k) {   // captured with another number of vectors
    (void)hipGraphExecDestroy(ex);
    ex = nullptr;
  }
  if (ex) return ex;
  if (defl) m->defl_graph_k = m->defl_k;
  // capture on a private stream (the caller's may be the null stream); nothing
  // executes during capture, and the graph is then launched on the caller's stream
  if (!m->capture_stream &&
      hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking) != hipSuccess)
    return nullptr;
  // A capture that fails (or is invalidated) leaves the iterations to direct
  // launches from then on; its error is cleared so that it does not surface
  // as the failure of a later call.
  if (m->graphs_failed) return nullptr;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(m->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    m->graphs_failed = true;
    (void)hipGetLastError();
    return nullptr;
  }
  m->capturing = true;
  for (int i = 0; i < kGraphIters; ++i) cg_iteration(m, m->capture_stream, st, fp32, 0);
  m->capturing = false;
  if (hipStreamEndCapture(m->capture_stream, &g) != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    m->graphs_failed = true;
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    ex = nullptr;
    m->graphs_failed = true;
    (void)hipGetLastError();
  }
  (void)hipGraphDestroy(g);
  return ex;
}

// Conjugate gradients on (A - dA) z = rhs preconditioned by A^{-1}, from
// z = m->z = 0, with its scalars in *st (stop when |r| <= sqrt(tolsq) |rhs| or
// after st->max_iter iterations).  The cached rotations and the contact mask
// must describe the linearisation point.  Iterations run as captured graphs of
// kGraphIters, except that while a kernel class is being timed one chunk in
// kProfStride runs as direct launches (timed live).
// Algorithmic traffic of the fused solver, counted as the method's: the
// preconditioner A^{-1} r costs what the factor's two sweeps move (the packed
// entries of a sparse Cholesky factor of A_s, nested dissection with 64-node
// leaves, read once per sweep, 8 bytes each; half for FP32), not the dense
// n x n inverse this path holds instead.  Per launch one such product (plus
// the 3n-vectors r in, s out); per iteration that product, the rotation cache
// of every Gauss point (15 doubles, 19 with muscles), the connectivity and
// weights, the product with A (12 bytes per stored entry of the lower
// triangle of A_s, plus the 3N-vectors in and out) and the 3n-vectors r, q,
// w, s, p, z each read and written once.
double sparse_solve_bytes(const dpd_mesh* m, bool fp32) {
  return 2.0 * (fp32 ? 4.0 : 8.0) * (double)m->method_factor_nnz;
}

double dense_matvec_bytes(const dpd_mesh* m, bool fp32) {
  const double n = (double)m->hm.n_free;
  return sparse_solve_bytes(m, fp32) + 2.0 * 3.0 * n * 8.0;
}

double dense_iter_bytes(const dpd_mesh* m, bool fp32) {
  const double n = (double)m->hm.n_free, E = (double)m->hm.n_elems, N = (double)m->hm.n_nodes;
  const double rows = m->opt.muscle_k > 0.0 ? 19.0 : 15.0;
  const double a_lower = 0.5 * ((double)m->A.col.size() + n);
  return sparse_solve_bytes(m, fp32) + rows * 8.0 * E * 8.0 + 8.0 * E * 4.0 + E * 8.0 +
         12.0 * a_lower + 2.0 * 3.0 * N * 8.0 + 12.0 * 3.0 * n * 8.0;
}

// One fused solve on state st (reset beforehand with its tolerance and cap)
// for the right-hand side rhs_scale * rhs, into m->z (fixed rows stay zero).
// Asynchronous: the caller reads the state (iterations, curvature, abort) at
// its next synchronisation.  With pd_fallback a non-positive curvature leaves
// z = A^{-1} rhs, the plain PD step.
dpd_status cg_dense_async(dpd_mesh* m, hipStream_t s, IterState* st, const double* rhs, double rhs_scale,
                          bool fp32, bool pd_fallback, const double* nb2_ref) {
  if (fp32 && !m->ainv32) return fail(m, DPD_ESTATE, "no FP32 copy of the dense inverse");
  // while timed, every launch adds its own device-clock duration, iterations
  // and itself to m->prof_acc (HIP events around a cooperative launch would
  // also bracket the host's enqueue time)
  ProfAcc* acc = m->prof_class == DPD_PROF_CG_DENSE && !m->capturing ? m->prof_acc : nullptr;
  HIPCHECK(m, launch_cg_dense(m->dm, m->dcg, s, m->dense_blocks, fp32, m->cache, rhs, rhs_scale,
                              pd_fallback ? 1 : 0, m->z, st, acc, nb2_ref));
  return DPD_OK;
}

dpd_status check_aborted(dpd_mesh* m, int st_idx) {
  if (m->h_st[st_idx].aborted || m->h_st[0].aborted)
    return fail(m, DPD_EHIP, "fused conjugate-gradient solver: grid barrier timed out");
  return DPD_OK;
}

dpd_status cg_dense(dpd_mesh* m, hipStream_t s, IterState* st, const double* rhs, bool fp32) {
  const int st_idx = st == m->st ? 0 : 1;
  dpd_status rc = cg_dense_async(m, s, st, rhs, 1.0, fp32, false);
  if (rc != DPD_OK) return rc;
  rc = read_state(m, s);
  if (rc != DPD_OK) return rc;
  return check_aborted(m, st_idx);
}

// ---------------------------------------------------------------- deflation
//
// The adjoint systems (A - dA) z = xbar are solved by CG preconditioned by
// A^{-1}; its iteration count grows with 1 / (1 - lambda_max(A^{-1} dA)), and the
// largest eigenvalues belong to a few slow modes (near-rigid rotations and the
// softest bending modes).  Keeping the search directions H-orthogonal to a
// space W holding approximations of those modes removes them from the
// iteration (deflated CG): the solution is the same, the contraction is set by
// the next eigenvalues.  W is built by Lanczos on B = dA A^{-1} = I - H A^{-1},
// which is self-adjoint in <u, v> = u^T A^{-1} v: with Q the Lanczos vectors and
// S = A^{-1} Q, an eigenvector u = Q y of B gives w = A^{-1} u = S y with
// dA w = lambda A w.  W is rebuilt every deflation_refresh backward steps; H W
// and E = W^T H W follow the linearisation point every step.

constexpr int kLanczosSteps = 40;

// Eigen-decomposition of a symmetric n x n matrix (row-major) by cyclic Jacobi
// rotations; eigenvalues in w, eigenvectors in the columns of V.
void sym_eig_jacobi(int n, std::vector<double> a, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? diag : off) += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    if (off <= 1e-30 * std::max(diag, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

dpd_status defl_alloc(dpd_mesh* m) {
  if (m->defl_W) return DPD_OK;
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  const int64_t blocks = (m->dm.N + kBlock - 1) / kBlock;
  dpd_status st;
  if ((st = dev_alloc(m, &m->defl_W, kDeflMax * n3)) != DPD_OK ||
      (st = dev_alloc(m, &m->defl_HW, kDeflMax * n3)) != DPD_OK ||
      (st = dev_alloc(m, &m->defl_Q, (kLanczosSteps + 1) * n3)) != DPD_OK ||
      (st = dev_alloc(m, &m->defl_S, (kLanczosSteps + 1) * n3)) != DPD_OK ||
      (st = dev_alloc(m, &m->defl_part, std::max<int64_t>((kDeflMax + 2) * blocks, 256 * 64))) != DPD_OK ||
      (st = dev_alloc(m, &m->defl_dots, 64)) != DPD_OK || (st = dev_alloc(m, &m->defl_coef, 64)) != DPD_OK ||
      (st = dev_alloc(m, &m->defl_state, 1)) != DPD_OK)
    return st;
  HIPCHECK(m, hipHostMalloc((void**)&m->h_defl, 64 * 64 * sizeof(double), hipHostMallocDefault));
  m->defl_steps = kLanczosSteps + 1;
  return DPD_OK;
}

// Device multi-dot out = X^T y (cnt vectors) copied to m->h_defl (synchronizes).
dpd_status defl_dots_host(dpd_mesh* m, hipStream_t s, const double* X, int cnt, const double* y) {
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  launch_multi_dot(s, X, cnt, y, n3, m->defl_part, m->defl_dots);
  HIPCHECK(m, hipMemcpyAsync(m->h_defl, m->defl_dots, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  return DPD_OK;
}

// y += sign * X c for host coefficients c (cnt of them).
dpd_status defl_axpy_host(dpd_mesh* m, hipStream_t s, double* y, const double* X, int cnt, const double* c,
                          double sign) {
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  // the coefficients are staged through pinned memory: wait for their previous use first
  HIPCHECK(m, hipStreamSynchronize(s));
  std::memcpy(m->h_defl, c, cnt * sizeof(double));
  HIPCHECK(m, hipMemcpyAsync(m->defl_coef, m->h_defl, cnt * sizeof(double), hipMemcpyHostToDevice, s));
  launch_multi_axpy(s, y, X, cnt, m->defl_coef, n3, sign);
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

// H p with the cached linearisation point (fixed rows zero).
void defl_hessian(dpd_mesh* m, hipStream_t s, const double* p, double* out) {
  launch_elem_hvp(m->dm, s, p, m->cache, m->fe, nullptr);
  launch_node_hvp(m->dm, s, p, m->fe, nullptr, out, nullptr, m->partials, 0, 0, 0);
}

// Lanczos on B = I - H A^{-1} (A^{-1} inner product) from a fixed start
// vector, full reorthogonalization; W = the Ritz vectors S y of B's k largest
// Ritz values.
dpd_status defl_build(dpd_mesh* m, hipStream_t s, bool fp32) {
  dpd_status rc;
  if ((rc = defl_alloc(m)) != DPD_OK) return rc;
  const int64_t N = m->dm.N, n3 = 3 * N;
  const int K = std::min(kDeflMax, m->opt.deflation);
  const int ms = kLanczosSteps;
  double* Q = m->defl_Q;
  double* S = m->defl_S;
  // start vector: a fixed pseudo-random field on the free nodes
  {
    std::vector<double> u(n3, 0.0);
    uint64_t x = 0x9e3779b97f4a7c15ull;
    for (int64_t c = 0; c < 3; ++c)
      for (int64_t n = 0; n < N; ++n) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        if (!m->hm.fixed[n]) u[c * N + n] = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
      }
    HIPCHECK(m, hipMemcpyAsync(Q, u.data(), n3 * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHECK(m, hipStreamSynchronize(s));
  }
  solve(m, s, fp32, Q, S, 1.0, 0, nullptr);
  if ((rc = defl_dots_host(m, s, Q, 1, S)) != DPD_OK) return rc;
  double b0 = std::sqrt(std::max(m->h_defl[0], 0.0));
  if (!(b0 > 0.0)) return DPD_OK;
  launch_lincomb(s, n3, Q, 1.0 / b0, Q, 0.0, nullptr);
  launch_lincomb(s, n3, S, 1.0 / b0, S, 0.0, nullptr);
  std::vector<double> alpha, beta;
  int steps = 0;
  for (int j = 0; j < ms; ++j) {
    double* w = Q + (j + 1) * n3;
    double* sw = S + (j + 1) * n3;
    defl_hessian(m, s, S + j * n3, sw);                   // H S_j (staged in the next S slot)
    launch_lincomb(s, n3, w, 1.0, Q + j * n3, -1.0, sw);  // w = Q_j - H S_j = B Q_j
    // full reorthogonalization against Q_0..Q_j in the A^{-1} inner product, twice
    std::vector<double> c(j + 1);
    for (int pass = 0; pass < 2; ++pass) {
      if ((rc = defl_dots_host(m, s, S, j + 1, w)) != DPD_OK) return rc;
      std::copy(m->h_defl, m->h_defl + j + 1, c.begin());
      if (pass == 0) alpha.push_back(c[j]);
      if ((rc = defl_axpy_host(m, s, w, Q, j + 1, c.data(), -1.0)) != DPD_OK) return rc;
    }
    solve(m, s, fp32, w, sw, 1.0, 0, nullptr);
    if ((rc = defl_dots_host(m, s, w, 1, sw)) != DPD_OK) return rc;
    const double bj = std::sqrt(std::max(m->h_defl[0], 0.0));
    steps = j + 1;
    if (!(bj > 1e-10 * std::fabs(alpha[0]) + 1e-300)) break;
    beta.push_back(bj);
    launch_lincomb(s, n3, w, 1.0 / bj, w, 0.0, nullptr);
    launch_lincomb(s, n3, sw, 1.0 / bj, sw, 0.0, nullptr);
  }
  // Ritz pairs of the tridiagonal T (steps x steps)
  std::vector<double> T((size_t)steps * steps, 0.0), theta, Y;
  for (int i = 0; i < steps; ++i) {
    T[(size_t)i * steps + i] = alpha[i];
    if (i + 1 < steps) T[(size_t)i * steps + i + 1] = T[(size_t)(i + 1) * steps + i] = beta[i];
  }
  sym_eig_jacobi(steps, T, theta, Y);
  std::vector<int> order(steps);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return theta[a] > theta[b]; });
  const int k = std::min(K, steps);
  HIPCHECK(m, hipMemsetAsync(m->defl_W, 0, k * n3 * sizeof(double), s));
  for (int j = 0; j < k; ++j) {
    std::vector<double> y(steps);
    for (int i = 0; i < steps; ++i) y[i] = Y[(size_t)i * steps + order[j]];
    if ((rc = defl_axpy_host(m, s, m->defl_W + j * n3, S, steps, y.data(), 1.0)) != DPD_OK) return rc;
  }
  HIPCHECK(m, hipStreamSynchronize(s));
  m->defl_k = k;
  m->defl_age = 0;
  return DPD_OK;
}

// Per backward step (the cache holds the linearisation point): rebuild W when
// due, then H W and E^{-1} = (W^T H W)^{-1}.  Leaves deflation off for this
// step when E is not positive definite.
dpd_status defl_prepare(dpd_mesh* m, hipStream_t s, bool fp32) {
  dpd_status rc;
  m->defl_active = false;
  const int refresh = m->opt.deflation_refresh > 0 ? m->opt.deflation_refresh : 25;
  if (m->defl_k == 0 || m->defl_age >= refresh)
    if ((rc = defl_build(m, s, fp32)) != DPD_OK) return rc;
  m->defl_age += 1;
  const int k = m->defl_k;
  if (k == 0) return DPD_OK;
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  for (int j = 0; j < k; ++j) defl_hessian(m, s, m->defl_W + j * n3, m->defl_HW + j * n3);
  std::vector<double> E((size_t)k * k);
  for (int j = 0; j < k; ++j) {
    if ((rc = defl_dots_host(m, s, m->defl_W, k, m->defl_HW + j * n3)) != DPD_OK) return rc;
    for (int i = 0; i < k; ++i) E[(size_t)i * k + j] = m->h_defl[i];
  }
  // symmetrize and invert by Gauss-Jordan (k <= 16), requiring positive pivots
  std::vector<double> a((size_t)k * 2 * k, 0.0);
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < k; ++j) a[(size_t)i * 2 * k + j] = 0.5 * (E[(size_t)i * k + j] + E[(size_t)j * k + i]);
    a[(size_t)i * 2 * k + k + i] = 1.0;
  }
  for (int c = 0; c < k; ++c) {
    const double piv = a[(size_t)c * 2 * k + c];
    if (!(piv > 0.0) || !std::isfinite(piv)) return DPD_OK;
    for (int j = 0; j < 2 * k; ++j) a[(size_t)c * 2 * k + j] /= piv;
    for (int i = 0; i < k; ++i) {
      if (i == c) continue;
      const double f = a[(size_t)i * 2 * k + c];
      for (int j = 0; j < 2 * k; ++j) a[(size_t)i * 2 * k + j] -= f * a[(size_t)c * 2 * k + j];
    }
  }
  DeflState h{};
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) h.einv[i * kDeflMax + j] = a[(size_t)i * 2 * k + k + j];
  HIPCHECK(m, hipMemcpy(m->defl_state, &h, sizeof(DeflState), hipMemcpyHostToDevice));
  m->defl_active = true;
  return DPD_OK;
}

// z0 = W E^{-1} W^T rhs into m->z (zeroed before), r0 = rhs - HW E^{-1} W^T rhs into m->cg_r.
dpd_status deflated_start(dpd_mesh* m, hipStream_t s, const double* rhs) {
  dpd_status rc;
  const int k = m->defl_k;
  if ((rc = defl_dots_host(m, s, m->defl_W, k, rhs)) != DPD_OK) return rc;
  std::vector<double> c(m->h_defl, m->h_defl + k), a(k, 0.0);
  DeflState h{};
  HIPCHECK(m, hipMemcpy(&h, m->defl_state, sizeof(DeflState), hipMemcpyDeviceToHost));
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) a[i] += h.einv[i * kDeflMax + j] * c[j];
  if ((rc = defl_axpy_host(m, s, m->z, m->defl_W, k, a.data(), 1.0)) != DPD_OK) return rc;
  if ((rc = defl_axpy_host(m, s, m->cg_r, m->defl_HW, k, a.data(), -1.0)) != DPD_OK) return rc;
  return DPD_OK;
}

// Galerkin start of the adjoint solve: z_start = Z c with (Z^T H Z) c = Z^T xbar
// over the stored solutions Z (the H-norm best approximation of the solution
// in their span; eigenvalues of Z^T H Z below 1e-12 of the largest dropped).
// Needs the adjoint cache at the current point.  Leaves z_start unset when
// no solution is stored.
dpd_status galerkin_start(dpd_mesh* m, hipStream_t s) {
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  dpd_status rc;
  if (!m->gal_Z) {
    if ((rc = dev_alloc(m, &m->gal_Z, kGalMax * n3)) != DPD_OK) return rc;
    if ((rc = dev_alloc(m, &m->gal_HZ, kGalMax * n3)) != DPD_OK) return rc;
    // multi-dot partials: at most 256 chunks per vector; the small system: kGalMax
    // columns of G and Z^T xbar
    if ((rc = dev_alloc(m, &m->gal_part, 256 * kGalMax)) != DPD_OK) return rc;
    if ((rc = dev_alloc(m, &m->gal_dots, (kGalMax + 1) * kGalMax)) != DPD_OK) return rc;
    if ((rc = dev_alloc(m, &m->gal_coef, kGalMax)) != DPD_OK) return rc;
    HIPCHECK(m, hipHostMalloc((void**)&m->h_gal, (kGalMax + 1) * kGalMax * sizeof(double), hipHostMallocDefault));
  }
  const int k = m->gal_n;
  if (k == 0) return DPD_OK;
  for (int j = 0; j < k; ++j) defl_hessian(m, s, m->gal_Z + j * n3, m->gal_HZ + j * n3);
  for (int j = 0; j < k; ++j)
    launch_multi_dot(s, m->gal_Z, k, m->gal_HZ + j * n3, n3, m->gal_part, m->gal_dots + j * kGalMax);
  launch_multi_dot(s, m->gal_Z, k, m->xbar, n3, m->gal_part, m->gal_dots + kGalMax * kGalMax);
  HIPCHECK(m, hipMemcpyAsync(m->h_gal, m->gal_dots, (kGalMax + 1) * kGalMax * sizeof(double),
                             hipMemcpyDeviceToHost, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  std::vector<double> G((size_t)k * k), w, V, c(k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      G[(size_t)i * k + j] = 0.5 * (m->h_gal[j * kGalMax + i] + m->h_gal[i * kGalMax + j]);
  const double* b = m->h_gal + kGalMax * kGalMax;
  sym_eig_jacobi(k, G, w, V);
  double wmax = 0.0;
  for (double x : w) wmax = std::max(wmax, x);
  for (int e = 0; e < k; ++e) {
    if (!(w[e] > 1e-12 * wmax)) continue;
    double vb = 0.0;
    for (int i = 0; i < k; ++i) vb += V[(size_t)i * k + e] * b[i];
    for (int i = 0; i < k; ++i) c[i] += V[(size_t)i * k + e] * vb / w[e];
  }
  std::memcpy(m->h_gal, c.data(), k * sizeof(double));
  HIPCHECK(m, hipMemcpyAsync(m->gal_coef, m->h_gal, k * sizeof(double), hipMemcpyHostToDevice, s));
  launch_fill(s, n3, m->z_start, 0.0);
  launch_multi_axpy(s, m->z_start, m->gal_Z, k, m->gal_coef, n3, 1.0);
  return DPD_OK;
}

dpd_status conjugate_gradient(dpd_mesh* m, hipStream_t s, IterState* st, const double* rhs, bool fp32,
                              int max_it, int check_every, const double* z0) {
  if (m->dense_blocks > 0 && m->opt.fused_cg) return cg_dense(m, s, st, rhs, fp32);
  dpd_status rc;
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  const int st_idx = st == m->st ? 0 : 1;
  launch_fill(s, n3, m->z, 0.0);
  launch_fill(s, n3, m->p, 0.0);
  launch_fill(s, n3, m->q, 0.0);
  launch_lincomb(s, n3, m->cg_r, 1.0, rhs, 0.0, nullptr);
  launch_dot(m->dm, s, rhs, rhs, st, m->partials, 0);
  if (z0 && st == m->st && !m->defl_active && m->warm_st) {
    // warm start: z = z0, r = rhs - H z0, kept only if |r| < |rhs| (decided
    // on the device; the stopping test stays relative to |rhs|)
    launch_lincomb(s, n3, m->z, 1.0, z0, 0.0, nullptr);
    defl_hessian(m, s, m->z, m->q);
    launch_lincomb(s, n3, m->cg_r, 1.0, rhs, -1.0, m->q);
    launch_fill(s, n3, m->q, 0.0);
    launch_dot(m->dm, s, rhs, rhs, m->warm_st, m->partials, 0);
    launch_dot(m->dm, s, m->cg_r, m->cg_r, m->warm_st + 1, m->partials, 0);
    launch_warm_select(s, n3, m->z, m->cg_r, rhs, m->warm_st);
  }
  if (st == m->st && m->defl_active && !m->batcher) {
    // start from the solution's component in W: z0 = W E^{-1} W^T rhs, r0 = rhs - HW E^{-1} W^T rhs
    // (r0 is then orthogonal to W, and stays so)
    if ((rc = deflated_start(m, s, rhs)) != DPD_OK) return rc;
  }
  if (m->batcher) {
    // the iterations run in the batch engine's launches, together with other
    // handles' solves; the set-up above must be complete first
    HIPCHECK(m, hipStreamSynchronize(s));
    if ((rc = m->batcher->solve(m, st, fp32, max_it)) != DPD_OK)
      return fail(m, rc, "batched conjugate-gradient iterations failed");
    return read_state(m, s);   // callers read the final state from the host mirror
  }
  const int chunk = std::max(kGraphIters, check_every / kGraphIters * kGraphIters);
  // Iterations are enqueued in chunks between host checks; every kernel of an
  // iteration enqueued past convergence exits at once, but still costs a
  // launch.  The first chunk has check_every iterations, or, after a solve on
  // the same state, one more than that solve took (rounded up to whole
  // graphs, at most check_every); later ones are sized from the residual
  // reduction over the previous chunk: the iterations still needed at that
  // rate, rounded up to whole graphs (at most 4 chunks).
  int chunks = 0, next = chunk, k_prev = 0;
  if (m->cg_last[st_idx] > 0)
    next = std::min(chunk, (m->cg_last[st_idx] + 1 + kGraphIters - 1) / kGraphIters * kGraphIters);
  double rsq_prev = 0.0;
  for (int k = 0; k < max_it;) {
    const bool direct = !m->opt.use_graphs || (m->prof_class != DPD_PROF_OFF && chunks % kProfStride == 0);
    hipGraphExec_t ex = direct ? nullptr : cg_graph(m, s, st, fp32);
    for (int i = 0; i < next && k < max_it; i += kGraphIters) {
      if (ex) {
        HIPCHECK(m, hipGraphLaunch(ex, s));
        k += kGraphIters;
      } else {
        for (int j = 0; j < kGraphIters; ++j, ++k) cg_iteration(m, s, st, fp32, k);
      }
    }
    chunks += 1;
    if ((rc = read_state(m, s)) != DPD_OK) return rc;
    const IterState& h = m->h_st[st_idx];
    if (h.done) break;
    next = chunk;
    const double r_ref = chunks > 1 ? rsq_prev : h.nb2;
    const int it = chunks > 1 ? h.iter - k_prev : h.iter;
    if (it > 0 && h.rsq > 0.0 && h.rsq < r_ref && h.tolsq * h.nb2 < h.rsq) {
      const double need = std::log(h.tolsq * h.nb2 / h.rsq) / (std::log(h.rsq / r_ref) / it);
      if (std::isfinite(need) && need > 0.0) {
        const int want = ((int)std::ceil(need) + kGraphIters - 1) / kGraphIters * kGraphIters;
        next = std::max(kGraphIters, std::min(4 * chunk, want));
      }
    }
    rsq_prev = h.rsq;
    k_prev = h.iter;
  }
  if (chunks == 0 && (rc = read_state(m, s)) != DPD_OK) return rc;   // no iteration allowed
  m->cg_last[st_idx] = m->h_st[st_idx].iter;
  return DPD_OK;
}

}  // namespace

dpd_status dpd_backward_step(dpd_mesh* m, void* stream, const double* x, const double* v,
                             const double* act, const double* xn, const double* gx_next,
                             const double* gv_next, double* gx, double* gv, double* g_youngs,
                             double* g_act, dpd_stats* stats) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!x || !v || !xn || !gx_next || !gv_next || !gx || !gv)
    return fail(m, DPD_EINVAL, "null state pointer");
  if (gx == gx_next || gx == gv_next || gv == gx_next || gv == gv_next || gx == gv)
    return fail(m, DPD_EINVAL, "outputs must not alias inputs");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  const dpd_options& o = m->opt;
  const bool fp32 = o.precision == DPD_MIXED;
  if (fp32 && !m->have_fp32) return fail(m, DPD_ESTATE, "mixed precision needs FP32 panels (refactorize)");
  const int64_t n3 = 3 * (int64_t)m->dm.N;
  const int max_it = std::max(0, o.bwd_max_iter);
  launch_reset(s, m->st, o.bwd_rel_tol * o.bwd_rel_tol, max_it);
  // xbar = dL/dx_{i+1} + dL/dv_{i+1} / h  (v_{i+1} = (x_{i+1} - x_i)/h)
  launch_lincomb(s, n3, m->xbar, 1.0, gx_next, 1.0 / o.h, gv_next);
  launch_zero_fixed(m->dm, s, m->xbar);
  launch_adj_cache(m->dm, s, xn, act, m->cache, m->st);
  int fallbacks = 0;
  // With the fused solver the epilogue is enqueued with the solve and gated
  // on the device: it does nothing if the solve met non-positive curvature,
  // in which case the fallback below finishes the adjoint and runs it again.
  const bool gated = o.bwd_solver == DPD_BWD_PCG && m->dense_blocks > 0 && o.fused_cg;
  // warm start (dpd_options.bwd_warm_start): polynomial extrapolation in t of
  // the last adjoint solutions, order 0 (z_{t+1}), 1 (2 z_{t+1} - z_{t+2}) or
  // 2 (3 z_{t+1} - 3 z_{t+2} + z_{t+3}), as many as are held, built in z_start
  const bool warm = o.bwd_solver == DPD_BWD_PCG && o.bwd_warm_start > 0 && o.deflation <= 0;
  if (warm && !m->z_start) {
    for (double*& b : m->z_hist)
      if ((rc = dev_alloc(m, &b, n3)) != DPD_OK) return rc;
    if ((rc = dev_alloc(m, &m->z_start, n3)) != DPD_OK) return rc;
    if ((rc = dev_alloc(m, &m->warm_st, 2)) != DPD_OK) return rc;
    HIPCHECK(m, hipMemset(m->warm_st, 0, 2 * sizeof(IterState)));   // reduction tickets start at zero
  }
  const bool galerkin = warm && o.bwd_warm_start >= 4;
  const int order = warm && !galerkin ? std::min(std::min(o.bwd_warm_start, 3) - 1, m->z_hist_n - 1) : -1;
  bool have_start = order >= 0;
  if (galerkin) {
    const int cap = o.bwd_warm_start == 4 ? kGalDefault : std::min(o.bwd_warm_start, kGalMax);
    if (m->gal_cap != cap) {   // another number of kept solutions: start the history over
      m->gal_cap = cap;
      m->gal_n = m->gal_next = 0;
    }
    if ((rc = galerkin_start(m, s)) != DPD_OK) return rc;
    have_start = m->gal_n > 0;
  }
  if (order == 0) {
    launch_lincomb(s, n3, m->z_start, 1.0, m->z_hist[0], 0.0, nullptr);
  } else if (order == 1) {
    launch_lincomb(s, n3, m->z_start, 2.0, m->z_hist[0], -1.0, m->z_hist[1]);
  } else if (order == 2) {
    launch_lincomb(s, n3, m->z_start, 3.0, m->z_hist[0], -3.0, m->z_hist[1]);
    launch_lincomb(s, n3, m->z_start, 1.0, m->z_start, 1.0, m->z_hist[2]);
  }
  const double* z0 = have_start ? m->z_start : nullptr;
  if (gated) {
    if (z0) {
      // the fused solver solves H d = xbar - H z0 (start and safeguard decided
      // on the device), its stopping test relative to |xbar|; z = z0 + d
      defl_hessian(m, s, m->z_start, m->q);
      launch_lincomb(s, n3, m->cg_r, 1.0, m->xbar, -1.0, m->q);
      launch_dot(m->dm, s, m->xbar, m->xbar, m->warm_st, m->partials, 0);
      launch_dot(m->dm, s, m->cg_r, m->cg_r, m->warm_st + 1, m->partials, 0);
      launch_warm_select(s, n3, m->z_start, m->cg_r, m->xbar, m->warm_st);
      if ((rc = cg_dense_async(m, s, m->st, m->cg_r, 1.0, fp32, false, &m->warm_st[0].nb2)) != DPD_OK) return rc;
      launch_lincomb(s, n3, m->z, 1.0, m->z, 1.0, m->z_start);
      launch_zero_fixed(m->dm, s, m->z);
    } else if ((rc = cg_dense_async(m, s, m->st, m->xbar, 1.0, fp32, false)) != DPD_OK) {
      return rc;
    }
  } else if (o.bwd_solver == DPD_BWD_PCG) {
    m->defl_active = false;
    if (o.deflation > 0 && !m->batcher && (rc = defl_prepare(m, s, fp32)) != DPD_OK) return rc;
    rc = conjugate_gradient(m, s, m->st, m->xbar, fp32, max_it, o.check_every, z0);   // leaves h_st current
    m->defl_active = false;
    if (rc != DPD_OK) return rc;
    if (m->h_st->curvature) {
      // the paper's safeguard when the quasi-Newton step is not a descent:
      // continue with the plain fixed-point iteration from the current z
      fallbacks = 1;
      launch_reset(s, m->st, o.bwd_rel_tol * o.bwd_rel_tol, max_it);
      launch_dot(m->dm, s, m->xbar, m->xbar, m->st, m->partials, 0);
      if ((rc = fixed_point(m, s, xn, fp32, max_it)) != DPD_OK) return rc;
    }
  } else {
    launch_fill(s, n3, m->z, 0.0);
    launch_dot(m->dm, s, m->xbar, m->xbar, m->st, m->partials, 0);
    if ((rc = fixed_point(m, s, xn, fp32, max_it)) != DPD_OK) return rc;
  }
  launch_adj_epilogue(m->dm, s, x, v, m->z, gv_next, gx, gv, gated ? m->st : nullptr);
  if (g_youngs || g_act) launch_grad_params(m->dm, s, xn, m->z, m->cache, g_youngs, g_act, gated ? m->st : nullptr);
  HIPCHECK(m, hipGetLastError());
  if ((rc = read_state(m, s)) != DPD_OK) return rc;
  if (gated) {
    if ((rc = check_aborted(m, 0)) != DPD_OK) return rc;
    if (m->h_st->curvature) {
      // the paper's safeguard when the quasi-Newton step is not a descent:
      // continue with the plain fixed-point iteration from the current z
      fallbacks = 1;
      launch_reset(s, m->st, o.bwd_rel_tol * o.bwd_rel_tol, max_it);
      launch_dot(m->dm, s, m->xbar, m->xbar, m->st, m->partials, 0);
      if ((rc = fixed_point(m, s, xn, fp32, max_it)) != DPD_OK) return rc;
      launch_adj_epilogue(m->dm, s, x, v, m->z, gv_next, gx, gv);
      if (g_youngs || g_act) launch_grad_params(m->dm, s, xn, m->z, m->cache, g_youngs, g_act);
      HIPCHECK(m, hipGetLastError());
      if ((rc = read_state(m, s)) != DPD_OK) return rc;
    }
  }
  if (warm && !galerkin) {
    std::swap(m->z_hist[2], m->z_hist[1]);
    std::swap(m->z_hist[1], m->z_hist[0]);   // the oldest buffer takes the new solution
    launch_lincomb(s, n3, m->z_hist[0], 1.0, m->z, 0.0, nullptr);
    m->z_hist_n = std::min(3, m->z_hist_n + 1);
  } else if (galerkin) {
    launch_lincomb(s, n3, m->gal_Z + (int64_t)m->gal_next * n3, 1.0, m->z, 0.0, nullptr);
    m->gal_next = (m->gal_next + 1) % m->gal_cap;
    m->gal_n = std::min(m->gal_cap, m->gal_n + 1);
  }
  const IterState& h = *m->h_st;
  if (stats) {
    stats->bwd_iters = h.iter;
    stats->converged = h.converged;
    stats->fallbacks = fallbacks;
    stats->inverted_qps = h.inverted;
    stats->bwd_rel_res = h.nb2 > 0 ? std::sqrt(h.rsq / h.nb2) : 0.0;
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (h.nonfinite) return fail(m, DPD_ENONFINITE, "non-finite residual in the adjoint iteration");
  if (h.curvature) return fail(m, DPD_ECURVATURE, "non-positive curvature in the adjoint iteration");
  if (!h.converged) return DPD_NOT_CONVERGED;
  return DPD_OK;
}

dpd_status dpd_apply_inverse(dpd_mesh* m, void* stream, int32_t precision, const double* b, double* out) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!b || !out || b == out) return fail(m, DPD_EINVAL, "bad vector arguments");
  const bool fp32 = precision == DPD_MIXED;
  if (fp32 && !m->have_fp32) return fail(m, DPD_ESTATE, "no FP32 panels");
  hipStream_t s = (hipStream_t)stream;
  solve(m, s, fp32, b, out, 1.0, 0, nullptr);
  launch_zero_fixed(m->dm, s, out);
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

dpd_status dpd_gradient(dpd_mesh* m, void* stream, const double* x, const double* y, const double* act,
                        double* out) {
  if (!m || !x || !y || !out) return fail(m, DPD_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  launch_reset(s, m->st, 0.0, 0);
  launch_elem_forces(m->dm, s, x, act, m->fe, nullptr, nullptr);
  launch_node_residual(m->dm, s, x, y, m->fe, out, m->st, m->partials, 0, 0, 1);
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

dpd_status dpd_hessian_apply(dpd_mesh* m, void* stream, const double* x, const double* act,
                             const double* p, double* out) {
  if (!m || !x || !p || !out) return fail(m, DPD_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  launch_adj_cache(m->dm, s, x, act, m->cache, nullptr);
  launch_elem_hvp(m->dm, s, p, m->cache, m->fe, nullptr);
  launch_node_hvp(m->dm, s, p, m->fe, nullptr, out, nullptr, nullptr, 0, 0, 0);
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

namespace {

// Scratch of dpd_gradient_noalloc, one copy per GPU for the life of the
// process: the iteration state of the residual's grid reduction (its own
// 256-byte slot), the per-workgroup partial sums of the node pass and the
// element forces [3][8E].  A mesh of E elements has at most 8E nodes (every
// node is a voxel corner), so the node pass has at most 8E / kBlock + 1
// workgroups.
constexpr int64_t kNoAllocMaxElems = 16384;
constexpr int64_t kNoAllocStateBytes = 256;
constexpr int64_t kNoAllocPartialBytes = ((8 * (8 * kNoAllocMaxElems / kBlock + 1) + 255) / 256) * 256;
constexpr int64_t kNoAllocForceBytes = 24 * 8 * kNoAllocMaxElems;
constexpr int64_t kNoAllocBytes = kNoAllocStateBytes + kNoAllocPartialBytes + kNoAllocForceBytes;
static_assert(sizeof(IterState) <= kNoAllocStateBytes, "iteration state slot too small");

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kNoAllocMaxDevices] = {};

}  // namespace

// In host code this name stands for the array, not its device address: the
// address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
dpd_status noalloc_scratch(dpd_mesh* m, unsigned char** out) {
  int dev = -1;
  HIPCHECK(m, hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(m, DPD_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(m, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(m, DPD_EHIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return DPD_OK;
}

}  // namespace

dpd_status dpd_gradient_noalloc(dpd_mesh* m, void* stream, const double* x, const double* y,
                                const double* act, double* out) {
  if (!m || !x || !y || !out) return fail(m, DPD_EINVAL, "null argument");
  if ((int64_t)m->dm.E > kNoAllocMaxElems)
    return fail(m, DPD_EINVAL, "dpd_gradient_noalloc: the mesh has " + std::to_string(m->dm.E) +
                                   " elements, more than its scratch holds (" +
                                   std::to_string(kNoAllocMaxElems) + ")");
  unsigned char* base = nullptr;
  dpd_status rc = noalloc_scratch(m, &base);
  if (rc != DPD_OK) return rc;
  IterState* st = reinterpret_cast<IterState*>(base);
  double* partials = reinterpret_cast<double*>(base + kNoAllocStateBytes);
  double* fe = reinterpret_cast<double*>(base + kNoAllocStateBytes + kNoAllocPartialBytes);
  hipStream_t s = (hipStream_t)stream;
  // the reset kernel zeroes the reduction's ticket counter (kept from the last call)
  launch_reset(s, st, 0.0, 0);
  launch_elem_forces(m->dm, s, x, act, fe, nullptr, nullptr);
  launch_node_residual(m->dm, s, x, y, fe, out, st, partials, 0, 0, 1);
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

dpd_status dpd_rotations(dpd_mesh* m, void* stream, const double* x, double* R_out) {
  if (!m || !x || !R_out) return fail(m, DPD_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  launch_elem_forces(m->dm, s, x, nullptr, m->fe, R_out, nullptr);
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

dpd_status dpd_contact_prepare(dpd_mesh* m, void* stream, const int32_t* nodes_host, int32_t n_cand) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!nodes_host || n_cand < 1) return fail(m, DPD_EINVAL, "need at least one candidate node");
  if (m->hm.corners != 8) return fail(m, DPD_EINVAL, "complementarity contact is available on voxel meshes");
  const int N = (int)m->hm.n_nodes;
  std::vector<int32_t> cand(nodes_host, nodes_host + n_cand);
  std::vector<uint8_t> seen(N, 0);
  for (int32_t v : cand) {
    if (v < 0 || v >= N) return fail(m, DPD_EINVAL, "candidate node out of range");
    if (m->hm.fixed[v]) return fail(m, DPD_EINVAL, "candidate nodes must be free");
    if (seen[v]) return fail(m, DPD_EINVAL, "repeated candidate node");
    seen[v] = 1;
  }
  m->contact_n = 0;
  m->contact_cached.clear();
  m->contact_red_ok = false;
  if (n_cand > m->contact_cap) {
    if ((rc = dev_alloc(m, &m->contact_cand, n_cand)) != DPD_OK ||
        (rc = dev_alloc(m, &m->contact_B1, (int64_t)n_cand * N)) != DPD_OK ||
        (rc = dev_alloc(m, &m->contact_tgt, 3 * (int64_t)n_cand)) != DPD_OK ||
        (rc = dev_alloc(m, &m->contact_kind, n_cand)) != DPD_OK ||
        (rc = dev_alloc(m, &m->contact_left, n_cand)) != DPD_OK)
      return rc;
    m->contact_cap = n_cand;
  }
  if (!m->contact_mask && (rc = dev_alloc(m, &m->contact_mask, N)) != DPD_OK) return rc;
  if (!m->contact_set &&
      ((rc = dev_alloc(m, &m->contact_set, kContactMaxSet)) != DPD_OK ||
       (rc = dev_alloc(m, &m->contact_Sinv, (int64_t)kContactMaxSet * kContactMaxSet)) != DPD_OK ||
       (rc = dev_alloc(m, &m->contact_lam, 3 * (int64_t)kContactMaxSet)) != DPD_OK ||
       (rc = dev_alloc(m, &m->contact_status, 1)) != DPD_OK))
    return rc;
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(m, hipMemcpyAsync(m->contact_cand, cand.data(), sizeof(int32_t) * n_cand, hipMemcpyHostToDevice, s));
  const int64_t n3 = 3 * (int64_t)N;
  launch_fill(s, n3, m->y, 0.0);  // fixed rows stay 0 in every solution below
  for (int k0 = 0; k0 < n_cand; k0 += 3) {
    launch_fill(s, n3, m->r, 0.0);
    launch_contact_unit(s, N, n_cand, m->contact_cand, k0, m->r);
    solve(m, s, false, m->r, m->y, 1.0, 0, nullptr);
    launch_contact_collect(s, N, n_cand, k0, m->y, m->contact_B1);
  }
  HIPCHECK(m, hipGetLastError());
  HIPCHECK(m, hipStreamSynchronize(s));
  m->contact_n = n_cand;
  return DPD_OK;
}

}  // extern "C"

namespace {

// Make `set` (ascending candidate indices, at most kContactMaxSet) the set
// whose capacitance inverse is cached: factorize and invert it unless it is
// the cached one already (host synchronisation only then).
dpd_status contact_use_set(dpd_mesh* m, hipStream_t s, const int32_t* set, int32_t c) {
  if (c == 0 || (m->contact_cached.size() == (size_t)c && std::equal(set, set + c, m->contact_cached.begin())))
    return DPD_OK;
  m->contact_cached.clear();
  HIPCHECK(m, hipMemcpyAsync(m->contact_set, set, sizeof(int32_t) * c, hipMemcpyHostToDevice, s));
  HIPCHECK(m, launch_contact_factor(s, m->dm.N, m->contact_cand, m->contact_set, c, m->contact_B1, m->contact_Sinv,
                                    m->contact_status));
  int32_t bad = 0;
  HIPCHECK(m, hipMemcpyAsync(&bad, m->contact_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  if (bad) return fail(m, DPD_ENOTSPD, "non-positive pivot in the contact capacitance matrix");
  m->contact_cached.assign(set, set + c);
  return DPD_OK;
}

// The set {i : kind[i] != 0} of a host kind array, ascending.
dpd_status contact_set_of(dpd_mesh* m, const std::vector<int32_t>& kind, std::vector<int32_t>* set) {
  set->clear();
  for (int32_t i = 0; i < (int32_t)kind.size(); ++i)
    if (kind[i]) set->push_back(i);
  if ((int)set->size() > kContactMaxSet) return fail(m, DPD_EINVAL, "contact set exceeds 120 nodes");
  return DPD_OK;
}

// mask = Dirichlet flags with the set's nodes added (from the device kinds).
dpd_status contact_mask(dpd_mesh* m, hipStream_t s) {
  HIPCHECK(m, hipMemcpyAsync(m->contact_mask, m->dm.fixed, (size_t)m->dm.N, hipMemcpyDeviceToDevice, s));
  launch_contact_mark(s, m->contact_n, m->contact_cand, m->contact_kind, m->contact_mask);
  return DPD_OK;
}

// Where A^{-1} is held dense, (A_{C̄×C̄})^{-1} of the current set is formed once
// (a rank-c downdate of the dense inverse) and each reduced global step is one
// dense launch; *dense reports whether that path is taken.
dpd_status contact_use_dense(dpd_mesh* m, hipStream_t s, const int32_t* set, int32_t c, bool* dense) {
  const int n = m->dcg.n;
  *dense = m->dense_blocks > 0 && m->opt.fused_cg && m->ainv64 && n >= 1 && n <= kContactDenseMaxRows;
  if (!*dense) return DPD_OK;
  dpd_status rc;
  if (!m->contact_W &&
      ((rc = dev_alloc(m, &m->contact_W, (int64_t)n * n)) != DPD_OK ||
       (rc = dev_alloc(m, &m->contact_T, (int64_t)n * kContactMaxSet)) != DPD_OK ||
       (rc = dev_alloc(m, &m->contact_inc, n)) != DPD_OK))
    return rc;
  if (m->contact_red_ok && m->contact_red.size() == (size_t)c && std::equal(set, set + c, m->contact_red.begin()))
    return DPD_OK;
  HIPCHECK(m, launch_contact_reduced_inverse(s, n, m->dcg.inv, m->contact_cand, m->contact_set, c, m->ainv64,
                                             m->contact_Sinv, m->contact_T, m->contact_inc, m->contact_W));
  m->contact_red.assign(set, set + c);
  m->contact_red_ok = true;
  return DPD_OK;
}

// The whole inner loop of one contact set in one cooperative launch (dense
// path with contact_fused): x0 holds the start iterate and receives the last;
// x1 is work.  Algorithmic bytes per iteration: W, the element forces written
// and read, connectivity and weights, node incidences, and x, y (or xbar)
// and the new x.
dpd_status contact_fused_loop(dpd_mesh* m, hipStream_t s, const DevMesh& dmc, int mode, double* x0,
                              const double* y, const double* act, int max_it) {
  const int n = m->dcg.n, N = m->dm.N;
  if (!m->contact_bar) {
    dpd_status rc = dev_alloc(m, &m->contact_bar, kContactBarWords);
    if (rc != DPD_OK) return rc;
  }
  const double E = m->dm.E;
  const double bytes = 8.0 * n * n + 2.0 * 24.0 * 8.0 * E + 40.0 * E + 32.0 * N + 72.0 * n;
  {
    ProfScope ps(m, s, DPD_PROF_CONTACT_FUSED, bytes, 6.0 * (double)n * n);
    HIPCHECK(m, launch_contact_fused(s, dmc, m->dcg, m->dense_blocks, m->contact_W, x0, y, act,
                                     mode ? m->cache : nullptr, m->st, m->contact_bar, mode, max_it));
  }
  uint32_t abort_word = 0;
  HIPCHECK(m, hipMemcpyAsync(&abort_word, m->contact_bar + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  dpd_status rc = read_state(m, s);
  if (rc != DPD_OK) return rc;
  if (abort_word) return fail(m, DPD_EHIP, "fused contact loop: a grid barrier timed out");
  return DPD_OK;
}

// The contact adjoint by conjugate gradients preconditioned with the set's
// reduced inverse, one cooperative launch, into m->z (from z = 0).
// Algorithmic bytes per iteration: W, the rotation cache, connectivity and
// weights, node incidences, and the own-row vectors.
dpd_status contact_fused_cg(dpd_mesh* m, hipStream_t s, const DevMesh& dmc, int max_it) {
  const int n = m->dcg.n, N = m->dm.N;
  if (!m->contact_bar) {
    dpd_status rc = dev_alloc(m, &m->contact_bar, kContactBarWords);
    if (rc != DPD_OK) return rc;
  }
  const double E = m->dm.E;
  const double rows = m->opt.muscle_k > 0.0 ? 19.0 : 15.0;
  const double bytes = 8.0 * n * n + 8.0 * rows * 8.0 * E + 40.0 * E + 32.0 * N + 8.0 * 3.0 * n * 6.0;
  {
    ProfScope ps(m, s, DPD_PROF_CONTACT_FUSED_CG, bytes, 6.0 * (double)n * n);
    HIPCHECK(m, launch_contact_fused_cg(s, dmc, m->dcg, m->dense_blocks, m->contact_W, m->z, m->xbar, m->cache,
                                        m->st, m->contact_bar, max_it));
  }
  uint32_t abort_word = 0;
  HIPCHECK(m, hipMemcpyAsync(&abort_word, m->contact_bar + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  dpd_status rc = read_state(m, s);
  if (rc != DPD_OK) return rc;
  if (abort_word) return fail(m, DPD_EHIP, "fused contact adjoint: a grid barrier timed out");
  return DPD_OK;
}

// x <- x - (A_{C̄×C̄})^{-1} r_{C̄} on the nodes outside the mask: one dense
// launch, or d = A^{-1} r into `d` by the factor's sweeps, the capacitance
// correction and the masked update.
dpd_status contact_reduced_step(dpd_mesh* m, hipStream_t s, int32_t c, bool dense, const double* r, double* d,
                                double* x, IterState* st, int k) {
  const int N = m->dm.N;
  if (dense) {
    const double n = m->dcg.n;
    ProfScope ps(m, s, DPD_PROF_CONTACT_DENSE, 8.0 * n * n + 72.0 * n, 6.0 * n * n, st == m->st ? 0 : 1, k,
                 false);
    HIPCHECK(m, launch_contact_dense_step(s, m->dcg.n, N, m->dcg.perm, m->contact_W, r, x, st));
    return DPD_OK;
  }
  solve(m, s, false, r, d, 1.0, 0, st, k);
  if (c > 0) launch_contact_lam(s, N, m->contact_cand, m->contact_set, c, m->contact_Sinv, d, m->contact_lam, st);
  ProfScope ps(m, s, DPD_PROF_CONTACT_DESCEND, 8.0 * ((double)c * N + 10.0 * N) + 8.0 * 4.0 * c,
               6.0 * (double)c * N, st == m->st ? 0 : 1, k, false);
  launch_contact_descend(s, N, m->contact_set, c, m->contact_B1, m->contact_lam, d, m->contact_mask, x, st);
  return DPD_OK;
}

}  // namespace

extern "C" {

dpd_status dpd_contact_forward_step(dpd_mesh* m, void* stream, const double* x, const double* v,
                                    const double* act, double* xn, double* vn, int32_t* kind_out,
                                    dpd_stats* stats) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!m->contact_n) return fail(m, DPD_ESTATE, "no contact candidates (call dpd_contact_prepare)");
  if (!x || !v || !xn || !vn || !kind_out) return fail(m, DPD_EINVAL, "null argument");
  if (xn == x || xn == v || vn == x || vn == v || xn == vn)
    return fail(m, DPD_EINVAL, "outputs must not alias inputs");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  const dpd_options& o = m->opt;
  const int N = m->dm.N, nc = m->contact_n;
  const int max_it = std::max(0, o.fwd_max_iter);
  DevMesh dmc = m->dm;  // the contact set joins the Dirichlet nodes
  dmc.fixed = m->contact_mask;
  launch_contact_detect(s, N, nc, m->contact_cand, o.h, x, v, m->contact_tgt, m->contact_kind, m->contact_left);
  std::vector<int32_t> kind(nc), next(nc), set;
  HIPCHECK(m, hipMemcpyAsync(kind.data(), m->contact_kind, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
  HIPCHECK(m, hipStreamSynchronize(s));
  int iters = 0, sets = 0;
  bool converged = true, nonfinite = false;
  double rel_res = 0.0;
  for (;;) {
    ++sets;
    if ((rc = contact_set_of(m, kind, &set)) != DPD_OK) return rc;
    const int32_t c = (int32_t)set.size();
    bool dense = false;
    if ((rc = contact_use_set(m, s, set.data(), c)) != DPD_OK ||
        (rc = contact_use_dense(m, s, set.data(), c, &dense)) != DPD_OK)
      return rc;
    if ((rc = contact_mask(m, s)) != DPD_OK) return rc;
    // Alg. 3's inner loop: x = y with x_C = x*, then local and reduced global
    // steps until |grad g| on the free nodes outside C meets the tolerance
    launch_reset(s, m->st, o.fwd_rel_tol * o.fwd_rel_tol, max_it);
    launch_prologue(dmc, s, x, v, m->y, xn, m->st, m->partials, o.fwd_abs_tol_rel);
    launch_contact_place(s, N, nc, m->contact_cand, m->contact_kind, m->contact_tgt, xn);
    const bool fused = dense && o.contact_fused;
    if (fused && (rc = contact_fused_loop(m, s, dmc, 0, xn, m->y, act, max_it)) != DPD_OK) return rc;
    for (int k = 0; !fused; ++k) {
      {
        ProfScope ps(m, s, DPD_PROF_ELEM_FORCES, elem_forces_bytes(m), 0.0, 0, k, false);
        launch_elem_forces(m->dm, s, xn, act, m->fe, nullptr, m->st);
      }
      launch_node_residual(dmc, s, xn, m->y, m->fe, m->r, m->st, m->partials, k, max_it, 0);
      if (k >= max_it) break;
      if ((rc = contact_reduced_step(m, s, c, dense, m->r, m->z, xn, m->st, k)) != DPD_OK) return rc;
      if ((k + 1) % o.check_every == 0) {
        if ((rc = read_state(m, s)) != DPD_OK) return rc;
        if (m->h_st->done) break;
      }
    }
    if ((rc = read_state(m, s)) != DPD_OK) return rc;
    iters += m->h_st->iter;
    converged = converged && m->h_st->converged;
    nonfinite = nonfinite || m->h_st->nonfinite;
    rel_res = std::max(rel_res, m->h_st->r0sq > 0 ? std::sqrt(m->h_st->rsq / m->h_st->r0sq) : 0.0);
    if (nonfinite) break;
    // contact forces r = grad g(x) on the set (eq:tic_1) and the update of C
    IterState* aux = m->st + 1;
    launch_reset(s, aux, 0.0, 0);
    launch_elem_forces(m->dm, s, xn, act, m->fe, nullptr, aux);
    launch_node_residual(m->dm, s, xn, m->y, m->fe, m->r, aux, m->partials, 0, 0, 1);
    launch_contact_active_set(s, N, nc, m->contact_cand, x, xn, m->r, m->contact_kind, m->contact_left,
                              m->contact_tgt);
    HIPCHECK(m, hipMemcpyAsync(next.data(), m->contact_kind, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(m, hipStreamSynchronize(s));
    if (next == kind) break;
    kind.swap(next);
    if (sets > 2 * nc + 1) return fail(m, DPD_ESTATE, "contact active set did not settle");
  }
  launch_velocity(m->dm, s, x, xn, vn);
  HIPCHECK(m, hipGetLastError());
  std::memcpy(kind_out, kind.data(), sizeof(int32_t) * nc);
  HIPCHECK(m, hipStreamSynchronize(s));
  if (stats) {
    stats->fwd_iters = iters;
    stats->fwd_outer = sets;
    stats->converged = converged;
    stats->inverted_qps = m->h_st->inverted;
    stats->fwd_rel_res = rel_res;
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (nonfinite) return fail(m, DPD_ENONFINITE, "non-finite residual in the forward iteration");
  if (!converged) return DPD_NOT_CONVERGED;
  return DPD_OK;
}

dpd_status dpd_contact_backward_step(dpd_mesh* m, void* stream, const double* x, const double* v,
                                     const double* act, const double* xn, const int32_t* kind_host,
                                     const double* gx_next, const double* gv_next, double* gx, double* gv,
                                     double* g_youngs, double* g_act, dpd_stats* stats) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!m->contact_n) return fail(m, DPD_ESTATE, "no contact candidates (call dpd_contact_prepare)");
  if (!x || !v || !xn || !kind_host || !gx_next || !gv_next || !gx || !gv)
    return fail(m, DPD_EINVAL, "null argument");
  if (gx == gx_next || gx == gv_next || gv == gx_next || gv == gv_next || gx == gv)
    return fail(m, DPD_EINVAL, "outputs must not alias inputs");
  const int N = m->dm.N, nc = m->contact_n;
  std::vector<int32_t> kind(kind_host, kind_host + nc), set;
  for (int32_t k : kind)
    if (k < 0 || k > 2) return fail(m, DPD_EINVAL, "contact kind must be 0, 1 or 2");
  if ((rc = contact_set_of(m, kind, &set)) != DPD_OK) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  const dpd_options& o = m->opt;
  const int32_t c = (int32_t)set.size();
  bool dense = false;
  if ((rc = contact_use_set(m, s, set.data(), c)) != DPD_OK ||
      (rc = contact_use_dense(m, s, set.data(), c, &dense)) != DPD_OK)
    return rc;
  HIPCHECK(m, hipMemcpyAsync(m->contact_kind, kind.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, s));
  if ((rc = contact_mask(m, s)) != DPD_OK) return rc;
  DevMesh dmc = m->dm;
  dmc.fixed = m->contact_mask;
  const int64_t n3 = 3 * (int64_t)N;
  const int max_it = std::max(0, o.bwd_max_iter);
  launch_reset(s, m->st, o.bwd_rel_tol * o.bwd_rel_tol, max_it);
  // xbar = dL/dx_{i+1} + dL/dv_{i+1} / h, kept on C (it reaches x* there)
  launch_lincomb(s, n3, m->xbar, 1.0, gx_next, 1.0 / o.h, gv_next);
  launch_zero_fixed(m->dm, s, m->xbar);
  launch_adj_cache(m->dm, s, xn, act, m->cache, m->st);
  launch_fill(s, n3, m->z, 0.0);
  launch_dot(dmc, s, m->xbar, m->xbar, m->st, m->partials, 0);
  // Alg. 5: z <- z - (A_{C̄×C̄})^{-1} ((A - dA) z - xbar)_{C̄}, z = 0 on C; with
  // the fused loop and bwd_solver = PCG, its quasi-Newton acceleration (CG
  // preconditioned by the reduced inverse), continued by Alg. 5's iteration
  // from the current z if it meets non-positive curvature
  const bool fused = dense && o.contact_fused;
  int fallbacks = 0;
  if (fused && o.bwd_solver == DPD_BWD_PCG) {
    if ((rc = contact_fused_cg(m, s, dmc, max_it)) != DPD_OK) return rc;
    if (m->h_st->curvature) {
      fallbacks = 1;
      launch_reset(s, m->st, o.bwd_rel_tol * o.bwd_rel_tol, max_it);
      launch_dot(dmc, s, m->xbar, m->xbar, m->st, m->partials, 0);
      if ((rc = contact_fused_loop(m, s, dmc, 1, m->z, m->xbar, nullptr, max_it)) != DPD_OK) return rc;
    }
  } else if (fused && (rc = contact_fused_loop(m, s, dmc, 1, m->z, m->xbar, nullptr, max_it)) != DPD_OK) {
    return rc;
  }
  for (int k = 0; !fused; ++k) {
    {
      ProfScope ps(m, s, DPD_PROF_ELEM_HVP, elem_hvp_bytes(m), elem_hvp_flops(m), 0, k, false);
      launch_elem_hvp(m->dm, s, m->z, m->cache, m->fe, m->st);
    }
    launch_node_hvp(dmc, s, m->z, m->fe, m->xbar, m->r, m->st, m->partials, 1, k, max_it);
    if (k >= max_it) break;
    if ((rc = contact_reduced_step(m, s, c, dense, m->r, m->p, m->z, m->st, k)) != DPD_OK) return rc;
    if ((k + 1) % o.check_every == 0) {
      if ((rc = read_state(m, s)) != DPD_OK) return rc;
      if (m->h_st->done) break;
    }
  }
  // r = (A - dA) z - xbar on every free node: -dL/dx* on C
  launch_elem_hvp(m->dm, s, m->z, m->cache, m->fe, nullptr);
  launch_node_hvp(m->dm, s, m->z, m->fe, m->xbar, m->r, nullptr, m->partials, 0, 0, 0);
  launch_adj_epilogue(dmc, s, x, v, m->z, gv_next, gx, gv);
  if (g_youngs || g_act) launch_grad_params(m->dm, s, xn, m->z, m->cache, g_youngs, g_act);
  launch_contact_target_vjp(s, N, nc, m->contact_cand, m->contact_kind, x, v, m->r, gx, gv);
  HIPCHECK(m, hipGetLastError());
  if ((rc = read_state(m, s)) != DPD_OK) return rc;
  const IterState& h = *m->h_st;
  if (stats) {
    stats->bwd_iters = h.iter;
    stats->converged = h.converged;
    stats->fallbacks = fallbacks;
    stats->inverted_qps = h.inverted;
    stats->bwd_rel_res = h.nb2 > 0 ? std::sqrt(h.rsq / h.nb2) : 0.0;
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (h.nonfinite) return fail(m, DPD_ENONFINITE, "non-finite residual in the adjoint iteration");
  if (!h.converged) return DPD_NOT_CONVERGED;
  return DPD_OK;
}

dpd_status dpd_contact_solve(dpd_mesh* m, void* stream, const int32_t* set_host, int32_t c,
                             const double* xstar, const double* b, double* x) {
  dpd_status rc = check_ready(m);
  if (rc != DPD_OK) return rc;
  if (!m->contact_n) return fail(m, DPD_ESTATE, "no contact candidates (call dpd_contact_prepare)");
  if (!b || !x || (c > 0 && (!set_host || !xstar))) return fail(m, DPD_EINVAL, "null argument");
  if (x == b) return fail(m, DPD_EINVAL, "x must not alias b");
  if (c < 0 || c > kContactMaxSet) return fail(m, DPD_EINVAL, "active set size must be 0..120");
  std::vector<uint8_t> seen(m->contact_n, 0);
  for (int32_t k = 0; k < c; ++k) {
    const int32_t v = set_host[k];
    if (v < 0 || v >= m->contact_n) return fail(m, DPD_EINVAL, "active-set index out of range");
    if (seen[v]) return fail(m, DPD_EINVAL, "repeated active-set index");
    seen[v] = 1;
  }
  hipStream_t s = (hipStream_t)stream;
  const int N = (int)m->hm.n_nodes;
  // a new active set: its capacitance matrix is factorized and inverted once
  if ((rc = contact_use_set(m, s, set_host, c)) != DPD_OK) return rc;
  launch_fill(s, 3 * (int64_t)N, x, 0.0);
  solve(m, s, false, b, x, 1.0, 0, nullptr);  // a1 = A^{-1} b
  if (c > 0) {
    launch_contact_lam(s, N, m->contact_cand, m->contact_set, c, m->contact_Sinv, x, m->contact_lam);
    {
      ProfScope ps(m, s, DPD_PROF_CONTACT_UPDATE,
                   8.0 * ((double)c * N + 6.0 * N) + 8.0 * 4.0 * c, 6.0 * (double)c * N);
      launch_contact_update(s, N, m->contact_set, c, m->contact_B1, m->contact_lam, x);
    }
    launch_contact_set(s, N, m->contact_cand, m->contact_set, c, xstar, x);
  }
  HIPCHECK(m, hipGetLastError());
  return DPD_OK;
}

dpd_status dpd_profile_start(dpd_mesh* m, int32_t kernel_class) {
  if (!m) return fail(nullptr, DPD_EINVAL, "null mesh");
  if (kernel_class < DPD_PROF_OFF || kernel_class > DPD_PROF_SOLVE_DAG)
    return fail(m, DPD_EINVAL, "unknown kernel class");
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    m->clock_khz = khz;
  if (kernel_class == DPD_PROF_CG_DENSE) {
    if (!m->prof_acc) {
      dpd_status st = dev_alloc(m, &m->prof_acc, 1);
      if (st != DPD_OK) return st;
    }
    HIPCHECK(m, hipMemset(m->prof_acc, 0, sizeof(ProfAcc)));
  } else if (kernel_class != DPD_PROF_OFF && kernel_class != DPD_PROF_SOLVE) {
    if (!m->prof_clock) {
      dpd_status st = dev_alloc(m, &m->prof_clock, 1);
      if (st != DPD_OK) return st;
    }
    HIPCHECK(m, hipMemset(m->prof_clock, 0, sizeof(LaunchClock)));
  }
  m->prof_class = kernel_class;
  m->prof_launches = 0;
  m->prof_seen = 0;
  m->prof_iters = 0;
  m->prof_ms = m->prof_bytes = m->prof_flops = m->prof_event_ms = 0.0;
  return DPD_OK;
}

dpd_status dpd_profile_read(dpd_mesh* m, void* stream, dpd_kernel_profile* out) {
  if (!m || !out) return fail(m, DPD_EINVAL, "null argument");
  HIPCHECK(m, hipStreamSynchronize((hipStream_t)stream));
  prof_harvest(m);
  if (m->prof_class == DPD_PROF_CG_DENSE && m->prof_acc) {
    ProfAcc a{};
    HIPCHECK(m, hipMemcpy(&a, m->prof_acc, sizeof(ProfAcc), hipMemcpyDeviceToHost));
    const bool fp32 = m->opt.precision == DPD_MIXED;
    const double n = (double)m->hm.n_free;
    m->prof_launches = (int64_t)a.launches;
    m->prof_iters = (int64_t)a.iters;
    m->prof_ms = (double)a.ticks / m->clock_khz;
    m->prof_event_ms = 0.0;
    m->prof_bytes = (double)a.launches * dense_matvec_bytes(m, fp32) + (double)a.iters * dense_iter_bytes(m, fp32);
    m->prof_flops = (double)a.launches * 6.0 * n * n +
                    (double)a.iters * (6.0 * n * n + 600.0 * 8.0 * (double)m->hm.n_elems);
  } else if (m->prof_class != DPD_PROF_OFF && m->prof_class != DPD_PROF_SOLVE && m->prof_clock) {
    LaunchClock c{};
    HIPCHECK(m, hipMemcpy(&c, m->prof_clock, sizeof(LaunchClock), hipMemcpyDeviceToHost));
    m->prof_launches = (int64_t)c.launches;
    m->prof_ms = (double)c.ticks / m->clock_khz;
    m->prof_event_ms = 0.0;
    m->prof_bytes = c.bytes;
    m->prof_flops = c.flops;
  }
  out->launches = m->prof_launches;
  out->iterations = m->prof_iters;
  out->event_ms = m->prof_event_ms;
  out->total_ms = m->prof_ms;
  out->bytes = m->prof_bytes;
  out->flops = m->prof_flops;
  m->prof_class = DPD_PROF_OFF;
  return DPD_OK;
}

const char* dpd_status_string(dpd_status s) {
  switch (s) {
    case DPD_OK: return "ok";
    case DPD_NOT_CONVERGED: return "not converged";
    case DPD_EINVAL: return "invalid argument";
    case DPD_ENOTSPD: return "matrix not positive definite";
    case DPD_ENOMEM: return "out of memory";
    case DPD_EHIP: return "HIP runtime error";
    case DPD_ESTATE: return "invalid state";
    case DPD_ENONFINITE: return "non-finite value";
    case DPD_ECURVATURE: return "non-positive curvature";
  }
  return "unknown status";
}

const char* dpd_last_error(const dpd_mesh* m) {
  if (m) return m->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
