// Batched conjugate-gradient engine (see batch.hpp): the preconditioned CG
// iteration of Sec. DiffPD's quasi-Newton acceleration, A^{-1}-preconditioned,
// for several handles at once.  Per iteration: the forward sweep level by
// level and the backward sweep level by level, each level one launch per
// kernel shape over every slot's tasks of that level (slots' trees aligned at
// their leaves for the forward sweep and at their roots for the backward
// sweep), then the element Hessian product, the node gather with the inner
// products, and the vector update, one launch each over all slots.
#include "batch.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "handle.hpp"
#include "internal.hpp"

namespace dpd {

namespace {

constexpr int kChunkMin = 4;    // iterations between state reads
constexpr int kChunkMax = 32;
constexpr int kChunkFirst = 8;

int blocks_of(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

Batcher::Batcher(int device, int max_slots) : device_(device), max_slots_(std::max(1, max_slots)) {
  thread_ = std::thread([this] { loop(); });
}

Batcher::~Batcher() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (thread_.joinable()) thread_.join();
}

BatchStats Batcher::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  return stats_;
}

dpd_status Batcher::solve(dpd_mesh* m, IterState* st, bool fp32, int max_it) {
  Job job;
  job.m = m;
  job.st = st;
  job.fp32 = fp32;
  job.max_it = std::max(0, max_it);
  std::unique_lock<std::mutex> lk(mu_);
  if (stop_) return DPD_ESTATE;
  incoming_.push_back(&job);
  cv_.notify_all();
  cv_.wait(lk, [&] { return job.done; });
  return job.rc;
}

bool Batcher::reserve(size_t slots, size_t tasks, size_t gathers) {
  if (slots > cap_slots_) {
    if (d_solve_) (void)hipFree(d_solve_);
    if (d_cg_) (void)hipFree(d_cg_);
    if (h_st_) (void)hipHostFree(h_st_);
    d_solve_ = nullptr;
    d_cg_ = nullptr;
    h_st_ = nullptr;
    cap_slots_ = 0;
    if (hipMalloc(&d_solve_, slots * sizeof(BatchSolveSlot)) != hipSuccess ||
        hipMalloc(&d_cg_, slots * sizeof(BatchCgSlot)) != hipSuccess ||
        hipHostMalloc(&h_st_, slots * sizeof(IterState), hipHostMallocDefault) != hipSuccess)
      return false;
    cap_slots_ = slots;
  }
  if (tasks > cap_tasks_) {
    if (d_tasks_) (void)hipFree(d_tasks_);
    d_tasks_ = nullptr;
    cap_tasks_ = 0;
    const size_t want = std::max(tasks, 2 * cap_tasks_);
    if (hipMalloc(&d_tasks_, want * sizeof(SweepTask)) != hipSuccess) return false;
    cap_tasks_ = want;
  }
  if (gathers > cap_gathers_) {
    if (d_gathers_) (void)hipFree(d_gathers_);
    d_gathers_ = nullptr;
    cap_gathers_ = 0;
    const size_t want = std::max(gathers, 2 * cap_gathers_);
    if (hipMalloc(&d_gathers_, want * sizeof(int2)) != hipSuccess) return false;
    cap_gathers_ = want;
  }
  return true;
}

// Slot descriptors and the launch list of the active set.
bool Batcher::build(const std::vector<Job*>& active) {
  const int ns = (int)active.size();
  std::vector<BatchSolveSlot> hs(ns);
  std::vector<BatchCgSlot> hc(ns);
  int eb = 0, nb = 0, max_levels = 0;
  for (int j = 0; j < ns; ++j) {
    dpd_mesh* m = active[j]->m;
    hs[j].S = m->ds;
    hs[j].b = m->cg_r;
    hs[j].out = m->s;
    hs[j].st = active[j]->st;
    hs[j].N = m->dm.N;
    BatchCgSlot& c = hc[j];
    c.M = m->dm;
    c.cache = m->cache;
    c.fe = m->fe;
    c.sv = m->s;
    c.r = m->cg_r;
    c.w = m->xbar_w;
    c.z = m->z;
    c.p = m->p;
    c.q = m->q;
    c.st = active[j]->st;
    c.partials = m->partials;
    c.elem_block0 = eb;
    c.node_block0 = nb;
    c.node_blocks = blocks_of(m->dm.N, kBlock);
    eb += blocks_of(m->dm.E, kElemsPerBlock);
    nb += c.node_blocks;
    max_levels = std::max(max_levels, m->S.n_levels);
  }
  std::vector<SweepTask> tasks;
  std::vector<int2> gathers;
  launches_.clear();
  // key: kind, lanes, LDS staging, precision -> tasks of that shape at this level index
  using Key = std::tuple<int, int, int, int>;
  for (int l = 0; l < max_levels; ++l) {  // forward, leaves first
    const int g0 = (int)gathers.size();
    std::map<Key, std::pair<std::vector<SweepTask>, int>> groups;
    for (int j = 0; j < ns; ++j) {
      const dpd_mesh* m = active[j]->m;
      const LevelPlan& P = m->plan;
      if (l >= m->S.n_levels) continue;
      const int n = P.fwd_off[l + 1] - P.fwd_off[l];
      if (!n) continue;
      const int ng = P.gather_off[l + 1] - P.gather_off[l];
      for (int i = 0; i < ng; ++i) gathers.push_back(make_int2(j, P.gather_cols[P.gather_off[l] + i]));
      const bool wide = P.fwd_wide[l] != 0;
      const Key key{wide ? 2 : 1, wide ? sweep_lanes(P.fwd_cols[l]) : 0, 0, active[j]->fp32 ? 1 : 0};
      auto& g = groups[key];
      g.second = std::max(g.second, P.fwd_cols[l]);
      for (int i = 0; i < n; ++i) {
        SweepTask t = P.fwd[P.fwd_off[l] + i];
        t.pad0 = j;
        t.pad1 = ng > 0 ? 1 : 0;
        g.first.push_back(t);
      }
    }
    if ((int)gathers.size() > g0)
      launches_.push_back(Launch{0, g0, (int)gathers.size() - g0, 0, 0, false, false});
    for (auto& kv : groups) {
      const int first = (int)tasks.size();
      tasks.insert(tasks.end(), kv.second.first.begin(), kv.second.first.end());
      launches_.push_back(Launch{std::get<0>(kv.first), first, (int)kv.second.first.size(), std::get<1>(kv.first),
                                 kv.second.second, false, std::get<3>(kv.first) != 0});
    }
  }
  for (int b = 0; b < max_levels; ++b) {  // backward, roots first
    std::map<Key, std::pair<std::vector<SweepTask>, int>> groups;
    for (int j = 0; j < ns; ++j) {
      const dpd_mesh* m = active[j]->m;
      const LevelPlan& P = m->plan;
      const int l = m->S.n_levels - 1 - b;
      if (l < 0) continue;
      const int n = P.bwd_off[l + 1] - P.bwd_off[l];
      if (!n) continue;
      const bool narrow = P.bwd_narrow[l] != 0;
      const bool lds = (int64_t)3 * P.bwd_rows[l] * (int64_t)sizeof(double) <= kSweepLdsBudget;
      const Key key{narrow ? 4 : 3, narrow ? 0 : sweep_lanes(P.bwd_rows[l]), (!narrow && lds) ? 1 : 0,
                    active[j]->fp32 ? 1 : 0};
      auto& g = groups[key];
      g.second = std::max(g.second, P.bwd_rows[l]);
      for (int i = 0; i < n; ++i) {
        SweepTask t = P.bwd[P.bwd_off[l] + i];
        t.pad0 = j;
        t.pad1 = 0;
        g.first.push_back(t);
      }
    }
    for (auto& kv : groups) {
      const int first = (int)tasks.size();
      tasks.insert(tasks.end(), kv.second.first.begin(), kv.second.first.end());
      launches_.push_back(Launch{std::get<0>(kv.first), first, (int)kv.second.first.size(), std::get<1>(kv.first),
                                 kv.second.second, std::get<2>(kv.first) != 0, std::get<3>(kv.first) != 0});
    }
  }
  if (!reserve((size_t)std::max(ns, max_slots_), tasks.size(), std::max<size_t>(1, gathers.size()))) return false;
  if (hipMemcpyAsync(d_solve_, hs.data(), ns * sizeof(BatchSolveSlot), hipMemcpyHostToDevice, stream_) !=
          hipSuccess ||
      hipMemcpyAsync(d_cg_, hc.data(), ns * sizeof(BatchCgSlot), hipMemcpyHostToDevice, stream_) != hipSuccess ||
      (!tasks.empty() && hipMemcpyAsync(d_tasks_, tasks.data(), tasks.size() * sizeof(SweepTask),
                                        hipMemcpyHostToDevice, stream_) != hipSuccess) ||
      (!gathers.empty() && hipMemcpyAsync(d_gathers_, gathers.data(), gathers.size() * sizeof(int2),
                                          hipMemcpyHostToDevice, stream_) != hipSuccess))
    return false;
  // the host vectors are released on return: the copies must have been made
  if (hipStreamSynchronize(stream_) != hipSuccess) return false;
  nslots_ = ns;
  elem_blocks_ = eb;
  node_blocks_ = nb;
  return true;
}

bool Batcher::run_chunk(int iterations) {
  for (int it = 0; it < iterations; ++it) {
    for (const Launch& L : launches_) {
      switch (L.kind) {
        case 0:
          launch_batch_sweep_gather(d_solve_, stream_, d_gathers_ + L.first, L.count);
          break;
        case 1:
          launch_batch_sweep_fwd(d_solve_, stream_, d_tasks_ + L.first, L.count, L.lds, L.fp32);
          break;
        case 2:
          launch_batch_sweep_fwd_wide(d_solve_, stream_, d_tasks_ + L.first, L.count, L.lpr, L.lds, L.fp32);
          break;
        case 3:
          launch_batch_sweep_bwd(d_solve_, stream_, d_tasks_ + L.first, L.count, L.lpr, L.use_lds, L.lds, L.fp32);
          break;
        default:
          launch_batch_sweep_bwd_narrow(d_solve_, stream_, d_tasks_ + L.first, L.count, L.lds, L.fp32);
          break;
      }
    }
    launch_batch_cg_iteration_tail(d_cg_, nslots_, elem_blocks_, node_blocks_, stream_);
  }
  return hipGetLastError() == hipSuccess;
}

bool Batcher::read_states(const std::vector<Job*>& active) {
  for (size_t j = 0; j < active.size(); ++j)
    if (hipMemcpyAsync(h_st_ + j, active[j]->st, sizeof(IterState), hipMemcpyDeviceToHost, stream_) != hipSuccess)
      return false;
  return hipStreamSynchronize(stream_) == hipSuccess;
}

// Iterations until the next state read: the fewest that any active solve
// still needs at the residual reduction rate it showed since the previous
// read (the first read after kChunkFirst), in multiples of kChunkMin.
int Batcher::next_chunk(const std::vector<Job*>& active) const {
  int chunk = kChunkMax;
  for (size_t j = 0; j < active.size(); ++j) {
    const Job& J = *active[j];
    const IterState& h = h_st_[j];
    int need = kChunkFirst;
    const int it = h.iter - J.iter_prev;
    if (J.rsq_prev > 0.0 && it > 0 && h.rsq > 0.0 && h.rsq < J.rsq_prev && h.tolsq * h.nb2 < h.rsq) {
      const double n = std::log(h.tolsq * h.nb2 / h.rsq) / (std::log(h.rsq / J.rsq_prev) / it);
      if (std::isfinite(n) && n > 0.0) need = (int)std::ceil(n);
    }
    need = std::min(need, J.max_it - J.iters);
    chunk = std::min(chunk, need);
  }
  chunk = (std::max(chunk, 1) + kChunkMin - 1) / kChunkMin * kChunkMin;
  return std::min(kChunkMax, chunk);
}

void Batcher::loop() {
  const bool ok_dev = hipSetDevice(device_) == hipSuccess &&
                      hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) == hipSuccess;
  std::vector<Job*> active;
  bool rebuild = false;
  int chunk = kChunkFirst;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || !incoming_.empty() || !active.empty(); });
      if (stop_ && incoming_.empty() && active.empty()) break;
      if (!incoming_.empty()) {
        active.insert(active.end(), incoming_.begin(), incoming_.end());
        incoming_.clear();
        rebuild = true;
        chunk = std::min(chunk, kChunkFirst);   // the new solves have no residual history
      }
    }
    bool ok = ok_dev;
    if (ok && rebuild) {
      ok = build(active);
      rebuild = false;
    }
    if (ok) ok = run_chunk(chunk);
    if (ok) ok = read_states(active);
    std::vector<Job*> still, finished;
    std::vector<IterState> still_h;
    for (size_t j = 0; j < active.size(); ++j) {
      Job* J = active[j];
      if (!ok) {
        J->rc = DPD_EHIP;
        finished.push_back(J);
        continue;
      }
      J->iters += chunk;
      const IterState& h = h_st_[j];
      if (h.done || h.iter >= J->max_it || J->iters >= J->max_it) {
        finished.push_back(J);
      } else {
        still.push_back(J);
        still_h.push_back(h);
      }
    }
    int next = kChunkFirst;
    if (ok && !still.empty()) {
      std::copy(still_h.begin(), still_h.end(), h_st_);
      next = next_chunk(still);
      for (size_t j = 0; j < still.size(); ++j) {
        still[j]->rsq_prev = h_st_[j].rsq;
        still[j]->iter_prev = h_st_[j].iter;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (ok) {
        stats_.iterations += chunk;
        stats_.slot_iterations += (int64_t)chunk * (int64_t)active.size();
        stats_.launches += (int64_t)chunk * (int64_t)(launches_.size() + 3);
        stats_.peak_slots = std::max(stats_.peak_slots, (int32_t)active.size());
      }
      for (Job* J : finished) J->done = true;
      stats_.solves += (int64_t)finished.size();
    }
    if (!finished.empty()) {
      cv_.notify_all();
      rebuild = true;
    }
    active.swap(still);
    chunk = next;
  }
  if (stream_) (void)hipStreamDestroy(stream_);
  if (d_solve_) (void)hipFree(d_solve_);
  if (d_cg_) (void)hipFree(d_cg_);
  if (d_tasks_) (void)hipFree(d_tasks_);
  if (d_gathers_) (void)hipFree(d_gathers_);
  if (h_st_) (void)hipHostFree(h_st_);
}

}  // namespace dpd
