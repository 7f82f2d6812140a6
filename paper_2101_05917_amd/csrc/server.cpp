// Rollout server: continuous batching of differentiable rollouts.
//
// Worker threads (one per slot) take queued requests in arrival order, run
// the host analysis, wait until the request's device footprint fits in the
// remaining HBM budget, then keep the request's factor and states resident
// while its forward and adjoint steps run on the worker's own HIP stream; a
// slot is refilled as soon as its request finishes.  With batching on, every
// request takes the multi-launch solver and every conjugate-gradient solve of
// a resident request (the Newton steps of its forward steps and the adjoint
// systems of its backward steps) runs in a shared batch engine: one launch per
// sweep level and kernel shape, and one for each of the element Hessian
// product, the node gather and the vector update, over all requests whose
// solves are under way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/diffpd.h"
#include "batch.hpp"
#include "handle.hpp"
#include "internal.hpp"

namespace {

struct Request {
  int64_t id = 0;
  std::vector<int32_t> cells, fixed;
  std::vector<double> youngs, loss_x;
  int64_t n_nodes = 0;
  int32_t steps = 0;
  dpd_options opt{};
  dpd_result res{};
  std::vector<double> gx, gv, gE;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct dpd_server {
  int64_t budget = 0;
  int32_t max_slots = 1;
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_mem, cv_done;
  std::deque<Request*> queue;
  std::vector<std::unique_ptr<Request>> all;
  int64_t used = 0, peak = 0;
  int32_t active = 0, peak_active = 0, pending = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::unique_ptr<dpd::Batcher> batcher;   // null: each slot iterates on its own stream
  bool verbose = false;                    // DPD_SERVER_VERBOSE set: failed requests reported on stderr
};

namespace {

// One whole rollout on stream s; fills r->res and the gradients.
void run_request(dpd_server* srv, Request* r, hipStream_t s) {
  dpd_mesh* m = nullptr;
  dpd_status st = dpd::create_host(r->cells.data(), (int64_t)r->cells.size() / 3, r->youngs.data(),
                                   r->fixed.empty() ? nullptr : r->fixed.data(),
                                   (int64_t)r->fixed.size() / 3, &r->opt, &m);
  // Everything a poll may read is published under srv->mu; the worker keeps
  // its running figures in locals until then.
  auto finish_fail = [&](dpd_status code) {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->res.status = code;
    r->res.state = DPD_REQ_FAILED;
    r->res.t_done = now_s(srv->t0);
  };
  if (st != DPD_OK) return finish_fail(st);
  m->batcher = srv->batcher.get();
  dpd_mesh_info info{};
  dpd_get_info(m, &info);
  const int64_t N = info.n_nodes, E = info.n_elements, T = r->steps;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->res.n_nodes = N;
    r->res.n_elements = E;
  }
  if (N != r->n_nodes || (int64_t)r->loss_x.size() != 3 * N) {
    dpd::destroy_synced(m);
    return finish_fail(DPD_EINVAL);
  }
  const int64_t n3 = 3 * N;
  const int64_t state_bytes = 8 * ((T + 1) * 2 * n3 + 5 * n3 + E);
  const int64_t fp = dpd::footprint_bytes(m) + state_bytes;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->res.footprint_bytes = fp;
  }
  if (fp > srv->budget) {
    dpd::destroy_synced(m);
    return finish_fail(DPD_ENOMEM);
  }
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_mem.wait(lk, [&] { return srv->used + fp <= srv->budget; });
    srv->used += fp;
    srv->peak = std::max(srv->peak, srv->used);
    srv->active += 1;
    srv->peak_active = std::max(srv->peak_active, srv->active);
    r->res.t_admit = now_s(srv->t0);
    r->res.state = DPD_REQ_RUNNING;
  }
  double* buf = nullptr;
  dpd_status result = DPD_OK;
  int64_t fwd_iters = 0, bwd_iters = 0;
  double loss = 0.0;
  auto soft = [&](dpd_status c) {
    if (c < 0) return false;
    if (c == DPD_NOT_CONVERGED) result = DPD_NOT_CONVERGED;
    return true;
  };
  do {
    if ((st = dpd::upload_device(m)) != DPD_OK) {
      m = nullptr;
      result = st;
      break;
    }
    if ((st = dpd_factorize(m, s)) != DPD_OK) {
      result = st;
      break;
    }
    if (hipMalloc(&buf, (size_t)state_bytes) != hipSuccess) {
      buf = nullptr;
      result = DPD_ENOMEM;
      break;
    }
    double* xs = buf;                       // [T+1][3N]
    double* vs = xs + (T + 1) * n3;         // [T+1][3N]
    double* gx = vs + (T + 1) * n3;
    double* gv = gx + n3;
    double* gx2 = gv + n3;
    double* gv2 = gx2 + n3;
    double* c = gv2 + n3;
    double* gE = c + n3;
    std::vector<double> X(n3);
    dpd_rest_positions(m, X.data());
    if (hipMemcpyAsync(xs, X.data(), n3 * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(vs, 0, n3 * 8, s) != hipSuccess) {
      result = DPD_EHIP;
      break;
    }
    bool ok = true;
    for (int64_t t = 0; t < T && ok; ++t) {
      dpd_stats fs{};
      const dpd_status c1 = dpd_forward_step(m, s, xs + t * n3, vs + t * n3, nullptr, xs + (t + 1) * n3,
                                             vs + (t + 1) * n3, &fs);
      ok = soft(c1);
      if (!ok) result = c1;
      fwd_iters += fs.fwd_iters;
    }
    if (!ok) break;
    std::vector<double> xT(n3);
    if (hipMemcpyAsync(xT.data(), xs + T * n3, n3 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(gx, r->loss_x.data(), n3 * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(gv, 0, n3 * 8, s) != hipSuccess || hipMemsetAsync(gE, 0, E * 8, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      result = DPD_EHIP;
      break;
    }
    double L = 0.0;
    for (int64_t i = 0; i < n3; ++i) L += r->loss_x[i] * xT[i];
    loss = L;
    for (int64_t t = T - 1; t >= 0 && ok; --t) {
      dpd_stats bs{};
      dpd_status c2 = dpd_backward_step(m, s, xs + t * n3, vs + t * n3, nullptr, xs + (t + 1) * n3, gx,
                                        gv, gx2, gv2, gE, nullptr, &bs);
      ok = soft(c2);
      if (!ok) result = c2;
      bwd_iters += bs.bwd_iters;
      std::swap(gx, gx2);
      std::swap(gv, gv2);
    }
    if (!ok) break;
    r->gx.resize(n3);
    r->gv.resize(n3);
    r->gE.resize(E);
    if (hipMemcpyAsync(r->gx.data(), gx, n3 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(r->gv.data(), gv, n3 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(r->gE.data(), gE, E * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      result = DPD_EHIP;
  } while (false);
  if (result < 0 && srv->verbose)
    std::fprintf(stderr, "dpd_server: request %lld failed (%s): %s\n", (long long)r->id, dpd_status_string(result),
                 m ? dpd_last_error(m) : "mesh upload");
  (void)hipStreamSynchronize(s);
  if (buf) (void)hipFree(buf);
  if (m) dpd::destroy_synced(m);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->used -= fp;
    srv->active -= 1;
    r->res.fwd_iters = fwd_iters;
    r->res.bwd_iters = bwd_iters;
    r->res.loss = loss;
    r->res.status = result;
    r->res.state = result < 0 ? DPD_REQ_FAILED : DPD_REQ_DONE;
    r->res.t_done = now_s(srv->t0);
  }
  srv->cv_mem.notify_all();
}

void worker(dpd_server* srv) {
  (void)hipSetDevice(srv->device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_work.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
      if (srv->queue.empty()) break;
      r = srv->queue.front();
      srv->queue.pop_front();
    }
    if (s) run_request(srv, r, s);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      if (!s) {
        r->res.status = DPD_EHIP;
        r->res.state = DPD_REQ_FAILED;
      }
      srv->pending -= 1;
    }
    srv->cv_done.notify_all();
  }
  if (s) (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

dpd_status dpd_server_create(int64_t budget, int32_t max_slots, int32_t batched, dpd_server** out) {
  if (!out || budget <= 0 || max_slots < 1) return DPD_EINVAL;
  dpd_server* srv = new dpd_server();
  srv->budget = budget;
  srv->max_slots = max_slots;
  (void)hipGetDevice(&srv->device);
  if (batched) srv->batcher = std::make_unique<dpd::Batcher>(srv->device, max_slots);
  srv->verbose = std::getenv("DPD_SERVER_VERBOSE") != nullptr;
  srv->t0 = std::chrono::steady_clock::now();
  for (int32_t i = 0; i < max_slots; ++i) srv->workers.emplace_back(worker, srv);
  *out = srv;
  return DPD_OK;
}

dpd_status dpd_server_batch_stats(dpd_server* srv, dpd_batch_stats* out) {
  if (!srv || !out) return DPD_EINVAL;
  std::memset(out, 0, sizeof(*out));
  if (!srv->batcher) return DPD_OK;
  const dpd::BatchStats b = srv->batcher->stats();
  out->iterations = b.iterations;
  out->slot_iterations = b.slot_iterations;
  out->launches = b.launches;
  out->solves = b.solves;
  out->peak_slots = b.peak_slots;
  return DPD_OK;
}

dpd_status dpd_server_submit(dpd_server* srv, const dpd_request* q, int64_t* ticket) {
  if (!srv || !q || !ticket || !q->cells_ijk || !q->youngs || !q->loss_x || q->n_cells <= 0 ||
      q->steps < 1 || q->n_nodes <= 0 || (q->n_fixed > 0 && !q->fixed_ijk))
    return DPD_EINVAL;
  auto r = std::make_unique<Request>();
  r->cells.assign(q->cells_ijk, q->cells_ijk + 3 * q->n_cells);
  r->youngs.assign(q->youngs, q->youngs + q->n_cells);
  if (q->n_fixed > 0) r->fixed.assign(q->fixed_ijk, q->fixed_ijk + 3 * q->n_fixed);
  r->loss_x.assign(q->loss_x, q->loss_x + 3 * q->n_nodes);
  r->n_nodes = q->n_nodes;
  r->steps = q->steps;
  r->opt = q->opt;
  // no stream capture in the workers: a capture under way in one worker makes
  // the synchronous runtime calls of another (a mesh upload's copies and
  // memsets) fail; the batch engine is what amortizes launches here
  r->opt.use_graphs = 0;
  // with the batch engine every request takes the multi-launch solver, whose
  // iterations the engine shares (not the fused dense solver's one
  // cooperative launch per request and solve)
  if (srv->batcher) r->opt.fused_cg = 0;
  r->res.state = DPD_REQ_QUEUED;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->id = (int64_t)srv->all.size();
    r->res.t_submit = now_s(srv->t0);
    *ticket = r->id;
    srv->queue.push_back(r.get());
    srv->all.push_back(std::move(r));
    srv->pending += 1;
  }
  srv->cv_work.notify_one();
  return DPD_OK;
}

dpd_status dpd_server_poll(dpd_server* srv, int64_t ticket, dpd_result* out, double* g_x0,
                           double* g_v0, double* g_youngs) {
  if (!srv || !out) return DPD_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (ticket < 0 || ticket >= (int64_t)srv->all.size()) return DPD_EINVAL;
  const Request& r = *srv->all[ticket];
  *out = r.res;
  if (r.res.state == DPD_REQ_DONE) {
    if (g_x0) std::memcpy(g_x0, r.gx.data(), r.gx.size() * 8);
    if (g_v0) std::memcpy(g_v0, r.gv.data(), r.gv.size() * 8);
    if (g_youngs) std::memcpy(g_youngs, r.gE.data(), r.gE.size() * 8);
  }
  return DPD_OK;
}

dpd_status dpd_server_drain(dpd_server* srv) {
  if (!srv) return DPD_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->pending == 0; });
  return DPD_OK;
}

dpd_status dpd_server_stats(dpd_server* srv, int64_t* peak_bytes, int32_t* peak_active) {
  if (!srv) return DPD_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (peak_bytes) *peak_bytes = srv->peak;
  if (peak_active) *peak_active = srv->peak_active;
  return DPD_OK;
}

void dpd_server_destroy(dpd_server* srv) {
  if (!srv) return;
  dpd_server_drain(srv);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  srv->batcher.reset();
  delete srv;
}

}  // extern "C"
