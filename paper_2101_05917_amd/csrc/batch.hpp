// Batched conjugate-gradient engine: the preconditioned CG solves of several
// mesh handles (the adjoint systems of Alg. 2's quasi-Newton acceleration and
// the forward Newton steps) advanced together, one batched launch per kernel
// shape and iteration instead of one launch per handle.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/diffpd.h"
#include "device.hpp"

namespace dpd {

// Counters of a batcher since its creation.
struct BatchStats {
  int64_t iterations = 0;       // batched iterations launched
  int64_t slot_iterations = 0;  // sum over those iterations of the solves taking part
  int64_t launches = 0;         // kernel launches made for them
  int64_t solves = 0;           // solves completed
  int32_t peak_slots = 0;       // most solves in one batch
};

// A thread of its own owns one HIP stream (default priority) and runs the
// batch: a caller hands over a prepared solve (state reset, vectors z, p, q
// zeroed, r = rhs, |rhs|^2 in the state, its stream's work complete) and blocks
// until the solve has finished; solves that arrive while a batch runs join it
// at the next chunk boundary, finished ones leave it there.  Each slot's blocks
// run exactly its own kernels' arithmetic (same tasks, same per-slot block
// indices and reduction order), so a handle's result does not depend on which
// other handles share its launches.
class Batcher {
 public:
  Batcher(int device, int max_slots);
  ~Batcher();
  Batcher(const Batcher&) = delete;
  Batcher& operator=(const Batcher&) = delete;

  // Run the prepared solve of handle m on its state st (device) to the end
  // (converged, non-positive curvature, non-finite or max_it iterations).
  dpd_status solve(dpd_mesh* m, IterState* st, bool fp32, int max_it);
  BatchStats stats();

 private:
  struct Job {
    dpd_mesh* m;
    IterState* st;
    bool fp32;
    int max_it;
    int iters = 0;            // iterations enqueued for it
    double rsq_prev = -1.0;   // |r|^2 at the previous boundary
    int iter_prev = 0;
    bool done = false;
    dpd_status rc = DPD_OK;
  };
  struct Launch {
    int kind;                 // 0 gather, 1 narrow forward, 2 wide forward, 3 backward columns, 4 narrow backward
    int first, count;
    int lpr, lds;             // lanes per row / column; LDS extent (columns or rows)
    bool use_lds, fp32;
  };

  void loop();
  bool build(const std::vector<Job*>& active);
  bool run_chunk(int iterations);
  bool read_states(const std::vector<Job*>& active);
  int next_chunk(const std::vector<Job*>& active) const;
  bool reserve(size_t slots, size_t tasks, size_t gathers);

  int device_, max_slots_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::vector<Job*> incoming_;
  bool stop_ = false;
  BatchStats stats_;
  std::thread thread_;

  // owned by the batch thread
  hipStream_t stream_ = nullptr;
  std::vector<Launch> launches_;
  int nslots_ = 0, elem_blocks_ = 0, node_blocks_ = 0;
  size_t cap_slots_ = 0, cap_tasks_ = 0, cap_gathers_ = 0;
  BatchSolveSlot* d_solve_ = nullptr;
  BatchCgSlot* d_cg_ = nullptr;
  SweepTask* d_tasks_ = nullptr;
  int2* d_gathers_ = nullptr;
  IterState* h_st_ = nullptr;   // pinned [cap_slots_]
};

}  // namespace dpd
