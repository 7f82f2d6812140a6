// Host-side test driver for the single-launch solve's queue (test
// infrastructure, not part of the library).
//
// Builds the library's sweep plan and its single-launch queue (build_dag) for
// a mesh, checks the queue's structure against the level plan, then plays the
// launch on the CPU: W simulated workgroups claim entries in queue order (one
// ahead, as the kernel does), an entry runs only when the kernel's wait
// conditions hold, and finishing it updates the counters as the kernel does.
// Random choices among the runnable workgroups explore many interleavings.
// Every value an entry reads (forward updates, gathered right-hand sides,
// forward and backward solutions) must have been written by an entry that
// finished before it, every value must be written exactly once, and the
// queue must drain (no interleaving may leave every workgroup waiting).
//
// usage: dag_check <input.bin>   (the input format of host_check, no
//        right-hand sides needed); exit 0 when every check passes.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../paper_2101_05917_amd/csrc/internal.hpp"

using namespace dpd;

#define CHECK(cond)                                                                \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__);       \
      std::exit(3);                                                                \
    }                                                                              \
  } while (0)

template <typename T>
static void rd(FILE* f, T* p, size_t n) {
  if (n && std::fread(p, sizeof(T), n, f) != n) throw std::runtime_error("short read");
}

struct Sim {
  const Symbolic& S;
  const LevelPlan& P;
  const DagPlan& D;
  // counters as in the kernel
  std::vector<uint32_t> cdone, tdone, gdone, bdone;
  // written flags: forward updates (per U position), gathered rhs, y, x (per internal column)
  std::vector<uint8_t> wU, wbt, wy, wx;

  Sim(const Symbolic& s, const LevelPlan& p, const DagPlan& d) : S(s), P(p), D(d) {}

  void reset() {
    const size_t ns = S.sn.size();
    cdone.assign(ns, 0);
    tdone.assign(ns, 0);
    gdone.assign(ns, 0);
    bdone.assign(ns, 0);
    wU.assign(S.u_size, 0);
    wbt.assign(S.n, 0);
    wy.assign(S.n, 0);
    wx.assign(S.n, 0);
  }

  bool ready(const DagEntry& e) const {
    const bool narrow = e.kind == kDagFwdNarrow || e.kind == kDagBwdNarrow;
    const int nsub = narrow ? e.n : 1;
    for (int k = 0; k < nsub; ++k) {
      const int s = e.sn[k];
      const DagSn& d = D.sn[s];
      if (e.kind == kDagBwdCols || e.kind == kDagBwdNarrow) {
        if (d.parent >= 0) {
          if (bdone[d.parent] < (uint32_t)D.sn[d.parent].ntb) return false;
        } else if (tdone[s] < (uint32_t)d.ntf) {
          return false;
        }
      } else {
        if (cdone[s] < (uint32_t)d.nch) return false;
        if (e.kind != kDagGather && gdone[s] < (uint32_t)d.ngt) return false;
      }
    }
    return true;
  }

  void read_rhs_column(int j, bool pre) {
    if (pre) {
      CHECK(wbt[j]);
      return;
    }
    for (int k = S.cptr[j]; k < S.cptr[j + 1]; ++k) CHECK(wU[S.cidx[k]]);
  }

  void fwd_task(const SweepTask& t, bool pre) {
    for (int c = 0; c < t.ncols; ++c) read_rhs_column(t.col0 + c, pre);
    for (int r = t.first; r < t.first + t.count; ++r) {
      if (r < t.ncols) {
        CHECK(!wy[t.col0 + r]);
        wy[t.col0 + r] = 1;
      } else {
        const int64_t u = t.u_off + (r - t.ncols);
        CHECK(u >= 0 && u < (int64_t)wU.size() && !wU[u]);
        wU[u] = 1;
      }
    }
  }

  void bwd_task(const SweepTask& t) {
    for (int c = 0; c < t.ncols; ++c) CHECK(wy[t.col0 + c]);
    for (int r = 0; r < t.nrows; ++r) CHECK(wx[S.rows[t.rows_off + r]]);
    for (int c = t.first; c < t.first + t.count; ++c) {
      CHECK(!wx[t.col0 + c]);
      wx[t.col0 + c] = 1;
    }
  }

  void run(const DagEntry& e) {
    switch (e.kind) {
      case kDagGather:
        for (int i = 0; i < e.n; ++i) {
          const int j = P.gather_cols[e.first + i];
          read_rhs_column(j, false);
          CHECK(!wbt[j]);
          wbt[j] = 1;
        }
        gdone[e.sn[0]] += 1;
        return;
      case kDagFwdNarrow:
      case kDagFwdWide:
        for (int i = 0; i < e.n; ++i) {
          const SweepTask& t = P.fwd[e.first + i];
          fwd_task(t, (e.flags & 1) != 0);
          const int s = t.sn;
          if (++tdone[s] == (uint32_t)D.sn[s].ntf && D.sn[s].parent >= 0) cdone[D.sn[s].parent] += 1;
        }
        return;
      default:
        for (int i = 0; i < e.n; ++i) {
          const SweepTask& t = P.bwd[e.first + i];
          bwd_task(t);
          bdone[t.sn] += 1;
        }
        return;
    }
  }

  // One launch with W resident workgroups.  Events, chosen at random among
  // those possible: a workgroup starts and claims its first entry; a
  // workgroup holding an entry claims the next one (the kernel does this
  // before waiting); a workgroup whose entry's waits hold runs it and moves on
  // to the entry it claimed ahead.  Returns the number of events.
  int64_t launch(int W, uint64_t seed) {
    reset();
    std::mt19937_64 rng(seed);
    const int nq = (int)D.q.size();
    int next = 0;
    std::vector<int> started(W, 0), cur(W, -1), ahead(W, -1);
    int64_t events = 0, finished = 0;
    struct Ev { int kind, w; };
    std::vector<Ev> evs;
    while (finished < nq) {
      evs.clear();
      for (int w = 0; w < W; ++w) {
        if (!started[w]) {
          evs.push_back({0, w});
        } else if (cur[w] < nq) {
          if (ahead[w] < 0) evs.push_back({1, w});
          else if (ready(D.q[cur[w]])) evs.push_back({2, w});
        }
      }
      CHECK(!evs.empty());   // every workgroup waiting: the launch would hang
      const Ev ev = evs[rng() % evs.size()];
      const int w = ev.w;
      if (ev.kind == 0) {
        started[w] = 1;
        cur[w] = next++;
      } else if (ev.kind == 1) {
        ahead[w] = next++;
      } else {
        run(D.q[cur[w]]);
        ++finished;
        cur[w] = ahead[w];
        ahead[w] = -1;
      }
      ++events;
    }
    for (int j = 0; j < S.n; ++j) CHECK(wy[j] && wx[j]);
    for (size_t u = 0; u < wU.size(); ++u) CHECK(wU[u]);
    return events;
  }
};

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t nc, nfx;
  rd(in, &nc, 1);
  std::vector<int32_t> cells(3 * nc);
  std::vector<double> youngs(nc);
  rd(in, cells.data(), cells.size());
  rd(in, youngs.data(), youngs.size());
  rd(in, &nfx, 1);
  std::vector<int32_t> fixed(3 * nfx);
  rd(in, fixed.data(), fixed.size());
  double ov[17];
  rd(in, ov, 17);
  dpd_options o{};
  o.dx = ov[0]; o.rho = ov[1]; o.nu = ov[2]; o.h = ov[3];
  for (int k = 0; k < 3; ++k) { o.gravity[k] = ov[4 + k]; o.origin[k] = ov[7 + k]; o.fiber[k] = ov[14 + k]; }
  o.contact_k = ov[10]; o.friction_mu = ov[11]; o.friction_eps = ov[12]; o.muscle_k = ov[13];
  int32_t leaf_max, sep_max;
  rd(in, &leaf_max, 1);
  rd(in, &sep_max, 1);
  std::fclose(in);
  HostMesh m;
  const std::string err = build_mesh(cells.data(), nc, youngs.data(), fixed.data(), nfx, o, m);
  if (!err.empty()) {
    std::fprintf(stderr, "build_mesh: %s\n", err.c_str());
    return 4;
  }
  Csr A;
  assemble_As(m, o, A);
  Symbolic S;
  analyse(m, A, leaf_max, sep_max, S);
  LevelPlan P;
  build_plan(S, P);
  DagPlan D;
  const int64_t budget = 60 * 1024;
  build_dag(S, P, budget, D);
  if (!D.usable) {
    std::printf("plan not usable (LDS); the level launches are used\n");
    return 0;
  }

  // structure: every level task and gathered column in exactly one entry,
  // forward entries first, levels in order, counts per supernode
  const int ns = (int)S.sn.size();
  CHECK((int)D.sn.size() == ns);
  std::vector<int> seen_f(P.fwd.size(), 0), seen_b(P.bwd.size(), 0), seen_g(P.gather_cols.size(), 0);
  std::vector<int> ntf(ns, 0), ngt(ns, 0), ntb(ns, 0);
  int last_level = -1;
  bool in_bwd = false;
  for (size_t i = 0; i < D.q.size(); ++i) {
    const DagEntry& e = D.q[i];
    const bool bwd = e.kind == kDagBwdCols || e.kind == kDagBwdNarrow;
    CHECK(bwd == ((int)i >= D.n_fwd));
    if (bwd && !in_bwd) {
      in_bwd = true;
      last_level = S.n_levels;
    }
    CHECK(e.n >= 1);
    if (e.kind == kDagGather) {
      CHECK(e.n <= kDagGatherCols);
      const int s = e.sn[0];
      for (int k = 0; k < e.n; ++k) {
        const int g = e.first + k;
        CHECK(g >= 0 && g < (int)P.gather_cols.size());
        seen_g[g]++;
        CHECK(S.snode_of[P.gather_cols[g]] == s);
      }
      CHECK(S.sn[s].level >= last_level);
      last_level = S.sn[s].level;
      ngt[s]++;
      continue;
    }
    CHECK(e.n == 1);
    const std::vector<SweepTask>& tasks = bwd ? P.bwd : P.fwd;
    const int lvl = S.sn[tasks[e.first].sn].level;
    CHECK(bwd ? lvl <= last_level : lvl >= last_level);
    last_level = lvl;
    for (int k = 0; k < e.n; ++k) {
      const int t = e.first + k;
      CHECK(t >= 0 && t < (int)tasks.size());
      CHECK(tasks[t].sn == e.sn[k]);
      CHECK(S.sn[tasks[t].sn].level == lvl);
      (bwd ? seen_b : seen_f)[t]++;
      (bwd ? ntb : ntf)[tasks[t].sn]++;
      if (e.kind == kDagFwdNarrow) CHECK(!P.fwd_wide[lvl] && tasks[t].ncols <= kDagNarrowCols);
      if (e.kind == kDagFwdWide) CHECK(P.fwd_wide[lvl] && e.lpr == sweep_lanes(P.fwd_cols[lvl]));
      if (e.kind == kDagBwdNarrow) {
        CHECK(P.bwd_narrow[lvl]);
        CHECK(lds_bwd_narrow(tasks[t].ncols + tasks[t].nrows) <= D.bwd_region);
      }
      if (e.kind == kDagBwdCols) {
        CHECK(!P.bwd_narrow[lvl] && e.lpr == sweep_lanes(P.bwd_rows[lvl]));
        CHECK(e.flags & 2);
        CHECK(3 * (int64_t)P.bwd_rows[lvl] * 8 <= D.lds_bytes);
      }
      if (e.kind == kDagFwdWide) CHECK(3 * (int64_t)P.fwd_cols[lvl] * 8 <= D.lds_bytes);
    }
  }
  for (int v : seen_f) CHECK(v == 1);
  for (int v : seen_b) CHECK(v == 1);
  for (int v : seen_g) CHECK(v == 1);
  for (int s = 0; s < ns; ++s) {
    CHECK(D.sn[s].parent == S.sn[s].parent);
    CHECK(D.sn[s].nch == (int)S.children[s].size());
    CHECK(D.sn[s].ntf == ntf[s] && D.sn[s].ngt == ngt[s] && D.sn[s].ntb == ntb[s]);
    CHECK(ntf[s] >= 1 && ntb[s] >= 1);
  }
  CHECK(D.lds_bytes <= budget);
  CHECK((int64_t)D.bwd_region * 8 <= D.lds_bytes);

  // the launch played with many interleavings and workgroup counts
  Sim sim(S, P, D);
  int64_t plays = 0;
  for (int W : {1, 2, 7, 64, 512})
    for (uint64_t seed = 0; seed < 4; ++seed) {
      sim.launch(W, 1000 * W + seed);
      ++plays;
    }
  std::printf("supernodes %d levels %d entries %zu (forward %d) lds %lld plays %lld\n", ns, S.n_levels,
              D.q.size(), D.n_fwd, (long long)D.lds_bytes, (long long)plays);
  return 0;
}
