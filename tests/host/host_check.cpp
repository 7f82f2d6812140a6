// Host-side test driver (test infrastructure, not part of the library).
//
// Runs the library's host code (voxel ingestion, assembly of A_s, nested
// dissection, symbolic analysis, numeric factorization, panel construction,
// level schedule) and replays the GPU sweep kernels' index arithmetic task by
// task on the CPU, asserting every access stays inside its buffer.  Writes
// the node numbering, A_s and A^{-1} b for the given right-hand sides so the
// Python tests can compare them with the oracle.
//
// usage: host_check <input.bin> <output.bin>
#include <algorithm>
#include <cmath>
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../paper_2101_05917_amd/csrc/internal.hpp"

using namespace dpd;

#define CHECK(cond)                                                                   \
  do {                                                                                \
    if (!(cond)) {                                                                    \
      std::fprintf(stderr, "bounds check failed: %s (line %d)\n", #cond, __LINE__); \
      std::exit(3);                                                                   \
    }                                                                                 \
  } while (0)

template <typename T>
static void rd(FILE* f, T* p, size_t n) {
  if (n && std::fread(p, sizeof(T), n, f) != n) throw std::runtime_error("short read");
}
template <typename T>
static void wr(FILE* f, const T* p, size_t n) {
  if (n) std::fwrite(p, sizeof(T), n, f);
}

static int find_item_h(const int32_t* prefix, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Replay of the device factorization (factor_gpu.hip) on the CPU, workgroup
// by workgroup and lane by lane with the kernels' index arithmetic and a
// bounds check on every access; returns the panels it produces.
static std::vector<double> replay_device_factor(const Symbolic& S, const Csr& A, const FactorPlan& FP) {
  const int NB = kFactorNB, TT = kFactorTile, TH = 256;
  std::vector<double> F(FP.front_size, 0.0), P(S.panel_size, 0.0);
  const int ns = (int)FP.fronts.size();
  for (int c = 0; c < S.n; ++c) {
    const int s = S.snode_of[c];
    CHECK(s >= 0 && s < ns);
    const FrontDesc f = FP.fronts[s];
    const int j = c - f.col0;
    CHECK(j >= 0 && j < f.nc);
    const int64_t idx = f.panel_off + (int64_t)j * f.ld + j;
    CHECK(idx >= 0 && idx < S.panel_size);
    P[idx] = 1.0;
  }
  CHECK(FP.a_dst.size() == FP.a_src.size());
  for (size_t i = 0; i < FP.a_dst.size(); ++i) {
    CHECK(FP.a_dst[i] >= 0 && FP.a_dst[i] < FP.front_size);
    CHECK(FP.a_src[i] >= 0 && FP.a_src[i] < (int32_t)A.val.size());
    F[FP.a_dst[i]] = A.val[FP.a_src[i]];
  }
  auto fidx = [&](const FrontDesc& f, int64_t r, int64_t c) {
    CHECK(r >= 0 && r < f.ld && c >= 0 && c < f.ld);
    const int64_t i = f.front_off + r + c * f.ld;
    CHECK(i >= 0 && i < FP.front_size);
    return i;
  };
  auto pidx = [&](const FrontDesc& f, int64_t r, int64_t c) {
    CHECK(r >= 0 && r < f.ld && c >= 0 && c < f.nc);
    const int64_t i = f.panel_off + r + c * f.ld;
    CHECK(i >= 0 && i < S.panel_size);
    return i;
  };
  for (const FactorOp& op : FP.ops) {
    CHECK(op.n > 0 && op.list_off >= 0 && (size_t)op.list_off + 2 * op.n + 1 + op.blocks <= FP.ints.size());
    const int32_t* items = &FP.ints[op.list_off];
    const int32_t* pre = items + op.n;
    CHECK(pre[0] == 0 && pre[op.n] == op.blocks);
    for (int b = 0; b < op.blocks; ++b) {
      const int it = items[2 * op.n + 1 + b];
      CHECK(it == find_item_h(pre, op.n, b));
      CHECK(pre[it] <= b && b < pre[it + 1]);
      CHECK(items[it] >= 0 && items[it] < ns);
      const FrontDesc f = FP.fronts[items[it]];
      const int local = b - pre[it];
      if (op.kind == kFactorExtend) {
        CHECK(f.parent >= 0 && f.parent < ns);
        const FrontDesc pa = FP.fronts[f.parent];
        for (int w = 0; w < TH / 64; ++w) {
          const int q = local * (TH / 64) + w;
          if (q >= f.nrows) continue;
          CHECK(f.rows_off + q < (int64_t)FP.relmap.size());
          const int rq = FP.relmap[f.rows_off + q];
          for (int lane = 0; lane < 64; ++lane)
            for (int p0 = q + lane; p0 < f.nrows; p0 += 256)
              for (int k = 0; k < 4; ++k) {
                const int pc = std::min(p0 + 64 * k, f.nrows - 1);   // clamped load index
                CHECK(f.rows_off + pc < (int64_t)FP.relmap.size());
                const int rp = FP.relmap[f.rows_off + pc];
                (void)F[fidx(pa, rp, rq)];
                (void)F[fidx(f, f.nc + pc, f.nc + q)];
                if (p0 + 64 * k >= f.nrows) continue;
                CHECK(rp >= rq);
                F[fidx(pa, rp, rq)] += F[fidx(f, f.nc + pc, f.nc + q)];
              }
        }
      } else if (op.kind == kFactorPanel) {
        const int kb = std::min(NB, f.nc - op.k0), k0 = op.k0, k1 = k0 + kb;
        CHECK(kb > 0);
        const int PR = TH / 4;   // rows (or panel columns) per workgroup, four lanes each
        const int rows_chunks = (f.ld - k1 + PR - 1) / PR;
        double D[32][33], Li[32][33];
        for (int i = 0; i < NB; ++i)
          for (int j = 0; j < NB; ++j) {
            D[i][j] = (i < kb && j <= i) ? F[fidx(f, k0 + i, k0 + j)] : (i == j ? 1.0 : 0.0);
            Li[i][j] = 0.0;
          }
        for (int j = 0; j < kb; ++j) {
          CHECK(D[j][j] > 0.0);
          const double sd = std::sqrt(D[j][j]);
          for (int i = j; i < kb; ++i) D[i][j] = (i == j) ? sd : D[i][j] / sd;
          for (int t = j + 1; t < kb; ++t)
            for (int i = t; i < kb; ++i) D[i][t] -= D[i][j] * D[t][j];
        }
        for (int j = 0; j < kb; ++j) {
          Li[j][j] = 1.0 / D[j][j];
          for (int i = j + 1; i < kb; ++i) {
            double v = 0.0;
            for (int t = j; t < i; ++t) v += D[i][t] * Li[t][j];
            Li[i][j] = -v / D[i][i];
          }
        }
        CHECK(local < rows_chunks + (k1 + PR - 1) / PR);
        for (int slot = 0; slot < PR; ++slot) {
          double x[32];
          std::vector<int64_t> at(kb);
          if (local < rows_chunks) {
            const int i = k1 + local * PR + slot;
            if (i >= f.ld) continue;
            for (int t = 0; t < kb; ++t) at[t] = fidx(f, i, k0 + t);
            for (int t = 0; t < NB; ++t) x[t] = t < kb ? F[at[t]] : 0.0;
            for (int j = 0; j < kb; ++j) {
              double sum = 0.0;
              for (int t = 0; t < NB; ++t) sum += Li[j][t] * x[t];
              F[at[j]] = sum;
            }
          } else {
            const int c = (local - rows_chunks) * PR + slot;
            if (c >= k1) continue;
            for (int t = 0; t < kb; ++t) at[t] = pidx(f, k0 + t, c);
            for (int t = 0; t < NB; ++t) x[t] = t < kb ? P[at[t]] : 0.0;
            for (int j = 0; j < kb; ++j) {
              double sum = 0.0;
              for (int t = 0; t < NB; ++t) sum += Li[j][t] * x[t];
              P[at[j]] = sum;
            }
          }
        }
      } else {
        CHECK(op.kind == kFactorUpdate);
        const int kb = std::min(NB, f.nc - op.k0), k0 = op.k0, k1 = k0 + kb, m = f.ld - k1;
        CHECK(kb > 0 && m > 0);
        const int T = (m + TT - 1) / TT, nsy = T * (T + 1) / 2, tc = (k1 + TT - 1) / TT;
        CHECK(local < nsy + T * tc);
        const bool syrk = local < nsy;
        int ti, tj;
        if (syrk) {
          ti = (int)((std::sqrt(8.0 * local + 1.0) - 1.0) * 0.5);
          while ((ti + 1) * (ti + 2) / 2 <= local) ++ti;
          while (ti * (ti + 1) / 2 > local) --ti;
          tj = local - ti * (ti + 1) / 2;
          CHECK(tj >= 0 && tj <= ti && ti < T);
        } else {
          ti = (local - nsy) / tc;
          tj = (local - nsy) % tc;
          CHECK(ti < T && tj < tc);
        }
        for (int p = 0; p < TT; ++p)
          for (int q = 0; q < TT; ++q) {
            const int gp = ti * TT + p, gq = tj * TT + q;
            if (gp >= m) continue;
            if (syrk ? (gq > gp) : (gq >= k1)) continue;
            double acc = 0.0;
            for (int t = 0; t < kb; ++t) {
              const double xv = F[fidx(f, k1 + gp, k0 + t)];
              const double yv = syrk ? F[fidx(f, k1 + gq, k0 + t)] : P[pidx(f, k0 + t, gq)];
              acc += xv * yv;
            }
            if (syrk) F[fidx(f, k1 + gp, k1 + gq)] -= acc;
            else P[pidx(f, k1 + gp, gq)] -= acc;
          }
      }
    }
  }
  // row-major copy: the transpose launch's table and indices
  {
    const FactorOp& op = FP.transpose;
    CHECK(op.kind == kFactorTranspose && op.n == ns);
    CHECK((size_t)op.list_off + 2 * op.n + 1 + op.blocks <= FP.ints.size());
    const int32_t* items = &FP.ints[op.list_off];
    const int32_t* pre = items + op.n;
    std::vector<double> T(S.panel_size, -1.0);
    for (int b = 0; b < op.blocks; ++b) {
      const int it = items[2 * op.n + 1 + b];
      CHECK(it == find_item_h(pre, op.n, b));
      const FrontDesc f = FP.fronts[items[it]];
      const int64_t total = (int64_t)f.ld * f.nc;
      for (int tid = 0; tid < TH; ++tid)
        for (int k = 0; k < 4; ++k) {
          const int64_t e = (int64_t)(b - pre[it]) * kFactorTransposeChunk + tid + k * TH;
          const int64_t ec = std::min(e, total - 1);
          const int64_t r = ec / f.nc, c = ec - r * f.nc;
          const int64_t src = f.panel_off + c * f.ld + r;
          CHECK(src >= 0 && src < S.panel_size);
          if (e < total) {
            CHECK(f.panel_off + e < S.panel_size);
            T[f.panel_off + e] = P[src];
          }
        }
    }
    const std::vector<double> ref = transpose_panels<double>(S, P);
    for (int64_t i = 0; i < S.panel_size; ++i) CHECK(T[i] == ref[i]);
  }
  return P;
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t nc, nfx, nrhs;
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
  HostMesh m;
  std::string err = build_mesh(cells.data(), nc, youngs.data(), fixed.data(), nfx, o, m);
  if (!err.empty()) {
    std::fprintf(stderr, "build_mesh: %s\n", err.c_str());
    return 4;
  }
  const int64_t N = m.n_nodes, nf = m.n_free;
  rd(in, &nrhs, 1);
  std::vector<double> B(nrhs * 3 * N);
  rd(in, B.data(), B.size());
  std::fclose(in);

  Csr A;
  assemble_As(m, o, A);
  Symbolic S;
  analyse(m, A, leaf_max, sep_max, S);
  LevelPlan P;
  build_plan(S, P);
  std::vector<double> panel;
  if (!factor_panels(S, A, panel, err)) {
    std::fprintf(stderr, "factor: %s\n", err.c_str());
    return 5;
  }
  CHECK((int64_t)panel.size() == S.panel_size);
  {
    // the device factorization's plan and arithmetic, replayed: the same panels
    // to rounding; the sweeps below then run on the replayed panels
    FactorPlan FP;
    const std::string perr = build_factor_plan(S, A, FP);
    if (!perr.empty()) {
      std::fprintf(stderr, "factor plan: %s\n", perr.c_str());
      return 6;
    }
    const std::vector<double> dev = replay_device_factor(S, A, FP);
    double dmax = 0.0, pmax = 0.0;
    for (int64_t i = 0; i < S.panel_size; ++i) {
      dmax = std::max(dmax, std::abs(dev[i] - panel[i]));
      pmax = std::max(pmax, std::abs(panel[i]));
    }
    if (std::getenv("HOST_CHECK_LEVELS")) std::fprintf(stderr, "device-factor replay: max |diff| %.3e of %.3e\n", dmax, pmax);
    CHECK(dmax <= 1e-11 * pmax);
    panel = dev;
  }
  // structural checks of the plan
  for (const SweepTask& t : P.fwd) {
    CHECK(t.sn >= 0 && t.sn < (int32_t)S.sn.size());
    const Supernode& sn = S.sn[t.sn];
    CHECK(t.first >= 0 && t.count > 0 && t.count <= kBlock && t.first + t.count <= sn.ncols + sn.nrows);
  }
  for (int32_t l = 0; l < S.n_levels; ++l)
    for (int32_t ti = P.bwd_off[l]; ti < P.bwd_off[l + 1]; ++ti) {
      const SweepTask& t = P.bwd[ti];
      const Supernode& sn = S.sn[t.sn];
      CHECK(sn.level == l);
      CHECK(t.first >= 0 && t.count > 0 && t.first + t.count <= sn.ncols);
      CHECK(P.bwd_narrow[l] ? t.count <= 64 : t.count <= kColsPerTask);
    }
  CHECK((int32_t)P.gather_off.size() == S.n_levels + 1);
  for (int32_t l = 0; l < S.n_levels; ++l)
    for (int32_t g = P.gather_off[l]; g < P.gather_off[l + 1]; ++g) {
      const int32_t j = P.gather_cols[g];
      CHECK(j >= 0 && j < nf && S.sn[S.snode_of[j]].level == l && P.fwd_wide[l]);
      CHECK(S.cptr[j] <= S.cptr[j + 1] && S.cptr[j + 1] <= (int32_t)S.cidx.size());
    }
  std::vector<int32_t> perm_pub(nf);
  for (int64_t i = 0; i < nf; ++i) perm_pub[i] = m.free_nodes[S.perm[i]];
  const std::vector<double> panelT = transpose_panels<double>(S, panel);

  std::vector<double> X((size_t)nrhs * 3 * N, 0.0);
  for (int64_t rhs = 0; rhs < nrhs; ++rhs) {
    const double* b = &B[rhs * 3 * N];
    double* out = &X[rhs * 3 * N];
    std::vector<double> y_int(3 * nf, 0.0), x_int(3 * nf, 0.0), U(3 * S.u_size, 0.0);
    // forward levels (k_sweep_fwd)
    for (int32_t l = 0; l < S.n_levels; ++l)
      for (int32_t ti = P.fwd_off[l]; ti < P.fwd_off[l + 1]; ++ti) {
        const SweepTask t = P.fwd[ti];
        const Supernode& sn = S.sn[t.sn];
        const int nc_ = sn.ncols, ld = sn.ncols + sn.nrows;
        CHECK(nc_ <= P.fwd_cols[l]);
        std::vector<double> bs(3 * P.fwd_cols[l]);
        for (int c = 0; c < nc_; ++c) {
          const int j = sn.col0 + c;
          CHECK(j >= 0 && j < nf);
          const int node = perm_pub[j];
          CHECK(node >= 0 && node < N);
          double v[3] = {b[node], b[N + node], b[2 * N + node]};
          for (int k = S.cptr[j]; k < S.cptr[j + 1]; ++k) {
            const int64_t pos = 3 * (int64_t)S.cidx[k];
            CHECK(pos >= 0 && pos + 2 < (int64_t)U.size());
            for (int q = 0; q < 3; ++q) v[q] += U[pos + q];
          }
          for (int q = 0; q < 3; ++q) bs[q * nc_ + c] = v[q];
        }
        for (int tid = 0; tid < t.count; ++tid) {
          const int r = t.first + tid;
          const int cend = r < nc_ ? r + 1 : nc_;
          double a[3] = {0, 0, 0};
          for (int c = 0; c < cend; ++c) {
            // narrow kernel reads the column-major panel, wide kernel the row-major copy
            const int64_t pi = P.fwd_wide[l] ? sn.panel_off + (int64_t)r * nc_ + c
                                             : sn.panel_off + r + (int64_t)c * ld;
            CHECK(pi >= 0 && pi < S.panel_size);
            const double pv = P.fwd_wide[l] ? panelT[pi] : panel[pi];
            for (int q = 0; q < 3; ++q) a[q] += pv * bs[q * nc_ + c];
          }
          if (r < nc_) {
            for (int q = 0; q < 3; ++q) y_int[q * nf + sn.col0 + r] = a[q];
          } else {
            const int64_t pos = 3 * (sn.u_off + (r - nc_));
            CHECK(pos >= 0 && pos + 2 < (int64_t)U.size());
            for (int q = 0; q < 3; ++q) U[pos + q] = a[q];
          }
        }
      }
    // backward levels (k_sweep_bwd)
    for (int32_t l = S.n_levels - 1; l >= 0; --l)
      for (int32_t ti = P.bwd_off[l]; ti < P.bwd_off[l + 1]; ++ti) {
        const SweepTask t = P.bwd[ti];
        const Supernode& sn = S.sn[t.sn];
        const int nc_ = sn.ncols, ld = sn.ncols + sn.nrows;
        CHECK(ld <= P.bwd_rows[l]);
        CHECK(P.bwd_narrow[l] ? (t.first == 0 && t.count == nc_ && nc_ <= 64 && ld <= 2048)
                              : t.count <= kColsPerTask);
        for (int cc = 0; cc < t.count; ++cc) {
          const int c = t.first + cc;
          const int cw = c;   // first row read: the column's own row (zeros above it are skipped)
          double a[3] = {0, 0, 0};
          for (int r = cw; r < ld; ++r) {
            const int64_t pi = P.bwd_narrow[l] ? sn.panel_off + (int64_t)r * nc_ + c
                                               : sn.panel_off + (int64_t)c * ld + r;
            CHECK(pi >= 0 && pi < S.panel_size);
            int j;
            const double* src;
            if (r < nc_) {
              j = sn.col0 + r;
              src = y_int.data();
            } else {
              CHECK(sn.rows_off + (r - nc_) < (int64_t)S.rows.size());
              j = S.rows[sn.rows_off + (r - nc_)];
              src = x_int.data();
            }
            CHECK(j >= 0 && j < nf);
            const double pv = P.bwd_narrow[l] ? panelT[pi] : panel[pi];
            for (int q = 0; q < 3; ++q) a[q] += pv * src[q * nf + j];
          }
          const int j = sn.col0 + c;
          for (int q = 0; q < 3; ++q) x_int[q * nf + j] = a[q];
          const int node = perm_pub[j];
          for (int q = 0; q < 3; ++q) out[q * N + node] = a[q];
        }
      }
  }

  if (std::getenv("HOST_CHECK_LEVELS")) {
    for (int32_t l = 0; l < S.n_levels; ++l) {
      int nsn = 0, maxld = 0, maxnc = 0;
      for (auto& sn : S.sn)
        if (sn.level == l) {
          nsn++;
          maxld = std::max(maxld, sn.ncols + sn.nrows);
          maxnc = std::max(maxnc, sn.ncols);
        }
      std::fprintf(stderr, "level %2d supernodes %5d fwd_tasks %6d bwd_tasks %6d max_nc %5d max_ld %5d fwd_MB %8.2f\n",
                   l, nsn, P.fwd_off[l + 1] - P.fwd_off[l], P.bwd_off[l + 1] - P.bwd_off[l], maxnc, maxld,
                   P.fwd_bytes[l] / 1e6);
    }
  }
  FILE* f = std::fopen(argv[2], "wb");
  int64_t hdr[8] = {N, nf, (int64_t)A.col.size(), (int64_t)S.sn.size(), S.n_levels, S.packed_nnz,
                    (int64_t)P.fwd.size(), (int64_t)P.bwd.size()};
  wr(f, hdr, 8);
  wr(f, m.node_ijk.data(), m.node_ijk.size());
  wr(f, m.mass.data(), m.mass.size());
  wr(f, m.free_nodes.data(), m.free_nodes.size());
  wr(f, A.ptr.data(), A.ptr.size());
  wr(f, A.col.data(), A.col.size());
  wr(f, A.val.data(), A.val.size());
  wr(f, X.data(), X.size());
  std::fclose(f);
  return 0;
}
