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
