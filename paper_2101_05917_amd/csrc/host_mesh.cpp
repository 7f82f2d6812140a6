// Voxel ingestion, node numbering and assembly of the scalar node matrix.
//
// Discretization (paper Sec. Background and supplemental Sec. Energy
// Definitions): trilinear cubic voxels, energies integrated at the 2x2x2
// Gauss points, lumped mass.  Every term of A = M/h^2 + sum_c w_c G_c^T G_c
// (eq:pd_global) with the energies used here acts identically on the x, y
// and z coordinates, so A = I_3 (x) A_s with A_s an N x N scalar matrix:
//   A_s = diag(m)/h^2 + sum_q w_q B_q^T B_q + sum_q w_m b_q b_q^T + k [contact]
// with B_q the 3x8 shape-gradient matrix and b_q = B_q^T m (fibre).
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "internal.hpp"

namespace dpd {

void reference_gradients(double Bxi[8][3][8]) {
  const double g = 1.0 / std::sqrt(3.0);
  for (int q = 0; q < 8; ++q) {
    double xi[3];
    for (int k = 0; k < 3; ++k) xi[k] = ((q >> k) & 1) ? g : -g;
    for (int a = 0; a < 8; ++a) {
      double s[3];
      for (int k = 0; k < 3; ++k) s[k] = ((a >> k) & 1) ? 1.0 : -1.0;
      for (int j = 0; j < 3; ++j) {
        double v = 0.125 * s[j];
        for (int k = 0; k < 3; ++k)
          if (k != j) v *= 1.0 + s[k] * xi[k];
        Bxi[q][j][a] = v;
      }
    }
  }
}

static inline int64_t key3(int64_t i, int64_t j, int64_t k) {
  return ((k + (1 << 20)) << 42) | ((j + (1 << 20)) << 21) | (i + (1 << 20));
}

std::string build_mesh(const int32_t* cells, int64_t n_cells, const double* youngs,
                       const int32_t* fixed_ijk, int64_t n_fixed, const dpd_options& o,
                       HostMesh& m) {
  if (n_cells <= 0 || !cells || !youngs) return "no cells";
  if (!(o.dx > 0) || !(o.rho > 0) || !(o.h > 0)) return "dx, rho and h must be positive";
  if (!(o.nu >= 0.0 && o.nu < 0.5)) return "nu must lie in [0, 0.5)";
  if (o.contact_k < 0 || o.muscle_k < 0 || o.friction_mu < 0) return "negative contact/muscle/friction";
  if (!(o.volume_scale >= 0.0) || !std::isfinite(o.volume_scale)) return "volume_scale must be >= 0";
  for (int64_t e = 0; e < n_cells; ++e)
    if (!(youngs[e] > 0) || !std::isfinite(youngs[e])) return "Young's moduli must be positive";
  for (int64_t e = 0; e < 3 * n_cells; ++e)
    if (cells[e] < -(1 << 19) || cells[e] >= (1 << 19)) return "voxel index out of range";

  // unique corners, sorted lexicographically with i fastest
  std::vector<int64_t> keys;
  keys.reserve(8 * n_cells);
  {
    std::vector<int64_t> ck(n_cells);
    for (int64_t e = 0; e < n_cells; ++e) ck[e] = key3(cells[3 * e], cells[3 * e + 1], cells[3 * e + 2]);
    std::sort(ck.begin(), ck.end());
    if (std::adjacent_find(ck.begin(), ck.end()) != ck.end()) return "duplicate voxels";
  }
  for (int64_t e = 0; e < n_cells; ++e)
    for (int a = 0; a < 8; ++a)
      keys.push_back(key3(cells[3 * e] + (a & 1), cells[3 * e + 1] + ((a >> 1) & 1),
                          cells[3 * e + 2] + ((a >> 2) & 1)));
  std::vector<int64_t> nodes = keys;
  std::sort(nodes.begin(), nodes.end());
  nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
  const int64_t N = (int64_t)nodes.size(), E = n_cells;
  m.n_nodes = N;
  m.n_elems = E;
  m.node_ijk.resize(3 * N);
  for (int64_t n = 0; n < N; ++n) {
    int64_t k = nodes[n];
    m.node_ijk[3 * n + 0] = (int32_t)((k & ((1LL << 21) - 1)) - (1 << 20));
    m.node_ijk[3 * n + 1] = (int32_t)(((k >> 21) & ((1LL << 21) - 1)) - (1 << 20));
    m.node_ijk[3 * n + 2] = (int32_t)((k >> 42) - (1 << 20));
  }
  for (int c = 0; c < 3; ++c) {
    m.grid_min[c] = m.node_ijk[c];
    m.grid_max[c] = m.node_ijk[c];
  }
  for (int64_t n = 0; n < N; ++n)
    for (int c = 0; c < 3; ++c) {
      m.grid_min[c] = std::min(m.grid_min[c], m.node_ijk[3 * n + c]);
      m.grid_max[c] = std::max(m.grid_max[c], m.node_ijk[3 * n + c]);
    }
  m.conn.resize(8 * E);
  for (int64_t t = 0; t < 8 * E; ++t)
    m.conn[t] = (int32_t)(std::lower_bound(nodes.begin(), nodes.end(), keys[t]) - nodes.begin());

  m.youngs.assign(youngs, youngs + E);
  m.mass.assign(N, 0.0);
  const double share = o.rho * o.dx * o.dx * o.dx / 8.0;
  for (int64_t t = 0; t < 8 * E; ++t) m.mass[m.conn[t]] += share;

  m.X.resize(3 * N);
  for (int64_t n = 0; n < N; ++n)
    for (int c = 0; c < 3; ++c) m.X[c * N + n] = o.origin[c] + o.dx * m.node_ijk[3 * n + c];

  m.fixed.assign(N, 0);
  for (int64_t f = 0; f < n_fixed; ++f) {
    int64_t k = key3(fixed_ijk[3 * f], fixed_ijk[3 * f + 1], fixed_ijk[3 * f + 2]);
    auto it = std::lower_bound(nodes.begin(), nodes.end(), k);
    if (it == nodes.end() || *it != k) return "fixed node is not a mesh node";
    m.fixed[it - nodes.begin()] = 1;
  }
  m.free_index.assign(N, -1);
  m.free_nodes.clear();
  for (int64_t n = 0; n < N; ++n)
    if (!m.fixed[n]) {
      m.free_index[n] = (int32_t)m.free_nodes.size();
      m.free_nodes.push_back((int32_t)n);
    }
  m.n_free = (int64_t)m.free_nodes.size();
  if (m.n_free == 0) return "every node is fixed";

  m.is_contact.assign(N, 0);
  m.contact.clear();
  if (o.contact_k > 0) {
    for (int64_t n = 0; n < N; ++n)
      if (m.node_ijk[3 * n + 2] == m.grid_min[2]) {
        m.is_contact[n] = 1;
        m.contact.push_back((int32_t)n);
      }
  }
  m.node_inc.assign(8 * N, -1);
  std::vector<int> cnt(N, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < 8; ++a) {
      int32_t n = m.conn[8 * e + a];
      m.node_inc[(int64_t)cnt[n] * N + n] = (int32_t)(8 * e + a);
      cnt[n]++;
    }
  return "";
}

void assemble_As(const HostMesh& m, const dpd_options& o, Csr& A) {
  double Bxi[8][3][8];
  reference_gradients(Bxi);
  const double dx = o.dx, Vq = dx * dx * dx / 8.0, s = 2.0 / dx;
  // K0[a][b] = V_q sum_q sum_j dN_a/dX_j dN_b/dX_j ; Km[a][b] = V_q sum_q (gradN_a.m)(gradN_b.m)
  double K0[8][8] = {}, Km[8][8] = {};
  for (int q = 0; q < 8; ++q)
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b) {
        double acc = 0, ma = 0, mb = 0;
        for (int j = 0; j < 3; ++j) {
          acc += Bxi[q][j][a] * Bxi[q][j][b] * s * s;
          ma += Bxi[q][j][a] * s * o.fiber[j];
          mb += Bxi[q][j][b] * s * o.fiber[j];
        }
        K0[a][b] += Vq * acc;
        Km[a][b] += Vq * ma * mb;
      }
  const int64_t nf = m.n_free;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(nf);
  for (int64_t e = 0; e < m.n_elems; ++e) {
    const double mu = m.youngs[e] / (2.0 * (1.0 + o.nu));
    // w_q = 2 mu V_q (+ the volume term's volume_scale lambda V_q), V_q folded into K0
    const double lam = m.youngs[e] * o.nu / ((1.0 + o.nu) * (1.0 - 2.0 * o.nu));
    const double w = 2.0 * mu + o.volume_scale * lam;
    for (int a = 0; a < 8; ++a) {
      int32_t ia = m.free_index[m.conn[8 * e + a]];
      if (ia < 0) continue;
      for (int b = 0; b < 8; ++b) {
        int32_t ib = m.free_index[m.conn[8 * e + b]];
        if (ib < 0) continue;
        double v = w * K0[a][b] + o.muscle_k * Km[a][b];
        rows[ia].push_back({ib, v});
      }
    }
  }
  A.n = (int32_t)nf;
  A.ptr.assign(nf + 1, 0);
  A.col.clear();
  A.val.clear();
  const double h2 = o.h * o.h;
  for (int64_t i = 0; i < nf; ++i) {
    int32_t node = m.free_nodes[i];
    double diag = m.mass[node] / h2 + (m.is_contact[node] ? o.contact_k : 0.0);
    rows[i].push_back({(int32_t)i, diag});
    auto& r = rows[i];
    std::stable_sort(r.begin(), r.end(), [](auto& x, auto& y) { return x.first < y.first; });
    size_t k = 0;
    while (k < r.size()) {
      int32_t c = r[k].first;
      double v = 0;
      while (k < r.size() && r[k].first == c) v += r[k++].second;
      A.col.push_back(c);
      A.val.push_back(v);
    }
    A.ptr[i + 1] = (int64_t)A.col.size();
    std::vector<std::pair<int32_t, double>>().swap(r);
  }
}

}  // namespace dpd
