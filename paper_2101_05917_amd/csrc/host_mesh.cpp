// Voxel and tetrahedral mesh ingestion, node numbering and assembly of the
// scalar node matrix.
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

// Linear tetrahedra (the voxel reading with one integration point per element
// of weight V_e): F = D_s D_m^{-1}, lumped mass rho V_e / 4 per corner, the
// ground penalty on the nodes of minimal rest height.
std::string build_tet_mesh(const double* X, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                           const double* youngs, const int32_t* fixed_nodes, int64_t n_fixed, const dpd_options& o,
                           HostMesh& m) {
  if (n_nodes <= 0 || n_tets <= 0 || !X || !tets || !youngs) return "no nodes or tetrahedra";
  if (n_nodes >= (1LL << 31) || 4 * n_tets >= (1LL << 31)) return "mesh too large";
  if (!(o.rho > 0) || !(o.h > 0)) return "rho and h must be positive";
  if (!(o.nu >= 0.0 && o.nu < 0.5)) return "nu must lie in [0, 0.5)";
  if (o.contact_k < 0 || o.friction_mu < 0) return "negative contact/friction";
  if (o.muscle_k != 0.0 || o.volume_scale != 0.0) return "tetrahedral meshes take the corotated term only";
  const int64_t N = n_nodes, E = n_tets;
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!std::isfinite(X[i])) return "non-finite node position";
  for (int64_t e = 0; e < E; ++e)
    if (!(youngs[e] > 0) || !std::isfinite(youngs[e])) return "Young's moduli must be positive";
  for (int64_t t = 0; t < 4 * E; ++t)
    if (tets[t] < 0 || tets[t] >= N) return "tetrahedron corner out of range";
  m.corners = 4;
  m.n_nodes = N;
  m.n_elems = E;
  m.node_ijk.clear();
  m.node_inc.clear();
  m.conn.assign(tets, tets + 4 * E);
  m.youngs.assign(youngs, youngs + E);
  m.X.resize(3 * N);
  for (int64_t n = 0; n < N; ++n)
    for (int c = 0; c < 3; ++c) m.X[c * N + n] = X[3 * n + c];
  m.dminv.resize(9 * E);
  m.vol.resize(E);
  m.mass.assign(N, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t* t = tets + 4 * e;
    double D[9];   // columns: edges X_k - X_0
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) D[3 * i + k] = X[3 * (int64_t)t[k + 1] + i] - X[3 * (int64_t)t[0] + i];
    const double c00 = D[4] * D[8] - D[5] * D[7], c01 = D[5] * D[6] - D[3] * D[8], c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    double scale = 0.0;
    for (double v : D) scale = std::max(scale, std::fabs(v));
    if (!(std::fabs(det) > 1e-12 * scale * scale * scale)) return "degenerate tetrahedron";
    const double id = 1.0 / det;
    double* Di = &m.dminv[9 * e];   // inverse by cofactors, row-major
    Di[0] = c00 * id;
    Di[1] = (D[2] * D[7] - D[1] * D[8]) * id;
    Di[2] = (D[1] * D[5] - D[2] * D[4]) * id;
    Di[3] = c01 * id;
    Di[4] = (D[0] * D[8] - D[2] * D[6]) * id;
    Di[5] = (D[2] * D[3] - D[0] * D[5]) * id;
    Di[6] = c02 * id;
    Di[7] = (D[1] * D[6] - D[0] * D[7]) * id;
    Di[8] = (D[0] * D[4] - D[1] * D[3]) * id;
    m.vol[e] = std::fabs(det) / 6.0;
    for (int a = 0; a < 4; ++a) m.mass[t[a]] += o.rho * m.vol[e] / 4.0;
  }
  for (int64_t n = 0; n < N; ++n)
    if (!(m.mass[n] > 0.0)) return "a node belongs to no tetrahedron";
  m.fixed.assign(N, 0);
  for (int64_t f = 0; f < n_fixed; ++f) {
    if (fixed_nodes[f] < 0 || fixed_nodes[f] >= N) return "fixed node out of range";
    m.fixed[fixed_nodes[f]] = 1;
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
    double zmin = m.X[2 * N], zmax = m.X[2 * N];
    for (int64_t n = 0; n < N; ++n) {
      zmin = std::min(zmin, m.X[2 * N + n]);
      zmax = std::max(zmax, m.X[2 * N + n]);
    }
    const double tol = 1e-12 * std::max(1.0, std::max(std::fabs(zmin), std::fabs(zmax)));
    for (int64_t n = 0; n < N; ++n)
      if (m.X[2 * N + n] <= zmin + tol) {
        m.is_contact[n] = 1;
        m.contact.push_back((int32_t)n);
      }
  }
  m.inc_ptr.assign(N + 1, 0);
  for (int64_t t = 0; t < 4 * E; ++t) m.inc_ptr[tets[t] + 1]++;
  for (int64_t n = 0; n < N; ++n) m.inc_ptr[n + 1] += m.inc_ptr[n];
  m.inc.assign(4 * E, 0);
  std::vector<int32_t> fill(m.inc_ptr.begin(), m.inc_ptr.end() - 1);
  for (int64_t t = 0; t < 4 * E; ++t) m.inc[fill[tets[t]]++] = (int32_t)t;   // t = 4e + a, ascending
  return "";
}

// A_s of linear tetrahedra: diag(m)/h^2 + sum_e 2 mu_e V_e B_e B_e^T + k [contact],
// B_e the 4 x 3 matrix of shape gradients (rows: -sum of D_m^{-1}'s rows, then its rows).
static void assemble_As_tet(const HostMesh& m, const dpd_options& o, Csr& A) {
  const int64_t nf = m.n_free;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(nf);
  for (int64_t e = 0; e < m.n_elems; ++e) {
    const double* Di = &m.dminv[9 * e];
    double B[4][3];
    for (int j = 0; j < 3; ++j) {
      B[0][j] = -(Di[j] + Di[3 + j] + Di[6 + j]);
      for (int k = 0; k < 3; ++k) B[k + 1][j] = Di[3 * k + j];
    }
    const double w = 2.0 * m.youngs[e] / (2.0 * (1.0 + o.nu)) * m.vol[e];
    for (int a = 0; a < 4; ++a) {
      const int32_t ia = m.free_index[m.conn[4 * e + a]];
      if (ia < 0) continue;
      for (int b = 0; b < 4; ++b) {
        const int32_t ib = m.free_index[m.conn[4 * e + b]];
        if (ib < 0) continue;
        rows[ia].push_back({ib, w * (B[a][0] * B[b][0] + B[a][1] * B[b][1] + B[a][2] * B[b][2])});
      }
    }
  }
  A.n = (int32_t)nf;
  A.ptr.assign(nf + 1, 0);
  A.col.clear();
  A.val.clear();
  const double h2 = o.h * o.h;
  for (int64_t i = 0; i < nf; ++i) {
    const int32_t node = m.free_nodes[i];
    rows[i].push_back({(int32_t)i, m.mass[node] / h2 + (m.is_contact[node] ? o.contact_k : 0.0)});
    auto& r = rows[i];
    std::stable_sort(r.begin(), r.end(), [](auto& x, auto& y) { return x.first < y.first; });
    size_t k = 0;
    while (k < r.size()) {
      const int32_t c = r[k].first;
      double v = 0;
      while (k < r.size() && r[k].first == c) v += r[k++].second;
      A.col.push_back(c);
      A.val.push_back(v);
    }
    A.ptr[i + 1] = (int64_t)A.col.size();
    std::vector<std::pair<int32_t, double>>().swap(r);
  }
}

void assemble_As(const HostMesh& m, const dpd_options& o, Csr& A) {
  if (m.corners == 4) return assemble_As_tet(m, o, A);
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
