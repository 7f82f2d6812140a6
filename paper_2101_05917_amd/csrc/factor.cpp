// Ordering, symbolic analysis and numeric factorization of the scalar node
// matrix A_s, and construction of the panels the GPU triangular sweeps read.
//
// The paper factorizes the constant matrix A once and back-substitutes in
// every global step of the forward (Alg. 1) and backward (Alg. 2) iterations
// (Sec. Background, Projective Dynamics; Sec. Differentiable Projective
// Dynamics).  Here:
//   * nested dissection on the voxel grid (a grid plane separates the two
//     halves because hex neighbours differ by at most one in each index), or,
//     on tetrahedral meshes, by median splits of the rest positions with the
//     lower half's boundary nodes as separators;
//   * one supernode per dissection leaf and per separator (split into chunks
//     of at most sep_max columns), ordered children before parents;
//   * multifrontal Cholesky with dense fronts;
//   * per supernode s the panel [inv(L_ss); -L_Rs inv(L_ss)], so that both
//     sweeps become dense matrix-vector products with no intra-block
//     dependency chain:
//        forward   y_s = inv(L_ss) b~_s,   b_R -= (L_Rs inv(L_ss)) b~_s
//        backward  x_s = inv(L_ss)^T y_s - (L_Rs inv(L_ss))^T x_R
//     where b~_s is b_s minus the updates of s's descendants.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include <omp.h>

#include "internal.hpp"

namespace dpd {

namespace {

struct NdCtx {
  const HostMesh* m;
  const Csr* A;                              // adjacency of the free nodes (tetrahedra)
  int32_t leaf_max, sep_max;
  std::vector<std::vector<int32_t>> groups;  // emitted supernode node lists (free indices)
  std::vector<int8_t> side;                  // bisection side of each free node, -1 outside
};

void sort_lex(const HostMesh& m, std::vector<int32_t>& v) {
  if (m.node_ijk.empty()) {   // tetrahedra: by rest position (z, y, x), then id
    const int64_t N = m.n_nodes;
    std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
      const int64_t na = m.free_nodes[a], nb = m.free_nodes[b];
      for (int c = 2; c >= 0; --c)
        if (m.X[c * N + na] != m.X[c * N + nb]) return m.X[c * N + na] < m.X[c * N + nb];
      return a < b;
    });
    return;
  }
  std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) {
    const int32_t* pa = &m.node_ijk[3 * (int64_t)m.free_nodes[a]];
    const int32_t* pb = &m.node_ijk[3 * (int64_t)m.free_nodes[b]];
    if (pa[2] != pb[2]) return pa[2] < pb[2];
    if (pa[1] != pb[1]) return pa[1] < pb[1];
    return pa[0] < pb[0];
  });
}

void emit(NdCtx& c, std::vector<int32_t>& nodes, int32_t chunk) {
  sort_lex(*c.m, nodes);
  const int64_t n = (int64_t)nodes.size();
  const int64_t pieces = (n + chunk - 1) / chunk;
  for (int64_t p = 0; p < pieces; ++p) {
    int64_t b = n * p / pieces, e = n * (p + 1) / pieces;
    c.groups.emplace_back(nodes.begin() + b, nodes.begin() + e);
  }
}

void nd(NdCtx& c, std::vector<int32_t>& nodes) {
  if (nodes.empty()) return;
  const HostMesh& m = *c.m;
  if ((int64_t)nodes.size() <= c.leaf_max) {
    emit(c, nodes, c.sep_max);
    return;
  }
  int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (int32_t f : nodes) {
    const int32_t* p = &m.node_ijk[3 * (int64_t)m.free_nodes[f]];
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
  if (hi[ax] - lo[ax] < 2) {
    emit(c, nodes, c.sep_max);
    return;
  }
  const int32_t mid = lo[ax] + (hi[ax] - lo[ax]) / 2;
  std::vector<int32_t> left, right, sep;
  for (int32_t f : nodes) {
    int32_t v = m.node_ijk[3 * (int64_t)m.free_nodes[f] + ax];
    (v < mid ? left : (v > mid ? right : sep)).push_back(f);
  }
  std::vector<int32_t>().swap(nodes);
  nd(c, left);
  nd(c, right);
  if (!sep.empty()) emit(c, sep, c.sep_max);
}

// Nested dissection of an unstructured mesh (tetrahedra): split the nodes at
// the median of their rest positions along the longest extent; the nodes of
// the lower half with a neighbour (an off-diagonal entry of A_s) in the upper
// half form the separator, which leaves the two remaining parts unconnected.
void nd_graph(NdCtx& c, std::vector<int32_t>& nodes) {
  if (nodes.empty()) return;
  const HostMesh& m = *c.m;
  if ((int64_t)nodes.size() <= c.leaf_max) {
    emit(c, nodes, c.sep_max);
    return;
  }
  const int64_t N = m.n_nodes;
  double lo[3], hi[3];
  for (int k = 0; k < 3; ++k) lo[k] = hi[k] = m.X[k * N + m.free_nodes[nodes[0]]];
  for (int32_t f : nodes)
    for (int k = 0; k < 3; ++k) {
      const double v = m.X[k * N + m.free_nodes[f]];
      lo[k] = std::min(lo[k], v);
      hi[k] = std::max(hi[k], v);
    }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
  const size_t half = nodes.size() / 2;
  std::nth_element(nodes.begin(), nodes.begin() + half, nodes.end(), [&](int32_t a, int32_t b) {
    const double va = m.X[ax * N + m.free_nodes[a]], vb = m.X[ax * N + m.free_nodes[b]];
    return va != vb ? va < vb : a < b;
  });
  for (size_t i = 0; i < nodes.size(); ++i) c.side[nodes[i]] = i < half ? 0 : 1;
  std::vector<int32_t> left, right, sep;
  const Csr& A = *c.A;
  for (size_t i = 0; i < nodes.size(); ++i) {
    const int32_t f = nodes[i];
    if (i >= half) {
      right.push_back(f);
      continue;
    }
    bool cut = false;
    for (int64_t k = A.ptr[f]; k < A.ptr[f + 1] && !cut; ++k) cut = c.side[A.col[k]] == 1;
    (cut ? sep : left).push_back(f);
  }
  for (int32_t f : nodes) c.side[f] = -1;
  std::vector<int32_t>().swap(nodes);
  nd_graph(c, left);
  nd_graph(c, right);
  if (!sep.empty()) emit(c, sep, c.sep_max);
}

}  // namespace

void analyse(const HostMesh& m, const Csr& A, int32_t leaf_max, int32_t sep_max, Symbolic& S) {
  const int32_t n = A.n;
  NdCtx c{&m, &A, leaf_max, sep_max, {}, {}};
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  if (m.corners == 4) {
    c.side.assign(n, -1);
    nd_graph(c, all);
  } else {
    nd(c, all);
  }

  S.n = n;
  S.perm.clear();
  S.perm.reserve(n);
  S.sn.clear();
  for (auto& g : c.groups) {
    Supernode s;
    s.col0 = (int32_t)S.perm.size();
    s.ncols = (int32_t)g.size();
    S.sn.push_back(s);
    S.perm.insert(S.perm.end(), g.begin(), g.end());
  }
  S.iperm.assign(n, -1);
  for (int32_t i = 0; i < n; ++i) S.iperm[S.perm[i]] = i;
  const int32_t ns = (int32_t)S.sn.size();
  S.snode_of.assign(n, -1);
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t j = 0; j < S.sn[s].ncols; ++j) S.snode_of[S.sn[s].col0 + j] = s;

  S.children.assign(ns, {});
  S.rows.clear();
  std::vector<int32_t> mark(n, -1), buf;
  int64_t panel = 0, u = 0, packed = 0;
  S.n_levels = 0;
  for (int32_t s = 0; s < ns; ++s) {
    Supernode& sn = S.sn[s];
    const int32_t end = sn.col0 + sn.ncols;
    buf.clear();
    for (int32_t j = sn.col0; j < end; ++j) {
      const int32_t f = S.perm[j];
      for (int64_t k = A.ptr[f]; k < A.ptr[f + 1]; ++k) {
        const int32_t i = S.iperm[A.col[k]];
        if (i >= end && mark[i] != s) {
          mark[i] = s;
          buf.push_back(i);
        }
      }
    }
    int32_t lvl = 0;
    for (int32_t ch : S.children[s]) {
      const Supernode& cs = S.sn[ch];
      lvl = std::max(lvl, cs.level + 1);
      for (int32_t p = 0; p < cs.nrows; ++p) {
        const int32_t i = S.rows[cs.rows_off + p];
        if (i >= end && mark[i] != s) {
          mark[i] = s;
          buf.push_back(i);
        }
      }
    }
    std::sort(buf.begin(), buf.end());
    sn.level = lvl;
    S.n_levels = std::max(S.n_levels, lvl + 1);
    sn.nrows = (int32_t)buf.size();
    sn.rows_off = (int64_t)S.rows.size();
    S.rows.insert(S.rows.end(), buf.begin(), buf.end());
    sn.parent = buf.empty() ? -1 : S.snode_of[buf[0]];
    if (sn.parent >= 0) S.children[sn.parent].push_back(s);
    sn.panel_off = panel;
    panel += (int64_t)(sn.ncols + sn.nrows) * sn.ncols;
    sn.u_off = u;
    u += sn.nrows;
    packed += (int64_t)sn.ncols * (sn.ncols + 1) / 2 + (int64_t)sn.nrows * sn.ncols;
  }
  S.panel_size = panel;
  S.u_size = u;
  S.packed_nnz = packed;

  // forward-update contributions to every internal row, in supernode order
  S.cptr.assign(n + 1, 0);
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t p = 0; p < S.sn[s].nrows; ++p) S.cptr[S.rows[S.sn[s].rows_off + p] + 1]++;
  for (int32_t i = 0; i < n; ++i) S.cptr[i + 1] += S.cptr[i];
  S.cidx.assign(S.cptr[n], 0);
  std::vector<int32_t> fill(S.cptr.begin(), S.cptr.end() - 1);
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t p = 0; p < S.sn[s].nrows; ++p) {
      const int32_t i = S.rows[S.sn[s].rows_off + p];
      S.cidx[fill[i]++] = (int32_t)(S.sn[s].u_off + p);
    }
}

namespace {

// Left-looking Cholesky of the ncols leading columns of an ld x ld front
// (column-major): produces L_ss in rows [0, n) and L_Rs in rows [n, ld).
bool panel_cholesky(double* F, int32_t n, int32_t ld) {
  for (int32_t j = 0; j < n; ++j) {
    double* cj = F + (int64_t)j * ld;
    for (int32_t k = 0; k < j; ++k) {
      const double* ck = F + (int64_t)k * ld;
      const double a = ck[j];
      if (a == 0.0) continue;
      for (int32_t i = j; i < ld; ++i) cj[i] -= ck[i] * a;
    }
    const double d = cj[j];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double s = std::sqrt(d);
    cj[j] = s;
    const double inv = 1.0 / s;
    for (int32_t i = j + 1; i < ld; ++i) cj[i] *= inv;
  }
  return true;
}

// U (r x r, lower, column-major) = F22 - L21 L21^T where F22 and L21 live in
// the front F (ld = n + r).
void schur_update(const double* F, int32_t n, int32_t ld, double* U) {
  const int32_t r = ld - n;
  for (int32_t j = 0; j < r; ++j)
    for (int32_t i = j; i < r; ++i) U[(int64_t)j * r + i] = F[(int64_t)(n + j) * ld + n + i];
  const int64_t work = (int64_t)r * r * n;
#pragma omp parallel for schedule(dynamic, 4) if (work > (1 << 22))
  for (int32_t j0 = 0; j0 < r; j0 += 4) {
    const int32_t jn = std::min(4, r - j0);
    for (int32_t k = 0; k < n; ++k) {
      const double* lk = F + (int64_t)k * ld + n;  // L21[:, k]
      double a[4] = {0, 0, 0, 0};
      for (int32_t t = 0; t < jn; ++t) a[t] = lk[j0 + t];
      if (jn == 4) {
        double* u0 = U + (int64_t)(j0 + 0) * r;
        double* u1 = U + (int64_t)(j0 + 1) * r;
        double* u2 = U + (int64_t)(j0 + 2) * r;
        double* u3 = U + (int64_t)(j0 + 3) * r;
        for (int32_t t = 0; t < 4; ++t) {
          double* ut = U + (int64_t)(j0 + t) * r;
          for (int32_t i = j0 + t; i < j0 + 4; ++i) ut[i] -= lk[i] * a[t];
        }
        for (int32_t i = j0 + 4; i < r; ++i) {
          const double l = lk[i];
          u0[i] -= l * a[0];
          u1[i] -= l * a[1];
          u2[i] -= l * a[2];
          u3[i] -= l * a[3];
        }
      } else {
        for (int32_t t = 0; t < jn; ++t) {
          double* ut = U + (int64_t)(j0 + t) * r;
          for (int32_t i = j0 + t; i < r; ++i) ut[i] -= lk[i] * a[t];
        }
      }
    }
  }
}

// Panel [inv(L11); -L21 inv(L11)] (ld x n, column-major) from the factored front.
// The lower block is stored negated so both sweeps only add.
void make_panel(const double* F, int32_t n, int32_t ld, double* P) {
  // inverse of the lower-triangular L11, column by column
  std::vector<double> T((int64_t)n * n, 0.0);
#pragma omp parallel for schedule(dynamic, 8) if ((int64_t)n * n * n > (1 << 21))
  for (int32_t j = 0; j < n; ++j) {
    double* t = T.data() + (int64_t)j * n;
    t[j] = 1.0;
    for (int32_t k = j; k < n; ++k) {
      const double* lk = F + (int64_t)k * ld;
      t[k] /= lk[k];
      const double tk = t[k];
      if (tk == 0.0) continue;
      for (int32_t i = k + 1; i < n; ++i) t[i] -= lk[i] * tk;
    }
  }
  const int32_t r = ld - n;
#pragma omp parallel for schedule(dynamic, 4) if ((int64_t)r * n * n > (1 << 21))
  for (int32_t j = 0; j < n; ++j) {
    double* pc = P + (int64_t)j * ld;
    const double* t = T.data() + (int64_t)j * n;
    for (int32_t i = 0; i < n; ++i) pc[i] = t[i];
    double* w = pc + n;
    for (int32_t i = 0; i < r; ++i) w[i] = 0.0;
    for (int32_t k = j; k < n; ++k) {
      const double tk = t[k];
      if (tk == 0.0) continue;
      const double* l = F + (int64_t)k * ld + n;
      for (int32_t i = 0; i < r; ++i) w[i] -= l[i] * tk;
    }
  }
}

}  // namespace

bool factor_panels(const Symbolic& S, const Csr& A, std::vector<double>& panels, std::string& err) {
  const int32_t n = S.n, ns = (int32_t)S.sn.size();
  panels.assign(S.panel_size, 0.0);
  std::vector<int32_t> loc(n, -1);
  std::vector<std::vector<double>> upd(ns);
  std::vector<double> F;
  for (int32_t s = 0; s < ns; ++s) {
    const Supernode& sn = S.sn[s];
    const int32_t nc = sn.ncols, nr = sn.nrows, ld = nc + nr;
    for (int32_t j = 0; j < nc; ++j) loc[sn.col0 + j] = j;
    for (int32_t p = 0; p < nr; ++p) loc[S.rows[sn.rows_off + p]] = nc + p;
    F.assign((int64_t)ld * ld, 0.0);
    const int32_t end = sn.col0 + nc;
    for (int32_t j = sn.col0; j < end; ++j) {
      const int32_t f = S.perm[j];
      const int32_t lj = loc[j];
      for (int64_t k = A.ptr[f]; k < A.ptr[f + 1]; ++k) {
        const int32_t i = S.iperm[A.col[k]];
        if (i < j) continue;
        F[(int64_t)lj * ld + loc[i]] += A.val[k];
      }
    }
    for (int32_t ch : S.children[s]) {
      const Supernode& cs = S.sn[ch];
      const int32_t r = cs.nrows;
      const double* U = upd[ch].data();
      const int32_t* R = &S.rows[cs.rows_off];
      for (int32_t q = 0; q < r; ++q) {
        const int64_t lq = (int64_t)loc[R[q]] * ld;
        for (int32_t p = q; p < r; ++p) F[lq + loc[R[p]]] += U[(int64_t)q * r + p];
      }
      std::vector<double>().swap(upd[ch]);
    }
    if (!panel_cholesky(F.data(), nc, ld)) {
      err = "non-positive pivot in supernode " + std::to_string(s);
      return false;
    }
    if (nr > 0) {
      upd[s].assign((int64_t)nr * nr, 0.0);
      schur_update(F.data(), nc, ld, upd[s].data());
    }
    make_panel(F.data(), nc, ld, panels.data() + sn.panel_off);
  }
  return true;
}

static SweepTask make_task(const Supernode& sn, int32_t s, int32_t first, int32_t count) {
  SweepTask t{};
  t.sn = s;
  t.first = first;
  t.count = count;
  t.col0 = sn.col0;
  t.ncols = sn.ncols;
  t.nrows = sn.nrows;
  t.panel_off = sn.panel_off;
  t.rows_off = sn.rows_off;
  t.u_off = sn.u_off;
  return t;
}

void build_plan(const Symbolic& S, LevelPlan& P) {
  const int32_t L = S.n_levels;
  std::vector<std::vector<int32_t>> by_level(L);
  for (int32_t s = 0; s < (int32_t)S.sn.size(); ++s) by_level[S.sn[s].level].push_back(s);
  P.fwd.clear();
  P.bwd.clear();
  P.fwd_off.assign(L + 1, 0);
  P.bwd_off.assign(L + 1, 0);
  P.fwd_cols.assign(L, 0);
  P.bwd_rows.assign(L, 0);
  P.fwd_wide.assign(L, 0);
  P.bwd_narrow.assign(L, 0);
  const int64_t target = 2048;  // workgroups wanted per level
  for (int32_t l = 0; l < L; ++l) {
    P.fwd_off[l] = (int32_t)P.fwd.size();
    P.bwd_off[l] = (int32_t)P.bwd.size();
    int64_t rows = 0, cols = 0;
    int32_t max_nc = 0;
    for (int32_t s : by_level[l]) {
      rows += S.sn[s].ncols + S.sn[s].nrows;
      cols += S.sn[s].ncols;
      max_nc = std::max(max_nc, S.sn[s].ncols);
    }
    const bool wide = max_nc > 64;
    P.fwd_wide[l] = wide ? 1 : 0;
    int32_t max_ld = 0;
    for (int32_t s : by_level[l]) max_ld = std::max(max_ld, S.sn[s].ncols + S.sn[s].nrows);
    // many small supernodes: one backward task each (LDS holds 3 x ld doubles
    // and 1024 x 3 partial sums, within 64 KiB)
    const bool narrow_b = !wide && (int64_t)by_level[l].size() >= 256 && lds_bwd_narrow(max_ld) * 8 <= 65536;
    P.bwd_narrow[l] = narrow_b ? 1 : 0;
    // wide forward: one pass of a task's waves (16 waves x 64 / lanes-per-row
    // rows), so the block's staged right-hand sides serve that many rows;
    // backward: likewise one pass of columns (16 x 64 / lanes-per-column)
    const int32_t rpt = (kWideTaskThreads / 64) * (64 / sweep_lanes(max_nc));
    const int32_t cpt = (kWideTaskThreads / 64) * (64 / sweep_lanes(max_ld));
    for (int32_t s : by_level[l]) {
      const Supernode& sn = S.sn[s];
      const int32_t ld = sn.ncols + sn.nrows;
      const int32_t fstep = wide ? rpt : 64;   // narrow forward: 64 rows per task
      for (int32_t f = 0; f < ld; f += fstep) P.fwd.push_back(make_task(sn, s, f, std::min(fstep, ld - f)));
      if (narrow_b)
        P.bwd.push_back(make_task(sn, s, 0, sn.ncols));
      else
        for (int32_t f = 0; f < sn.ncols; f += cpt) P.bwd.push_back(make_task(sn, s, f, std::min(cpt, sn.ncols - f)));
      P.fwd_cols[l] = std::max(P.fwd_cols[l], sn.ncols);
      P.bwd_rows[l] = std::max(P.bwd_rows[l], ld);
    }
  }
  P.fwd_off[L] = (int32_t)P.fwd.size();   // the last level's task range is read below
  P.bwd_off[L] = (int32_t)P.bwd.size();
  // pre-gather on wide levels whose supernodes are split into several tasks
  P.gather_off.assign(L + 1, 0);
  P.gather_cols.clear();
  for (int32_t l = 0; l < L; ++l) {
    P.gather_off[l] = (int32_t)P.gather_cols.size();
    const int32_t ntask = P.fwd_off[l + 1] - P.fwd_off[l];
    const int32_t nsn = (int32_t)by_level[l].size();
    int32_t max_nc = 0;
    for (int32_t s : by_level[l]) max_nc = std::max(max_nc, S.sn[s].ncols);
    int64_t contribs = 0;
    for (int32_t s : by_level[l]) contribs += S.cptr[S.sn[s].col0 + S.sn[s].ncols] - S.cptr[S.sn[s].col0];
    if (P.fwd_wide[l] && ntask >= 4 * nsn && max_nc >= 256 && contribs > 0)
      for (int32_t s : by_level[l])
        for (int32_t c = 0; c < S.sn[s].ncols; ++c) P.gather_cols.push_back(S.sn[s].col0 + c);
  }
  P.gather_off[L] = (int32_t)P.gather_cols.size();
  P.fwd_bytes.assign(L, 0.0);
  P.bwd_bytes.assign(L, 0.0);
  P.fwd_flops.assign(L, 0.0);
  P.bwd_flops.assign(L, 0.0);
  for (int32_t l = 0; l < L; ++l)
    for (int32_t s : by_level[l]) {
      const Supernode& sn = S.sn[s];
      const double nc = sn.ncols, nr = sn.nrows, nnz = nc * (nc + 1) / 2 + nr * nc;
      double contribs = 0;
      for (int32_t j = sn.col0; j < sn.col0 + sn.ncols; ++j) contribs += S.cptr[j + 1] - S.cptr[j];
      // forward: panel, b_s and incoming updates read, y_s and outgoing updates written;
      // a pre-gathered level's sweep kernel reads the gathered b~_s instead (the
      // gather pass, a kernel of its own, moves the updates)
      const bool pre = P.gather_off[l + 1] > P.gather_off[l];
      P.fwd_bytes[l] += pre ? 8.0 * nnz + 24.0 * nc + 24.0 * (nc + nr)
                            : 8.0 * nnz + 24.0 * (nc + contribs) + 24.0 * (nc + nr) + 4.0 * contribs;
      // backward: panel, y_s and x_R read, x_s written (internal and public copies)
      P.bwd_bytes[l] += 8.0 * nnz + 24.0 * (nc + nr) + 4.0 * nr + 48.0 * nc;
      P.fwd_flops[l] += 6.0 * nnz;
      P.bwd_flops[l] += 6.0 * nnz;
    }
  P.fwd_off[L] = (int32_t)P.fwd.size();
  P.bwd_off[L] = (int32_t)P.bwd.size();
}


void build_dag(const Symbolic& S, const LevelPlan& P, int64_t lds_budget_bytes, DagPlan& D) {
  const int32_t L = S.n_levels, ns = (int32_t)S.sn.size();
  D.q.clear();
  D.bwd_region = 0;
  D.usable = true;
  D.sn.assign(ns, DagSn{});
  for (int32_t s = 0; s < ns; ++s) {
    D.sn[s].parent = S.sn[s].parent;
    D.sn[s].nch = (int32_t)S.children[s].size();
  }
  int64_t lds = 0;
  auto entry = [](int32_t kind, int32_t n, int32_t first, int32_t lpr, int32_t flags) {
    DagEntry e{};
    e.kind = kind;
    e.n = n;
    e.first = first;
    e.lpr = lpr;
    e.flags = flags;
    for (int k = 0; k < kDagSub; ++k) e.sn[k] = -1;
    return e;
  };
  for (int32_t l = 0; l < L; ++l) {
    // gathers of the level: runs of at most kDagGatherCols columns of one supernode
    for (int32_t g = P.gather_off[l]; g < P.gather_off[l + 1];) {
      const int32_t s = S.snode_of[P.gather_cols[g]];
      int32_t n = 1;
      while (n < kDagGatherCols && g + n < P.gather_off[l + 1] && S.snode_of[P.gather_cols[g + n]] == s) ++n;
      DagEntry e = entry(kDagGather, n, g, 0, 0);
      e.sn[0] = s;
      D.q.push_back(e);
      D.sn[s].ngt += 1;
      g += n;
    }
    const int32_t t0 = P.fwd_off[l], t1 = P.fwd_off[l + 1];
    if (P.fwd_wide[l]) {
      const int32_t lpr = sweep_lanes(P.fwd_cols[l]);
      const int32_t pre = P.gather_off[l + 1] > P.gather_off[l] ? 1 : 0;
      lds = std::max<int64_t>(lds, 3 * (int64_t)P.fwd_cols[l] * 8);
      for (int32_t t = t0; t < t1; ++t) {
        DagEntry e = entry(kDagFwdWide, 1, t, lpr, pre);
        e.sn[0] = P.fwd[t].sn;
        D.q.push_back(e);
      }
    } else {
      // one task per entry on the whole workgroup
      lds = std::max<int64_t>(lds, lds_fwd_narrow(kDagNarrowCols) * 8);
      for (int32_t t = t0; t < t1; ++t) {
        DagEntry e = entry(kDagFwdNarrow, 1, t, 0, 0);
        e.sn[0] = P.fwd[t].sn;
        D.q.push_back(e);
      }
    }
    for (int32_t t = t0; t < t1; ++t) D.sn[P.fwd[t].sn].ntf += 1;
  }
  D.n_fwd = (int32_t)D.q.size();
  for (int32_t l = L - 1; l >= 0; --l) {
    const int32_t t0 = P.bwd_off[l], t1 = P.bwd_off[l + 1];
    if (P.bwd_narrow[l]) {
      // one task per entry on the whole workgroup
      D.bwd_region = std::max<int32_t>(D.bwd_region, (int32_t)lds_bwd_narrow(P.bwd_rows[l]));
      lds = std::max<int64_t>(lds, (int64_t)D.bwd_region * 8);
      for (int32_t t = t0; t < t1; ++t) {
        DagEntry e = entry(kDagBwdNarrow, 1, t, 0, 0);
        e.sn[0] = P.bwd[t].sn;
        D.q.push_back(e);
      }
    } else {
      const int32_t lpr = sweep_lanes(P.bwd_rows[l]);
      const int64_t need = 3 * (int64_t)P.bwd_rows[l] * 8;
      const int32_t staged = need <= lds_budget_bytes ? 2 : 0;
      if (staged) lds = std::max(lds, need);
      else D.usable = false;   // the kernel stages every column task's vector in LDS
      for (int32_t t = t0; t < t1; ++t) {
        DagEntry e = entry(kDagBwdCols, 1, t, lpr, staged);
        e.sn[0] = P.bwd[t].sn;
        D.q.push_back(e);
      }
    }
    for (int32_t t = t0; t < t1; ++t) D.sn[P.bwd[t].sn].ntb += 1;
  }
  D.lds_bytes = lds;
  if (lds > lds_budget_bytes) D.usable = false;
}

std::string build_factor_plan(const Symbolic& S, const Csr& A, FactorPlan& P) {
  const int32_t ns = (int32_t)S.sn.size();
  P = FactorPlan{};
  P.fronts.resize(ns);
  int64_t off = 0;
  for (int32_t s = 0; s < ns; ++s) {
    const Supernode& sn = S.sn[s];
    FrontDesc& f = P.fronts[s];
    f.front_off = off;
    f.panel_off = sn.panel_off;
    f.rows_off = sn.rows_off;
    f.ld = sn.ncols + sn.nrows;
    f.nc = sn.ncols;
    f.nrows = sn.nrows;
    f.parent = sn.parent;
    f.col0 = sn.col0;
    off += (int64_t)f.ld * f.ld;
    const double n = sn.ncols, r = sn.nrows;
    P.flops += n * n * n / 3.0 + n * n * r + n * r * r + n * n * n / 3.0 + r * n * n;
  }
  P.front_size = off;
  // entries of A on or below the diagonal of each supernode's columns
  std::vector<int32_t> loc(S.n, -1);
  for (int32_t s = 0; s < ns; ++s) {
    const Supernode& sn = S.sn[s];
    const FrontDesc& f = P.fronts[s];
    for (int32_t j = 0; j < sn.ncols; ++j) loc[sn.col0 + j] = j;
    for (int32_t p = 0; p < sn.nrows; ++p) loc[S.rows[sn.rows_off + p]] = sn.ncols + p;
    for (int32_t j = sn.col0; j < sn.col0 + sn.ncols; ++j) {
      const int32_t fr = S.perm[j];
      for (int64_t k = A.ptr[fr]; k < A.ptr[fr + 1]; ++k) {
        const int32_t i = S.iperm[A.col[k]];
        if (i < j) continue;
        const int32_t li = loc[i];
        if (li < 0 || li >= f.ld) return "entry of A outside its supernode's front";
        P.a_dst.push_back(f.front_off + (int64_t)loc[j] * f.ld + li);
        P.a_src.push_back((int32_t)k);
      }
    }
    // the rows of s's children in s's front
    for (int32_t ch : S.children[s]) {
      const Supernode& cs = S.sn[ch];
      for (int32_t p = 0; p < cs.nrows; ++p) {
        const int32_t li = loc[S.rows[cs.rows_off + p]];
        if (li < 0 || li >= f.ld) return "child row outside its parent's front";
        if (P.relmap.size() < S.rows.size()) P.relmap.resize(S.rows.size(), -1);
        P.relmap[cs.rows_off + p] = li;
      }
    }
    for (int32_t j = 0; j < sn.ncols; ++j) loc[sn.col0 + j] = -1;
    for (int32_t p = 0; p < sn.nrows; ++p) loc[S.rows[sn.rows_off + p]] = -1;
  }
  P.relmap.resize(S.rows.size(), -1);
  for (int32_t s = 0; s < ns; ++s)
    if (S.sn[s].parent >= 0)
      for (int32_t p = 0; p < S.sn[s].nrows; ++p)
        if (P.relmap[S.sn[s].rows_off + p] < 0) return "child row without a position in its parent";

  auto add_op = [&](int32_t kind, int32_t level, int32_t k0, const std::vector<int32_t>& items,
                    const std::vector<int64_t>& blocks) {
    FactorOp op{};
    op.kind = kind;
    op.level = level;
    op.k0 = k0;
    op.n = (int32_t)items.size();
    op.list_off = (int32_t)P.ints.size();
    P.ints.insert(P.ints.end(), items.begin(), items.end());
    int64_t acc = 0;
    P.ints.push_back(0);
    for (int64_t b : blocks) {
      acc += b;
      P.ints.push_back((int32_t)acc);
    }
    op.blocks = (int32_t)acc;
    if (acc >= (int64_t)1 << 30) return false;
    for (size_t i = 0; i < blocks.size(); ++i)
      for (int64_t b = 0; b < blocks[i]; ++b) P.ints.push_back((int32_t)i);
    if (acc > 0 && kind != kFactorTranspose) P.ops.push_back(op);
    if (kind == kFactorTranspose) P.transpose = op;
    return (int64_t)P.ints.size() < (int64_t)1 << 31;
  };
  const int64_t TT = kFactorTile, NB = kFactorNB;
  for (int32_t l = 0; l < S.n_levels; ++l) {
    std::vector<int32_t> lev;
    int32_t max_nc = 0;
    size_t max_ch = 0;
    for (int32_t s = 0; s < ns; ++s)
      if (S.sn[s].level == l) {
        lev.push_back(s);
        max_nc = std::max(max_nc, S.sn[s].ncols);
        max_ch = std::max(max_ch, S.children[s].size());
      }
    // extend-add, one launch per sibling rank (fronts of one launch are distinct)
    for (size_t c = 0; c < max_ch; ++c) {
      std::vector<int32_t> items;
      std::vector<int64_t> blocks;
      for (int32_t s : lev)
        if (S.children[s].size() > c) {
          const int32_t ch = S.children[s][c];
          if (S.sn[ch].nrows <= 0) return "child without rows";
          items.push_back(ch);
          blocks.push_back((S.sn[ch].nrows + 3) / 4);
        }
      if (!add_op(kFactorExtend, l, 0, items, blocks)) return "extend-add launch too large";
    }
    for (int32_t k0 = 0; k0 < max_nc; k0 += (int32_t)NB) {
      std::vector<int32_t> i1, i2;
      std::vector<int64_t> b1, b2;
      for (int32_t s : lev) {
        const FrontDesc& f = P.fronts[s];
        if (f.nc <= k0) continue;
        const int64_t kb = std::min<int64_t>(NB, f.nc - k0), k1 = k0 + kb, m = f.ld - k1;
        i1.push_back(s);
        b1.push_back((m + 63) / 64 + (k1 + 63) / 64);   // rows, then panel columns, 64 per workgroup
        if (m > 0) {
          const int64_t T = (m + TT - 1) / TT;
          i2.push_back(s);
          b2.push_back(T * (T + 1) / 2 + T * ((k1 + TT - 1) / TT));
        }
      }
      if (!add_op(kFactorPanel, l, k0, i1, b1)) return "panel launch too large";
      if (!add_op(kFactorUpdate, l, k0, i2, b2)) return "update launch too large";
    }
  }
  {
    std::vector<int32_t> all(ns);
    std::vector<int64_t> blocks(ns);
    for (int32_t s = 0; s < ns; ++s) {
      all[s] = s;
      const int64_t e = (int64_t)P.fronts[s].ld * P.fronts[s].nc;
      blocks[s] = (e + kFactorTransposeChunk - 1) / kFactorTransposeChunk;
    }
    if (!add_op(kFactorTranspose, -1, 0, all, blocks)) return "transpose launch too large";
  }
  for (int64_t d : P.a_dst)
    if (d < 0 || d >= P.front_size) return "front position out of range";
  for (int32_t k : P.a_src)
    if (k < 0 || k >= (int64_t)A.val.size()) return "entry index out of range";
  return "";
}

}  // namespace dpd
