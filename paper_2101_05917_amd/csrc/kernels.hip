// HIP kernels (gfx950) of the PD step and its adjoint.
//
//  * Local step (Alg. 1, eq:pd_energy_single): one thread per Gauss point,
//    eight lanes per hex element.  The element's eight node positions are
//    staged in LDS, each lane forms its deformation gradient F_q, projects it
//    onto SO(3) (closest rotation, supplemental Sec. Energy Definitions) and
//    the lanes of an element exchange their stresses through LDS to produce
//    the eight nodal force vectors of the element.  No atomics: element
//    forces go to an element-major buffer and a node-centric kernel gathers
//    the (at most eight) contributions of each node in a fixed order.
//  * Residual: grad g(x) = M (x - y)/h^2 + sum_c w_c G_c^T (G_c x - p_c)
//    (eq:energy_grad), whose norm drives the stopping test; the global step
//    is then x <- x - A^{-1} grad g(x), the correction form of Alg. 1.
//  * Adjoint local step (eq:matrix_split): dA p through the differential of
//    the polar decomposition at cached rotations.
//  * Global step: level-scheduled supernodal sweeps over precomputed panels
//    [inv(L_ss); -L_Rs inv(L_ss)] (dense matrix-vector products per level).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>

#include "device.hpp"
#include "device_math.hpp"

namespace dpd {

thread_local ClockArg g_launch_clock;

// ------------------------------------------------------------------ forward local step

__global__ void __launch_bounds__(kBlock) k_elem_forces(DevMesh M, const double* __restrict__ x,
                                                        const double* __restrict__ act,
                                                        double* __restrict__ fe,
                                                        double* __restrict__ R_out,
                                                        IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  __shared__ ElemTile T;
  const int le = threadIdx.x >> 3, q = threadIdx.x & 7;
  const int e = blockIdx.x * kElemsPerBlock + le;
  const bool valid = e < M.E;
  const GradTable G = grad_table(M.dx);
  gather_nodes(M, x, T, le, q, e, valid);
  __syncthreads();
  if (valid) {
    double F[9], R[9];
    deformation_gradient(T, le, q, G, F);
    if (M.local32)
      closest_rotation_mixed(F, R);
    else
      closest_rotation(F, R);
    if (st && det3(F) <= 0.0) atomicAdd(&st->inverted, 1);
    const double w = M.w_e[e];
    double* P = T.Ps[le][q];
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = w * (F[i] - R[i]);
    if (M.wv_e) {
      // volume-preserving term: projection onto det D = 1 (D = R where det F <= 0)
      VolumeProj vp;
      volume_project(F, R, vp);
      double D[9];
      if (vp.ok) volume_matrix(R, vp.V, vp.Dd, D);
      else
#pragma unroll
        for (int i = 0; i < 9; ++i) D[i] = R[i];
      const double wv = M.wv_e[e];
#pragma unroll
      for (int i = 0; i < 9; ++i) P[i] += wv * (F[i] - D[i]);
    }
    if (R_out) {
      const int64_t Q = 8 * (int64_t)M.E, qi = 8 * (int64_t)e + q;
#pragma unroll
      for (int i = 0; i < 9; ++i) R_out[i * Q + qi] = R[i];
    }
    if (M.muscle_k > 0.0) {
      // fibre projection onto |p| = r (supplemental, muscle fibers)
      const double m0 = M.fiber[0], m1 = M.fiber[1], m2 = M.fiber[2];
      const double f0 = F[0] * m0 + F[1] * m1 + F[2] * m2;
      const double f1 = F[3] * m0 + F[4] * m1 + F[5] * m2;
      const double f2 = F[6] * m0 + F[7] * m1 + F[8] * m2;
      const double r = act ? act[e] : 1.0;
      const double nf = sqrt(f0 * f0 + f1 * f1 + f2 * f2);
      double p0, p1, p2;
      if (nf > 0.0) {
        p0 = r * f0 / nf;
        p1 = r * f1 / nf;
        p2 = r * f2 / nf;
      } else {
        p0 = r * m0;
        p1 = r * m1;
        p2 = r * m2;
      }
      const double wm = M.muscle_k * M.Vq;
      const double d0 = wm * (f0 - p0), d1 = wm * (f1 - p1), d2 = wm * (f2 - p2);
      P[0] += d0 * m0; P[1] += d0 * m1; P[2] += d0 * m2;
      P[3] += d1 * m0; P[4] += d1 * m1; P[5] += d1 * m2;
      P[6] += d2 * m0; P[7] += d2 * m1; P[8] += d2 * m2;
    }
  }
  __syncthreads();
  element_forces_out(M, T, le, q, e, valid, G, fe);
  clock_exit(ck);
}


// r = M (x - y)/h^2 + sum w G^T (G x - p) + ground term; |r|^2 -> stopping test.
__global__ void __launch_bounds__(kBlock) k_node_residual(DevMesh M, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ fe,
                                                          double* __restrict__ r, IterState* st,
                                                          double* partials, int k, int max_iter,
                                                          int fixed_iters) {
  if (st->done) return;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (n < M.N) {
    const int64_t N = M.N;
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    if (!M.fixed[n]) {
      node_force(M, fe, n, r0, r1, r2);
      const double c = M.mass[n] / (M.h * M.h);
      r0 += c * (x[n] - y[n]);
      r1 += c * (x[N + n] - y[N + n]);
      r2 += c * (x[2 * N + n] - y[2 * N + n]);
      if (M.contact[n]) {
        const double z = x[2 * N + n];
        if (z < 0.0) r2 += M.contact_k * z;
      }
      acc = r0 * r0 + r1 * r1 + r2 * r2;
    }
    r[n] = r0;
    r[N + n] = r1;
    r[2 * N + n] = r2;
  }
  double tot;
  if (grid_sum(acc, partials, st, &tot)) {
    st->rsq = tot;
    st->iter = k;
    if (k == 0) st->r0sq = tot;
    if (!isfinite(tot)) {
      st->nonfinite = 1;
      st->done = 1;
    } else if (!fixed_iters && (tot <= st->tolsq * st->r0sq || tot <= st->atolsq)) {
      st->converged = 1;
      st->done = 1;
    }
    if (k >= max_iter) st->done = 1;
  }
}

__global__ void k_reset_state(IterState* st, double tolsq, int max_iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->max_iter = max_iter;
    st->r0sq = st->rsq = st->atolsq = 0.0;
    st->tolsq = tolsq;
    st->nb2 = st->rs = st->pq = st->alpha = st->beta = st->acc = 0.0;
    st->iter = st->done = st->converged = st->nonfinite = st->curvature = st->inverted = 0;
    st->aborted = st->solves = 0;
    st->g_prev = -1.0;
    st->eta = 0.0;
    st->counter = 0u;
  }
}

// y = x + h v + h^2 (g + f_fric / m); x^0 = y with Dirichlet nodes at rest.
// The explicit friction acts on ground-contact nodes below the ground.
__global__ void __launch_bounds__(kBlock) k_prologue(DevMesh M, const double* __restrict__ x,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ y, double* __restrict__ xn,
                                                     IterState* st, double* partials,
                                                     double abs_tol_rel) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (n < M.N) {
    const int64_t N = M.N;
    double ft0 = 0.0, ft1 = 0.0;
    if (M.contact[n] && M.friction_mu > 0.0) {
      const double z = x[2 * N + n];
      const double fn = M.contact_k * fmax(0.0, -z);
      const double v0 = v[n], v1 = v[N + n];
      const double s = sqrt(v0 * v0 + v1 * v1 + M.friction_eps * M.friction_eps);
      ft0 = -M.friction_mu * fn * v0 / s;
      ft1 = -M.friction_mu * fn * v1 / s;
    }
    const double h = M.h, m = M.mass[n];
    const double y0 = x[n] + h * v[n] + h * h * (M.g[0] + ft0 / m);
    const double y1 = x[N + n] + h * v[N + n] + h * h * (M.g[1] + ft1 / m);
    const double y2 = x[2 * N + n] + h * v[2 * N + n] + h * h * M.g[2];
    y[n] = y0;
    y[N + n] = y1;
    y[2 * N + n] = y2;
    if (M.fixed[n]) {
      xn[n] = M.X[n];
      xn[N + n] = M.X[N + n];
      xn[2 * N + n] = M.X[2 * N + n];
    } else {
      xn[n] = y0;
      xn[N + n] = y1;
      xn[2 * N + n] = y2;
      const double c = m / (h * h);
      acc = c * c * (y0 * y0 + y1 * y1 + y2 * y2);
    }
  }
  double tot;
  if (grid_sum(acc, partials, st, &tot)) st->atolsq = abs_tol_rel * abs_tol_rel * tot;
}

__global__ void __launch_bounds__(kBlock) k_velocity(int N, double inv_h, const double* __restrict__ x,
                                                     const double* __restrict__ xn,
                                                     double* __restrict__ vn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * (int64_t)N) vn[i] = (xn[i] - x[i]) * inv_h;
}

// Zero the fixed-node rows of a [3][N] vector (outputs of a solve are defined
// on free nodes only).
__global__ void k_zero_fixed(DevMesh M, double* v) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < M.N && M.fixed[n]) {
    v[n] = 0.0;
    v[(int64_t)M.N + n] = 0.0;
    v[2 * (int64_t)M.N + n] = 0.0;
  }
}

// ------------------------------------------------------------------ adjoint

// Per Gauss point at x_{i+1}: R (9), inv(tr(S) I - S) (6), and for muscles the unit
// fibre image n (3) and r/|f| (1): cache layout [19][Q].
constexpr int kCacheRows = 19;

__global__ void __launch_bounds__(kBlock) k_adj_cache(DevMesh M, const double* __restrict__ x,
                                                      const double* __restrict__ act,
                                                      double* __restrict__ cache, IterState* st,
                                                      const IterState* gate, int elem_blocks) {
  if (gate && gate->done) return;
  if ((int)blockIdx.x >= elem_blocks) {
    // ground contact active at the linearisation point (height below zero):
    // the contact term of A - dA is k on the vertical coordinate there
    const int n = (blockIdx.x - elem_blocks) * blockDim.x + threadIdx.x;
    if (n < M.N) M.cmask[n] = (M.contact[n] && x[2 * (int64_t)M.N + n] < 0.0) ? 1 : 0;
    return;
  }
  __shared__ ElemTile T;
  const int le = threadIdx.x >> 3, q = threadIdx.x & 7;
  const int e = blockIdx.x * kElemsPerBlock + le;
  const bool valid = e < M.E;
  const GradTable G = grad_table(M.dx);
  gather_nodes(M, x, T, le, q, e, valid);
  __syncthreads();
  if (!valid) return;
  double F[9], R[9], Ki[6];
  deformation_gradient(T, le, q, G, F);
  if (M.local32)
    closest_rotation_mixed(F, R);
  else
    closest_rotation(F, R);
  const bool ok = rotation_kinv(F, R, Ki);
  if (st && (!ok || det3(F) <= 0.0)) atomicAdd(&st->inverted, 1);
  const int64_t Q = 8 * (int64_t)M.E, qi = 8 * (int64_t)e + q;
#pragma unroll
  for (int i = 0; i < 9; ++i) cache[i * Q + qi] = R[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) cache[(9 + i) * Q + qi] = Ki[i];
  if (M.wv_e) {
    VolumeProj vp;
    volume_project(F, R, vp);
    double Gm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, r[3] = {0, 0, 0}, k[3] = {0, 0, 0};
    if (vp.ok) volume_derivative_data(vp, Gm, r, k);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      cache[(kVolV + i) * Q + qi] = vp.V[i];
      cache[(kVolG + i) * Q + qi] = Gm[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cache[(kVolR + i) * Q + qi] = r[i];
      cache[(kVolK + i) * Q + qi] = k[i];
      cache[(kVolD + i) * Q + qi] = vp.Dd[i];
    }
    cache[kVolOk * Q + qi] = vp.ok ? 1.0 : 0.0;
  }
  if (M.muscle_k > 0.0) {
    const double m0 = M.fiber[0], m1 = M.fiber[1], m2 = M.fiber[2];
    const double f0 = F[0] * m0 + F[1] * m1 + F[2] * m2;
    const double f1 = F[3] * m0 + F[4] * m1 + F[5] * m2;
    const double f2 = F[6] * m0 + F[7] * m1 + F[8] * m2;
    const double nf = sqrt(f0 * f0 + f1 * f1 + f2 * f2);
    const double r = act ? act[e] : 1.0;
    if (nf > 0.0) {
      cache[15 * Q + qi] = f0 / nf;
      cache[16 * Q + qi] = f1 / nf;
      cache[17 * Q + qi] = f2 / nf;
      cache[18 * Q + qi] = r / nf;
    } else {
      cache[15 * Q + qi] = m0;
      cache[16 * Q + qi] = m1;
      cache[17 * Q + qi] = m2;
      cache[18 * Q + qi] = 0.0;
    }
  }
}

// dA p per element (the adjoint local step): corner forces of block bid's
// elements into fe.
__device__ inline void elem_hvp_block(const DevMesh& M, const double* __restrict__ p,
                                      const double* __restrict__ cache, double* __restrict__ fe, int bid) {
  __shared__ ElemTile T;
  const int le = threadIdx.x >> 3, q = threadIdx.x & 7;
  const int e = bid * kElemsPerBlock + le;
  const bool valid = e < M.E;
  const GradTable G = grad_table(M.dx);
  gather_nodes(M, p, T, le, q, e, valid);
  __syncthreads();
  if (valid) hvp_stress(M, T, le, q, e, G, cache);
  __syncthreads();
  element_forces_out(M, T, le, q, e, valid, G, fe);
}

__global__ void __launch_bounds__(kBlock) k_elem_hvp(DevMesh M, const double* __restrict__ p,
                                                     const double* __restrict__ cache,
                                                     double* __restrict__ fe, const IterState* st,
                                                     ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  elem_hvp_block(M, p, cache, fe, blockIdx.x);
  clock_exit(ck);
}

// out = (A - dA) p (- rhs if given); mode 0: plain; mode 1: out = H p - rhs and
// |out|^2 / nb2 drives the fixed-point stopping test.
__global__ void __launch_bounds__(kBlock) k_node_hvp(DevMesh M, const double* __restrict__ p,
                                                     const double* __restrict__ fe,
                                                     const double* __restrict__ rhs,
                                                     double* __restrict__ out, IterState* st,
                                                     double* partials, int mode, int k, int max_iter) {
  if (st && st->done) return;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (n < M.N) {
    const int64_t N = M.N;
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if (!M.fixed[n]) {
      node_force(M, fe, n, o0, o1, o2);
      const double c = M.mass[n] / (M.h * M.h);
      const double p0 = p[n], p1 = p[N + n], p2 = p[2 * N + n];
      o0 += c * p0;
      o1 += c * p1;
      o2 += c * p2;
      if (M.cmask[n]) o2 += M.contact_k * p2;
      if (rhs) {
        o0 -= rhs[n];
        o1 -= rhs[N + n];
        o2 -= rhs[2 * N + n];
      }
      acc = o0 * o0 + o1 * o1 + o2 * o2;
    }
    out[n] = o0;
    out[N + n] = o1;
    out[2 * N + n] = o2;
  }
  if (mode == 0) return;
  double tot;
  if (grid_sum(acc, partials, st, &tot)) {
    st->rsq = tot;
    st->iter = k;
    if (!isfinite(tot)) {
      st->nonfinite = 1;
      st->done = 1;
    } else if (tot <= st->tolsq * st->nb2) {
      st->converged = 1;
      st->done = 1;
    }
    if (k >= max_iter) st->done = 1;
  }
}

// |a|^2 over free nodes into st->nb2 (and rsq); a zero norm ends the iteration.
__global__ void __launch_bounds__(kBlock) k_dot(DevMesh M, const double* __restrict__ a,
                                                const double* __restrict__ b, IterState* st,
                                                double* partials, int what) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (n < M.N && !M.fixed[n]) {
    const int64_t N = M.N;
    acc = a[n] * b[n] + a[N + n] * b[N + n] + a[2 * N + n] * b[2 * N + n];
  }
  double tot;
  if (grid_sum(acc, partials, st, &tot)) {
    st->nb2 = tot;
    st->rsq = tot;
    if (!(tot > 0.0)) {
      st->converged = 1;
      st->done = 1;
    }
  }
}

// Two grid sums at once (same fixed order as grid_sum).
__device__ inline bool grid_sum2(double a, double b, double* partials, IterState* st, double* ta,
                                 double* tb, int bid, int nblk) {
  __shared__ double ws[kBlock / 64];
  __shared__ int last;
  const double ba = block_sum(a, ws);
  const double bb = block_sum(b, ws);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partials[2 * bid], ba, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[2 * bid + 1], bb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t t =
        __hip_atomic_fetch_add(&st->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == (uint32_t)nblk - 1);
  }
  __syncthreads();
  if (!last) return false;
  double sa = 0.0, sb = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    sa += __hip_atomic_load(&partials[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sb += __hip_atomic_load(&partials[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  sa = block_sum(sa, ws);
  sb = block_sum(sb, ws);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&st->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *ta = sa;
    *tb = sb;
  }
  return threadIdx.x == 0;
}

// Conjugate gradients in the Chronopoulos-Gear arrangement, which needs one
// grid reduction per iteration: with s = M^{-1} r and w = H s,
//   gamma = r.s, delta = w.s, beta = gamma/gamma_old,
//   alpha = gamma / (delta - beta gamma / alpha_old)   (= gamma / p^T H p),
//   p = s + beta p, q = w + beta q, z += alpha p, r -= alpha q.
// This step forms w = H s (node part) and both inner products; block bid of nblk.
__device__ inline void cg_hvp_dots_block(const DevMesh& M, const double* __restrict__ sv,
                                         const double* __restrict__ fe, const double* __restrict__ r,
                                         double* __restrict__ w, IterState* st, double* partials, int bid,
                                         int nblk) {
  const int n = bid * blockDim.x + threadIdx.x;
  double rs = 0.0, ws_ = 0.0;
  if (n < M.N) {
    const int64_t N = M.N;
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if (!M.fixed[n]) {
      node_force(M, fe, n, o0, o1, o2);
      const double c = M.mass[n] / (M.h * M.h);
      const double s0 = sv[n], s1 = sv[N + n], s2 = sv[2 * N + n];
      o0 += c * s0;
      o1 += c * s1;
      o2 += c * s2;
      if (M.cmask[n]) o2 += M.contact_k * s2;
      rs = r[n] * s0 + r[N + n] * s1 + r[2 * N + n] * s2;
      ws_ = o0 * s0 + o1 * s1 + o2 * s2;
    }
    w[n] = o0;
    w[N + n] = o1;
    w[2 * N + n] = o2;
  }
  double gamma, delta;
  if (grid_sum2(rs, ws_, partials, st, &gamma, &delta, bid, nblk)) {
    const bool first = st->iter == 0;
    const double beta = first ? 0.0 : gamma / st->rs;
    const double den = first ? delta : delta - beta * gamma / st->alpha;
    if (!(den > 0.0) || !isfinite(den) || !isfinite(gamma)) {
      st->curvature = 1;
      st->done = 1;
    } else {
      st->beta = beta;
      st->alpha = gamma / den;
      st->rs = gamma;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_hvp_dots(DevMesh M, const double* __restrict__ sv,
                                                        const double* __restrict__ fe,
                                                        const double* __restrict__ r,
                                                        double* __restrict__ w, IterState* st,
                                                        double* partials) {
  if (st->done) return;
  cg_hvp_dots_block(M, sv, fe, r, w, st, partials, blockIdx.x, gridDim.x);
}

// p = s + beta p; q = w + beta q; z += alpha p; r -= alpha q; |r|^2 -> stopping test.
__device__ inline void cg_step_block(const DevMesh& M, double* __restrict__ z, double* __restrict__ r,
                                     double* __restrict__ p, double* __restrict__ q,
                                     const double* __restrict__ sv, const double* __restrict__ w, IterState* st,
                                     double* partials, int bid, int nblk) {
  const double alpha = st->alpha, beta = st->beta;
  const int n = bid * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (n < M.N && !M.fixed[n]) {
    const int64_t N = M.N;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = c * N + n;
      const double pi = sv[i] + beta * p[i];
      const double qi = w[i] + beta * q[i];
      p[i] = pi;
      q[i] = qi;
      z[i] += alpha * pi;
      const double ri = r[i] - alpha * qi;
      r[i] = ri;
      acc += ri * ri;
    }
  }
  double tot;
  if (grid_sum_at(acc, partials, st, &tot, bid, nblk)) {
    st->rsq = tot;
    st->iter += 1;
    if (!isfinite(tot)) {
      st->nonfinite = 1;
      st->done = 1;
    } else if (tot <= st->tolsq * st->nb2) {
      st->converged = 1;
      st->done = 1;
    }
    if (st->iter >= st->max_iter) st->done = 1;
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_step(DevMesh M, double* __restrict__ z, double* __restrict__ r,
                                                    double* __restrict__ p, double* __restrict__ q,
                                                    const double* __restrict__ sv,
                                                    const double* __restrict__ w, IterState* st,
                                                    double* partials) {
  if (st->done) return;
  cg_step_block(M, z, r, p, q, sv, w, st, partials, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- deflated iterations

__global__ void __launch_bounds__(kBlock) k_cg_hvp_dots_defl(DevMesh M, const double* __restrict__ sv,
                                                             const double* __restrict__ fe,
                                                             const double* __restrict__ r, double* __restrict__ w,
                                                             IterState* st, double* partials,
                                                             const double* __restrict__ HW, int k, DeflState* D) {
  if (st->done) return;
  __shared__ double ws[kBlock / 64];
  __shared__ int last;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = M.N, n3 = 3 * N;
  double v[kDeflMax + 2];
#pragma unroll
  for (int j = 0; j < kDeflMax + 2; ++j) v[j] = 0.0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (n < M.N) {
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if (!M.fixed[n]) {
      node_force(M, fe, n, o0, o1, o2);
      const double c = M.mass[n] / (M.h * M.h);
      s0 = sv[n];
      s1 = sv[N + n];
      s2 = sv[2 * N + n];
      o0 += c * s0;
      o1 += c * s1;
      o2 += c * s2;
      if (M.cmask[n]) o2 += M.contact_k * s2;
      v[0] = r[n] * s0 + r[N + n] * s1 + r[2 * N + n] * s2;
      v[1] = o0 * s0 + o1 * s1 + o2 * s2;
#pragma unroll
      for (int j = 0; j < kDeflMax; ++j)
        if (j < k) v[2 + j] = HW[j * n3 + n] * s0 + HW[j * n3 + N + n] * s1 + HW[j * n3 + 2 * N + n] * s2;
    }
    w[n] = o0;
    w[N + n] = o1;
    w[2 * N + n] = o2;
  }
  const int nv = k + 2, nb = gridDim.x;
#pragma unroll
  for (int j = 0; j < kDeflMax + 2; ++j) {
    if (j >= nv) break;
    const double b = block_sum(v[j], ws);
    if (threadIdx.x == 0) __hip_atomic_store(&partials[j * nb + blockIdx.x], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) {
    const uint32_t t = __hip_atomic_fetch_add(&st->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == (uint32_t)nb - 1);
  }
  __syncthreads();
  if (!last) return;
  double tot[kDeflMax + 2];
#pragma unroll
  for (int j = 0; j < kDeflMax + 2; ++j) {
    tot[j] = 0.0;
    if (j >= nv) continue;
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
      a += __hip_atomic_load(&partials[j * nb + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tot[j] = block_sum(a, ws);
  }
  if (threadIdx.x != 0) return;
  __hip_atomic_store(&st->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double gamma = tot[0], delta = tot[1];
  double mc = 0.0;
  for (int i = 0; i < k; ++i) {
    double m = 0.0;
    for (int j = 0; j < k; ++j) m += D->einv[i * kDeflMax + j] * tot[2 + j];
    D->mu[i] = m;
    mc += m * tot[2 + i];
  }
  const bool first = st->iter == 0;
  const double beta = first ? 0.0 : gamma / st->rs;
  const double den = (first ? delta : delta - beta * gamma / st->alpha) - mc;
  if (!(den > 0.0) || !isfinite(den) || !isfinite(gamma)) {
    st->curvature = 1;
    st->done = 1;
  } else {
    st->beta = beta;
    st->alpha = gamma / den;
    st->rs = gamma;
  }
}

__global__ void __launch_bounds__(kBlock) k_cg_step_defl(DevMesh M, double* __restrict__ z, double* __restrict__ r,
                                                         double* __restrict__ p, double* __restrict__ q,
                                                         const double* __restrict__ sv,
                                                         const double* __restrict__ w, IterState* st,
                                                         double* partials, const double* __restrict__ W,
                                                         const double* __restrict__ HW, int k,
                                                         const DeflState* __restrict__ D) {
  if (st->done) return;
  const double alpha = st->alpha, beta = st->beta;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (n < M.N && !M.fixed[n]) {
    const int64_t N = M.N, n3 = 3 * N;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = c * N + n;
      double pi = sv[i] + beta * p[i], qi = w[i] + beta * q[i];
      for (int j = 0; j < k; ++j) {
        const double m = D->mu[j];
        pi -= m * W[j * n3 + i];
        qi -= m * HW[j * n3 + i];
      }
      p[i] = pi;
      q[i] = qi;
      z[i] += alpha * pi;
      const double ri = r[i] - alpha * qi;
      r[i] = ri;
      acc += ri * ri;
    }
  }
  double tot;
  if (grid_sum(acc, partials, st, &tot)) {
    st->rsq = tot;
    st->iter += 1;
    if (!isfinite(tot)) {
      st->nonfinite = 1;
      st->done = 1;
    } else if (tot <= st->tolsq * st->nb2) {
      st->converged = 1;
      st->done = 1;
    }
    if (st->iter >= st->max_iter) st->done = 1;
  }
}

// Partial dot products of chunk blockIdx.x for vector blockIdx.y.
__global__ void __launch_bounds__(kBlock) k_multi_dot_part(const double* __restrict__ X, const double* __restrict__ y,
                                                           int64_t n, int64_t chunk, double* __restrict__ partials) {
  __shared__ double ws[kBlock / 64];
  const double* x = X + (int64_t)blockIdx.y * n;
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
  double a = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) a += x[i] * y[i];
  a = block_sum(a, ws);
  if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = a;
}

__global__ void __launch_bounds__(kBlock) k_multi_dot_sum(const double* __restrict__ partials, int chunks,
                                                          double* __restrict__ out) {
  __shared__ double ws[kBlock / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < chunks; i += blockDim.x) a += partials[(int64_t)blockIdx.x * chunks + i];
  a = block_sum(a, ws);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

__global__ void __launch_bounds__(kBlock) k_multi_axpy(double* __restrict__ y, const double* __restrict__ X, int cnt,
                                                       const double* __restrict__ c, int64_t n, double sign) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int j = 0; j < cnt; ++j) a += c[j] * X[(int64_t)j * n + i];
  y[i] += sign * a;
}

// ---------------------------------------------------------------- batched iterations
//
// The same three steps over several handles' conjugate-gradient solves in one
// launch: the blocks of slot j are [block0, block0 + nblk) of the grid, and
// each block runs exactly the arithmetic of the single-handle kernel's block
// (bid = its index within the slot), so a slot's results do not depend on the
// other slots of the batch.  A slot whose solve has finished does nothing.

__device__ inline int batch_slot(const BatchCgSlot* __restrict__ slots, int nslots, int elem) {
  const int b = blockIdx.x;
  int j = 0;
  for (int i = 1; i < nslots; ++i)
    if ((elem ? slots[i].elem_block0 : slots[i].node_block0) <= b) j = i;
  return j;
}

__global__ void __launch_bounds__(kBlock) k_batch_elem_hvp(const BatchCgSlot* __restrict__ slots, int nslots) {
  const int j = batch_slot(slots, nslots, 1);
  const BatchCgSlot& S = slots[j];
  if (S.st->done) return;
  elem_hvp_block(S.M, S.sv, S.cache, S.fe, blockIdx.x - S.elem_block0);
}

__global__ void __launch_bounds__(kBlock) k_batch_cg_hvp_dots(const BatchCgSlot* __restrict__ slots, int nslots) {
  const int j = batch_slot(slots, nslots, 0);
  const BatchCgSlot& S = slots[j];
  if (S.st->done) return;
  cg_hvp_dots_block(S.M, S.sv, S.fe, S.r, S.w, S.st, S.partials, blockIdx.x - S.node_block0, S.node_blocks);
}

__global__ void __launch_bounds__(kBlock) k_batch_cg_step(const BatchCgSlot* __restrict__ slots, int nslots) {
  const int j = batch_slot(slots, nslots, 0);
  const BatchCgSlot& S = slots[j];
  if (S.st->done) return;
  cg_step_block(S.M, S.z, S.r, S.p, S.q, S.sv, S.w, S.st, S.partials, blockIdx.x - S.node_block0,
                S.node_blocks);
}

// Backward epilogue: dL/dy = M z/h^2 (eq:chain_rule); through
// y = x + h v + h^2 M^{-1}(M g + f_fric(x, v)) and v_{i+1} = (x_{i+1} - x)/h.
// dL/df_fric = h^2 M^{-1} dL/dy = z.
__global__ void __launch_bounds__(kBlock) k_adj_epilogue(DevMesh M, const double* __restrict__ x,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ z,
                                                         const double* __restrict__ gv_next,
                                                         double* __restrict__ gx,
                                                         double* __restrict__ gv, const IterState* gate) {
  if (gate && gate->curvature) return;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= M.N) return;
  const int64_t N = M.N;
  const double h = M.h;
  const bool fixed = M.fixed[n];
  const double c = fixed ? 0.0 : M.mass[n] / (h * h);
  double dy[3], ox[3], ov[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dy[k] = fixed ? 0.0 : c * z[k * N + n];
    ox[k] = dy[k] - gv_next[k * N + n] / h;
    ov[k] = h * dy[k];
  }
  if (!fixed && M.contact[n] && M.friction_mu > 0.0) {
    const double zz = x[2 * N + n];
    const double k = M.contact_k, mu = M.friction_mu;
    const double fn = k * fmax(0.0, -zz);
    const double dfn = zz < 0.0 ? -k : 0.0;
    const double v0 = v[n], v1 = v[N + n];
    const double s2 = v0 * v0 + v1 * v1 + M.friction_eps * M.friction_eps;
    const double s = sqrt(s2);
    const double w0 = z[n], w1 = z[N + n];
    ox[2] += -mu * dfn * (w0 * v0 + w1 * v1) / s;
    const double a = -mu * fn / s, b = mu * fn / (s * s2);
    const double vw = v0 * w0 + v1 * w1;
    ov[0] += a * w0 + b * v0 * vw;
    ov[1] += a * w1 + b * v1 * vw;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gx[k * N + n] = ox[k];
    gv[k * N + n] = ov[k];
  }
}

// dL/dE_e += -V_q/(1+nu) sum_q <G_q z, F_q - R_q>;  dL/dr_e = sum_q w_m <G_m,q z, n_q>.
__global__ void __launch_bounds__(kBlock) k_grad_params(DevMesh M, const double* __restrict__ xn,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ cache,
                                                        double* __restrict__ g_youngs,
                                                        double* __restrict__ g_act, const IterState* gate) {
  if (gate && gate->curvature) return;
  __shared__ ElemTile T;
  __shared__ double Zs[kElemsPerBlock][8][3];
  __shared__ double red[kElemsPerBlock][8][2];
  const int le = threadIdx.x >> 3, q = threadIdx.x & 7;
  const int e = blockIdx.x * kElemsPerBlock + le;
  const bool valid = e < M.E;
  const GradTable G = grad_table(M.dx);
  gather_nodes(M, xn, T, le, q, e, valid);
  if (valid) {
    const int nd = M.conn[(int64_t)q * M.E + e];
    Zs[le][q][0] = z[nd];
    Zs[le][q][1] = z[(int64_t)M.N + nd];
    Zs[le][q][2] = z[2 * (int64_t)M.N + nd];
  }
  __syncthreads();
  double ge = 0.0, ga = 0.0;
  if (valid) {
    const int64_t Q = 8 * (int64_t)M.E, qi = 8 * (int64_t)e + q;
    double F[9], dF[9];
    deformation_gradient(T, le, q, G, F);
#pragma unroll
    for (int i = 0; i < 9; ++i) dF[i] = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double b0 = bgrad(q, 0, a, G), b1 = bgrad(q, 1, a, G), b2 = bgrad(q, 2, a, G);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double zi = Zs[le][a][i];
        dF[3 * i + 0] += zi * b0;
        dF[3 * i + 1] += zi * b1;
        dF[3 * i + 2] += zi * b2;
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) ge += dF[i] * (F[i] - cache[i * Q + qi]);
    ge *= -M.Vq / (1.0 + M.nu);
    if (M.wv_e) {
      // through the volume weight: -dw_v/dE <G z, F - D>, D = R V diag(Dd) V^T (= R where det F <= 0)
      double R[9], V[9], Dd[3], D[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        R[i] = cache[i * Q + qi];
        V[i] = cache[(kVolV + i) * Q + qi];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) Dd[i] = cache[(kVolD + i) * Q + qi];
      volume_matrix(R, V, Dd, D);
      double gv = 0.0;
#pragma unroll
      for (int i = 0; i < 9; ++i) gv += dF[i] * (F[i] - D[i]);
      ge -= M.dwv_dE * gv;
    }
    if (M.muscle_k > 0.0) {
      const double m0 = M.fiber[0], m1 = M.fiber[1], m2 = M.fiber[2];
      const double d0 = dF[0] * m0 + dF[1] * m1 + dF[2] * m2;
      const double d1 = dF[3] * m0 + dF[4] * m1 + dF[5] * m2;
      const double d2 = dF[6] * m0 + dF[7] * m1 + dF[8] * m2;
      ga = M.muscle_k * M.Vq *
           (d0 * cache[15 * Q + qi] + d1 * cache[16 * Q + qi] + d2 * cache[17 * Q + qi]);
    }
    red[le][q][0] = ge;
    red[le][q][1] = ga;
  }
  __syncthreads();
  if (valid && q == 0) {
    double se = 0.0, sa = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      se += red[le][k][0];
      sa += red[le][k][1];
    }
    if (g_youngs) g_youngs[e] += se;
    if (g_act) g_act[e] = sa;
  }
}

// out = a x + b y over 3N entries (y may be null: out = a x)
__global__ void __launch_bounds__(kBlock) k_lincomb(int64_t n, double* out, double a,
                                                    const double* x, double b,
                                                    const double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void __launch_bounds__(kBlock) k_warm_select(int64_t n, double* __restrict__ z0, double* __restrict__ r,
                                                        const double* __restrict__ b, const IterState* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || w[1].nb2 < w[0].nb2) return;
  z0[i] = 0.0;
  r[i] = b[i];
}

__global__ void __launch_bounds__(kBlock) k_fill(int64_t n, double* __restrict__ out, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

// ------------------------------------------------------------------ launchers

static inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

void launch_lincomb(hipStream_t s, int64_t n, double* out, double a, const double* x, double b,
                    const double* y) {
  hipLaunchKernelGGL(k_lincomb, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, out, a, x, b, y);
}

// Occupies the stream for a bounded time (a fixed number of s_sleep periods of
// 64 x 127 shader clocks each) so that the launches enqueued behind it are all
// in the queue when it ends; it touches no memory and always finishes.
__global__ void k_hold(int periods) {
  for (int i = 0; i < periods; ++i) __builtin_amdgcn_s_sleep(127);
}

void launch_hold(hipStream_t s, int periods) {
  hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, s, periods);
}

void launch_fill(hipStream_t s, int64_t n, double* out, double v) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, out, v);
}

void launch_warm_select(hipStream_t s, int64_t n, double* z0, double* r, const double* b, const IterState* w) {
  hipLaunchKernelGGL(k_warm_select, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, z0, r, b, w);
}

void launch_reset(hipStream_t s, IterState* st, double tolsq, int max_iter) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, st, tolsq, max_iter);
}

void launch_prologue(const DevMesh& M, hipStream_t s, const double* x, const double* v, double* y,
                     double* xn, IterState* st, double* partials, double abs_tol_rel) {
  hipLaunchKernelGGL(k_prologue, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, x, v, y, xn, st,
                     partials, abs_tol_rel);
}

void launch_elem_forces(const DevMesh& M, hipStream_t s, const double* x, const double* act,
                        double* fe, double* R_out, IterState* st) {
  if (M.corners == 4) return launch_tet_forces(M, s, x, fe, R_out, st);
  const int nb = (M.E + kElemsPerBlock - 1) / kElemsPerBlock;
  DPD_LAUNCH(k_elem_forces, dim3(nb), dim3(kBlock), 0, s, M, x, act, fe, R_out, st);
}

void launch_node_residual(const DevMesh& M, hipStream_t s, const double* x, const double* y,
                          const double* fe, double* r, IterState* st, double* partials, int k,
                          int max_iter, int fixed_iters) {
  hipLaunchKernelGGL(k_node_residual, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, x, y, fe, r, st,
                     partials, k, max_iter, fixed_iters);
}

void launch_velocity(const DevMesh& M, hipStream_t s, const double* x, const double* xn, double* vn) {
  hipLaunchKernelGGL(k_velocity, dim3(blocks_for(3 * (int64_t)M.N)), dim3(kBlock), 0, s, M.N,
                     1.0 / M.h, x, xn, vn);
}

void launch_zero_fixed(const DevMesh& M, hipStream_t s, double* v) {
  hipLaunchKernelGGL(k_zero_fixed, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, v);
}





void launch_adj_cache(const DevMesh& M, hipStream_t s, const double* x, const double* act,
                      double* cache, IterState* st, const IterState* gate) {
  if (M.corners == 4) return launch_tet_adj_cache(M, s, x, cache, st, gate);
  const int nb = (M.E + kElemsPerBlock - 1) / kElemsPerBlock;
  hipLaunchKernelGGL(k_adj_cache, dim3(nb + blocks_for(M.N)), dim3(kBlock), 0, s, M, x, act, cache, st, gate,
                     nb);
}

// Newton forward step, inner-solve set-up on the device (no host round trip):
// unless the outer iteration has finished (then the inner state is marked
// done, so the solve and the update that follow do nothing), the forcing term
// eta (fixed, or Eisenstat-Walker "choice 2": 0.9 (|g_k| / |g_{k-1}|)^2,
// safeguarded by 0.9 eta_{k-1}^2 above 0.1, capped at eta_max, and kept above
// half the outer tolerance relative to |g_k|) and the iteration cap.
__global__ void k_newton_inner(IterState* outer, IterState* inner, double eta_max, int adaptive,
                               double rel_tol, int inner_max_iter, int max_iter) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (inner->aborted) {   // a fused solve of this batch failed: stop the step, keep the flag
    outer->aborted = 1;
    outer->done = 1;
  }
  inner->r0sq = inner->rsq = inner->atolsq = 0.0;
  inner->nb2 = inner->rs = inner->pq = inner->alpha = inner->beta = inner->acc = 0.0;
  inner->iter = inner->converged = inner->nonfinite = inner->curvature = inner->inverted = 0;
  inner->aborted = 0;
  inner->counter = 0u;
  if (outer->done || outer->solves >= max_iter) {
    outer->done = 1;
    inner->done = 1;
    return;
  }
  inner->done = 0;
  double eta = eta_max;
  const double gk = sqrt(outer->rsq);
  if (adaptive) {
    if (outer->g_prev > 0.0 && gk > 0.0) {
      double e = 0.9 * (gk / outer->g_prev) * (gk / outer->g_prev);
      const double safe = 0.9 * outer->eta * outer->eta;
      if (safe > 0.1) e = fmax(e, safe);
      eta = fmin(eta_max, fmax(e, 0.5 * rel_tol * sqrt(outer->r0sq) / gk));
    }
    outer->g_prev = gk;
  }
  outer->eta = eta;
  inner->tolsq = eta * eta;
  inner->max_iter = max(1, min(inner_max_iter, max_iter - outer->solves));
}

// x += z after the inner solve, and the solve's iterations added to the
// outer count (unless the outer iteration had already finished).
__global__ void __launch_bounds__(kBlock) k_newton_update(int64_t n3, IterState* outer, const IterState* inner,
                                                          double* __restrict__ xn, const double* __restrict__ z) {
  if (outer->done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) xn[i] += z[i];
  if (i == 0) outer->solves += max(1, inner->iter);
}

void launch_newton_inner(hipStream_t s, IterState* outer, IterState* inner, double eta_max, int adaptive,
                         double rel_tol, int inner_max_iter, int max_iter) {
  hipLaunchKernelGGL(k_newton_inner, dim3(1), dim3(64), 0, s, outer, inner, eta_max, adaptive, rel_tol,
                     inner_max_iter, max_iter);
}

void launch_newton_update(hipStream_t s, int64_t n3, IterState* outer, const IterState* inner, double* xn,
                          const double* z) {
  hipLaunchKernelGGL(k_newton_update, dim3((unsigned)((n3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n3, outer,
                     inner, xn, z);
}

void launch_elem_hvp(const DevMesh& M, hipStream_t s, const double* p, const double* cache,
                     double* fe, const IterState* st) {
  if (M.corners == 4) return launch_tet_hvp(M, s, p, cache, fe, st);
  const int nb = (M.E + kElemsPerBlock - 1) / kElemsPerBlock;
  DPD_LAUNCH(k_elem_hvp, dim3(nb), dim3(kBlock), 0, s, M, p, cache, fe, st);
}

void launch_node_hvp(const DevMesh& M, hipStream_t s, const double* p, const double* fe,
                     const double* rhs, double* out, IterState* st, double* partials, int mode, int k,
                     int max_iter) {
  hipLaunchKernelGGL(k_node_hvp, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, p, fe, rhs, out,
                     st, partials, mode, k, max_iter);
}

void launch_dot(const DevMesh& M, hipStream_t s, const double* a, const double* b, IterState* st,
                double* partials, int what) {
  hipLaunchKernelGGL(k_dot, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, a, b, st, partials, what);
}


void launch_cg_hvp_dots(const DevMesh& M, hipStream_t s, const double* sv, const double* fe,
                        const double* r, double* w, IterState* st, double* partials) {
  hipLaunchKernelGGL(k_cg_hvp_dots, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, sv, fe, r, w, st,
                     partials);
}

void launch_cg_step(const DevMesh& M, hipStream_t s, double* z, double* r, double* p, double* q,
                    const double* sv, const double* w, IterState* st, double* partials) {
  hipLaunchKernelGGL(k_cg_step, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, z, r, p, q, sv, w, st,
                     partials);
}


void launch_batch_cg_iteration_tail(const BatchCgSlot* slots, int nslots, int elem_blocks, int node_blocks,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_batch_elem_hvp, dim3(elem_blocks), dim3(kBlock), 0, s, slots, nslots);
  hipLaunchKernelGGL(k_batch_cg_hvp_dots, dim3(node_blocks), dim3(kBlock), 0, s, slots, nslots);
  hipLaunchKernelGGL(k_batch_cg_step, dim3(node_blocks), dim3(kBlock), 0, s, slots, nslots);
}

void launch_cg_hvp_dots_defl(const DevMesh& M, hipStream_t s, const double* sv, const double* fe, const double* r,
                             double* w, IterState* st, double* partials, const double* HW, int k, DeflState* D) {
  hipLaunchKernelGGL(k_cg_hvp_dots_defl, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, sv, fe, r, w, st, partials,
                     HW, k, D);
}

void launch_cg_step_defl(const DevMesh& M, hipStream_t s, double* z, double* r, double* p, double* q,
                         const double* sv, const double* w, IterState* st, double* partials, const double* W,
                         const double* HW, int k, const DeflState* D) {
  hipLaunchKernelGGL(k_cg_step_defl, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, z, r, p, q, sv, w, st, partials,
                     W, HW, k, D);
}

void launch_multi_dot(hipStream_t s, const double* X, int cnt, const double* y, int64_t n, double* partials,
                      double* out) {
  const int chunks = (int)std::min<int64_t>(256, (n + kBlock * 4 - 1) / (kBlock * 4));
  const int64_t chunk = (n + chunks - 1) / chunks;
  hipLaunchKernelGGL(k_multi_dot_part, dim3(chunks, cnt), dim3(kBlock), 0, s, X, y, n, chunk, partials);
  hipLaunchKernelGGL(k_multi_dot_sum, dim3(cnt), dim3(kBlock), 0, s, partials, chunks, out);
}

void launch_multi_axpy(hipStream_t s, double* y, const double* X, int cnt, const double* c, int64_t n, double sign) {
  hipLaunchKernelGGL(k_multi_axpy, dim3(blocks_for(n)), dim3(kBlock), 0, s, y, X, cnt, c, n, sign);
}

void launch_adj_epilogue(const DevMesh& M, hipStream_t s, const double* x, const double* v,
                         const double* z, const double* gv_next, double* gx, double* gv, const IterState* gate) {
  hipLaunchKernelGGL(k_adj_epilogue, dim3(blocks_for(M.N)), dim3(kBlock), 0, s, M, x, v, z, gv_next,
                     gx, gv, gate);
}

void launch_grad_params(const DevMesh& M, hipStream_t s, const double* xn, const double* z,
                        const double* cache, double* g_youngs, double* g_act, const IterState* gate) {
  if (M.corners == 4) return launch_tet_grad_params(M, s, xn, z, cache, g_youngs, gate);
  const int nb = (M.E + kElemsPerBlock - 1) / kElemsPerBlock;
  hipLaunchKernelGGL(k_grad_params, dim3(nb), dim3(kBlock), 0, s, M, xn, z, cache, g_youngs, g_act, gate);
}

}  // namespace dpd
