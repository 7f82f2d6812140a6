// The inner loop of a time step with contact in one cooperative launch, for
// meshes whose reduced inverse W = (A_{C̄×C̄})^{-1} is held dense (Sec.
// Contact; Alg. 3's PD iterations, mode 0, or Alg. 5's adjoint iterations,
// mode 1).  Workgroup b owns the internal rows [b R, b R + R) (the fused
// solver's partition, with its lists of the elements touching those rows).
// One iteration:
//   phase 1  the workgroup's elements (one per 8 lanes, a Gauss point and a
//            corner per lane): mode 0, the projections at x_k (corotated,
//            muscle); mode 1, the adjoint stress differential at z_k from the
//            cached rotations; corner forces in LDS; then the residual of the
//            own rows (zero on the contact set; formed as the residual kernels
//            form it, in the same order), published with the rows' partial
//            norm.  (Elements shared by workgroups are evaluated in each, so
//            Gauss points with det F <= 0 are not counted here.)
//   barrier
//   phase 2  every workgroup gathers the whole residual into LDS and sums the
//            partial norms in workgroup order (the same bits everywhere, so
//            every workgroup takes the same stopping decision: mode 0 against
//            the first norm and the absolute floor, mode 1 against |xbar|),
//            then updates its own rows, x <- x - W r, and publishes them.
//   wait     for the workgroups owning rows at its element corners (instead of
//            a second barrier; the residual and the partial norms are double-
//            buffered by iteration parity for the workgroups still reading)
// The iterate's own rows live in LDS between iterations.  Workgroup 0 records
// the iteration state.  The data workgroups exchange (iterate, residual,
// partial norms) is written and read with device-coherent accesses
// (agent-scope relaxed atomics), so the barrier needs no cache write-back or
// invalidation and W stays cached.  The barrier has two levels (a counter per
// group of workgroups, one flag per group polled by wave 0 of every
// workgroup) and a bounded wait: a workgroup that times out raises the abort
// word, on which every workgroup leaves.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "contact.hpp"
#include "device.hpp"
#include "device_math.hpp"

namespace dpd {

namespace {

constexpr uint32_t kFusedSpin = 1u << 22;  // polls (with s_sleep) before a barrier gives up (seconds)
constexpr int kFBarGroups = 8;
constexpr int kFBarStride = 64;                 // uint32 words between group counters (own cache lines)
constexpr int kFBarFlags = 16;                  // first group flag; word 1 is the abort word

__device__ inline double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct FusedContact {
  DevMesh M;               // contact set and Dirichlet nodes masked
  int32_t n, rows;         // free rows; rows per workgroup
  int32_t mode, max_iter;  // 0: forward PD, 1: adjoint
  const double* W;         // [n][n]
  double* x0;              // [3][N] the iterate (input and output)
  const double* y;         // mode 0: y; mode 1: xbar
  const double* act;       // mode 0: muscle actuation or null
  const double* cache;     // mode 1: per-Gauss-point rotation cache
  IterState* st;
  uint32_t* bar;           // [kContactBarWords] group counters, flags, abort word
};

// Every wave waits for its own device-coherent stores, then workgroup b counts
// in at group b mod 8; the arrival that completes the group for this round
// raises the group's flag to the round; wave 0 polls the flags (one load).
__device__ bool fused_barrier(uint32_t* bar, uint32_t& round) {
  __shared__ int ok;
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  round += 1;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const uint32_t G = gridDim.x, g = blockIdx.x % kFBarGroups;
    const uint32_t ngroups = G < (uint32_t)kFBarGroups ? G : (uint32_t)kFBarGroups;
    if (lane == 0) {
      const uint32_t gsize = G / kFBarGroups + (g < G % kFBarGroups ? 1u : 0u);
      const uint32_t t =
          __hip_atomic_fetch_add(&bar[kFBarStride * (g + 1)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (t + 1 == round * gsize)
        __hip_atomic_store(&bar[kFBarFlags + g], round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int good = 1;
    for (uint32_t spin = 0;; ++spin) {
      const uint32_t v = (uint32_t)lane < ngroups
                             ? __hip_atomic_load(&bar[kFBarFlags + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : round;
      if (__all(v >= round)) break;
      const uint32_t ab = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ab != 0u || spin >= kFusedSpin) {
        if (lane == 0) __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// After phase 2: once its own rows of the iterate are stored, the workgroup
// waits for its own stores, raises its ready count to seq, and waits until the
// ready counts of the workgroups owning rows at its element corners (nbr)
// reach seq.  Bounded like the barrier, sharing its abort word.
__device__ bool publish_wait(uint32_t* ready, const int32_t* __restrict__ nbr, int nnb, uint32_t seq,
                             uint32_t* bar) {
  __shared__ int ok;
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(&ready[blockIdx.x], seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = 1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nnb; i += blockDim.x) {
    const int g = nbr[i];
    for (uint32_t spin = 0;; ++spin) {
      if (__hip_atomic_load(&ready[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= seq) break;
      if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spin >= kFusedSpin) {
        __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return ok != 0;
}

__global__ void __launch_bounds__(kDenseBlock) k_contact_fused(FusedContact P, DenseCG D, ClockArg ck) {
  if (P.st->done) return;
  clock_enter(ck);
  extern __shared__ double rv[];  // [3][n] the residual, internal order
  __shared__ ElemTileT<kDenseElems> Tl;
  __shared__ double fl[kDenseElems][8][3];  // corner forces
  __shared__ double ws[kDenseBlock / 64];
  __shared__ double tot_s;
  __shared__ double own_x[3 * kDenseMaxRows], own_y[3 * kDenseMaxRows];
  __shared__ double row_c[kDenseMaxRows];
  __shared__ int row_node[kDenseMaxRows], row_inc[kDenseMaxRows][8], row_free[kDenseMaxRows];
  __shared__ int row_pen[kDenseMaxRows];
  constexpr int MR = kDenseMaxRows;
  const DevMesh& M = P.M;
  const int n = P.n, tid = threadIdx.x, b = blockIdx.x, G_ = gridDim.x;
  const int64_t N = M.N;
  const int j0 = min(n, b * P.rows), j1 = min(n, j0 + P.rows), R = j1 - j0;
  const GradTable G = grad_table(M.dx);
  const double tolsq = P.st->tolsq, atolsq = P.st->atolsq, nb2 = P.st->nb2;
  // published residual [2][3][n] and partial norms [2][G], by iteration parity:
  // a workgroup may start iteration k + 1 while others still read iteration k's
  const int32_t* nbrs = D.nbr + D.nbr_off[b];
  const int nnb = D.nbr_off[b + 1] - D.nbr_off[b];
  uint32_t pub = 0;

  // the workgroup's elements and rows
  const int e0 = D.blk_eoff[b], ne = D.blk_eoff[b + 1] - e0;
  const int le = tid >> 3, a = tid & 7;
  const bool ev = le < ne;
  const int el = ev ? D.blk_elems[e0 + le] : 0;
  const int corner = ev ? M.conn[(int64_t)a * M.E + el] : 0;
  if (tid < R) {
    const int node = D.perm[j0 + tid];
    row_node[tid] = node;
    row_c[tid] = M.mass[node] / (M.h * M.h);
    row_free[tid] = M.fixed[node] ? 0 : 1;  // the contact set is masked
    row_pen[tid] = P.mode == 0 ? (M.contact[node] ? 1 : 0) : (M.cmask[node] ? 1 : 0);
#pragma unroll
    for (int q = 0; q < 8; ++q) row_inc[tid][q] = D.row_inc[8 * (j0 + tid) + q];
  }
  __syncthreads();
  if (tid < 3 * R) {
    const int c = tid / R, i = tid % R;
    const int64_t node = row_node[i];
    own_x[c * MR + i] = P.x0[c * N + node];
    own_y[c * MR + i] = P.y[c * N + node];
  }
  const int lane = tid & 63, wid = tid >> 6, waves = blockDim.x >> 6;
  uint32_t round = 0;
  double r0sq = 0.0;
  int k = 0;
  for (;; ++k) {
    double* rg = D.r + (k & 1) * 3 * n;
    double* part = D.part + (k & 1) * G_;
    // ---- phase 1: element corners of the iterate (device-coherent loads;
    // Dirichlet corners: the rest position, or 0 for the adjoint direction);
    // the adjoint's cache entries of this lane's Gauss point in the same round
    double cq[19];
    if (ev && P.mode == 1) load_gauss_cache(M, P.cache, el, a, cq);
    if (ev) {
      double u0, u1, u2;
      if (D.inv[corner] < 0) {
        u0 = P.mode == 0 ? M.X[corner] : 0.0;
        u1 = P.mode == 0 ? M.X[N + corner] : 0.0;
        u2 = P.mode == 0 ? M.X[2 * N + corner] : 0.0;
      } else {
        u0 = ld_dev(&P.x0[corner]);
        u1 = ld_dev(&P.x0[N + corner]);
        u2 = ld_dev(&P.x0[2 * N + corner]);
      }
      Tl.xs[le][a][0] = u0;
      Tl.xs[le][a][1] = u1;
      Tl.xs[le][a][2] = u2;
    }
    __syncthreads();
    if (ev) {
      const int q = a;
      if (P.mode == 1) {
        double dF[9];
        deformation_gradient(Tl, le, q, G, dF);
        hvp_stress_from_dF(M, Tl.Ps[le][q], dF, M.w_e[el], cq);
      } else {
        double F[9], Rm[9];
        deformation_gradient(Tl, le, q, G, F);
        if (M.local32)
          closest_rotation_mixed(F, Rm);
        else
          closest_rotation(F, Rm);
        const double w = M.w_e[el];
        double* Ps = Tl.Ps[le][q];
#pragma unroll
        for (int i = 0; i < 9; ++i) Ps[i] = w * (F[i] - Rm[i]);
        if (M.muscle_k > 0.0) {
          // fibre projection onto |p| = r (supplemental, muscle fibers)
          const double m0 = M.fiber[0], m1 = M.fiber[1], m2 = M.fiber[2];
          const double f0 = F[0] * m0 + F[1] * m1 + F[2] * m2;
          const double f1 = F[3] * m0 + F[4] * m1 + F[5] * m2;
          const double f2 = F[6] * m0 + F[7] * m1 + F[8] * m2;
          const double r = P.act ? P.act[el] : 1.0;
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
          Ps[0] += d0 * m0; Ps[1] += d0 * m1; Ps[2] += d0 * m2;
          Ps[3] += d1 * m0; Ps[4] += d1 * m1; Ps[5] += d1 * m2;
          Ps[6] += d2 * m0; Ps[7] += d2 * m1; Ps[8] += d2 * m2;
        }
      }
    }
    __syncthreads();
    if (ev) corner_force(Tl, le, a, G, fl[le][a][0], fl[le][a][1], fl[le][a][2]);
    __syncthreads();
    // own rows' residual, as the residual kernels form it (same order)
    double acc = 0.0;
    if (tid < R) {
      const int i = tid;
      double r0 = 0.0, r1 = 0.0, r2 = 0.0;
      if (row_free[i]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int code = row_inc[i][q];
          if (code >= 0) {
            r0 += fl[code >> 3][code & 7][0];
            r1 += fl[code >> 3][code & 7][1];
            r2 += fl[code >> 3][code & 7][2];
          }
        }
        const double c = row_c[i];
        const double u0 = own_x[i], u1 = own_x[MR + i], u2 = own_x[2 * MR + i];
        if (P.mode == 0) {
          r0 += c * (u0 - own_y[i]);
          r1 += c * (u1 - own_y[MR + i]);
          r2 += c * (u2 - own_y[2 * MR + i]);
          if (row_pen[i] && u2 < 0.0) r2 += M.contact_k * u2;
        } else {
          r0 += c * u0;
          r1 += c * u1;
          r2 += c * u2;
          if (row_pen[i]) r2 += M.contact_k * u2;
          r0 -= own_y[i];
          r1 -= own_y[MR + i];
          r2 -= own_y[2 * MR + i];
        }
        acc = r0 * r0 + r1 * r1 + r2 * r2;
      }
      st_dev(&rg[j0 + i], r0);
      st_dev(&rg[n + j0 + i], r1);
      st_dev(&rg[2 * n + j0 + i], r2);
    }
    const double bsum = block_sum(acc, ws);
    if (tid == 0) st_dev(&part[b], bsum);
    if (!fused_barrier(P.bar, round)) return;
    // ---- phase 2: the whole residual and its norm, the decision, own rows.
    // Wave 0 issues its loads of the partial norms (at most 4 per lane, G <=
    // 256) together with its share of the residual.
    double pv[4] = {0.0, 0.0, 0.0, 0.0};
    if (tid < 64) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = 64 * u + lane;
        if (g < G_) pv[u] = ld_dev(&part[g]);
      }
    }
    for (int i = tid; i < 3 * n; i += blockDim.x) rv[i] = ld_dev(&rg[i]);
    if (tid < 64) {
      // fixed order: each lane's partials, then the wave's sum
      const double t = wave_sum(((pv[0] + pv[1]) + pv[2]) + pv[3]);
      if (tid == 0) tot_s = t;
    }
    __syncthreads();
    const double tot = tot_s;
    if (k == 0) r0sq = tot;
    int done = 0, conv = 0, bad = 0;
    if (!isfinite(tot)) {
      bad = 1;
      done = 1;
    } else if (P.mode == 0 ? (tot <= tolsq * r0sq || tot <= atolsq) : (tot <= tolsq * nb2)) {
      conv = 1;
      done = 1;
    }
    if (k >= P.max_iter) done = 1;
    if (b == 0 && tid == 0) {
      P.st->rsq = tot;
      P.st->iter = k;
      if (P.mode == 0 && k == 0) P.st->r0sq = tot;
      if (bad) P.st->nonfinite = 1;
      if (conv) P.st->converged = 1;
      if (done) P.st->done = 1;
    }
    if (done) break;
    for (int i = wid; i < R; i += waves) {
      const double* row = P.W + (int64_t)(j0 + i) * n;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int jb = lane; jb < n; jb += 8 * 64) {
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = jb + 64 * u;
          w[u] = j < n ? row[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = jb + 64 * u;
          if (j < n) {
            s0 += w[u] * rv[j];
            s1 += w[u] * rv[n + j];
            s2 += w[u] * rv[2 * n + j];
          }
        }
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      if (lane == 0) {
        const int64_t node = row_node[i];
        const double x0n = own_x[i] - s0, x1n = own_x[MR + i] - s1, x2n = own_x[2 * MR + i] - s2;
        own_x[i] = x0n;
        own_x[MR + i] = x1n;
        own_x[2 * MR + i] = x2n;
        st_dev(&P.x0[node], x0n);
        st_dev(&P.x0[N + node], x1n);
        st_dev(&P.x0[2 * N + node], x2n);
      }
    }
    if (!publish_wait(D.ready, nbrs, nnb, ++pub, P.bar)) return;
  }
  ClockArg c2 = ck;
  c2.bytes = ck.bytes * (double)(k + 1);
  c2.flops = ck.flops * (double)(k + 1);
  clock_exit(c2);
}

// Alg. 5's system solved by conjugate gradients preconditioned with the set's
// reduced inverse W (the quasi-Newton acceleration of the adjoint, on the
// reduced system; Chronopoulos-Gear arrangement, one exchange of partial sums
// per iteration).  Same partition and exchange as k_contact_fused; per
// iteration, with the whole residual r_k in LDS:
//   own rows of s = W r_k, published; wait for the neighbours' rows;
//   w = (A - dA) s on the own rows (elements touching them; zero on the set),
//   partial sums r.s, s.w, r.r published;  barrier;
//   every workgroup sums the partials in workgroup order (same bits), stops
//   when |r_k| <= tol |xbar| (or at the cap, or on non-positive curvature,
//   recorded for the host's fallback), else updates its rows of p, q, z, r and
//   publishes r;  barrier;  gather r_{k+1}.
// z (own rows, in LDS) is written to x0 at the end.
__global__ void __launch_bounds__(kDenseBlock) k_contact_fused_cg(FusedContact P, DenseCG D, ClockArg ck) {
  if (P.st->done) return;
  clock_enter(ck);
  extern __shared__ double rv[];  // [3][n] r_k, internal order
  __shared__ ElemTileT<kDenseElems> Tl;
  __shared__ double fl[kDenseElems][8][3];
  __shared__ double ws[kDenseBlock / 64];
  __shared__ double sums[3];
  constexpr int MR = kDenseMaxRows;
  __shared__ double own_z[3 * MR], own_r[3 * MR], own_p[3 * MR], own_q[3 * MR], own_s[3 * MR];
  __shared__ double row_c[MR];
  __shared__ int row_node[MR], row_inc[MR][8], row_free[MR], row_pen[MR];
  const DevMesh& M = P.M;
  const int n = P.n, tid = threadIdx.x, b = blockIdx.x, G_ = gridDim.x;
  const int64_t N = M.N;
  const int j0 = min(n, b * P.rows), j1 = min(n, j0 + P.rows), R = j1 - j0;
  const GradTable G = grad_table(M.dx);
  const double tolsq = P.st->tolsq, nb2 = P.st->nb2;
  double* rg = D.r;      // [3][n] published r
  double* sg = D.q;      // [3][n] published s
  double* part = D.part; // [3][G] published partial sums
  const int32_t* nbrs = D.nbr + D.nbr_off[b];
  const int nnb = D.nbr_off[b + 1] - D.nbr_off[b];
  const int e0 = D.blk_eoff[b], ne = D.blk_eoff[b + 1] - e0;
  const int le = tid >> 3, a = tid & 7;
  const bool ev = le < ne;
  const int el = ev ? D.blk_elems[e0 + le] : 0;
  const int corner = ev ? M.conn[(int64_t)a * M.E + el] : 0;
  const int crow = ev ? D.inv[corner] : -1;
  if (tid < R) {
    const int node = D.perm[j0 + tid];
    row_node[tid] = node;
    row_c[tid] = M.mass[node] / (M.h * M.h);
    row_free[tid] = M.fixed[node] ? 0 : 1;  // the contact set is masked
    row_pen[tid] = M.cmask[node] ? 1 : 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) row_inc[tid][q] = D.row_inc[8 * (j0 + tid) + q];
  }
  __syncthreads();
  // r_0 = xbar on the free rows outside the set, z = p = q = 0
  if (tid < 3 * R) {
    const int c = tid / R, i = tid % R;
    const double v = row_free[i] ? P.y[c * N + row_node[i]] : 0.0;
    own_r[c * MR + i] = v;
    own_z[c * MR + i] = 0.0;
    own_p[c * MR + i] = 0.0;
    own_q[c * MR + i] = 0.0;
    st_dev(&rg[c * n + j0 + i], v);
  }
  const int lane = tid & 63, wid = tid >> 6, waves = blockDim.x >> 6;
  uint32_t round = 0, pub = 0;
  double gamma_old = 1.0, alpha_old = 1.0;
  int k = 0;
  bool alive = fused_barrier(P.bar, round);
  for (; alive; ++k) {
    for (int i = tid; i < 3 * n; i += blockDim.x) rv[i] = ld_dev(&rg[i]);
    __syncthreads();
    // s = W r on the own rows (the set's rows of W are 0), published
    for (int i = wid; i < R; i += waves) {
      const double* row = P.W + (int64_t)(j0 + i) * n;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int jb = lane; jb < n; jb += 8 * 64) {
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = jb + 64 * u;
          w[u] = j < n ? row[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = jb + 64 * u;
          if (j < n) {
            s0 += w[u] * rv[j];
            s1 += w[u] * rv[n + j];
            s2 += w[u] * rv[2 * n + j];
          }
        }
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      if (lane == 0) {
        own_s[i] = s0;
        own_s[MR + i] = s1;
        own_s[2 * MR + i] = s2;
        st_dev(&sg[j0 + i], s0);
        st_dev(&sg[n + j0 + i], s1);
        st_dev(&sg[2 * n + j0 + i], s2);
      }
    }
    if (!publish_wait(D.ready, nbrs, nnb, ++pub, P.bar)) return;
    // w = (A - dA) s on the own rows
    double cq[19];
    if (ev) load_gauss_cache(M, P.cache, el, a, cq);
    if (ev) {
      double u0 = 0.0, u1 = 0.0, u2 = 0.0;  // Dirichlet corners: 0
      if (crow >= 0) {
        u0 = ld_dev(&sg[crow]);
        u1 = ld_dev(&sg[n + crow]);
        u2 = ld_dev(&sg[2 * n + crow]);
      }
      Tl.xs[le][a][0] = u0;
      Tl.xs[le][a][1] = u1;
      Tl.xs[le][a][2] = u2;
    }
    __syncthreads();
    if (ev) {
      double dF[9];
      deformation_gradient(Tl, le, a, G, dF);
      hvp_stress_from_dF(M, Tl.Ps[le][a], dF, M.w_e[el], cq);
    }
    __syncthreads();
    if (ev) corner_force(Tl, le, a, G, fl[le][a][0], fl[le][a][1], fl[le][a][2]);
    __syncthreads();
    double pg = 0.0, pd = 0.0, pr = 0.0;
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    if (tid < R) {
      const int i = tid;
      if (row_free[i]) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int code = row_inc[i][q];
          if (code >= 0) {
            w0 += fl[code >> 3][code & 7][0];
            w1 += fl[code >> 3][code & 7][1];
            w2 += fl[code >> 3][code & 7][2];
          }
        }
        const double c = row_c[i];
        const double s0 = own_s[i], s1 = own_s[MR + i], s2 = own_s[2 * MR + i];
        w0 += c * s0;
        w1 += c * s1;
        w2 += c * s2;
        if (row_pen[i]) w2 += M.contact_k * s2;
        const double r0 = own_r[i], r1 = own_r[MR + i], r2 = own_r[2 * MR + i];
        pg = r0 * s0 + r1 * s1 + r2 * s2;
        pd = s0 * w0 + s1 * w1 + s2 * w2;
        pr = r0 * r0 + r1 * r1 + r2 * r2;
      }
    }
    const double bg = block_sum(pg, ws);
    const double bd = block_sum(pd, ws);
    const double br = block_sum(pr, ws);
    if (tid == 0) {
      st_dev(&part[b], bg);
      st_dev(&part[G_ + b], bd);
      st_dev(&part[2 * G_ + b], br);
    }
    if (!fused_barrier(P.bar, round)) return;
    if (tid < 64) {
      double tg = 0.0, td = 0.0, tr = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int g = 64 * u + lane;
        if (g < G_) {
          tg += ld_dev(&part[g]);
          td += ld_dev(&part[G_ + g]);
          tr += ld_dev(&part[2 * G_ + g]);
        }
      }
      tg = wave_sum(tg);
      td = wave_sum(td);
      tr = wave_sum(tr);
      if (tid == 0) {
        sums[0] = tg;
        sums[1] = td;
        sums[2] = tr;
      }
    }
    __syncthreads();
    const double gamma = sums[0], delta = sums[1], rsq = sums[2];
    int done = 0, conv = 0, bad = 0, curv = 0;
    double alpha = 0.0, beta = 0.0;
    if (!isfinite(rsq)) {
      bad = 1;
      done = 1;
    } else if (rsq <= tolsq * nb2) {
      conv = 1;
      done = 1;
    } else if (k >= P.max_iter) {
      done = 1;
    } else {
      beta = k == 0 ? 0.0 : gamma / gamma_old;
      const double den = k == 0 ? delta : delta - beta * gamma / alpha_old;
      if (!(den > 0.0) || !(gamma > 0.0)) {
        curv = 1;
        done = 1;
      } else {
        alpha = gamma / den;
      }
    }
    if (b == 0 && tid == 0) {
      P.st->rsq = rsq;
      P.st->iter = k;
      if (bad) P.st->nonfinite = 1;
      if (conv) P.st->converged = 1;
      if (curv) P.st->curvature = 1;
      if (done) P.st->done = 1;
    }
    if (done) break;
    if (tid < 3 * R) {
      const int c = tid / R, i = tid % R, o = c * MR + i;
      own_p[o] = own_s[o] + beta * own_p[o];
    }
    // q = w + beta q: w of own row i is held by thread i
    if (tid < R) {
      const int i = tid;
      own_q[i] = w0 + beta * own_q[i];
      own_q[MR + i] = w1 + beta * own_q[MR + i];
      own_q[2 * MR + i] = w2 + beta * own_q[2 * MR + i];
    }
    __syncthreads();
    if (tid < 3 * R) {
      const int c = tid / R, i = tid % R, o = c * MR + i;
      own_z[o] += alpha * own_p[o];
      const double rn = own_r[o] - alpha * own_q[o];
      own_r[o] = rn;
      st_dev(&rg[c * n + j0 + i], rn);
    }
    gamma_old = gamma;
    alpha_old = alpha;
    if (!fused_barrier(P.bar, round)) return;
  }
  if (!alive) return;
  __syncthreads();
  if (tid < 3 * R) {
    const int c = tid / R, i = tid % R;
    P.x0[c * N + row_node[i]] = own_z[c * MR + i];
  }
  ClockArg c2 = ck;
  c2.bytes = ck.bytes * (double)(k + 1);
  c2.flops = ck.flops * (double)(k + 1);
  clock_exit(c2);
}

__global__ void k_contact_fused_reset(uint32_t* bar, uint32_t* ready, int G) {
  for (int i = threadIdx.x; i < kContactBarWords; i += blockDim.x) bar[i] = 0u;
  for (int i = threadIdx.x; i < G; i += blockDim.x) ready[i] = 0u;
}

}  // namespace

hipError_t launch_contact_fused_cg(hipStream_t s, const DevMesh& Mmask, const DenseCG& D, int blocks,
                                   const double* W, double* z, const double* xbar, const double* cache,
                                   IterState* st, uint32_t* bar, int max_iter) {
  if (D.n < 1 || D.n > kContactDenseMaxRows || blocks < 1 || blocks > 256 || D.rows > kDenseMaxRows)
    return hipErrorInvalidValue;
  FusedContact P{};
  P.M = Mmask;
  P.n = D.n;
  P.rows = D.rows;
  P.mode = 1;
  P.max_iter = max_iter;
  P.W = W;
  P.x0 = z;
  P.y = xbar;
  P.cache = cache;
  P.st = st;
  P.bar = bar;
  hipLaunchKernelGGL(k_contact_fused_reset, dim3(1), dim3(256), 0, s, bar, D.ready, blocks);
  ClockArg ck = take_launch_clock();
  DenseCG Dv = D;
  void* args[] = {&P, &Dv, &ck};
  return hipLaunchCooperativeKernel((const void*)k_contact_fused_cg, dim3(blocks), dim3(kDenseBlock), args,
                                    (unsigned)contact_dense_lds(D.n), s);
}

hipError_t launch_contact_fused(hipStream_t s, const DevMesh& Mmask, const DenseCG& D, int blocks,
                                const double* W, double* x, const double* y, const double* act, const double* cache,
                                IterState* st, uint32_t* bar, int mode, int max_iter) {
  if (D.n < 1 || D.n > kContactDenseMaxRows || blocks < 1 || blocks > 256 || D.rows > kDenseMaxRows)
    return hipErrorInvalidValue;
  FusedContact P{};
  P.M = Mmask;
  P.n = D.n;
  P.rows = D.rows;
  P.mode = mode;
  P.max_iter = max_iter;
  P.W = W;
  P.x0 = x;
  P.y = y;
  P.act = act;
  P.cache = cache;
  P.st = st;
  P.bar = bar;
  hipLaunchKernelGGL(k_contact_fused_reset, dim3(1), dim3(256), 0, s, bar, D.ready, blocks);
  ClockArg ck = take_launch_clock();
  DenseCG Dv = D;
  void* args[] = {&P, &Dv, &ck};
  return hipLaunchCooperativeKernel((const void*)k_contact_fused, dim3(blocks), dim3(kDenseBlock), args,
                                    (unsigned)contact_dense_lds(D.n), s);
}

}  // namespace dpd
