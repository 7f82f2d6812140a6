// Preconditioned conjugate gradients on (A - dA) z = rhs in one cooperative
// launch, for meshes whose free nodes are few enough to hold A^{-1} as a dense
// matrix (n <= 2048 free nodes, at most 32 MB in FP64).
//
// The method is the one of the multi-launch path: the quasi-Newton solve that
// uses the constant PD matrix A as preconditioner of the adjoint and Newton
// systems (Sec. 5, eq:matrix_split), in the Chronopoulos-Gear arrangement of
// conjugate gradients (one fused pair of inner products per iteration):
//   s_k = A^{-1} r_k,  w_k = H s_k,  gamma_k = r_k.s_k,  delta_k = w_k.s_k,
//   beta_k = gamma_k / gamma_{k-1},  alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1}),
//   p_k = s_k + beta_k p_{k-1},  q_k = w_k + beta_k q_{k-1},
//   z_{k+1} = z_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k q_k.
// What changes is the schedule: the launch-per-kernel path spends most of its
// time between kernels at these sizes, so here every workgroup stays resident
// and an iteration has two phases:
//   phase 1 (k+1): every workgroup forms r_{k+1} for all rows in LDS from the
//       previous phase's vectors (no barrier needed for the update) and
//       |r_{k+1}|^2 from them (the same sum, in the same order, everywhere),
//       the owner of a row stores it with p, q and z, and then multiplies its
//       rows of A^{-1} (read once per iteration, coalesced) by r_{k+1};
//   phase 2 (k): the stopping test on |r_k|^2, then H s_k on the owned rows:
//       the hex elements around them are evaluated in LDS (8 lanes per
//       element), their corner forces gathered per node in the same fixed
//       incidence order as the multi-launch kernels, and the two partial inner
//       products are published.
// Phase 2 needs s_k only at the corners of the workgroup's elements, so
// between phase 1 and phase 2 a workgroup publishes its rows of s (a ready
// count per workgroup) and waits only for the workgroups that own rows at its
// corners; phase 1 needs w_k and the partial products of every workgroup, so a
// grid barrier follows phase 2.  Reductions are deterministic: every workgroup
// adds the published partials in the same order.  r, q, w and the partials
// alternate between two buffers, so that no workgroup overwrites a vector
// another one may still read.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "device_math.hpp"

namespace dpd {

namespace {

constexpr uint32_t kSpinLimit = 1u << 22;  // about 4 s of polling: then abort

// Vectors that workgroups exchange inside the launch are written and read
// with device-coherent accesses (agent-scope relaxed atomic loads and stores,
// which bypass the per-XCD caches' stale copies) so that the barrier needs no
// cache write-back or invalidation: A^{-1} and the other read-only data stay
// cached across iterations.
__device__ inline double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier of a cooperative launch, two levels: workgroup b counts
// in at the counter of group b mod 8 (one 256-byte line each); the workgroup
// that completes its group's count for this round stores the round number in
// the group's flag (the eight flags share one line), and wave 0 of every
// workgroup polls the eight flags with one load.  Every wave first waits until
// its own device-coherent stores have completed.  The wait is bounded: a
// workgroup that times out raises the abort flag, every workgroup that sees
// the flag stops waiting, and all of them leave the kernel, so the launch
// always drains.  Returns false after an abort.
constexpr int kBarGroups = 8;
constexpr int kBarStride = 64;   // uint32 entries between counters
constexpr int kBarFlags = 16;    // first group flag (bar[0] unused, bar[1] abort)
constexpr int kBarWords = kBarStride * (kBarGroups + 1);
static_assert(kBarWords == kDenseBarWords, "barrier buffer size");
static_assert(kBarFlags + kBarGroups <= kBarStride, "flags share the first line");

__device__ inline bool grid_barrier(uint32_t* bar, uint32_t& round) {
  __shared__ int ok;
  __syncthreads();
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  round += 1;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const uint32_t G = gridDim.x, g = blockIdx.x % kBarGroups;
    const uint32_t ngroups = G < (uint32_t)kBarGroups ? G : (uint32_t)kBarGroups;
    if (lane == 0) {
      const uint32_t gsize = G / kBarGroups + (g < G % kBarGroups ? 1u : 0u);
      const uint32_t t =
          __hip_atomic_fetch_add(&bar[kBarStride * (g + 1)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (t + 1 == round * gsize)
        __hip_atomic_store(&bar[kBarFlags + g], round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int good = 1;
    for (uint32_t spin = 0;; ++spin) {
      const uint32_t v = (uint32_t)lane < ngroups
                             ? __hip_atomic_load(&bar[kBarFlags + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : round;
      if (__all(v >= round)) break;
      const uint32_t ab = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ab != 0u || spin >= kSpinLimit) {
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

// Publication of s without a grid barrier: once its rows of s are stored, the
// workgroup waits until its own stores have completed and raises its ready
// count to seq, then waits until the ready counts of the nnb workgroups in nbr
// (the owners of rows at its element corners) reach seq.  The wait is bounded
// like the barrier's and shares its abort flag.  Returns false after an abort.
__device__ inline bool publish_wait(uint32_t* ready, const int32_t* __restrict__ nbr, int nnb, uint32_t seq,
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
    const int w = nbr[i];
    for (uint32_t spin = 0;; ++spin) {
      if (__hip_atomic_load(&ready[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= seq) break;
      if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spin >= kSpinLimit) {
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

// Shape-function gradients dN_a/dX_j at Gauss point q, gt[(q * 8 + a) * 3 + j],
// staged in LDS once per launch and read there, so that no lane keeps its
// 48 table entries in registers across the iteration loop.
__device__ inline void deformation_gradient_tab(const ElemTileT<kDenseElems>& T, int le, int q,
                                                const double* gt, double F[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double b0 = gt[(q * 8 + a) * 3], b1 = gt[(q * 8 + a) * 3 + 1], b2 = gt[(q * 8 + a) * 3 + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double xi = T.xs[le][a][i];
      F[3 * i + 0] += xi * b0;
      F[3 * i + 1] += xi * b1;
      F[3 * i + 2] += xi * b2;
    }
  }
}

__device__ inline void corner_force_tab(const ElemTileT<kDenseElems>& T, int le, int a, const double* gt,
                                        double& f0, double& f1, double& f2) {
  f0 = f1 = f2 = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double b0 = gt[(q * 8 + a) * 3], b1 = gt[(q * 8 + a) * 3 + 1], b2 = gt[(q * 8 + a) * 3 + 2];
    const double* P = T.Ps[le][q];
    f0 += P[0] * b0 + P[1] * b1 + P[2] * b2;
    f1 += P[3] * b0 + P[4] * b1 + P[5] * b2;
    f2 += P[6] * b0 + P[7] * b1 + P[8] * b2;
  }
}

// Sum over the workgroup, returned to every lane.
__device__ inline double block_all(double v, double* ws, double* bc) {
  v = block_sum(v, ws);
  if (threadIdx.x == 0) *bc = v;
  __syncthreads();
  const double out = *bc;
  __syncthreads();
  return out;
}

// s[rows j0..j0+R) = A^{-1}[rows] r, r staged in LDS (rv, [3][n]); `rows`
// points at the workgroup's R rows of A^{-1} (in LDS or in device memory).
// One wave per row (R <= 8 waves), lanes over the columns with eight loads of
// the row in flight per lane, then three wave sums.  The result is stored
// device-coherently and in the owner's LDS copy.
template <typename T>
__device__ __forceinline__ void dense_rows(const T* __restrict__ rows, int n, const double* rv, int j0, int R,
                                           double* __restrict__ s_glob, double* own_s) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = wid; i < R; i += kDenseBlock / 64) {
    const T* row = rows + (int64_t)i * n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int c = lane;
    for (; c + 7 * 64 < n; c += 8 * 64) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = (double)row[c + 64 * u];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int cu = c + 64 * u;
        a0 += p[u] * rv[cu];
        a1 += p[u] * rv[n + cu];
        a2 += p[u] * rv[2 * n + cu];
      }
    }
    for (; c < n; c += 64) {
      const double pc = (double)row[c];
      a0 += pc * rv[c];
      a1 += pc * rv[n + c];
      a2 += pc * rv[2 * n + c];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      const int j = j0 + i;
      st_dev(&s_glob[j], a0);
      st_dev(&s_glob[n + j], a1);
      st_dev(&s_glob[2 * n + j], a2);
      own_s[i] = a0;
      own_s[kDenseMaxRows + i] = a1;
      own_s[2 * kDenseMaxRows + i] = a2;
    }
  }
  __syncthreads();
}

// Two sums over the workgroup in one pass, valid in lane 0 only.
__device__ inline void block_sum2(double& a, double& b, double* ws2) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    ws2[2 * wid] = a;
    ws2[2 * wid + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      ta += ws2[2 * w];
      tb += ws2[2 * w + 1];
    }
    a = ta;
    b = tb;
  }
}

// Two sums over the workgroup in one pass, returned to every lane.
__device__ inline void block_all2(double& a, double& b, double* ws2, double* bc2) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    ws2[2 * wid] = a;
    ws2[2 * wid + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      ta += ws2[2 * w];
      tb += ws2[2 * w + 1];
    }
    bc2[0] = ta;
    bc2[1] = tb;
  }
  __syncthreads();
  a = bc2[0];
  b = bc2[1];
  __syncthreads();
}

template <typename T, bool kVecLds, bool kAinvLds>
__global__ void __launch_bounds__(kDenseBlock) k_cg_dense(DevMesh M, DenseCG D, const T* __restrict__ ainv,
                                                          const double* __restrict__ cache,
                                                          const double* __restrict__ rhs, double rhs_scale,
                                                          int pd_fallback, double* __restrict__ z_out,
                                                          IterState* st, ProfAcc* prof) {
  // a solve whose state is already finished (the Newton forward step enqueues
  // solves ahead of its convergence test) does nothing
  if (st->done) return;
  extern __shared__ double lds[];
  // r_k of every row in LDS ([3][n]); with kVecLds also q_k of every row, so
  // that r and q never go through device memory (every workgroup forms the
  // same values from the same inputs), else they are exchanged through D.r, D.q
  // With kAinvLds the workgroup's R rows of A^{-1} are copied to LDS once per
  // launch (after the vectors).
  double* rv = lds;
  double* ql = lds + 3 * D.n;
  T* arows = reinterpret_cast<T*>(lds + (kVecLds ? 6 : 3) * D.n);
  __shared__ ElemTileT<kDenseElems> Tl;
  // corner forces [kDenseElems][8][3] share storage with the tile's node
  // values, which are dead once the stresses are formed
  double* fl = &Tl.xs[0][0][0];
  __shared__ double ws[kDenseBlock / 64];
  __shared__ double bc;
  __shared__ double ws2[2 * (kDenseBlock / 64)], bc2[2];
  // the workgroup's own rows: r_k, s_k, p, z (owner-private), node data
  __shared__ double own_r[3 * kDenseMaxRows], own_s[3 * kDenseMaxRows], own_s0[3 * kDenseMaxRows];
  __shared__ double own_p[3 * kDenseMaxRows], own_z[3 * kDenseMaxRows];
  __shared__ double row_c[kDenseMaxRows], row_k[kDenseMaxRows];
  __shared__ int row_node[kDenseMaxRows], row_inc[kDenseMaxRows][8];
  __shared__ int el_rows[kDenseElems][8];
  __shared__ double gt[8 * 8 * 3];
  constexpr int MR = kDenseMaxRows;

  const int n = D.n, N = M.N, tid = threadIdx.x, b = blockIdx.x, G_ = gridDim.x;
  const int j0 = min(n, b * D.rows), j1 = min(n, j0 + D.rows), R = j1 - j0;
  const double tolsq = st->tolsq;
  const int max_iter = st->max_iter;
  const GradTable G = grad_table(M.dx);
  const uint64_t clk0 = wall_clock64();
  uint32_t round = 0, pub = 0;
  bool alive = true;
  const int32_t* nbrs = D.nbr + D.nbr_off[b];
  const int nnb = D.nbr_off[b + 1] - D.nbr_off[b];
  if (tid < 8 * 8 * 3) {
    const int q = tid / 24, a0 = (tid / 3) % 8, jj = tid % 3;
    gt[tid] = bgrad(q, jj, a0, G);
  }

  // ---- per-launch staging: the workgroup's elements (one per 8 lanes, lane
  // a = Gauss point a = corner a) with their cache entries in registers
  const int e0 = D.blk_eoff[b], ne = D.blk_eoff[b + 1] - e0;
  const int le = tid >> 3, a = tid & 7;
  const bool ev = le < ne;
  const int el = ev ? D.blk_elems[e0 + le] : 0;
  double we = 0.0;
  if (ev) {
    we = M.w_e[el];
    el_rows[le][a] = D.inv[M.conn[(int64_t)a * M.E + el]];
  }
  if (tid < R) {
    const int node = D.perm[j0 + tid];
    row_node[tid] = node;
    row_c[tid] = M.mass[node] / (M.h * M.h);
    row_k[tid] = M.cmask[node] ? M.contact_k : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) row_inc[tid][q] = D.row_inc[8 * (j0 + tid) + q];
  }

  // ---- phase 1 (k = 0): r_0 = rhs on the free rows, p = q = z = 0, s_0 = A^{-1} r_0
  for (int i = tid; i < n; i += kDenseBlock) {
    const int node = D.perm[i];
    rv[i] = rhs_scale * rhs[node];
    rv[n + i] = rhs_scale * rhs[(int64_t)N + node];
    rv[2 * n + i] = rhs_scale * rhs[2 * (int64_t)N + node];
  }
  if (kVecLds)
    for (int i = tid; i < 3 * n; i += kDenseBlock) ql[i] = 0.0;
  if (kAinvLds)
    for (int i = tid; i < R * n; i += kDenseBlock) arows[i] = ainv[(int64_t)j0 * n + i];
  const T* my_rows = kAinvLds ? arows : ainv + (int64_t)j0 * n;
  __syncthreads();
  if (tid < 3 * R) {
    const int c = tid / R, i = tid % R, j = j0 + i;
    const double v = rv[c * n + j];
    if (!kVecLds) {
      st_dev(&D.r[c * n + j], v);
      st_dev(&D.q[c * n + j], 0.0);
      st_dev(&D.q[3 * n + c * n + j], 0.0);
    }
    own_r[c * MR + i] = v;
    own_p[c * MR + i] = 0.0;
    own_z[c * MR + i] = 0.0;
  }
  double acc = 0.0;
  for (int i = tid; i < 3 * n; i += kDenseBlock) acc += rv[i] * rv[i];
  double rsq_next = block_all(acc, ws, &bc);   // |r_0|^2, the same bits in every workgroup
  dense_rows<T>(my_rows, n, rv, j0, R, D.s, own_s);
  if (tid < 3 * MR) own_s0[tid] = own_s[tid];
  alive = publish_wait(D.ready, nbrs, nnb, ++pub, D.bar);

  double nb2 = 0.0, rsq = 0.0, rs_old = 0.0, alpha_old = 0.0, alpha = 0.0, beta = 0.0;
  int k = 0, converged = 0, nonfinite = 0, curvature = 0;
  for (; alive; ++k) {
    // ---- phase 2 (k): one round of device-coherent loads (s_k at the
    // workgroup's element corners), the stopping test, then w_k = H s_k on the
    // own rows and the two inner products
    // cache entries of this lane's Gauss point: read-only and L2-resident,
    // loaded in the same round as the device-coherent loads below; the index
    // is made opaque to the compiler so that it does not keep 19 loop-invariant
    // addresses live in registers across the iteration loop
    double cq[19];
    if (ev) {
      int qi = 8 * el + a;
      __asm__ volatile("" : "+v"(qi));
      const int Q = 8 * M.E, rows = M.muscle_k > 0.0 ? 19 : 15;
#pragma unroll
      for (int i = 0; i < 19; ++i) cq[i] = i < rows ? cache[i * Q + qi] : 0.0;
    }
    double sv0 = 0.0, sv1 = 0.0, sv2 = 0.0;
    if (ev) {
      const int row = el_rows[le][a];
      if (row >= 0) {
        sv0 = ld_dev(&D.s[row]);
        sv1 = ld_dev(&D.s[n + row]);
        sv2 = ld_dev(&D.s[2 * n + row]);
      }
    }
    rsq = rsq_next;
    if (k == 0) nb2 = D.nb2_ref ? *D.nb2_ref : rsq;
    if (!isfinite(rsq)) {
      nonfinite = 1;
      break;
    }
    if (rsq <= tolsq * nb2) {
      converged = 1;
      break;
    }
    if (k >= max_iter) break;
    if (ev) {
      Tl.xs[le][a][0] = sv0;
      Tl.xs[le][a][1] = sv1;
      Tl.xs[le][a][2] = sv2;
    }
    __syncthreads();
    if (ev) {
      double dF[9];
      deformation_gradient_tab(Tl, le, a, gt, dF);
      hvp_stress_from_dF(M, Tl.Ps[le][a], dF, we, cq);
    }
    __syncthreads();
    if (ev) {
      double f0, f1, f2;
      corner_force_tab(Tl, le, a, gt, f0, f1, f2);
      double* o = fl + (le * 8 + a) * 3;
      o[0] = f0;
      o[1] = f1;
      o[2] = f2;
    }
    __syncthreads();
    double gam = 0.0, del = 0.0;
    if (tid < R) {
      const int j = j0 + tid;
      double o0 = 0.0, o1 = 0.0, o2 = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int code = row_inc[tid][q];
        if (code >= 0) {
          o0 += fl[3 * code];
          o1 += fl[3 * code + 1];
          o2 += fl[3 * code + 2];
        }
      }
      const double s0 = own_s[tid], s1 = own_s[MR + tid], s2 = own_s[2 * MR + tid];
      const double cm = row_c[tid];
      o0 += cm * s0;
      o1 += cm * s1;
      o2 += cm * s2;
      o2 += row_k[tid] * s2;
      double* wk = D.w + (k & 1) * 3 * n;
      st_dev(&wk[j], o0);
      st_dev(&wk[n + j], o1);
      st_dev(&wk[2 * n + j], o2);
      gam = own_r[tid] * s0 + own_r[MR + tid] * s1 + own_r[2 * MR + tid] * s2;
      del = o0 * s0 + o1 * s1 + o2 * s2;
    }
    block_sum2(gam, del, ws2);   // totals in lane 0 only
    if (tid == 0) {
      st_dev(&D.part[2 * ((k & 1) * G_ + b)], gam);
      st_dev(&D.part[2 * ((k & 1) * G_ + b) + 1], del);
    }
    if (!(alive = grid_barrier(D.bar, round))) break;

    // ---- phase 1 (k + 1): one round of device-coherent loads (gamma and delta
    // partials, w_k, q_{k-1}, r_k on every row), the scalars, r_{k+1} for every
    // row into LDS, the owner's updates, then s_{k+1} = A^{-1} r_{k+1}
    const double pg = tid < G_ ? ld_dev(&D.part[2 * ((k & 1) * G_ + tid)]) : 0.0;
    const double pd = tid < G_ ? ld_dev(&D.part[2 * ((k & 1) * G_ + tid) + 1]) : 0.0;
    const double* wk = D.w + (k & 1) * 3 * n;            // w_k
    const double* qprev = D.q + ((k + 1) & 1) * 3 * n;   // q_{k-1}
    double* qcur = D.q + (k & 1) * 3 * n;                // q_k
    const double* rk = D.r + (k & 1) * 3 * n;            // r_k
    double* rnext = D.r + ((k + 1) & 1) * 3 * n;         // r_{k+1}
    constexpr int kBatch = 8;
    double wv[kBatch], qv[kBatch], rr[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = u * kDenseBlock + tid;
      wv[u] = qv[u] = rr[u] = 0.0;
      if (i < 3 * n) {
        wv[u] = ld_dev(&wk[i]);
        qv[u] = kVecLds ? ql[i] : ld_dev(&qprev[i]);
        rr[u] = kVecLds ? rv[i] : ld_dev(&rk[i]);
      }
    }
    double gamma = pg, delta = pd;
    block_all2(gamma, delta, ws2, bc2);
    beta = k == 0 ? 0.0 : gamma / rs_old;
    const double den = k == 0 ? delta : delta - beta * gamma / alpha_old;
    if (!(den > 0.0) || !isfinite(den) || !isfinite(gamma)) {
      curvature = 1;
      // the forward Newton step falls back to one plain PD step, A^{-1} rhs = s_0
      if (pd_fallback && tid < 3 * MR) own_z[tid] = own_s0[tid];
      __syncthreads();
      break;
    }
    alpha = gamma / den;
    rs_old = gamma;
    alpha_old = alpha;
    double racc = 0.0;
    for (int base = 0; base < 3 * n; base += kBatch * kDenseBlock) {
      if (base > 0) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int i = base + u * kDenseBlock + tid;
          wv[u] = qv[u] = rr[u] = 0.0;
          if (i < 3 * n) {
            wv[u] = ld_dev(&wk[i]);
            qv[u] = kVecLds ? ql[i] : ld_dev(&qprev[i]);
            rr[u] = kVecLds ? rv[i] : ld_dev(&rk[i]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int i = base + u * kDenseBlock + tid;
        if (i < 3 * n) {
          const double qi = wv[u] + beta * qv[u];
          const double ri = rr[u] - alpha * qi;
          rv[i] = ri;
          racc += ri * ri;
          if (kVecLds) ql[i] = qi;
          const int c = (i >= n) + (i >= 2 * n), j = i - c * n;
          if (j >= j0 && j < j1) {
            const int o = c * MR + (j - j0);
            if (!kVecLds) {
              st_dev(&qcur[i], qi);
              st_dev(&rnext[i], ri);
            }
            own_r[o] = ri;
            const double pi = own_s[o] + beta * own_p[o];
            own_p[o] = pi;
            own_z[o] += alpha * pi;
          }
        }
      }
    }
    rsq_next = block_all(racc, ws, &bc);   // |r_{k+1}|^2, the same bits in every workgroup
    dense_rows<T>(my_rows, n, rv, j0, R, D.s, own_s);
    if (!(alive = publish_wait(D.ready, nbrs, nnb, ++pub, D.bar))) break;
  }

  // solution rows to the public layout (fixed rows are left as they are)
  if (tid < 3 * R) {
    const int c = tid / R, i = tid % R;
    z_out[(int64_t)c * N + row_node[i]] = own_z[c * MR + i];
  }
  if (b == 0 && tid == 0) {
    st->iter = k;
    st->rsq = rsq;
    st->nb2 = nb2;
    st->rs = rs_old;
    st->alpha = alpha;
    st->beta = beta;
    st->converged = converged;
    st->nonfinite = nonfinite;
    st->curvature = curvature;
    st->aborted = (!alive || __hip_atomic_load(&D.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) ? 1 : 0;
    if (prof) {
      atomicAdd(&prof->ticks, (unsigned long long)(wall_clock64() - clk0));
      atomicAdd(&prof->iters, (unsigned long long)k);
      atomicAdd(&prof->launches, 1ull);
    }
    st->done = 1;
  }
}

__global__ void k_bar_reset(uint32_t* bar, uint32_t* ready, int G) {
  for (int i = threadIdx.x; i < kBarWords; i += blockDim.x) bar[i] = 0u;
  for (int i = threadIdx.x; i < G; i += blockDim.x) ready[i] = 0u;
}

__global__ void __launch_bounds__(kBlock) k_unit_rhs(int N, int n, const int32_t* __restrict__ perm, int j0,
                                                     double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * (int64_t)N) return;
  const int c = (int)(i / N), node = (int)(i % N);
  b[i] = (j0 + c < n && perm[j0 + c] == node) ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(kBlock) k_collect_rows(int N, int n, const int32_t* __restrict__ perm, int j0,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ ainv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int node = perm[i];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (j0 + c < n) ainv[(int64_t)(j0 + c) * n + i] = x[(int64_t)c * N + node];
}

__global__ void __launch_bounds__(kBlock) k_to_fp32(int64_t count, const double* __restrict__ in,
                                                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (float)in[i];
}

}  // namespace

size_t cg_dense_lds_bytes(int n, int rows, int mode, bool fp32) {
  size_t b = (size_t)((mode & kDenseVecLds) ? 6 : 3) * n * sizeof(double);
  if (mode & kDenseAinvLds) b += (size_t)rows * n * (fp32 ? sizeof(float) : sizeof(double));
  return b;
}

namespace {
template <typename T>
const void* dense_kernel_t(int mode) {
  switch (mode & 3) {
    case 0: return (const void*)k_cg_dense<T, false, false>;
    case kDenseVecLds: return (const void*)k_cg_dense<T, true, false>;
    case kDenseAinvLds: return (const void*)k_cg_dense<T, false, true>;
    default: return (const void*)k_cg_dense<T, true, true>;
  }
}
const void* dense_kernel(bool fp32, int mode) {
  return fp32 ? dense_kernel_t<float>(mode) : dense_kernel_t<double>(mode);
}
}  // namespace

int cg_dense_max_blocks(int n, int rows, int mode, bool fp32) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = cg_dense_lds_bytes(n, rows, mode, fp32);
  const void* fn = dense_kernel(fp32, mode);
  if (lds > 48 * 1024 &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kDenseBlock, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per_cu * cus;
}

hipError_t launch_cg_dense(const DevMesh& M, const DenseCG& D, hipStream_t s, int blocks, bool fp32,
                           const double* cache, const double* rhs, double rhs_scale, int pd_fallback,
                           double* z_out, IterState* st, ProfAcc* prof, const double* nb2_ref) {
  hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, s, D.bar, D.ready, blocks);
  const int mode = fp32 ? D.mode32 : D.mode64;
  const size_t lds = cg_dense_lds_bytes(D.n, D.rows, mode, fp32);
  DevMesh m = M;
  DenseCG d = D;
  d.nb2_ref = nb2_ref;
  IterState* stp = st;
  const double* cp = cache;
  const double* rp = rhs;
  double* zp = z_out;
  double sc = rhs_scale;
  int pf = pd_fallback;
  ProfAcc* pa = prof;
  if (fp32) {
    const float* a = D.ainv32;
    void* args[] = {&m, &d, &a, &cp, &rp, &sc, &pf, &zp, &stp, &pa};
    return hipLaunchCooperativeKernel(dense_kernel(true, mode), dim3(blocks), dim3(kDenseBlock), args,
                                      (unsigned)lds, s);
  }
  const double* a = D.ainv64;
  void* args[] = {&m, &d, &a, &cp, &rp, &sc, &pf, &zp, &stp, &pa};
  return hipLaunchCooperativeKernel(dense_kernel(false, mode), dim3(blocks), dim3(kDenseBlock), args,
                                    (unsigned)lds, s);
}

void launch_unit_rhs(hipStream_t s, int N, int n, const int32_t* perm, int j0, double* b) {
  const int64_t t = 3 * (int64_t)N;
  hipLaunchKernelGGL(k_unit_rhs, dim3((unsigned)((t + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, N, n, perm,
                     j0, b);
}

void launch_collect_rows(hipStream_t s, int N, int n, const int32_t* perm, int j0, const double* x,
                         double* ainv) {
  hipLaunchKernelGGL(k_collect_rows, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N, n, perm, j0, x,
                     ainv);
}

void launch_to_fp32(hipStream_t s, int64_t count, const double* in, float* out) {
  hipLaunchKernelGGL(k_to_fp32, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, count, in,
                     out);
}

}  // namespace dpd
