// Global step with a contact set (Sec. Contact, the low-rank update of
// Alg. 4): x with x_C = x* and A_{C̄×C̄} x_{C̄} = b_{C̄}, computed from the
// factor of A without refactorizing the reduced matrix.
//
// The candidate nodes' columns of A^{-1} are precomputed once (the paper's
// caching of A^{-1} I_{I×C}; with A = I_3 (x) A_s one scalar column per node,
// B1[k][node] = (A_s^{-1} e_{cand k})[node]).  A solve then needs one global
// solve a1 = A^{-1} b and a correction in the columns of the active set:
//   x = a1 + B1_C lam,   (A^{-1})_{C×C} lam = -(a1)_C,   x_C = x*.
// Rows outside C then satisfy A x = b, and x_C = 0 before x* is written, so
// A_{C̄×C̄} x_{C̄} = b_{C̄}.  This is the Woodbury identity in capacitance form:
// the small system is c x c and SPD (a principal block of A^{-1}) instead of
// the paper's 2c x 2c I - V P^T B3.  Its inverse depends on the active set
// only, which stays fixed through Alg. 3's inner iterations, so it is
// computed (Cholesky in LDS) when the set changes and reused otherwise.
#include <hip/hip_runtime.h>

#include "contact.hpp"
#include "device.hpp"

namespace dpd {

namespace {

// b = e_{cand k} in coordinate c for the three candidates k = k0 + c.
__global__ void k_contact_unit(int N, int n_cand, const int32_t* __restrict__ cand, int k0, double* b) {
  const int c = threadIdx.x;
  if (c < 3 && k0 + c < n_cand) b[(int64_t)c * N + cand[k0 + c]] = 1.0;
}

// B1[k0 + c][node] = x[c][node]: the solution of the unit right-hand side of
// candidate k0 + c (rows of fixed nodes are 0).
__global__ void __launch_bounds__(kBlock) k_contact_collect(int N, int n_cand, int k0,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ B1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * (int64_t)N) return;
  const int c = (int)(i / N), node = (int)(i % N);
  if (k0 + c < n_cand) B1[(int64_t)(k0 + c) * N + node] = x[i];
}

// One workgroup, once per active set: S = B1[set][cand[set]] (c x c, SPD),
// S = L L^T, then Sinv = S^{-1} into device memory.
//  * Cholesky, one barrier per column: in step j, column j - 1 is scaled by
//    its pivot's square root while the trailing block is updated with
//    column j's unscaled entries, S[i][k] -= S[i][j] S[k][j] / S[j][j]; the
//    two touch disjoint entries.  The diagonal of L goes to ld.
//  * Inversion: thread j computes column j of L^{-1} by forward substitution
//    and keeps it in row j of the strict upper triangle (its diagonal in
//    dinv), which nothing else reads.
//  * Sinv[a][b] = sum_{i >= max(a, b)} L^{-1}[i][a] L^{-1}[i][b].
// status = 1 on a non-positive pivot.
__global__ void __launch_bounds__(kContactThreads) k_contact_factor(int N, const int32_t* __restrict__ cand,
                                                                    const int32_t* __restrict__ set, int c,
                                                                    const double* __restrict__ B1,
                                                                    double* __restrict__ Sinv, int* status) {
  extern __shared__ double lds[];
  double* S = lds;            // [c][c]
  double* ld = lds + c * c;   // [c] diagonal of L
  double* dinv = ld + c;      // [c] diagonal of L^{-1}
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < c * c; idx += nt) {
    const int k = idx / c, l = idx % c;
    S[idx] = B1[(int64_t)set[k] * N + cand[set[l]]];
  }
  __syncthreads();
  for (int j = 0; j <= c; ++j) {
    if (j > 0) {
      const double d = S[(j - 1) * c + (j - 1)];
      const double l = d > 0.0 ? sqrt(d) : 1.0;
      if (tid == 0) ld[j - 1] = l;
      for (int i = j + tid; i < c; i += nt) S[i * c + (j - 1)] /= l;
    }
    if (j < c) {
      const double d = S[j * c + j];
      if (tid == 0 && !(d > 0.0)) bad = 1;
      const double rd = d > 0.0 ? 1.0 / d : 0.0;
      const int m = c - j - 1;
      for (int idx = tid; idx < m * (m + 1) / 2; idx += nt) {
        // idx -> (i, k), 0 <= k <= i < m, row by row over the lower triangle
        int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= idx) ++i;
        while (i * (i + 1) / 2 > idx) --i;
        const int k = idx - i * (i + 1) / 2;
        const int ii = j + 1 + i, kk = j + 1 + k;
        S[ii * c + kk] -= S[ii * c + j] * S[kk * c + j] * rd;
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < c; j += nt) {
    const double wj = 1.0 / ld[j];
    dinv[j] = wj;
    for (int i = j + 1; i < c; ++i) {
      double acc = S[i * c + j] * wj;
      for (int k = j + 1; k < i; ++k) acc += S[i * c + k] * S[j * c + k];
      S[j * c + i] = -acc / ld[i];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < c * c; idx += nt) {
    const int a = idx / c, b = idx % c;
    if (b > a) continue;
    double acc = dinv[a] * (a == b ? dinv[a] : S[b * c + a]);
    for (int i = a + 1; i < c; ++i) acc += S[a * c + i] * S[b * c + i];
    Sinv[a * c + b] = acc;
    Sinv[b * c + a] = acc;
  }
  if (tid == 0) *status = bad;
}

// lam[comp][a] = -sum_b Sinv[a][b] a1[comp][cand[set[b]]]: one workgroup,
// the set's entries of a1 gathered into LDS once, then a wave per row of Sinv
// (lanes over its columns, coalesced) and three wave sums.
__global__ void __launch_bounds__(kContactThreads) k_contact_lam(int N, const int32_t* __restrict__ cand,
                                                                 const int32_t* __restrict__ set, int c,
                                                                 const double* __restrict__ Sinv,
                                                                 const double* __restrict__ a1,
                                                                 double* __restrict__ lam, const IterState* st) {
  if (st && st->done) return;
  __shared__ double t[3 * kContactMaxSet];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 3 * c; idx += blockDim.x) {
    const int comp = idx / c, k = idx % c;
    t[idx] = a1[(int64_t)comp * N + cand[set[k]]];
  }
  __syncthreads();
  const int lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  for (int a = wid; a < c; a += nw) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = lane; b < c; b += 64) {
      const double v = Sinv[a * c + b];
      s0 += v * t[b];
      s1 += v * t[c + b];
      s2 += v * t[2 * c + b];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    if (lane == 0) {
      lam[a] = -s0;
      lam[c + a] = -s1;
      lam[2 * c + a] = -s2;
    }
  }
}

// x[comp][node] += sum_k B1[set[k]][node] lam[comp][k] for every node (the
// columns of the active set, streamed once; fixed rows of B1 are 0).
__global__ void __launch_bounds__(kBlock) k_contact_update(int N, const int32_t* __restrict__ set, int c,
                                                           const double* __restrict__ B1,
                                                           const double* __restrict__ lam, double* __restrict__ x,
                                                           ClockArg ck) {
  clock_enter(ck);
  __shared__ double sl[3 * kContactMaxSet];
  __shared__ int ss[kContactMaxSet];
  for (int idx = threadIdx.x; idx < 3 * c; idx += blockDim.x) sl[idx] = lam[idx];
  for (int k = threadIdx.x; k < c; k += blockDim.x) ss[k] = set[k];
  __syncthreads();
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node < N) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 8
    for (int k = 0; k < c; ++k) {
      const double bk = B1[(int64_t)ss[k] * N + node];
      a0 += bk * sl[k];
      a1 += bk * sl[c + k];
      a2 += bk * sl[2 * c + k];
    }
    x[node] += a0;
    x[(int64_t)N + node] += a1;
    x[2 * (int64_t)N + node] += a2;
  }
  clock_exit(ck);
}

// One reduced global step of Alg. 3 (or Alg. 5) in correction form: with
// d = A^{-1} r and lam from d, x <- x - (d + B1_C lam) at every node outside
// the mask (Dirichlet nodes and the contact set, whose rows stay at their
// prescribed values).  d + B1_C lam vanishes on C, so this is
// x_{C̄} <- x_{C̄} - (A_{C̄×C̄})^{-1} r_{C̄}.
__global__ void __launch_bounds__(kBlock) k_contact_descend(int N, const int32_t* __restrict__ set, int c,
                                                            const double* __restrict__ B1,
                                                            const double* __restrict__ lam,
                                                            const double* __restrict__ d,
                                                            const uint8_t* __restrict__ mask,
                                                            double* __restrict__ x, const IterState* st,
                                                            ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  __shared__ double sl[3 * kContactMaxSet];
  __shared__ int ss[kContactMaxSet];
  for (int idx = threadIdx.x; idx < 3 * c; idx += blockDim.x) sl[idx] = lam[idx];
  for (int k = threadIdx.x; k < c; k += blockDim.x) ss[k] = set[k];
  __syncthreads();
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node < N && !mask[node]) {
    double a0 = d[node], a1 = d[(int64_t)N + node], a2 = d[2 * (int64_t)N + node];
#pragma unroll 8
    for (int k = 0; k < c; ++k) {
      const double bk = B1[(int64_t)ss[k] * N + node];
      a0 += bk * sl[k];
      a1 += bk * sl[c + k];
      a2 += bk * sl[2 * c + k];
    }
    x[node] -= a0;
    x[(int64_t)N + node] -= a1;
    x[2 * (int64_t)N + node] -= a2;
  }
  clock_exit(ck);
}

// Collision detection against the ground plane z = 0 for every candidate
// (Sec. Contact, remarks on friction: the target is where the ray
// x_j + t v_j, 0 <= t <= h, meets the plane, t = 0 included).  In contact
// when z_j + h v_z <= 0 and v_z <= 0; kind 1 (ray): z_j >= 0 and v_z < 0,
// target x_j + t v_j at t = -z_j / v_z; kind 2 (static): a node on the plane
// not moving along z, or one below it, target (x_j, y_j, 0); kind 0: no
// contact.  Products and sums are rounded one by one (no fused
// multiply-add), so the decision and the target are those of the plain
// formula.  `left` (a node has left the set in this step) is cleared.
__global__ void k_contact_detect(int N, int n_cand, const int32_t* __restrict__ cand, double h,
                                 const double* __restrict__ x, const double* __restrict__ v,
                                 double* __restrict__ tgt, int32_t* __restrict__ kind,
                                 uint8_t* __restrict__ left) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cand) return;
  const int64_t j = cand[i];
  const double z = x[2 * N + j], vz = v[2 * N + j];
  double p0 = x[j], p1 = x[N + j];
  int k = 0;
  if (__dadd_rn(z, __dmul_rn(h, vz)) <= 0.0 && vz <= 0.0) {
    if (z >= 0.0 && vz < 0.0) {
      const double t = -z / vz;
      p0 = __dadd_rn(p0, __dmul_rn(t, v[j]));
      p1 = __dadd_rn(p1, __dmul_rn(t, v[N + j]));
      k = 1;
    } else {
      k = 2;
    }
  }
  kind[i] = k;
  left[i] = 0;
  tgt[i] = p0;
  tgt[n_cand + i] = p1;
  tgt[2 * n_cand + i] = 0.0;
}

// mask[cand[i]] = 1 for the candidates in the set (on a copy of the Dirichlet
// flags).
__global__ void k_contact_mark(int n_cand, const int32_t* __restrict__ cand, const int32_t* __restrict__ kind,
                               uint8_t* __restrict__ mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cand && kind[i]) mask[cand[i]] = 1;
}

// x at the set's nodes = their targets.
__global__ void k_contact_place(int N, int n_cand, const int32_t* __restrict__ cand,
                                const int32_t* __restrict__ kind, const double* __restrict__ tgt,
                                double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cand || !kind[i]) return;
  const int64_t j = cand[i];
  x[j] = tgt[i];
  x[N + j] = tgt[n_cand + i];
  x[2 * N + j] = tgt[2 * n_cand + i];
}

// Active-set update of Alg. 3 from the reduced solution xn and r = grad g(xn)
// (eq:tic_1, the contact forces on the set): a node of the set whose normal
// force r_z is negative leaves it, unless it has left once in this step; a
// node outside it below the plane joins it with the target (x0_j, y0_j, 0)
// of its start-of-step position x0 (kind 2).
__global__ void k_contact_active_set(int N, int n_cand, const int32_t* __restrict__ cand,
                                     const double* __restrict__ x0, const double* __restrict__ xn,
                                     const double* __restrict__ r, int32_t* __restrict__ kind,
                                     uint8_t* __restrict__ left, double* __restrict__ tgt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cand) return;
  const int64_t j = cand[i];
  if (kind[i]) {
    if (r[2 * N + j] < 0.0 && !left[i]) {
      kind[i] = 0;
      left[i] = 1;
    }
  } else if (xn[2 * N + j] < 0.0) {
    kind[i] = 2;
    tgt[i] = x0[j];
    tgt[n_cand + i] = x0[N + j];
    tgt[2 * n_cand + i] = 0.0;
  }
}

// dL/dx* = xbar_C - (H z)_C = -r_C (r = H z - xbar), carried to x and v of
// the step's start through the targets: kind 2, x* = (x, y, 0); kind 1,
// x* = (x + t v_x, y + t v_y, 0) with t = -z / v_z (dt/dz = -1 / v_z,
// dt/dv_z = z / v_z^2).  The rows are distinct nodes: no two threads meet.
__global__ void k_contact_target_vjp(int N, int n_cand, const int32_t* __restrict__ cand,
                                     const int32_t* __restrict__ kind, const double* __restrict__ x,
                                     const double* __restrict__ v, const double* __restrict__ r,
                                     double* __restrict__ gx, double* __restrict__ gv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cand || !kind[i]) return;
  const int64_t j = cand[i];
  const double a = -r[j], b = -r[N + j];
  gx[j] += a;
  gx[N + j] += b;
  if (kind[i] == 1) {
    const double z = x[2 * N + j], vx = v[j], vy = v[N + j], vz = v[2 * N + j];
    const double t = -z / vz, sxy = vx * a + vy * b;
    gv[j] += t * a;
    gv[N + j] += t * b;
    gx[2 * N + j] += -sxy / vz;
    gv[2 * N + j] += sxy * z / (vz * vz);
  }
}

// Dense reduced inverse for meshes whose A^{-1} is held dense (internal
// order, n free nodes): W = A^{-1} - A^{-1}_{:,C} S^{-1} A^{-1}_{C,:}, the
// inverse of A_{C̄×C̄} on the rows and columns outside C, with the rows and
// columns of C set to 0.  T = A^{-1}_{:,C} S^{-1} first ([n][c]), then W by
// rows, thread j over the columns (coalesced), the row's T in LDS.
__global__ void __launch_bounds__(256) k_contact_red_t(int n, const int32_t* __restrict__ inv,
                                                       const int32_t* __restrict__ cand,
                                                       const int32_t* __restrict__ set, int c,
                                                       const double* __restrict__ Ainv,
                                                       const double* __restrict__ Sinv, double* __restrict__ T) {
  __shared__ double row[kContactMaxSet];
  const int i = blockIdx.x;
  for (int a = threadIdx.x; a < c; a += blockDim.x) row[a] = Ainv[(int64_t)i * n + inv[cand[set[a]]]];
  __syncthreads();
  for (int b = threadIdx.x; b < c; b += blockDim.x) {
    double acc = 0.0;
    for (int a = 0; a < c; ++a) acc += row[a] * Sinv[a * c + b];
    T[(int64_t)i * c + b] = acc;
  }
}

__global__ void __launch_bounds__(256) k_contact_red_w(int n, const int32_t* __restrict__ inv,
                                                       const int32_t* __restrict__ cand,
                                                       const int32_t* __restrict__ set, int c,
                                                       const double* __restrict__ Ainv,
                                                       const double* __restrict__ T, uint8_t* __restrict__ in_c,
                                                       double* __restrict__ W) {
  __shared__ double trow[kContactMaxSet];
  __shared__ int cb[kContactMaxSet];
  const int i = blockIdx.y;
  for (int b = threadIdx.x; b < c; b += blockDim.x) {
    trow[b] = T[(int64_t)i * c + b];
    cb[b] = inv[cand[set[b]]];
  }
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double w = 0.0;
  if (!in_c[i] && !in_c[j]) {
    w = Ainv[(int64_t)i * n + j];
    for (int b = 0; b < c; ++b) w -= trow[b] * Ainv[(int64_t)cb[b] * n + j];
  }
  W[(int64_t)i * n + j] = w;
}

__global__ void k_contact_zero_u8(int n, uint8_t* __restrict__ a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// in_c[row] = 1 for the internal rows of the set's nodes (on a zeroed array).
__global__ void k_contact_red_mark(const int32_t* __restrict__ inv, const int32_t* __restrict__ cand,
                                   const int32_t* __restrict__ set, int c, uint8_t* __restrict__ in_c) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < c) in_c[inv[cand[set[a]]]] = 1;
}

// x[perm[i]] -= sum_j W[i][j] r[perm[j]] for the n free rows: the reduced
// global step x_{C̄} <- x_{C̄} - (A_{C̄×C̄})^{-1} r_{C̄} in one launch (W's rows and
// columns of C are 0, so x_C keeps its value bit for bit).  Each workgroup
// gathers r into LDS ([3][n], internal order); a wave takes rows in turn,
// lanes over the columns (coalesced rows of W), three wave sums.
__global__ void __launch_bounds__(kContactDenseThreads) k_contact_dense_step(
    int n, int N, const int32_t* __restrict__ perm, const double* __restrict__ W, const double* __restrict__ r,
    double* __restrict__ x, const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double rl[];  // [3][n]
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int64_t p = perm[j];
    rl[j] = r[p];
    rl[n + j] = r[N + p];
    rl[2 * n + j] = r[2 * (int64_t)N + p];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  for (int i = blockIdx.x * waves + wid; i < n; i += gridDim.x * waves) {
    const double* row = W + (int64_t)i * n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    // eight loads in flight per lane before their products (a row is at most
    // 32 loads per lane)
    for (int j0 = lane; j0 < n; j0 += 8 * 64) {
      double w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + 64 * u;
        w[u] = j < n ? row[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + 64 * u;
        if (j < n) {
          s0 += w[u] * rl[j];
          s1 += w[u] * rl[n + j];
          s2 += w[u] * rl[2 * n + j];
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    if (lane == 0) {
      const int64_t p = perm[i];
      x[p] -= s0;
      x[N + p] -= s1;
      x[2 * (int64_t)N + p] -= s2;
    }
  }
  clock_exit(ck);
}

// x at the active set's nodes = x* ([3][c]).
__global__ void k_contact_set(int N, const int32_t* __restrict__ cand, const int32_t* __restrict__ set, int c,
                              const double* __restrict__ xstar, double* __restrict__ x) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * c) return;
  const int comp = idx / c, k = idx % c;
  x[(int64_t)comp * N + cand[set[k]]] = xstar[idx];
}

}  // namespace

size_t contact_factor_lds(int c) { return ((size_t)c * c + 2 * (size_t)c) * sizeof(double); }

void launch_contact_unit(hipStream_t s, int N, int n_cand, const int32_t* cand, int k0, double* b) {
  hipLaunchKernelGGL(k_contact_unit, dim3(1), dim3(64), 0, s, N, n_cand, cand, k0, b);
}

void launch_contact_collect(hipStream_t s, int N, int n_cand, int k0, const double* x, double* B1) {
  const int64_t t = 3 * (int64_t)N;
  hipLaunchKernelGGL(k_contact_collect, dim3((unsigned)((t + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, N, n_cand,
                     k0, x, B1);
}

hipError_t launch_contact_factor(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c,
                                 const double* B1, double* Sinv, int* status) {
  const size_t lds = contact_factor_lds(c);
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_contact_factor, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_contact_factor, dim3(1), dim3(kContactThreads), lds, s, N, cand, set, c, B1, Sinv, status);
  return hipGetLastError();
}

void launch_contact_lam(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c, const double* Sinv,
                        const double* a1, double* lam, const IterState* st) {
  hipLaunchKernelGGL(k_contact_lam, dim3(1), dim3(kContactThreads), 0, s, N, cand, set, c, Sinv, a1, lam, st);
}

void launch_contact_descend(hipStream_t s, int N, const int32_t* set, int c, const double* B1, const double* lam,
                            const double* d, const uint8_t* mask, double* x, const IterState* st) {
  DPD_LAUNCH(k_contact_descend, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N, set, c, B1, lam, d, mask,
             x, st);
}

static unsigned cand_blocks(int n_cand) { return (unsigned)((n_cand + 255) / 256); }

void launch_contact_detect(hipStream_t s, int N, int n_cand, const int32_t* cand, double h, const double* x,
                           const double* v, double* tgt, int32_t* kind, uint8_t* left) {
  hipLaunchKernelGGL(k_contact_detect, dim3(cand_blocks(n_cand)), dim3(256), 0, s, N, n_cand, cand, h, x, v, tgt,
                     kind, left);
}

void launch_contact_mark(hipStream_t s, int n_cand, const int32_t* cand, const int32_t* kind, uint8_t* mask) {
  hipLaunchKernelGGL(k_contact_mark, dim3(cand_blocks(n_cand)), dim3(256), 0, s, n_cand, cand, kind, mask);
}

void launch_contact_place(hipStream_t s, int N, int n_cand, const int32_t* cand, const int32_t* kind,
                          const double* tgt, double* x) {
  hipLaunchKernelGGL(k_contact_place, dim3(cand_blocks(n_cand)), dim3(256), 0, s, N, n_cand, cand, kind, tgt, x);
}

void launch_contact_active_set(hipStream_t s, int N, int n_cand, const int32_t* cand, const double* x0,
                               const double* xn, const double* r, int32_t* kind, uint8_t* left, double* tgt) {
  hipLaunchKernelGGL(k_contact_active_set, dim3(cand_blocks(n_cand)), dim3(256), 0, s, N, n_cand, cand, x0, xn, r,
                     kind, left, tgt);
}

hipError_t launch_contact_reduced_inverse(hipStream_t s, int n, const int32_t* inv, const int32_t* cand,
                                          const int32_t* set, int c, const double* Ainv, const double* Sinv,
                                          double* T, uint8_t* in_c, double* W) {
  hipLaunchKernelGGL(k_contact_zero_u8, dim3((n + 255) / 256), dim3(256), 0, s, n, in_c);
  if (c > 0) {
    hipLaunchKernelGGL(k_contact_red_mark, dim3((c + 63) / 64), dim3(64), 0, s, inv, cand, set, c, in_c);
    hipLaunchKernelGGL(k_contact_red_t, dim3(n), dim3(256), 0, s, n, inv, cand, set, c, Ainv, Sinv, T);
  }
  hipLaunchKernelGGL(k_contact_red_w, dim3((n + 255) / 256, n), dim3(256), 0, s, n, inv, cand, set, c, Ainv, T, in_c,
                     W);
  return hipGetLastError();
}

size_t contact_dense_lds(int n) { return 3 * (size_t)n * sizeof(double); }

hipError_t launch_contact_dense_step(hipStream_t s, int n, int N, const int32_t* perm, const double* W,
                                     const double* r, double* x, const IterState* st) {
  if (n < 1 || n > kContactDenseMaxRows) return hipErrorInvalidValue;
  const size_t lds = contact_dense_lds(n);  // at most 48 KiB: no attribute needed
  const int waves = kContactDenseThreads / 64;
  const unsigned blocks = (unsigned)((n + waves - 1) / waves);
  DPD_LAUNCH(k_contact_dense_step, dim3(blocks), dim3(kContactDenseThreads), lds, s, n, N, perm, W, r, x, st);
  return hipGetLastError();
}

void launch_contact_target_vjp(hipStream_t s, int N, int n_cand, const int32_t* cand, const int32_t* kind,
                               const double* x, const double* v, const double* r, double* gx, double* gv) {
  hipLaunchKernelGGL(k_contact_target_vjp, dim3(cand_blocks(n_cand)), dim3(256), 0, s, N, n_cand, cand, kind, x, v,
                     r, gx, gv);
}

void launch_contact_update(hipStream_t s, int N, const int32_t* set, int c, const double* B1, const double* lam,
                           double* x) {
  DPD_LAUNCH(k_contact_update, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N, set, c, B1, lam, x);
}

void launch_contact_set(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c, const double* xstar,
                        double* x) {
  hipLaunchKernelGGL(k_contact_set, dim3((3 * c + 63) / 64), dim3(64), 0, s, N, cand, set, c, xstar, x);
}

}  // namespace dpd
