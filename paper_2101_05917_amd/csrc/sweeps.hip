// Level-scheduled supernodal triangular sweeps (gfx950): the global step
// x = A^{-1} b of Alg. 1 and Alg. 2 with the factor of A computed once.
//
// Every supernode s stores the panel P_s = [inv(L_ss); -L_Rs inv(L_ss)]
// (ncols + nrows rows, ncols columns) in column-major order, plus a row-major
// copy.  A level of the elimination tree is a set of independent dense
// matrix-vector products with three right-hand sides (x, y, z):
//   forward   y_s = inv(L_ss) b~_s and the updates -L_Rs inv(L_ss) b~_s of
//             s's ancestors, b~_s = b_s + (updates of s's descendants);
//   backward  x_s = P_s^T [y_s; x_R].
// Updates are gathered by their consumer in a fixed order (no atomics).
//
// Each kernel launch processes one level; a task (one workgroup) is one block
// of rows or columns of one supernode.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dpd {

namespace {

constexpr int kGroup = 256;  // threads per task

// Accesses to the vectors that tasks exchange (right-hand sides gathered
// ahead, forward updates, the two sweeps' solutions).  Between launches plain
// loads and stores suffice; inside the single-launch solve (kCoh) they are
// device-coherent (agent-scope relaxed atomics), so a task sees what a task
// on another XCD wrote without cache write-backs or invalidations, and the
// read-only panels stay cached.
template <bool kCoh>
__device__ inline double ldx(const double* p) {
  if constexpr (kCoh) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool kCoh>
__device__ inline void stx(double* p, double v) {
  if constexpr (kCoh) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// b~ for the task's supernode into bs[3][nc]: pre-gathered (bt) or gathered here.
template <bool kCoh = false>
__device__ inline void stage_rhs(const DevSolve& S, const SweepTask& t, const double* __restrict__ b,
                                 int N, bool pre, int tid, double* bs, int nthreads = kGroup) {
  const int nc = t.ncols;
  for (int c = tid; c < nc; c += nthreads) {
    const int j = t.col0 + c;
    double v0, v1, v2;
    if (pre) {
      v0 = ldx<kCoh>(S.bt + j);
      v1 = ldx<kCoh>(S.bt + (int64_t)S.nf + j);
      v2 = ldx<kCoh>(S.bt + 2 * (int64_t)S.nf + j);
    } else {
      const int node = S.perm_pub[j];
      v0 = b[node];
      v1 = b[(int64_t)N + node];
      v2 = b[2 * (int64_t)N + node];
      // four contributions at a time, their loads issued together
      int k = S.cptr[j];
      const int k1 = S.cptr[j + 1];
      const double* U = S.U;
      for (; k + 3 < k1; k += 4) {
        const int64_t p0 = 3 * (int64_t)S.cidx[k], p1 = 3 * (int64_t)S.cidx[k + 1];
        const int64_t p2 = 3 * (int64_t)S.cidx[k + 2], p3 = 3 * (int64_t)S.cidx[k + 3];
        v0 += (ldx<kCoh>(U + p0) + ldx<kCoh>(U + p1)) + (ldx<kCoh>(U + p2) + ldx<kCoh>(U + p3));
        v1 += (ldx<kCoh>(U + p0 + 1) + ldx<kCoh>(U + p1 + 1)) + (ldx<kCoh>(U + p2 + 1) + ldx<kCoh>(U + p3 + 1));
        v2 += (ldx<kCoh>(U + p0 + 2) + ldx<kCoh>(U + p1 + 2)) + (ldx<kCoh>(U + p2 + 2) + ldx<kCoh>(U + p3 + 2));
      }
      for (; k < k1; ++k) {
        const int64_t pos = 3 * (int64_t)S.cidx[k];
        v0 += ldx<kCoh>(U + pos);
        v1 += ldx<kCoh>(U + pos + 1);
        v2 += ldx<kCoh>(U + pos + 2);
      }
    }
    bs[c] = v0;
    bs[nc + c] = v1;
    bs[2 * nc + c] = v2;
  }
}

template <bool kCoh = false>
__device__ inline void store_fwd_row(const DevSolve& S, const SweepTask& t, int r, double a0, double a1,
                                     double a2) {
  if (r < t.ncols) {
    const int j = t.col0 + r;
    stx<kCoh>(S.y_int + j, a0);
    stx<kCoh>(S.y_int + (int64_t)S.nf + j, a1);
    stx<kCoh>(S.y_int + 2 * (int64_t)S.nf + j, a2);
  } else {
    const int64_t pos = 3 * (t.u_off + (r - t.ncols));
    stx<kCoh>(S.U + pos, a0);
    stx<kCoh>(S.U + pos + 1, a1);
    stx<kCoh>(S.U + pos + 2, a2);
  }
}

// v[3][ld] = [y_s; x_R] for the backward task.
template <bool kCoh = false>
__device__ inline void stage_solution(const DevSolve& S, const SweepTask& t, int tid, double* vs,
                                      int nthreads = kGroup) {
  const int nc = t.ncols, ld = t.ncols + t.nrows;
  const int64_t nf = S.nf;
  const int* rows = S.rows + t.rows_off;
  for (int r = tid; r < ld; r += nthreads) {
    const double* src = S.y_int;
    int j = t.col0 + r;
    if (r >= nc) {
      src = S.x_int;
      j = rows[r - nc];
    }
    vs[r] = ldx<kCoh>(src + j);
    vs[ld + r] = ldx<kCoh>(src + nf + j);
    vs[2 * ld + r] = ldx<kCoh>(src + 2 * nf + j);
  }
}

template <bool kCoh = false>
__device__ inline void store_bwd_col(const DevSolve& S, const SweepTask& t, int c, double x0, double x1,
                                     double x2, double* __restrict__ out, int N, double alpha,
                                     int accumulate) {
  const int j = t.col0 + c;
  const int64_t nf = S.nf;
  stx<kCoh>(S.x_int + j, x0);
  stx<kCoh>(S.x_int + nf + j, x1);
  stx<kCoh>(S.x_int + 2 * nf + j, x2);
  const int node = S.perm_pub[j];
  if (accumulate) {
    out[node] += alpha * x0;
    out[(int64_t)N + node] += alpha * x1;
    out[2 * (int64_t)N + node] += alpha * x2;
  } else {
    out[node] = alpha * x0;
    out[(int64_t)N + node] = alpha * x1;
    out[2 * (int64_t)N + node] = alpha * x2;
  }
}

// Forward task, blocks of at most 64 columns: 64 panel rows, lane per row
// (column-major panel, coalesced across lanes), the columns split over the
// NT / 64 waves (c = wave mod NT / 64) so that each row has that many streams
// of loads in flight; the partial sums meet in LDS (after the staged
// right-hand sides) and are added in wave order.
// Every thread of the workgroup calls it (its barriers are the workgroup's).
template <typename T, int NT, bool kCoh = false>
__device__ inline void fwd_narrow_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panel,
                                       const double* __restrict__ b, int N, bool active, int tid,
                                       double* bs) {
  constexpr int kW = NT / 64;
  __syncthreads();
  if (active) stage_rhs<kCoh>(S, t, b, N, false, tid, bs, NT);
  __syncthreads();
  const int nc = active ? t.ncols : 0, ld = active ? t.ncols + t.nrows : 0;
  const int lane = tid & 63, wid = tid >> 6;
  const bool act = active && lane < t.count;
  const int r = t.first + (act ? lane : 0);
  const T* P = panel + t.panel_off + r;
  const int cend = act ? (r < nc ? r + 1 : nc) : 0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  int c = wid;
  for (; c + 3 * kW < cend; c += 4 * kW) {
    const double p0 = (double)P[(int64_t)c * ld], p1 = (double)P[(int64_t)(c + kW) * ld];
    const double p2 = (double)P[(int64_t)(c + 2 * kW) * ld], p3 = (double)P[(int64_t)(c + 3 * kW) * ld];
    a0 += p0 * bs[c] + p1 * bs[c + kW] + p2 * bs[c + 2 * kW] + p3 * bs[c + 3 * kW];
    a1 += p0 * bs[nc + c] + p1 * bs[nc + c + kW] + p2 * bs[nc + c + 2 * kW] + p3 * bs[nc + c + 3 * kW];
    a2 += p0 * bs[2 * nc + c] + p1 * bs[2 * nc + c + kW] + p2 * bs[2 * nc + c + 2 * kW] +
          p3 * bs[2 * nc + c + 3 * kW];
  }
  for (; c < cend; c += kW) {
    const double p = (double)P[(int64_t)c * ld];
    a0 += p * bs[c];
    a1 += p * bs[nc + c];
    a2 += p * bs[2 * nc + c];
  }
  double* red = bs + 3 * nc;   // [kW][64][3]
  if (active) {
    red[(wid * 64 + lane) * 3 + 0] = a0;
    red[(wid * 64 + lane) * 3 + 1] = a1;
    red[(wid * 64 + lane) * 3 + 2] = a2;
  }
  __syncthreads();
  if (wid == 0 && act) {
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      x0 += red[(k * 64 + lane) * 3 + 0];
      x1 += red[(k * 64 + lane) * 3 + 1];
      x2 += red[(k * 64 + lane) * 3 + 2];
    }
    store_fwd_row<kCoh>(S, t, r, x0, x1, x2);
  }
}

// Forward task, wide blocks: LPR lanes per panel row on the row-major copy
// (64 / LPR rows per wave), each lane walking the row's columns with stride
// LPR, then a reduction over the row's LPR lanes.  LPR is chosen per level so
// that every lane reads at least about eight entries of its row.  A task of NT
// lanes (16 waves) covers one pass of rows, so the block's right-hand sides
// staged in LDS serve 16 x 64 / LPR rows.
template <typename T, int LPR, int NT, bool kCoh = false>
__device__ inline void fwd_wide_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panelT,
                                     const double* __restrict__ b, int N, bool pre, bool active, int tid,
                                     double* bs) {
  __syncthreads();
  if (active) stage_rhs<kCoh>(S, t, b, N, pre, tid, bs, NT);
  __syncthreads();
  if (!active) return;
  constexpr int RPW = 64 / LPR;
  const int nc = t.ncols;
  const int lane = tid & 63, wid = tid >> 6, sub = lane / LPR, li = lane % LPR;
  const T* Pb = panelT + t.panel_off;
  for (int base = wid * RPW; base < t.count; base += (NT / 64) * RPW) {
    const int rr = base + sub;
    const bool act = rr < t.count;
    const int r = t.first + rr;
    const T* row = Pb + (int64_t)(act ? r : 0) * nc;
    const int cend = !act ? 0 : (r < nc ? r + 1 : nc);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int c = li;
    for (; c + 3 * LPR < cend; c += 4 * LPR) {
      const double p0 = (double)row[c], p1 = (double)row[c + LPR];
      const double p2 = (double)row[c + 2 * LPR], p3 = (double)row[c + 3 * LPR];
      a0 += p0 * bs[c] + p1 * bs[c + LPR] + p2 * bs[c + 2 * LPR] + p3 * bs[c + 3 * LPR];
      a1 += p0 * bs[nc + c] + p1 * bs[nc + c + LPR] + p2 * bs[nc + c + 2 * LPR] + p3 * bs[nc + c + 3 * LPR];
      a2 += p0 * bs[2 * nc + c] + p1 * bs[2 * nc + c + LPR] + p2 * bs[2 * nc + c + 2 * LPR] +
            p3 * bs[2 * nc + c + 3 * LPR];
    }
    for (; c < cend; c += LPR) {
      const double p = (double)row[c];
      a0 += p * bs[c];
      a1 += p * bs[nc + c];
      a2 += p * bs[2 * nc + c];
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, 64);
      a1 += __shfl_xor(a1, off, 64);
      a2 += __shfl_xor(a2, off, 64);
    }
    if (act && li == 0) store_fwd_row<kCoh>(S, t, r, a0, a1, a2);
  }
}

// Backward task: LPR lanes per panel column (64 / LPR columns per wave), each
// lane walking the column's rows from the diagonal down with stride LPR
// (column-major panel, contiguous), then a reduction over the column's lanes;
// v from LDS (kLds) or from global memory.  LPR is chosen per level so that
// every lane reads at least about eight entries of its column.
template <typename T, bool kLds, int LPR, int NT, bool kCoh = false>
__device__ inline void bwd_cols_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panel,
                                     double* __restrict__ out, int N, double alpha, int accumulate,
                                     bool active, int tid, double* vs) {
  __syncthreads();
  if (kLds && active) stage_solution<kCoh>(S, t, tid, vs, NT);
  __syncthreads();
  if (!active) return;
  constexpr int CPW = 64 / LPR;
  const int nc = t.ncols, ld = t.ncols + t.nrows;
  const int64_t nf = S.nf;
  const int* rows = S.rows + t.rows_off;
  const int lane = tid & 63, wid = tid >> 6, sub = lane / LPR, li = lane % LPR;
  for (int base = wid * CPW; base < t.count; base += (NT / 64) * CPW) {
    const int cc = base + sub;
    const bool act = cc < t.count;
    const int col = t.first + (act ? cc : 0);
    const T* Pc = panel + t.panel_off + (int64_t)col * ld;
    const int rend = act ? ld : 0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    auto term = [&](int r, double p) {
      double v0, v1, v2;
      if (kLds) {
        v0 = vs[r];
        v1 = vs[ld + r];
        v2 = vs[2 * ld + r];
      } else {
        const double* src = S.y_int;
        int j = t.col0 + r;
        if (r >= nc) {
          src = S.x_int;
          j = rows[r - nc];
        }
        v0 = ldx<kCoh>(src + j);
        v1 = ldx<kCoh>(src + nf + j);
        v2 = ldx<kCoh>(src + 2 * nf + j);
      }
      a0 += p * v0;
      a1 += p * v1;
      a2 += p * v2;
    };
    // rows above the diagonal are zeros: start at the column's own row;
    // four panel loads in flight per lane
    int r = col + li;
    for (; r + 3 * LPR < rend; r += 4 * LPR) {
      const double p0 = (double)Pc[r], p1 = (double)Pc[r + LPR];
      const double p2 = (double)Pc[r + 2 * LPR], p3 = (double)Pc[r + 3 * LPR];
      term(r, p0);
      term(r + LPR, p1);
      term(r + 2 * LPR, p2);
      term(r + 3 * LPR, p3);
    }
    for (; r < rend; r += LPR) term(r, (double)Pc[r]);
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, 64);
      a1 += __shfl_xor(a1, off, 64);
      a2 += __shfl_xor(a2, off, 64);
    }
    if (act && li == 0) store_bwd_col<kCoh>(S, t, col, a0, a1, a2, out, N, alpha, accumulate);
  }
}

// Backward task of a small supernode (at most 64 columns) on NT lanes: lane
// t takes column c = t mod W and row class t / W, with W the power of two
// at least the block's width (lanes are not left idle on narrow blocks), so
// each of the NT / W row classes walks every (NT / W)-th row of the
// row-major copy from the diagonal down (coalesced across the columns);
// the classes' partial sums meet in LDS and are added in class order.
// vs holds 3 ld doubles followed by NT x 3 reduction slots.
template <typename T, int NT, bool kCoh = false>
__device__ inline void bwd_narrow_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panelT,
                                       double* __restrict__ out, int N, double alpha, int accumulate,
                                       bool active, int tid, double* vs) {
  __syncthreads();
  if (active) stage_solution<kCoh>(S, t, tid, vs, NT);
  __syncthreads();
  const int nc = active ? t.ncols : 0, ld = active ? t.ncols + t.nrows : 0;
  double* red = vs + 3 * ld;
  const int W = nc <= 8 ? 8 : (nc <= 16 ? 16 : (nc <= 32 ? 32 : 64));
  const int parts = NT / W;
  const int c = tid % W, part = tid / W;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (active && c < nc) {
    const T* Pc = panelT + t.panel_off + c;
    // first row >= c (rows above the diagonal are zeros) in this class
    int r = c + ((part - c) % parts + parts) % parts;
    for (; r + 3 * parts < ld; r += 4 * parts) {
      const double p0 = (double)Pc[(int64_t)r * nc], p1 = (double)Pc[(int64_t)(r + parts) * nc];
      const double p2 = (double)Pc[(int64_t)(r + 2 * parts) * nc], p3 = (double)Pc[(int64_t)(r + 3 * parts) * nc];
      a0 += p0 * vs[r] + p1 * vs[r + parts] + p2 * vs[r + 2 * parts] + p3 * vs[r + 3 * parts];
      a1 += p0 * vs[ld + r] + p1 * vs[ld + r + parts] + p2 * vs[ld + r + 2 * parts] + p3 * vs[ld + r + 3 * parts];
      a2 += p0 * vs[2 * ld + r] + p1 * vs[2 * ld + r + parts] + p2 * vs[2 * ld + r + 2 * parts] +
            p3 * vs[2 * ld + r + 3 * parts];
    }
    for (; r < ld; r += parts) {
      const double p = (double)Pc[(int64_t)r * nc];
      a0 += p * vs[r];
      a1 += p * vs[ld + r];
      a2 += p * vs[2 * ld + r];
    }
  }
  if (active) {
    red[tid * 3 + 0] = a0;
    red[tid * 3 + 1] = a1;
    red[tid * 3 + 2] = a2;
  }
  __syncthreads();
  if (active && part == 0 && c < nc) {
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    for (int k = 0; k < parts; ++k) {
      x0 += red[(k * W + c) * 3 + 0];
      x1 += red[(k * W + c) * 3 + 1];
      x2 += red[(k * W + c) * 3 + 2];
    }
    store_bwd_col<kCoh>(S, t, c, x0, x1, x2, out, N, alpha, accumulate);
  }
}

// ---------------------------------------------------------------- per-level kernels

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sweep_fwd(DevSolve S, const SweepTask* __restrict__ tasks,
                                                      const T* __restrict__ panel, const double* __restrict__ b,
                                                      int N, const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double lds[];
  fwd_narrow_task<T, kBlock>(S, tasks[blockIdx.x], panel, b, N, true, threadIdx.x, lds);
  clock_exit(ck);
}

template <typename T, int LPR>
__global__ void __launch_bounds__(kWideTaskThreads) k_sweep_fwd_wide(DevSolve S, const SweepTask* __restrict__ tasks,
                                                                     const T* __restrict__ panelT,
                                                                     const double* __restrict__ b, int N, int pre,
                                                                     const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double lds[];
  fwd_wide_task<T, LPR, kWideTaskThreads>(S, tasks[blockIdx.x], panelT, b, N, pre != 0, true, threadIdx.x, lds);
  clock_exit(ck);
}

// Right-hand sides of one level with the descendants' updates added, once per
// column: bt[j] = b[perm j] + sum of the updates of row j (wave per column).
__global__ void __launch_bounds__(kBlock) k_sweep_gather(DevSolve S, const int32_t* __restrict__ cols,
                                                         int ncols, const double* __restrict__ b, int N,
                                                         const IterState* st) {
  if (st && st->done) return;
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= ncols) return;
  const int j = cols[w];
  const int k0 = S.cptr[j], k1 = S.cptr[j + 1];
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int k = k0 + lane; k < k1; k += 64) {
    const int64_t pos = 3 * (int64_t)S.cidx[k];
    v0 += S.U[pos];
    v1 += S.U[pos + 1];
    v2 += S.U[pos + 2];
  }
  v0 = wsum(v0);
  v1 = wsum(v1);
  v2 = wsum(v2);
  if (lane == 0) {
    const int node = S.perm_pub[j];
    S.bt[j] = b[node] + v0;
    S.bt[(int64_t)S.nf + j] = b[(int64_t)N + node] + v1;
    S.bt[2 * (int64_t)S.nf + j] = b[2 * (int64_t)N + node] + v2;
  }
}

template <typename T, bool kLds, int LPR>
__global__ void __launch_bounds__(kWideTaskThreads) k_sweep_bwd(DevSolve S, const SweepTask* __restrict__ tasks,
                                                                const T* __restrict__ panel,
                                                                double* __restrict__ out, int N, double alpha,
                                                                int accumulate, const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double lds[];
  bwd_cols_task<T, kLds, LPR, kWideTaskThreads>(S, tasks[blockIdx.x], panel, out, N, alpha, accumulate, true,
                                                threadIdx.x, lds);
  clock_exit(ck);
}

template <typename T>
__global__ void __launch_bounds__(kWideTaskThreads) k_sweep_bwd_narrow(DevSolve S, const SweepTask* __restrict__ tasks,
                                                             const T* __restrict__ panelT,
                                                             double* __restrict__ out, int N, double alpha,
                                                             int accumulate, const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double lds[];
  bwd_narrow_task<T, kWideTaskThreads>(S, tasks[blockIdx.x], panelT, out, N, alpha, accumulate, true, threadIdx.x,
                                       lds);
  clock_exit(ck);
}

// ---------------------------------------------------------------- batched level kernels
//
// Tasks of several handles' solves in one launch: each task names its slot
// (pad0), whose factor and vectors it uses, and runs the level kernel's own
// task code, so a slot's result is bitwise what its own level launches give.
// Every batched solve is out = A^{-1} b.

template <typename T>
__device__ inline const T* col_panel(const DevSolve& S);
template <>
__device__ inline const double* col_panel<double>(const DevSolve& S) { return S.panel64; }
template <>
__device__ inline const float* col_panel<float>(const DevSolve& S) { return S.panel32; }
template <typename T>
__device__ inline const T* row_panel(const DevSolve& S);
template <>
__device__ inline const double* row_panel<double>(const DevSolve& S) { return S.panelT64; }
template <>
__device__ inline const float* row_panel<float>(const DevSolve& S) { return S.panelT32; }

template <typename T>
__global__ void __launch_bounds__(kBlock) k_batch_sweep_fwd(const BatchSolveSlot* __restrict__ slots,
                                                            const SweepTask* __restrict__ tasks) {
  const SweepTask t = tasks[blockIdx.x];
  const BatchSolveSlot& B = slots[t.pad0];
  if (B.st && B.st->done) return;
  const DevSolve S = B.S;
  extern __shared__ double lds[];
  fwd_narrow_task<T, kBlock>(S, t, col_panel<T>(S), B.b, B.N, true, threadIdx.x, lds);
}

template <typename T, int LPR>
__global__ void __launch_bounds__(kWideTaskThreads) k_batch_sweep_fwd_wide(const BatchSolveSlot* __restrict__ slots,
                                                                           const SweepTask* __restrict__ tasks) {
  const SweepTask t = tasks[blockIdx.x];
  const BatchSolveSlot& B = slots[t.pad0];
  if (B.st && B.st->done) return;
  const DevSolve S = B.S;
  extern __shared__ double lds[];
  fwd_wide_task<T, LPR, kWideTaskThreads>(S, t, row_panel<T>(S), B.b, B.N, t.pad1 != 0, true, threadIdx.x, lds);
}

// k_sweep_gather's arithmetic on (slot, column) entries, wave per entry.
__global__ void __launch_bounds__(kBlock) k_batch_sweep_gather(const BatchSolveSlot* __restrict__ slots,
                                                               const int2* __restrict__ cols, int ncols) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= ncols) return;
  const int2 e = cols[w];
  const BatchSolveSlot& B = slots[e.x];
  if (B.st && B.st->done) return;
  const DevSolve& S = B.S;
  const int j = e.y;
  const int k0 = S.cptr[j], k1 = S.cptr[j + 1];
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int k = k0 + lane; k < k1; k += 64) {
    const int64_t pos = 3 * (int64_t)S.cidx[k];
    v0 += S.U[pos];
    v1 += S.U[pos + 1];
    v2 += S.U[pos + 2];
  }
  v0 = wsum(v0);
  v1 = wsum(v1);
  v2 = wsum(v2);
  if (lane == 0) {
    const int node = S.perm_pub[j];
    const int64_t N = B.N;
    S.bt[j] = B.b[node] + v0;
    S.bt[(int64_t)S.nf + j] = B.b[N + node] + v1;
    S.bt[2 * (int64_t)S.nf + j] = B.b[2 * N + node] + v2;
  }
}

template <typename T, bool kLds, int LPR>
__global__ void __launch_bounds__(kWideTaskThreads) k_batch_sweep_bwd(const BatchSolveSlot* __restrict__ slots,
                                                                      const SweepTask* __restrict__ tasks) {
  const SweepTask t = tasks[blockIdx.x];
  const BatchSolveSlot& B = slots[t.pad0];
  if (B.st && B.st->done) return;
  const DevSolve S = B.S;
  extern __shared__ double lds[];
  bwd_cols_task<T, kLds, LPR, kWideTaskThreads>(S, t, col_panel<T>(S), B.out, B.N, 1.0, 0, true, threadIdx.x,
                                                lds);
}

template <typename T>
__global__ void __launch_bounds__(kWideTaskThreads) k_batch_sweep_bwd_narrow(const BatchSolveSlot* __restrict__ slots,
                                                                             const SweepTask* __restrict__ tasks) {
  const SweepTask t = tasks[blockIdx.x];
  const BatchSolveSlot& B = slots[t.pad0];
  if (B.st && B.st->done) return;
  const DevSolve S = B.S;
  extern __shared__ double lds[];
  bwd_narrow_task<T, kWideTaskThreads>(S, t, row_panel<T>(S), B.out, B.N, 1.0, 0, true, threadIdx.x, lds);
}

// ---------------------------------------------------------------- single-launch solve

constexpr uint32_t kDagSpinLimit = 1u << 22;  // about 4 s of polling per wait: then abort

__device__ inline uint32_t ldu(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t addu(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (one lane) until the entry's dependencies are met; false after an abort
// (this wait timed out, or another one did).
__device__ inline bool dag_wait(const DagEntry& e, const DagSn* __restrict__ sni, uint32_t* ctr, int ns) {
  uint32_t* cdone = ctr + kDagHeader;
  uint32_t* tdone = cdone + ns;
  uint32_t* gdone = tdone + ns;
  uint32_t* bdone = gdone + ns;
  const int nsub = (e.kind == kDagFwdNarrow || e.kind == kDagBwdNarrow) ? e.n : 1;
  // unrolled: constant indices keep the entry in registers
#pragma unroll
  for (int k = 0; k < kDagSub; ++k) {
    if (k >= nsub) break;
    const int s = e.sn[k];
    const DagSn d = sni[s];
    const uint32_t* w1 = nullptr;
    const uint32_t* w2 = nullptr;
    uint32_t n1 = 0, n2 = 0;
    if (e.kind == kDagBwdCols || e.kind == kDagBwdNarrow) {
      if (d.parent >= 0) {
        w1 = bdone + d.parent;
        n1 = (uint32_t)sni[d.parent].ntb;
      } else {
        w1 = tdone + s;
        n1 = (uint32_t)d.ntf;
      }
    } else {
      w1 = cdone + s;
      n1 = (uint32_t)d.nch;
      if (e.kind != kDagGather) {
        w2 = gdone + s;
        n2 = (uint32_t)d.ngt;
      }
    }
    for (uint32_t spin = 0;; ++spin) {
      if (ldu(w1) >= n1 && (!w2 || ldu(w2) >= n2)) break;
      if (ldu(ctr + kDagAbort) != 0u || spin >= kDagSpinLimit) {
        __hip_atomic_store(ctr + kDagAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return true;
}

// Report the entry's level tasks done (one lane, after the workgroup's
// stores have completed).
__device__ inline void dag_signal(const DagEntry& e, const DagSn* __restrict__ sni, uint32_t* ctr, int ns) {
  uint32_t* cdone = ctr + kDagHeader;
  uint32_t* tdone = cdone + ns;
  uint32_t* gdone = tdone + ns;
  uint32_t* bdone = gdone + ns;
  if (e.kind == kDagGather) {
    addu(gdone + e.sn[0], 1u);
    return;
  }
  const bool narrow = e.kind == kDagFwdNarrow || e.kind == kDagBwdNarrow;
  const int nsub = narrow ? e.n : 1;
#pragma unroll
  for (int k = 0; k < kDagSub; ++k) {
    if (k >= nsub) break;
    const int s = e.sn[k];
    if (e.kind == kDagBwdCols || e.kind == kDagBwdNarrow) {
      addu(bdone + s, 1u);
    } else {
      const DagSn d = sni[s];
      if (addu(tdone + s, 1u) + 1u == (uint32_t)d.ntf && d.parent >= 0) addu(cdone + d.parent, 1u);
    }
  }
}

// The entry kinds of the single-launch solve.
// One narrow forward task on the workgroup's first 256 lanes (the level
// kernel's arithmetic; the other lanes only take part in the barriers).
template <typename T>
__device__ inline void dag_fwd_narrow(const DevSolve& S, const DagEntry& e, const SweepTask* __restrict__ fwd,
                                            const T* __restrict__ panel, const double* __restrict__ b, int N,
                                            bool ok, int tid, double* lds) {
  fwd_narrow_task<T, kBlock, true>(S, fwd[e.first], panel, b, N, ok && tid < kBlock, tid & (kBlock - 1), lds);
}

template <typename T>
__device__ inline void dag_fwd_wide(const DevSolve& S, const DagEntry& e, const SweepTask* __restrict__ fwd,
                                          const T* __restrict__ panelT, const double* __restrict__ b, int N,
                                          bool ok, int tid, double* lds) {
  const SweepTask& tk = fwd[e.first];
  const bool pre = (e.flags & 1) != 0;
  if (e.lpr == 64) fwd_wide_task<T, 64, kDagThreads, true>(S, tk, panelT, b, N, pre, ok, tid, lds);
  else if (e.lpr == 32) fwd_wide_task<T, 32, kDagThreads, true>(S, tk, panelT, b, N, pre, ok, tid, lds);
  else fwd_wide_task<T, 16, kDagThreads, true>(S, tk, panelT, b, N, pre, ok, tid, lds);
}

// Pre-gathered right-hand sides of up to 16 columns of one supernode, a wave
// per column (the arithmetic of k_sweep_gather).
__device__ inline void dag_gather(const DevSolve& S, const DagEntry& e, const int32_t* __restrict__ gcols,
                                        const double* __restrict__ b, int N, bool ok, int tid) {
  const int lane = tid & 63, w = tid >> 6;
  if (!ok || w >= e.n) return;
  const int j = gcols[e.first + w];
  const int k0 = S.cptr[j], k1 = S.cptr[j + 1];
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int k = k0 + lane; k < k1; k += 64) {
    const int64_t pos = 3 * (int64_t)S.cidx[k];
    v0 += ldx<true>(S.U + pos);
    v1 += ldx<true>(S.U + pos + 1);
    v2 += ldx<true>(S.U + pos + 2);
  }
  v0 = wsum(v0);
  v1 = wsum(v1);
  v2 = wsum(v2);
  if (lane == 0) {
    const int node = S.perm_pub[j];
    stx<true>(S.bt + j, b[node] + v0);
    stx<true>(S.bt + (int64_t)S.nf + j, b[(int64_t)N + node] + v1);
    stx<true>(S.bt + 2 * (int64_t)S.nf + j, b[2 * (int64_t)N + node] + v2);
  }
}

// The plan stages every backward column task's vector in LDS.
template <typename T>
__device__ inline void dag_bwd_cols(const DevSolve& S, const DagEntry& e, const SweepTask* __restrict__ bwd,
                                          const T* __restrict__ panel, double* __restrict__ out, int N,
                                          double alpha, int accumulate, bool ok, int tid, double* lds) {
  const SweepTask& tk = bwd[e.first];
  if (e.lpr == 64) bwd_cols_task<T, true, 64, kDagThreads, true>(S, tk, panel, out, N, alpha, accumulate, ok, tid, lds);
  else if (e.lpr == 32) bwd_cols_task<T, true, 32, kDagThreads, true>(S, tk, panel, out, N, alpha, accumulate, ok, tid, lds);
  else bwd_cols_task<T, true, 16, kDagThreads, true>(S, tk, panel, out, N, alpha, accumulate, ok, tid, lds);
}

// One narrow backward task on the whole workgroup (the level kernel's arithmetic).
template <typename T>
__device__ inline void dag_bwd_narrow(const DevSolve& S, const DagEntry& e, const SweepTask* __restrict__ bwd,
                                            const T* __restrict__ panelT, double* __restrict__ out, int N,
                                            double alpha, int accumulate, bool ok, int tid, double* lds,
                                            int bwd_region) {
  (void)bwd_region;
  bwd_narrow_task<T, kDagThreads, true>(S, bwd[e.first], panelT, out, N, alpha, accumulate, ok, tid, lds);
}

// Both sweeps of x = A^{-1} b in one launch: persistent workgroups take queue
// entries in order (a ticket claimed one entry ahead), wait for the entries
// they depend on, run them with the level kernels' arithmetic and report
// them.  Entries only depend on earlier ones and are claimed in order, so the
// lowest unfinished entry can always run and the queue drains.  Waits are
// bounded: a timeout raises the abort flag, every later wait gives up, the
// remaining entries are skipped, and the launch still drains; the last
// workgroup to leave zeroes the counters for the next launch and counts an
// aborted launch in a word the host reads.
template <typename T>
__global__ void __launch_bounds__(kDagThreads) k_solve_dag(
    DevSolve S, const DagEntry* __restrict__ q, int nq, const SweepTask* __restrict__ fwd,
    const SweepTask* __restrict__ bwd, const int32_t* __restrict__ gcols, const DagSn* __restrict__ sni,
    int ns, uint32_t* ctr, int bwd_region, const T* __restrict__ panel, const T* __restrict__ panelT,
    const double* __restrict__ b, double* __restrict__ out, int N, double alpha, int accumulate,
    const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double lds[];
  __shared__ int s_next, s_ok, s_last;
  const int tid = threadIdx.x;
  if (tid == 0) s_next = (int)addu(ctr + kDagTicket, 1u);
  __syncthreads();
  for (;;) {
    // uniform across the workgroup: the entry is read with scalar loads
    const int t = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();
    if (t >= nq) break;
    const DagEntry e = q[t];
    if (tid == 0) {
      s_next = (int)addu(ctr + kDagTicket, 1u);
      s_ok = dag_wait(e, sni, ctr, ns) ? 1 : 0;
    }
    __syncthreads();
    const bool ok = s_ok != 0;
    switch (e.kind) {
      case kDagFwdNarrow:
        dag_fwd_narrow<T>(S, e, fwd, panel, b, N, ok, tid, lds);
        break;
      case kDagFwdWide:
        dag_fwd_wide<T>(S, e, fwd, panelT, b, N, ok, tid, lds);
        break;
      case kDagGather:
        dag_gather(S, e, gcols, b, N, ok, tid);
        break;
      case kDagBwdCols:
        dag_bwd_cols<T>(S, e, bwd, panel, out, N, alpha, accumulate, ok, tid, lds);
        break;
      default:
        dag_bwd_narrow<T>(S, e, bwd, panelT, out, N, alpha, accumulate, ok, tid, lds, bwd_region);
        break;
    }
    // the entry's stores complete before it is reported
    __syncthreads();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0 && ok) dag_signal(e, sni, ctr, ns);
  }
  __syncthreads();
  if (tid == 0) {
    // this workgroup's counter updates complete before it counts itself out
    __builtin_amdgcn_s_waitcnt(0);
    s_last = addu(ctr + kDagExit, 1u) == gridDim.x - 1 ? 1 : 0;
  }
  __syncthreads();
  if (s_last) {
    uint32_t* cnt = ctr + kDagHeader;
    for (int i = tid; i < 4 * ns; i += kDagThreads)
      __hip_atomic_store(cnt + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
      if (ldu(ctr + kDagAbort) != 0u) addu(ctr + kDagAborts, 1u);
      __hip_atomic_store(ctr + kDagAbort, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctr + kDagTicket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctr + kDagExit, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  clock_exit(ck);
}

}  // namespace

// ---------------------------------------------------------------- launchers


void launch_sweep_fwd(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks, int lds_cols,
                      bool fp32, const double* b, int N, const IterState* st) {
  const size_t lds = (size_t)lds_fwd_narrow(lds_cols) * sizeof(double);
  if (fp32)
    DPD_LAUNCH(k_sweep_fwd<float>, dim3(ntasks), dim3(kBlock), lds, s, S, tasks, S.panel32, b, N, st);
  else
    DPD_LAUNCH(k_sweep_fwd<double>, dim3(ntasks), dim3(kBlock), lds, s, S, tasks, S.panel64, b, N, st);
}

void launch_sweep_fwd_wide(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks,
                           int lds_cols, bool fp32, const double* b, int N, const int32_t* gather_cols,
                           int n_gather, const IterState* st) {
  const size_t lds = (size_t)3 * lds_cols * sizeof(double);
  const int pre = gather_cols != nullptr && n_gather > 0;
  if (pre) {
    const int waves = kBlock / 64;
    hipLaunchKernelGGL(k_sweep_gather, dim3((n_gather + waves - 1) / waves), dim3(kBlock), 0, s, S,
                       gather_cols, n_gather, b, N, st);
  }
  // lanes per row: at least about eight columns per lane on the level's widest block
  const int lpr = sweep_lanes(lds_cols);
#define DPD_FWD_WIDE(T, L, P)                                                                       \
  DPD_LAUNCH((k_sweep_fwd_wide<T, L>), dim3(ntasks), dim3(kWideTaskThreads), lds, s, S, tasks, P, b, N, \
             pre, st)
  if (fp32) {
    if (lpr == 64) DPD_FWD_WIDE(float, 64, S.panelT32);
    else if (lpr == 32) DPD_FWD_WIDE(float, 32, S.panelT32);
    else DPD_FWD_WIDE(float, 16, S.panelT32);
  } else {
    if (lpr == 64) DPD_FWD_WIDE(double, 64, S.panelT64);
    else if (lpr == 32) DPD_FWD_WIDE(double, 32, S.panelT64);
    else DPD_FWD_WIDE(double, 16, S.panelT64);
  }
#undef DPD_FWD_WIDE
}

void launch_sweep_bwd(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks, int lds_rows,
                      bool use_lds, bool fp32, double* out, int N, double alpha, int accumulate,
                      const IterState* st) {
  const size_t lds = use_lds ? (size_t)3 * lds_rows * sizeof(double) : 0;
  // lanes per column: at least about eight rows per lane on the level's longest panel
  const int lpr = sweep_lanes(lds_rows);
#define DPD_BWD(T, K, L, P) \
  DPD_LAUNCH((k_sweep_bwd<T, K, L>), dim3(ntasks), dim3(kWideTaskThreads), K ? lds : 0, s, S, tasks, P, out, \
             N, alpha, accumulate, st)
#define DPD_BWD_L(T, K, P)                 \
  do {                                     \
    if (lpr == 64) DPD_BWD(T, K, 64, P);   \
    else if (lpr == 32) DPD_BWD(T, K, 32, P); \
    else DPD_BWD(T, K, 16, P);             \
  } while (0)
  if (fp32) {
    if (use_lds) DPD_BWD_L(float, true, S.panel32);
    else DPD_BWD_L(float, false, S.panel32);
  } else {
    if (use_lds) DPD_BWD_L(double, true, S.panel64);
    else DPD_BWD_L(double, false, S.panel64);
  }
#undef DPD_BWD_L
#undef DPD_BWD
}

void launch_sweep_bwd_narrow(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks,
                             int lds_rows, bool fp32, double* out, int N, double alpha, int accumulate,
                             const IterState* st) {
  const size_t lds = (size_t)lds_bwd_narrow(lds_rows) * sizeof(double);
  if (fp32)
    DPD_LAUNCH(k_sweep_bwd_narrow<float>, dim3(ntasks), dim3(kWideTaskThreads), lds, s, S, tasks, S.panelT32,
                       out, N, alpha, accumulate, st);
  else
    DPD_LAUNCH(k_sweep_bwd_narrow<double>, dim3(ntasks), dim3(kWideTaskThreads), lds, s, S, tasks, S.panelT64,
                       out, N, alpha, accumulate, st);
}

void launch_solve_dag(const DevSolve& S, const DevDag& D, hipStream_t s, bool fp32, const double* b, double* out,
                      int N, double alpha, int accumulate, const IterState* st) {
  if (fp32)
    DPD_LAUNCH(k_solve_dag<float>, dim3(D.grid), dim3(kDagThreads), D.lds_bytes, s, S, D.q, D.nq, D.fwd, D.bwd,
               D.gcols, D.sn, D.ns, D.ctr, D.bwd_region, S.panel32, S.panelT32, b, out, N, alpha, accumulate, st);
  else
    DPD_LAUNCH(k_solve_dag<double>, dim3(D.grid), dim3(kDagThreads), D.lds_bytes, s, S, D.q, D.nq, D.fwd, D.bwd,
               D.gcols, D.sn, D.ns, D.ctr, D.bwd_region, S.panel64, S.panelT64, b, out, N, alpha, accumulate, st);
}

void launch_batch_sweep_fwd(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks, int ntasks,
                            int lds_cols, bool fp32) {
  const size_t lds = (size_t)lds_fwd_narrow(lds_cols) * sizeof(double);
  if (fp32)
    hipLaunchKernelGGL(k_batch_sweep_fwd<float>, dim3(ntasks), dim3(kBlock), lds, s, slots, tasks);
  else
    hipLaunchKernelGGL(k_batch_sweep_fwd<double>, dim3(ntasks), dim3(kBlock), lds, s, slots, tasks);
}

void launch_batch_sweep_fwd_wide(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks, int ntasks,
                                 int lpr, int lds_cols, bool fp32) {
  const size_t lds = (size_t)3 * lds_cols * sizeof(double);
#define DPD_BFWD(T, L) \
  hipLaunchKernelGGL((k_batch_sweep_fwd_wide<T, L>), dim3(ntasks), dim3(kWideTaskThreads), lds, s, slots, tasks)
  if (fp32) {
    if (lpr == 64) DPD_BFWD(float, 64);
    else if (lpr == 32) DPD_BFWD(float, 32);
    else DPD_BFWD(float, 16);
  } else {
    if (lpr == 64) DPD_BFWD(double, 64);
    else if (lpr == 32) DPD_BFWD(double, 32);
    else DPD_BFWD(double, 16);
  }
#undef DPD_BFWD
}

void launch_batch_sweep_gather(const BatchSolveSlot* slots, hipStream_t s, const int2* cols, int ncols) {
  const int waves = kBlock / 64;
  hipLaunchKernelGGL(k_batch_sweep_gather, dim3((ncols + waves - 1) / waves), dim3(kBlock), 0, s, slots, cols,
                     ncols);
}

void launch_batch_sweep_bwd(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks, int ntasks,
                            int lpr, bool use_lds, int lds_rows, bool fp32) {
  const size_t lds = use_lds ? (size_t)3 * lds_rows * sizeof(double) : 0;
#define DPD_BBWD(T, K, L) \
  hipLaunchKernelGGL((k_batch_sweep_bwd<T, K, L>), dim3(ntasks), dim3(kWideTaskThreads), lds, s, slots, tasks)
#define DPD_BBWD_L(T, K)                    \
  do {                                      \
    if (lpr == 64) DPD_BBWD(T, K, 64);      \
    else if (lpr == 32) DPD_BBWD(T, K, 32); \
    else DPD_BBWD(T, K, 16);                \
  } while (0)
  if (fp32) {
    if (use_lds) DPD_BBWD_L(float, true);
    else DPD_BBWD_L(float, false);
  } else {
    if (use_lds) DPD_BBWD_L(double, true);
    else DPD_BBWD_L(double, false);
  }
#undef DPD_BBWD_L
#undef DPD_BBWD
}

void launch_batch_sweep_bwd_narrow(const BatchSolveSlot* slots, hipStream_t s, const SweepTask* tasks,
                                   int ntasks, int lds_rows, bool fp32) {
  const size_t lds = (size_t)lds_bwd_narrow(lds_rows) * sizeof(double);
  if (fp32)
    hipLaunchKernelGGL(k_batch_sweep_bwd_narrow<float>, dim3(ntasks), dim3(kWideTaskThreads), lds, s, slots, tasks);
  else
    hipLaunchKernelGGL(k_batch_sweep_bwd_narrow<double>, dim3(ntasks), dim3(kWideTaskThreads), lds, s, slots,
                       tasks);
}

const void* solve_dag_kernel(bool fp32) {
  return fp32 ? (const void*)k_solve_dag<float> : (const void*)k_solve_dag<double>;
}


}  // namespace dpd
