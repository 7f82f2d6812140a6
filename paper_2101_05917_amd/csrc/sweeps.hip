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

__device__ inline double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// b~ for the task's supernode into bs[3][nc]: pre-gathered (bt) or gathered here.
__device__ inline void stage_rhs(const DevSolve& S, const SweepTask& t, const double* __restrict__ b,
                                 int N, bool pre, int tid, double* bs, int nthreads = kGroup) {
  const int nc = t.ncols;
  for (int c = tid; c < nc; c += nthreads) {
    const int j = t.col0 + c;
    double v0, v1, v2;
    if (pre) {
      v0 = S.bt[j];
      v1 = S.bt[(int64_t)S.nf + j];
      v2 = S.bt[2 * (int64_t)S.nf + j];
    } else {
      const int node = S.perm_pub[j];
      v0 = b[node];
      v1 = b[(int64_t)N + node];
      v2 = b[2 * (int64_t)N + node];
      // four contributions at a time, their loads issued together
      int k = S.cptr[j];
      const int k1 = S.cptr[j + 1];
      for (; k + 3 < k1; k += 4) {
        const int64_t p0 = 3 * (int64_t)S.cidx[k], p1 = 3 * (int64_t)S.cidx[k + 1];
        const int64_t p2 = 3 * (int64_t)S.cidx[k + 2], p3 = 3 * (int64_t)S.cidx[k + 3];
        v0 += (S.U[p0] + S.U[p1]) + (S.U[p2] + S.U[p3]);
        v1 += (S.U[p0 + 1] + S.U[p1 + 1]) + (S.U[p2 + 1] + S.U[p3 + 1]);
        v2 += (S.U[p0 + 2] + S.U[p1 + 2]) + (S.U[p2 + 2] + S.U[p3 + 2]);
      }
      for (; k < k1; ++k) {
        const int64_t pos = 3 * (int64_t)S.cidx[k];
        v0 += S.U[pos];
        v1 += S.U[pos + 1];
        v2 += S.U[pos + 2];
      }
    }
    bs[c] = v0;
    bs[nc + c] = v1;
    bs[2 * nc + c] = v2;
  }
}

__device__ inline void store_fwd_row(const DevSolve& S, const SweepTask& t, int r, double a0, double a1,
                                     double a2) {
  if (r < t.ncols) {
    const int j = t.col0 + r;
    S.y_int[j] = a0;
    S.y_int[(int64_t)S.nf + j] = a1;
    S.y_int[2 * (int64_t)S.nf + j] = a2;
  } else {
    const int64_t pos = 3 * (t.u_off + (r - t.ncols));
    S.U[pos] = a0;
    S.U[pos + 1] = a1;
    S.U[pos + 2] = a2;
  }
}

// v[3][ld] = [y_s; x_R] for the backward task.
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
    vs[r] = src[j];
    vs[ld + r] = src[nf + j];
    vs[2 * ld + r] = src[2 * nf + j];
  }
}

__device__ inline void store_bwd_col(const DevSolve& S, const SweepTask& t, int c, double x0, double x1,
                                     double x2, double* __restrict__ out, int N, double alpha,
                                     int accumulate) {
  const int j = t.col0 + c;
  const int64_t nf = S.nf;
  S.x_int[j] = x0;
  S.x_int[nf + j] = x1;
  S.x_int[2 * nf + j] = x2;
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
// four waves (c = wave mod 4) so that each row has four streams of loads in
// flight; the four partial sums meet in LDS (after the staged right-hand
// sides) and are added in wave order.
template <typename T>
__device__ inline void fwd_narrow_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panel,
                                       const double* __restrict__ b, int N, bool active, int tid,
                                       double* bs) {
  __syncthreads();
  if (active) stage_rhs(S, t, b, N, false, tid, bs);
  __syncthreads();
  if (!active) return;
  const int nc = t.ncols, ld = t.ncols + t.nrows;
  const int lane = tid & 63, wid = tid >> 6;
  const bool act = lane < t.count;
  const int r = t.first + (act ? lane : 0);
  const T* P = panel + t.panel_off + r;
  const int cend = act ? (r < nc ? r + 1 : nc) : 0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  int c = wid;
  for (; c + 12 < cend; c += 16) {
    const double p0 = (double)P[(int64_t)c * ld], p1 = (double)P[(int64_t)(c + 4) * ld];
    const double p2 = (double)P[(int64_t)(c + 8) * ld], p3 = (double)P[(int64_t)(c + 12) * ld];
    a0 += p0 * bs[c] + p1 * bs[c + 4] + p2 * bs[c + 8] + p3 * bs[c + 12];
    a1 += p0 * bs[nc + c] + p1 * bs[nc + c + 4] + p2 * bs[nc + c + 8] + p3 * bs[nc + c + 12];
    a2 += p0 * bs[2 * nc + c] + p1 * bs[2 * nc + c + 4] + p2 * bs[2 * nc + c + 8] + p3 * bs[2 * nc + c + 12];
  }
  for (; c < cend; c += 4) {
    const double p = (double)P[(int64_t)c * ld];
    a0 += p * bs[c];
    a1 += p * bs[nc + c];
    a2 += p * bs[2 * nc + c];
  }
  double* red = bs + 3 * nc;   // [4][64][3]
  red[(wid * 64 + lane) * 3 + 0] = a0;
  red[(wid * 64 + lane) * 3 + 1] = a1;
  red[(wid * 64 + lane) * 3 + 2] = a2;
  __syncthreads();
  if (wid == 0 && act) {
    double x[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      x[q] = red[(0 * 64 + lane) * 3 + q] + red[(1 * 64 + lane) * 3 + q] + red[(2 * 64 + lane) * 3 + q] +
             red[(3 * 64 + lane) * 3 + q];
    store_fwd_row(S, t, r, x[0], x[1], x[2]);
  }
}

// Forward task, wide blocks: LPR lanes per panel row on the row-major copy
// (64 / LPR rows per wave), each lane walking the row's columns with stride
// LPR, then a reduction over the row's LPR lanes.  LPR is chosen per level so
// that every lane reads at least about eight entries of its row.  A task of NT
// lanes (16 waves) covers one pass of rows, so the block's right-hand sides
// staged in LDS serve 16 x 64 / LPR rows.
template <typename T, int LPR, int NT>
__device__ inline void fwd_wide_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panelT,
                                     const double* __restrict__ b, int N, bool pre, bool active, int tid,
                                     double* bs) {
  __syncthreads();
  if (active) stage_rhs(S, t, b, N, pre, tid, bs, NT);
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
    if (act && li == 0) store_fwd_row(S, t, r, a0, a1, a2);
  }
}

// Backward task: LPR lanes per panel column (64 / LPR columns per wave), each
// lane walking the column's rows from the diagonal down with stride LPR
// (column-major panel, contiguous), then a reduction over the column's lanes;
// v from LDS (kLds) or from global memory.  LPR is chosen per level so that
// every lane reads at least about eight entries of its column.
template <typename T, bool kLds, int LPR, int NT>
__device__ inline void bwd_cols_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panel,
                                     double* __restrict__ out, int N, double alpha, int accumulate,
                                     bool active, int tid, double* vs) {
  __syncthreads();
  if (kLds && active) stage_solution(S, t, tid, vs, NT);
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
        v0 = src[j];
        v1 = src[nf + j];
        v2 = src[2 * nf + j];
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
    if (act && li == 0) store_bwd_col(S, t, col, a0, a1, a2, out, N, alpha, accumulate);
  }
}

// Backward task of a small supernode (at most 64 columns): lanes over its
// columns on the row-major copy, rows split four ways, combined through LDS.
// vs holds 3 ld doubles followed by 4 x 64 x 3 reduction slots.
template <typename T>
__device__ inline void bwd_narrow_task(const DevSolve& S, const SweepTask& t, const T* __restrict__ panelT,
                                       double* __restrict__ out, int N, double alpha, int accumulate,
                                       bool active, int tid, double* vs) {
  __syncthreads();
  if (active) stage_solution(S, t, tid, vs);
  __syncthreads();
  const int nc = t.ncols, ld = t.ncols + t.nrows;
  double* red = vs + 3 * ld;
  const int c = tid & 63, part = tid >> 6;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (active && c < nc) {
    const T* Pc = panelT + t.panel_off + c;
    // first row >= c (rows above the diagonal are zeros) in this part's residue class
    int r = c + ((part - c) & 3);
    for (; r + 12 < ld; r += 16) {
      const double p0 = (double)Pc[(int64_t)r * nc], p1 = (double)Pc[(int64_t)(r + 4) * nc];
      const double p2 = (double)Pc[(int64_t)(r + 8) * nc], p3 = (double)Pc[(int64_t)(r + 12) * nc];
      a0 += p0 * vs[r] + p1 * vs[r + 4] + p2 * vs[r + 8] + p3 * vs[r + 12];
      a1 += p0 * vs[ld + r] + p1 * vs[ld + r + 4] + p2 * vs[ld + r + 8] + p3 * vs[ld + r + 12];
      a2 += p0 * vs[2 * ld + r] + p1 * vs[2 * ld + r + 4] + p2 * vs[2 * ld + r + 8] + p3 * vs[2 * ld + r + 12];
    }
    for (; r < ld; r += 4) {
      const double p = (double)Pc[(int64_t)r * nc];
      a0 += p * vs[r];
      a1 += p * vs[ld + r];
      a2 += p * vs[2 * ld + r];
    }
  }
  if (active) {
    red[(part * 64 + c) * 3 + 0] = a0;
    red[(part * 64 + c) * 3 + 1] = a1;
    red[(part * 64 + c) * 3 + 2] = a2;
  }
  __syncthreads();
  if (active && part == 0 && c < nc) {
    double x[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
      x[q] = red[(0 * 64 + c) * 3 + q] + red[(1 * 64 + c) * 3 + q] + red[(2 * 64 + c) * 3 + q] +
             red[(3 * 64 + c) * 3 + q];
    store_bwd_col(S, t, c, x[0], x[1], x[2], out, N, alpha, accumulate);
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
  fwd_narrow_task<T>(S, tasks[blockIdx.x], panel, b, N, true, threadIdx.x, lds);
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
__global__ void __launch_bounds__(kBlock) k_sweep_bwd_narrow(DevSolve S, const SweepTask* __restrict__ tasks,
                                                             const T* __restrict__ panelT,
                                                             double* __restrict__ out, int N, double alpha,
                                                             int accumulate, const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  extern __shared__ double lds[];
  bwd_narrow_task<T>(S, tasks[blockIdx.x], panelT, out, N, alpha, accumulate, true, threadIdx.x, lds);
  clock_exit(ck);
}

}  // namespace

// ---------------------------------------------------------------- launchers

void launch_sweep_fwd(const DevSolve& S, hipStream_t s, const SweepTask* tasks, int ntasks, int lds_cols,
                      bool fp32, const double* b, int N, const IterState* st) {
  const size_t lds = ((size_t)3 * lds_cols + 4 * 64 * 3) * sizeof(double);
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
  const size_t lds = ((size_t)3 * lds_rows + 4 * 64 * 3) * sizeof(double);
  if (fp32)
    DPD_LAUNCH(k_sweep_bwd_narrow<float>, dim3(ntasks), dim3(kBlock), lds, s, S, tasks, S.panelT32,
                       out, N, alpha, accumulate, st);
  else
    DPD_LAUNCH(k_sweep_bwd_narrow<double>, dim3(ntasks), dim3(kBlock), lds, s, S, tasks, S.panelT64,
                       out, N, alpha, accumulate, st);
}


}  // namespace dpd
