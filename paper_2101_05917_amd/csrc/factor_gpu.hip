// Multifrontal numeric Cholesky of A on the device and the panels of the
// triangular sweeps (the factorization that the global step of eq:pd_global
// precomputes once, Sec. Background).  The plan (factor.cpp) lists the
// launches; the dense work of a level's fronts advances one block column of
// kFactorNB at a time:
//   k_factor_panel   Cholesky factor of the diagonal block and its inverse
//                    (one wave), then the rows below the block and the
//                    panel's block row solved with that inverse;
//   k_factor_update  the trailing lower triangle and the panel's rows below
//                    the block updated by FP64 MFMA (16x16x4) on 64 x 64 tiles.
// The panel of a supernode is the first ncols columns of M^{-1} with
// M = [L11 0; L21 I]: [inv(L11); -L21 inv(L11)], obtained by forward
// substitution on [I; 0] alongside the factorization.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace dpd {

namespace {

constexpr int NB = kFactorNB;
constexpr int TT = kFactorTile;
constexpr int kThreads = 256;
constexpr int kPanelRows = kThreads / 4;   // rows (or panel columns) per panel-op workgroup

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Item of this workgroup (the op's per-workgroup table after its items and
// their prefix sums).
__device__ inline int item_of(const int32_t* __restrict__ items, int n) { return items[2 * n + 1 + blockIdx.x]; }

__global__ void __launch_bounds__(kThreads) k_factor_scatter(const int64_t* __restrict__ dst,
                                                             const int32_t* __restrict__ src,
                                                             const double* __restrict__ aval, int64_t n,
                                                             double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) F[dst[i]] = aval[src[i]];
}

// Ones on the diagonal of every panel's top block (the right-hand side [I; 0]).
__global__ void __launch_bounds__(kThreads) k_factor_identity(const FrontDesc* __restrict__ fd,
                                                              const int32_t* __restrict__ snode_of, int32_t n,
                                                              double* __restrict__ P) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const FrontDesc f = fd[snode_of[c]];
  const int j = c - f.col0;
  P[f.panel_off + (int64_t)j * f.ld + j] = 1.0;
}

// Extend-add: the child's update (trailing lower block of its front) into
// its parent's front, one wave per column of the update, four entries per
// lane in flight (the loads use clamped in-range indices, so they issue
// together; the stores are masked).
__global__ void __launch_bounds__(kThreads) k_factor_extend(const FrontDesc* __restrict__ fd,
                                                            const int32_t* __restrict__ items, int n,
                                                            const int32_t* __restrict__ relmap,
                                                            double* __restrict__ F) {
  const int32_t* pre = items + n;
  const int it = item_of(items, n);
  const FrontDesc ch = fd[items[it]];
  const FrontDesc pa = fd[ch.parent];
  const int r = ch.nrows;
  const int q = (blockIdx.x - pre[it]) * (kThreads / 64) + (threadIdx.x >> 6);
  if (q >= r) return;
  const double* __restrict__ U = F + ch.front_off + (int64_t)(ch.nc + q) * ch.ld + ch.nc;
  const int32_t* __restrict__ rel = relmap + ch.rows_off;
  double* __restrict__ col = F + pa.front_off + (int64_t)rel[q] * pa.ld;
  for (int p0 = q + (threadIdx.x & 63); p0 < r; p0 += 256) {
    int pp[4], rp[4];
    double u[4], c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pp[k] = min(p0 + 64 * k, r - 1);
      rp[k] = rel[pp[k]];
      u[k] = U[pp[k]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = col[rp[k]];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (p0 + 64 * k < r) col[rp[k]] = c[k] + u[k];
  }
}

// Lane l's value of v, for a wave-uniform l (two 32-bit lane reads).
__device__ inline double lane_value(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Inverse of the Cholesky factor of a diagonal block, on one wave: lane i
// holds row i of the block (entries t <= i, padded to NB x NB with an identity
// block) in a[].  Right-looking Cholesky: at step j the pivot column's entries
// are read across lanes before the pivot's square root, and every row below
// subtracts a_ij a_tj / a_jj from its entries t <= i.  Lane j then forms
// column j of L^{-1} by forward substitution into y[] (y[i] = (L^{-1})_ij).
// Returns false on a non-positive or non-finite pivot.
__device__ inline bool diag_inverse(double (&a)[NB], int lane, double (&y)[NB]) {
  bool bad = false;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double col[NB];
#pragma unroll
    for (int t = j; t < NB; ++t) col[t] = lane_value(a[j], t);
    const double d = col[j];
    const bool ok = d > 0.0 && __builtin_isfinite(d);
    bad = bad || !ok;
    const double dd = ok ? d : 1.0;
    const double inv_d = 1.0 / dd;
    const double sc = (lane > j) ? a[j] * inv_d : 0.0;
#pragma unroll
    for (int t = j + 1; t < NB; ++t) a[t] -= (t <= lane ? sc : 0.0) * col[t];
    const double sd = sqrt(dd);
    a[j] = (lane == j) ? sd : (lane > j ? a[j] * (1.0 / sd) : a[j]);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int u = 0; u < i; ++u) acc -= lane_value(a[u], i) * y[u];
    y[i] = acc / lane_value(a[i], i);
  }
  return !bad;
}

// Block column [k0, k0 + kb) of a front.  Wave 0 forms the inverse of the
// diagonal block's Cholesky factor, L_kk^{-1}, in LDS (every workgroup of the
// front does this).  Then the workgroup handles either
// 64 of the rows below (l = f L_kk^{-T} for each row f) or 64 of the panel's
// columns c < k0 + kb (y = L_kk^{-1} x on block row k), four lanes per row or
// column with NB / 4 outputs each: products with the inverse (inverted
// diagonal blocks, as in blocked triangular solves).  The four lanes of a row
// sit in one wave and load the whole row before any of them stores.  Global
// loads use clamped in-range addresses (the padding is selected afterwards),
// so each lane's loads issue together.  A non-positive or non-finite pivot
// sets *status.
__global__ void __launch_bounds__(kThreads) k_factor_panel(const FrontDesc* __restrict__ fd,
                                                           const int32_t* __restrict__ items, int n, int k0,
                                                           double* __restrict__ F, double* __restrict__ P,
                                                           int32_t* __restrict__ status) {
  __shared__ double Li[NB][NB + 1];
  const int32_t* pre = items + n;
  const int it = item_of(items, n);
  const FrontDesc f = fd[items[it]];
  const int kb = min(NB, f.nc - k0), k1 = k0 + kb;
  const int local = blockIdx.x - pre[it];
  const int rows_chunks = (f.ld - k1 + kPanelRows - 1) / kPanelRows;
  double* __restrict__ Fa = F + f.front_off;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int rr = min(lane, kb - 1);
    double a[NB], y[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) a[t] = Fa[(k0 + rr) + (int64_t)(k0 + min(t, rr)) * f.ld];
#pragma unroll
    for (int t = 0; t < NB; ++t) a[t] = (lane < kb && t <= lane) ? a[t] : (t == lane ? 1.0 : 0.0);
    if (!diag_inverse(a, lane, y) && lane == 0) atomicOr(status, 1);
    if (lane < NB)
#pragma unroll
      for (int i = 0; i < NB; ++i) Li[i][lane] = y[i];
  }
  __syncthreads();
  const int sub = threadIdx.x & 3, slot = threadIdx.x >> 2;
  double* __restrict__ v;
  int64_t stride;
  if (local < rows_chunks) {
    const int i = k1 + local * kPanelRows + slot;
    if (i >= f.ld) return;
    v = Fa + i + (int64_t)k0 * f.ld;
    stride = f.ld;
  } else {
    const int c = (local - rows_chunks) * kPanelRows + slot;
    if (c >= k1) return;
    v = P + f.panel_off + (int64_t)c * f.ld + k0;
    stride = 1;
  }
  double x[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) x[t] = v[min(t, kb - 1) * stride];
#pragma unroll
  for (int t = 0; t < NB; ++t) x[t] = t < kb ? x[t] : 0.0;
  constexpr int kOut = NB / 4;
#pragma unroll 1
  for (int q = 0; q < kOut; ++q) {
    const int jrow = sub * kOut + q;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int t = 0; t < NB; t += 2) {
      s0 += Li[jrow][t] * x[t];
      s1 += Li[jrow][t + 1] * x[t + 1];
    }
    if (jrow < kb) v[jrow * stride] = s0 + s1;
  }
}

// One 64 x 64 output tile C -= X Y of a front's block column k (inner
// dimension kb <= NB), on 4 waves of 32 x 32 each (2 x 2 MFMA blocks).
// Tiles 0 .. T(T+1)/2 - 1: the trailing lower triangle (X = L_{>k,k},
// Y = X^T); the rest: the panel rows below the block (X = L_{>k,k},
// Y = panel block row k, columns < k1).  The MFMA's A operand indexes the
// tile's columns and its B operand the rows, so that lanes 16g .. 16g + 15
// hold 16 consecutive rows of one column (each store writes 16-double runs).
__global__ void __launch_bounds__(kThreads) k_factor_update(const FrontDesc* __restrict__ fd,
                                                            const int32_t* __restrict__ items, int n, int k0,
                                                            double* __restrict__ F, double* __restrict__ P) {
  __shared__ double Xs[NB][TT + 1];   // Xs[t][p] = X[p][t]
  __shared__ double Ys[NB][TT + 1];   // Ys[t][q] = Y[t][q]
  const int32_t* pre = items + n;
  const int it = item_of(items, n);
  const FrontDesc f = fd[items[it]];
  const int kb = min(NB, f.nc - k0), k1 = k0 + kb, m = f.ld - k1;
  const int T = (m + TT - 1) / TT;
  const int local = blockIdx.x - pre[it];
  const int nsy = T * (T + 1) / 2;
  const bool syrk = local < nsy;
  int ti, tj;
  if (syrk) {
    ti = (int)((sqrt(8.0 * local + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= local) ++ti;
    while (ti * (ti + 1) / 2 > local) --ti;
    tj = local - ti * (ti + 1) / 2;
  } else {
    const int tc = (k1 + TT - 1) / TT;
    ti = (local - nsy) / tc;
    tj = (local - nsy) % tc;
  }
  const int64_t ld = f.ld;
  double* __restrict__ Fa = F + f.front_off;
  double* __restrict__ Pa = P + f.panel_off;
  const double* __restrict__ Lp = Fa + k1 + (int64_t)k0 * ld;   // L_{>k,k}: row p, column t at p + t ld
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pr = (w >> 1) * 32, qc = (w & 1) * 32;
  const int kl = lane >> 4, il = lane & 15;
  // the tile's current values first (clamped in-range addresses, so the loads
  // issue together and overlap the operand staging and the products)
  int64_t dst[2][2][4];
  bool keep[2][2][4];
  double old[2][2][4];
#pragma unroll
  for (int qb = 0; qb < 2; ++qb)
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gp = ti * TT + pr + pb * 16 + il;
        const int gq = tj * TT + qc + qb * 16 + 4 * e + kl;
        if (syrk) {
          keep[qb][pb][e] = gp < m && gq <= gp;
          dst[qb][pb][e] = f.front_off + (k1 + min(gp, m - 1)) + (int64_t)(k1 + min(gq, m - 1)) * ld;
        } else {
          keep[qb][pb][e] = gp < m && gq < k1;
          dst[qb][pb][e] = f.panel_off + (k1 + min(gp, m - 1)) + (int64_t)min(gq, k1 - 1) * ld;
        }
      }
  double* __restrict__ out = syrk ? F : P;
#pragma unroll
  for (int qb = 0; qb < 2; ++qb)
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int e = 0; e < 4; ++e) old[qb][pb][e] = out[dst[qb][pb][e]];
  constexpr int kPer = NB * TT / kThreads;
#pragma unroll
  for (int s2 = 0; s2 < kPer; ++s2) {
    const int idx = threadIdx.x + kThreads * s2;
    const int p = idx % TT, t = idx / TT;
    const int gp = ti * TT + p;
    const double v = Lp[min(gp, m - 1) + (int64_t)min(t, kb - 1) * ld];
    Xs[t][p] = (t < kb && gp < m) ? v : 0.0;
  }
  if (syrk) {
#pragma unroll
    for (int s2 = 0; s2 < kPer; ++s2) {
      const int idx = threadIdx.x + kThreads * s2;
      const int q = idx % TT, t = idx / TT;
      const int gq = tj * TT + q;
      const double v = Lp[min(gq, m - 1) + (int64_t)min(t, kb - 1) * ld];
      Ys[t][q] = (t < kb && gq < m) ? v : 0.0;
    }
  } else {
#pragma unroll
    for (int s2 = 0; s2 < kPer; ++s2) {
      const int idx = threadIdx.x + kThreads * s2;
      const int t = idx % NB, q = idx / NB;
      const int gq = tj * TT + q;
      const double v = Pa[(k0 + min(t, kb - 1)) + (int64_t)min(gq, k1 - 1) * ld];
      Ys[t][q] = (t < kb && gq < k1) ? v : 0.0;
    }
  }
  __syncthreads();
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < kb; t += 4) {
    const int kk = t + kl;
    const double a0 = Ys[kk][qc + il], a1 = Ys[kk][qc + 16 + il];
    const double b0 = Xs[kk][pr + il], b1 = Xs[kk][pr + 16 + il];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  // result (i, j) of a 16 x 16 block sits in lane j + 16 (i % 4), element i / 4
  // (the builtin's layout on gfx950): i indexes the tile's columns (A
  // operand), j its rows (B operand)
#pragma unroll
  for (int qb = 0; qb < 2; ++qb)
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (keep[qb][pb][e]) out[dst[qb][pb][e]] = old[qb][pb][e] - acc[qb][pb][e];
}

// Row-major copy of every panel: element (r, c) of a supernode at
// panel_off + r * nc + c; a workgroup copies kFactorTransposeChunk entries
// of one supernode, four per lane (loads issued together, stores masked).
__global__ void __launch_bounds__(kThreads) k_factor_transpose(const FrontDesc* __restrict__ fd,
                                                               const int32_t* __restrict__ items, int n,
                                                               const double* __restrict__ P,
                                                               double* __restrict__ out) {
  const int32_t* pre = items + n;
  const int it = item_of(items, n);
  const FrontDesc f = fd[items[it]];
  const int64_t total = (int64_t)f.ld * f.nc;
  const int64_t e0 = (int64_t)(blockIdx.x - pre[it]) * kFactorTransposeChunk + threadIdx.x;
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t e = min(e0 + k * kThreads, total - 1);
    const int64_t r = e / f.nc, c = e - r * f.nc;
    v[k] = P[f.panel_off + c * f.ld + r];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (e0 + k * kThreads < total) out[f.panel_off + e0 + k * kThreads] = v[k];
}

int grid_of(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

}  // namespace

void launch_factor_scatter(hipStream_t s, const int64_t* dst, const int32_t* src, const double* aval, int64_t n,
                           double* F) {
  if (n > 0) hipLaunchKernelGGL(k_factor_scatter, dim3(grid_of(n)), dim3(kThreads), 0, s, dst, src, aval, n, F);
}

void launch_factor_identity(hipStream_t s, const FrontDesc* fd, const int32_t* snode_of, int32_t n, double* P) {
  if (n > 0) hipLaunchKernelGGL(k_factor_identity, dim3(grid_of(n)), dim3(kThreads), 0, s, fd, snode_of, n, P);
}

void launch_factor_op(hipStream_t s, const FactorOp& op, const FrontDesc* fd, const int32_t* ints,
                      const int32_t* relmap, double* F, double* P, int32_t* status) {
  const int32_t* items = ints + op.list_off;
  switch (op.kind) {
    case kFactorExtend:
      hipLaunchKernelGGL(k_factor_extend, dim3(op.blocks), dim3(kThreads), 0, s, fd, items, op.n, relmap, F);
      break;
    case kFactorPanel:
      hipLaunchKernelGGL(k_factor_panel, dim3(op.blocks), dim3(kThreads), 0, s, fd, items, op.n, op.k0, F, P,
                         status);
      break;
    default:
      hipLaunchKernelGGL(k_factor_update, dim3(op.blocks), dim3(kThreads), 0, s, fd, items, op.n, op.k0, F, P);
      break;
  }
}

void launch_factor_transpose(hipStream_t s, const FactorOp& op, const FrontDesc* fd, const int32_t* ints,
                             const double* P, double* out) {
  if (op.blocks > 0)
    hipLaunchKernelGGL(k_factor_transpose, dim3(op.blocks), dim3(kThreads), 0, s, fd, ints + op.list_off, op.n, P,
                       out);
}

}  // namespace dpd
