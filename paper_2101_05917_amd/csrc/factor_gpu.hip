// Multifrontal numeric Cholesky of A on the device and the panels of the
// triangular sweeps (the factorization that the global step of eq:pd_global
// precomputes once, Sec. Background).  The plan (factor.cpp) lists the
// launches; the dense work of a level's fronts advances one block column of
// kFactorNB at a time:
//   k_factor_panel   Cholesky of the diagonal block in LDS, the rows below
//                    solved against it, and the panel's block row solved;
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

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Item of workgroup b: the largest i < n with prefix[i] <= b.
__device__ inline int find_item(const int32_t* __restrict__ prefix, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

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
// its parent's front, one wave per column of the update.
__global__ void __launch_bounds__(kThreads) k_factor_extend(const FrontDesc* __restrict__ fd,
                                                            const int32_t* __restrict__ items, int n,
                                                            const int32_t* __restrict__ relmap,
                                                            double* __restrict__ F) {
  const int32_t* pre = items + n;
  const int it = find_item(pre, n, blockIdx.x);
  const FrontDesc ch = fd[items[it]];
  const FrontDesc pa = fd[ch.parent];
  const int r = ch.nrows;
  const int q = (blockIdx.x - pre[it]) * (kThreads / 64) + (threadIdx.x >> 6);
  if (q >= r) return;
  const double* __restrict__ U = F + ch.front_off + (int64_t)(ch.nc + q) * ch.ld + ch.nc;
  const int32_t* __restrict__ rel = relmap + ch.rows_off;
  double* __restrict__ col = F + pa.front_off + (int64_t)rel[q] * pa.ld;
  for (int p = q + (threadIdx.x & 63); p < r; p += 64) col[rel[p]] += U[p];
}

// Block column [k0, k0 + kb) of a front: the diagonal block's Cholesky factor
// L_kk and its inverse (in LDS; every workgroup of the front computes them),
// then either a chunk of the rows below (l = f L_kk^{-T} for each row f) or a
// chunk of the panel's columns c < k0 + kb (y = L_kk^{-1} x on block row k).
// Both are products with the inverse (inverted diagonal blocks, as in blocked
// triangular solves), which keeps a row's 32 entries in registers and the
// inverse's rows in LDS.  A non-positive or non-finite pivot sets *status.
__global__ void __launch_bounds__(kThreads) k_factor_panel(const FrontDesc* __restrict__ fd,
                                                           const int32_t* __restrict__ items, int n, int k0,
                                                           double* __restrict__ F, double* __restrict__ P,
                                                           int32_t* __restrict__ status) {
  __shared__ double D[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  const int32_t* pre = items + n;
  const int it = find_item(pre, n, blockIdx.x);
  const FrontDesc f = fd[items[it]];
  const int kb = min(NB, f.nc - k0), k1 = k0 + kb;
  const int local = blockIdx.x - pre[it];
  const int rows_chunks = (f.ld - k1 + kThreads - 1) / kThreads;
  double* __restrict__ Fa = F + f.front_off;
  for (int idx = threadIdx.x; idx < NB * NB; idx += kThreads) {
    const int i = idx % NB, j = idx / NB;
    D[i][j] = (i < kb && j <= i) ? Fa[(k0 + i) + (int64_t)(k0 + j) * f.ld] : (i == j ? 1.0 : 0.0);
    Li[i][j] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    const double d = D[j][j];
    const bool bad = !(d > 0.0) || !__builtin_isfinite(d);
    const double sd = bad ? 1.0 : sqrt(d);
    if (bad && threadIdx.x == 0) atomicOr(status, 1);
    __syncthreads();
    for (int i = j + threadIdx.x; i < kb; i += kThreads) D[i][j] = (i == j) ? sd : D[i][j] / sd;
    __syncthreads();
    const int w = kb - j - 1;
    for (int idx = threadIdx.x; idx < w * w; idx += kThreads) {
      const int i = j + 1 + idx % w, t = j + 1 + idx / w;
      if (i >= t) D[i][t] -= D[i][j] * D[t][j];
    }
    __syncthreads();
  }
  // column j of L_kk^{-1} by forward substitution on e_j, one lane per column
  if (threadIdx.x < kb) {
    const int j = threadIdx.x;
    Li[j][j] = 1.0 / D[j][j];
    for (int i = j + 1; i < kb; ++i) {
      double v = 0.0;
      for (int t = j; t < i; ++t) v += D[i][t] * Li[t][j];
      Li[i][j] = -v / D[i][i];
    }
  }
  __syncthreads();
  double x[NB];
  double* __restrict__ v;
  int64_t stride;
  if (local < rows_chunks) {
    const int i = k1 + local * kThreads + threadIdx.x;
    if (i >= f.ld) return;
    v = Fa + i + (int64_t)k0 * f.ld;
    stride = f.ld;
  } else {
    const int c = (local - rows_chunks) * kThreads + threadIdx.x;
    if (c >= k1) return;
    v = P + f.panel_off + (int64_t)c * f.ld + k0;
    stride = 1;
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) x[t] = t < kb ? v[t * stride] : 0.0;
#pragma unroll 2
  for (int j = 0; j < kb; ++j) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) s += Li[j][t] * x[t];
    v[j * stride] = s;
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
  const int it = find_item(pre, n, blockIdx.x);
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
  for (int idx = threadIdx.x; idx < NB * TT; idx += kThreads) {
    const int p = idx % TT, t = idx / TT;
    const int gp = ti * TT + p;
    Xs[t][p] = (t < kb && gp < m) ? Lp[gp + (int64_t)t * ld] : 0.0;
  }
  if (syrk) {
    for (int idx = threadIdx.x; idx < NB * TT; idx += kThreads) {
      const int q = idx % TT, t = idx / TT;
      const int gq = tj * TT + q;
      Ys[t][q] = (t < kb && gq < m) ? Lp[gq + (int64_t)t * ld] : 0.0;
    }
  } else {
    for (int idx = threadIdx.x; idx < NB * TT; idx += kThreads) {
      const int t = idx % NB, q = idx / NB;
      const int gq = tj * TT + q;
      Ys[t][q] = (t < kb && gq < k1) ? Pa[(k0 + t) + (int64_t)gq * ld] : 0.0;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pr = (w >> 1) * 32, qc = (w & 1) * 32;
  const int kl = lane >> 4, il = lane & 15;
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
    for (int pb = 0; pb < 2; ++pb) {
      const int gp = ti * TT + pr + pb * 16 + il;
      if (gp >= m) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gq = tj * TT + qc + qb * 16 + 4 * e + kl;
        const double v = acc[qb][pb][e];
        if (syrk) {
          if (gq <= gp) Fa[(k1 + gp) + (int64_t)(k1 + gq) * ld] -= v;
        } else if (gq < k1) {
          Pa[(k1 + gp) + (int64_t)gq * ld] -= v;
        }
      }
    }
}

// Row-major copy of every panel: element (r, c) of a supernode at
// panel_off + r * nc + c.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_factor_transpose(const FrontDesc* __restrict__ fd, int ns,
                                                               int64_t total, const double* __restrict__ P,
                                                               T* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fd[mid].panel_off <= e) lo = mid;
    else hi = mid - 1;
  }
  const FrontDesc f = fd[lo];
  const int64_t local = e - f.panel_off;
  const int64_t r = local / f.nc, c = local % f.nc;
  out[e] = (T)P[f.panel_off + c * f.ld + r];
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

void launch_factor_transpose(hipStream_t s, const FrontDesc* fd, int ns, int64_t total, const double* P,
                             double* out) {
  if (total > 0)
    hipLaunchKernelGGL(k_factor_transpose<double>, dim3(grid_of(total)), dim3(kThreads), 0, s, fd, ns, total, P,
                       out);
}

}  // namespace dpd
