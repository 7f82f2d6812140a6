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
// the paper's 2c x 2c I - V P^T B3, and is factorized by Cholesky in LDS.
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

// One workgroup: S = B1[set][cand[set]] (c x c), y = a1 at the set's nodes
// (3 right-hand sides), S = L L^T by right-looking Cholesky, then
// lam = -L^{-T} L^{-1} y.  status = 1 on a non-positive pivot.
__global__ void __launch_bounds__(kContactThreads) k_contact_capacitance(int N, const int32_t* __restrict__ cand,
                                                                         const int32_t* __restrict__ set, int c,
                                                                         const double* __restrict__ B1,
                                                                         const double* __restrict__ a1,
                                                                         double* __restrict__ lam, int* status) {
  extern __shared__ double lds[];
  double* S = lds;          // [c][c], lower triangle becomes L
  double* y = lds + c * c;  // [3][c]
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < c * c; idx += nt) {
    const int k = idx / c, l = idx % c;
    S[idx] = B1[(int64_t)set[k] * N + cand[set[l]]];
  }
  for (int idx = tid; idx < 3 * c; idx += nt) {
    const int comp = idx / c, k = idx % c;
    y[idx] = a1[(int64_t)comp * N + cand[set[k]]];
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    if (tid == 0) {
      const double d = S[j * c + j];
      if (!(d > 0.0)) bad = 1;
      S[j * c + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double ljj = S[j * c + j];
    for (int i = j + 1 + tid; i < c; i += nt) S[i * c + j] /= ljj;
    __syncthreads();
    const int m = c - j - 1;
    for (int idx = tid; idx < m * m; idx += nt) {
      const int i = j + 1 + idx / m, k = j + 1 + idx % m;
      if (k <= i) S[i * c + k] -= S[i * c + j] * S[k * c + j];
    }
    __syncthreads();
  }
  for (int j = 0; j < c; ++j) {  // L z = y
    if (tid < 3) y[tid * c + j] /= S[j * c + j];
    __syncthreads();
    const int m = c - j - 1;
    for (int idx = tid; idx < 3 * m; idx += nt) {
      const int comp = idx / m, i = j + 1 + idx % m;
      y[comp * c + i] -= S[i * c + j] * y[comp * c + j];
    }
    __syncthreads();
  }
  for (int j = c - 1; j >= 0; --j) {  // L^T w = z
    if (tid < 3) y[tid * c + j] /= S[j * c + j];
    __syncthreads();
    for (int idx = tid; idx < 3 * j; idx += nt) {
      const int comp = idx / j, i = idx % j;
      y[comp * c + i] -= S[j * c + i] * y[comp * c + j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < 3 * c; idx += nt) lam[idx] = -y[idx];
  if (tid == 0) *status = bad;
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

// x at the active set's nodes = x* ([3][c]).
__global__ void k_contact_set(int N, const int32_t* __restrict__ cand, const int32_t* __restrict__ set, int c,
                              const double* __restrict__ xstar, double* __restrict__ x) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * c) return;
  const int comp = idx / c, k = idx % c;
  x[(int64_t)comp * N + cand[set[k]]] = xstar[idx];
}

}  // namespace

size_t contact_capacitance_lds(int c) { return ((size_t)c * c + 3 * (size_t)c) * sizeof(double); }

void launch_contact_unit(hipStream_t s, int N, int n_cand, const int32_t* cand, int k0, double* b) {
  hipLaunchKernelGGL(k_contact_unit, dim3(1), dim3(64), 0, s, N, n_cand, cand, k0, b);
}

void launch_contact_collect(hipStream_t s, int N, int n_cand, int k0, const double* x, double* B1) {
  const int64_t t = 3 * (int64_t)N;
  hipLaunchKernelGGL(k_contact_collect, dim3((unsigned)((t + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, N, n_cand,
                     k0, x, B1);
}

hipError_t launch_contact_capacitance(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c,
                                      const double* B1, const double* a1, double* lam, int* status) {
  const size_t lds = contact_capacitance_lds(c);
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_contact_capacitance,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_contact_capacitance, dim3(1), dim3(kContactThreads), lds, s, N, cand, set, c, B1, a1, lam,
                     status);
  return hipGetLastError();
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
