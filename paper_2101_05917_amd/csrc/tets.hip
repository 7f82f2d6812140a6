// Element kernels of linear tetrahedra: the forward local step (closest
// rotation of the constant deformation gradient F = D_s D_m^{-1}, eq:pd_energy_single),
// the backward prologue's rotation cache, the adjoint local step dA p
// (eq:matrix_split) and the parameter gradient dL/dE_e, one lane per element.
// The node gather, residual, conjugate-gradient and sweep kernels are shared
// with the voxel meshes (the gather runs over the compressed incidence).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "device_math.hpp"

namespace dpd {

namespace {

// Corner ids and shape gradients dN_a/dX of element e: rows of D_m^{-1} for
// corners 1..3 and minus their sum for corner 0.
struct TetGeom {
  int n[4];
  double B[4][3];
};

__device__ inline void tet_geom(const DevMesh& M, int e, TetGeom& g) {
  const int64_t E = M.E;
#pragma unroll
  for (int a = 0; a < 4; ++a) g.n[a] = M.conn[a * E + e];
  double Di[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Di[i] = M.dminv[i * E + e];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    g.B[1][j] = Di[j];
    g.B[2][j] = Di[3 + j];
    g.B[3][j] = Di[6 + j];
    g.B[0][j] = -(Di[j] + Di[3 + j] + Di[6 + j]);
  }
}

// F_ij = sum_a v_{a,i} dN_a/dX_j for a [3][N] field v.
__device__ inline void tet_gradient(const DevMesh& M, const TetGeom& g, const double* __restrict__ v, double F[9]) {
  const int64_t N = M.N;
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double va = v[i * N + g.n[a]];
#pragma unroll
      for (int j = 0; j < 3; ++j) F[3 * i + j] += va * g.B[a][j];
    }
  }
}

// Corner forces f_{a,i} = sum_j P_ij dN_a/dX_j (G^T of a stress-like P) into
// the [3][4E] buffer at 4e + a.
__device__ inline void tet_forces_out(const DevMesh& M, const TetGeom& g, int e, const double P[9],
                                      double* __restrict__ fe) {
  const int64_t E4 = 4 * (int64_t)M.E;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t idx = 4 * (int64_t)e + a;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      fe[i * E4 + idx] = P[3 * i] * g.B[a][0] + P[3 * i + 1] * g.B[a][1] + P[3 * i + 2] * g.B[a][2];
  }
}

__global__ void __launch_bounds__(kBlock) k_tet_forces(DevMesh M, const double* __restrict__ x,
                                                       double* __restrict__ fe, double* __restrict__ R_out,
                                                       IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < M.E) {
    TetGeom g;
    tet_geom(M, e, g);
    double F[9], R[9], P[9];
    tet_gradient(M, g, x, F);
    if (M.local32)
      closest_rotation_mixed(F, R);
    else
      closest_rotation(F, R);
    if (st && det3(F) <= 0.0) atomicAdd(&st->inverted, 1);
    const double w = M.w_e[e];
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = w * (F[i] - R[i]);
    if (R_out)
#pragma unroll
      for (int i = 0; i < 9; ++i) R_out[i * (int64_t)M.E + e] = R[i];
    tet_forces_out(M, g, e, P, fe);
  }
  clock_exit(ck);
}

// Per element: R (9) and inv(tr(S) I - S) (6) at x, layout [15][E]; the blocks
// past elem_blocks set the ground-contact mask of the nodes.
__global__ void __launch_bounds__(kBlock) k_tet_adj_cache(DevMesh M, const double* __restrict__ x,
                                                          double* __restrict__ cache, IterState* st,
                                                          const IterState* gate, int elem_blocks) {
  if (gate && gate->done) return;
  if ((int)blockIdx.x >= elem_blocks) {
    const int n = (blockIdx.x - elem_blocks) * blockDim.x + threadIdx.x;
    if (n < M.N) M.cmask[n] = (M.contact[n] && x[2 * (int64_t)M.N + n] < 0.0) ? 1 : 0;
    return;
  }
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M.E) return;
  TetGeom g;
  tet_geom(M, e, g);
  double F[9], R[9], Ki[6];
  tet_gradient(M, g, x, F);
  if (M.local32)
    closest_rotation_mixed(F, R);
  else
    closest_rotation(F, R);
  const bool ok = rotation_kinv(F, R, Ki);
  if (st && (!ok || det3(F) <= 0.0)) atomicAdd(&st->inverted, 1);
  const int64_t E = M.E;
#pragma unroll
  for (int i = 0; i < 9; ++i) cache[i * E + e] = R[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) cache[(9 + i) * E + e] = Ki[i];
}

// Corner forces of w (dF - dR[dF]) with dF = G p (the element part of (A - dA) p).
__global__ void __launch_bounds__(kBlock) k_tet_hvp(DevMesh M, const double* __restrict__ p,
                                                    const double* __restrict__ cache, double* __restrict__ fe,
                                                    const IterState* st, ClockArg ck) {
  if (st && st->done) return;
  clock_enter(ck);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < M.E) {
    TetGeom g;
    tet_geom(M, e, g);
    double dF[9], cq[19], P[9];
    tet_gradient(M, g, p, dF);
    const int64_t E = M.E;
#pragma unroll
    for (int i = 0; i < 15; ++i) cq[i] = cache[i * E + e];
#pragma unroll
    for (int i = 15; i < 19; ++i) cq[i] = 0.0;
    hvp_stress_from_dF(M, P, dF, M.w_e[e], cq);
    tet_forces_out(M, g, e, P, fe);
  }
  clock_exit(ck);
}

// dL/dE_e += -(G z) : (F - R) dw_e/dE_e with w_e = E_e V_e / (1 + nu).
__global__ void __launch_bounds__(kBlock) k_tet_grad_params(DevMesh M, const double* __restrict__ xn,
                                                            const double* __restrict__ z,
                                                            const double* __restrict__ cache,
                                                            double* __restrict__ g_youngs, const IterState* gate) {
  if (gate && gate->curvature) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M.E || !g_youngs) return;
  TetGeom g;
  tet_geom(M, e, g);
  double F[9], dF[9];
  tet_gradient(M, g, xn, F);
  tet_gradient(M, g, z, dF);
  const int64_t E = M.E;
  double ge = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) ge += dF[i] * (F[i] - cache[i * E + e]);
  g_youngs[e] += -ge * M.vol[e] / (1.0 + M.nu);
}

int tet_blocks(const DevMesh& M) { return (M.E + kBlock - 1) / kBlock; }

}  // namespace

void launch_tet_forces(const DevMesh& M, hipStream_t s, const double* x, double* fe, double* R_out, IterState* st) {
  DPD_LAUNCH(k_tet_forces, dim3(tet_blocks(M)), dim3(kBlock), 0, s, M, x, fe, R_out, st);
}

void launch_tet_adj_cache(const DevMesh& M, hipStream_t s, const double* x, double* cache, IterState* st,
                          const IterState* gate) {
  const int nb = tet_blocks(M);
  hipLaunchKernelGGL(k_tet_adj_cache, dim3(nb + (M.N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, M, x, cache, st,
                     gate, nb);
}

void launch_tet_hvp(const DevMesh& M, hipStream_t s, const double* p, const double* cache, double* fe,
                    const IterState* st) {
  DPD_LAUNCH(k_tet_hvp, dim3(tet_blocks(M)), dim3(kBlock), 0, s, M, p, cache, fe, st);
}

void launch_tet_grad_params(const DevMesh& M, hipStream_t s, const double* xn, const double* z, const double* cache,
                            double* g_youngs, const IterState* gate) {
  hipLaunchKernelGGL(k_tet_grad_params, dim3(tet_blocks(M)), dim3(kBlock), 0, s, M, xn, z, cache, g_youngs, gate);
}

}  // namespace dpd
