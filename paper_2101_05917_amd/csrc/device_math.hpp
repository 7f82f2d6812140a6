// Device-side building blocks shared by the kernels of the PD step, its
// adjoint and the fused dense conjugate-gradient solver (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"

namespace dpd {

// ------------------------------------------------------------------ helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; valid in thread 0.
__device__ inline double block_sum(double v, double* ws) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ws[i];
  __syncthreads();
  return t;
}

// Grid-wide sum with a deterministic order: each block publishes its partial,
// the last block to arrive sums the partials in block order.  Returns true in
// thread 0 of the last block, with the total in *total.  bid / nblk: this
// block's index among the nblk blocks taking part (a batched launch runs
// several such grids side by side).
__device__ inline bool grid_sum_at(double v, double* partials, IterState* st, double* total, int bid, int nblk) {
  __shared__ double ws[kBlock / 64];
  __shared__ int last;
  const double bs = block_sum(v, ws);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partials[bid], bs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t t =
        __hip_atomic_fetch_add(&st->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == (uint32_t)nblk - 1);
  }
  __syncthreads();
  if (!last) return false;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x)
    s += __hip_atomic_load(&partials[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // keep the order fixed: strided partial sums, then the block tree
  s = block_sum(s, ws);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&st->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *total = s;
  }
  return threadIdx.x == 0;
}

__device__ inline bool grid_sum(double v, double* partials, IterState* st, double* total) {
  return grid_sum_at(v, partials, st, total, blockIdx.x, gridDim.x);
}

// dN_a/dX_j at Gauss point q of a cubic voxel: (1/8) s_aj prod_{k != j}(1 +- g) * 2/dx,
// the factor being 1 + g when bits k of a and q agree and 1 - g otherwise.
struct GradTable {
  double c2, c1, c0;  // magnitudes for two, one, zero agreeing axes
};

__device__ inline double bgrad(int q, int j, int a, const GradTable& T) {
  const int x = ~(a ^ q);
  const int agree = ((x >> ((j + 1) % 3)) & 1) + ((x >> ((j + 2) % 3)) & 1);
  const double mag = agree == 2 ? T.c2 : (agree == 1 ? T.c1 : T.c0);
  return ((a >> j) & 1) ? mag : -mag;
}

__device__ inline GradTable grad_table(double dx) {
  const double g = 0.57735026918962576451;  // 1/sqrt(3)
  const double s = 2.0 / dx / 8.0;
  return {s * (1.0 + g) * (1.0 + g), s * (1.0 + g) * (1.0 - g), s * (1.0 - g) * (1.0 - g)};
}

// Closest rotation to F (row-major 3x3), i.e. argmax over SO(3) of tr(R^T F).
// With R = R(quat) this is the largest-eigenvalue eigenvector of a symmetric
// 4x4 matrix (Davenport's q-method); the eigenproblem is solved by cyclic
// Jacobi rotations (Golub & Van Loan, symmetric Schur decomposition).  T is
// the arithmetic type (FP64; FP32 for the mixed-precision local step, which
// then polishes the result in FP64).
template <typename T>
struct JacobiEps;
template <>
struct JacobiEps<double> {
  static constexpr double tiny = 1e-300, off = 1e-34;
};
template <>
struct JacobiEps<float> {
  static constexpr float tiny = 1e-30f, off = 1e-14f;
};

template <typename T>
__device__ inline void jrot(T (&B)[4][4], T (&V)[4][4], int p, int q) {
  const T apq = B[p][q];
  if (fabs(apq) <= JacobiEps<T>::tiny) return;
  const T tau = (B[q][q] - B[p][p]) / (T(2) * apq);
  const T t = (tau >= T(0) ? T(1) : T(-1)) / (fabs(tau) + sqrt(T(1) + tau * tau));
  const T c = T(1) / sqrt(T(1) + t * t), s = t * c;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k == p || k == q) continue;
    const T bkp = B[k][p], bkq = B[k][q];
    B[k][p] = B[p][k] = c * bkp - s * bkq;
    B[k][q] = B[q][k] = s * bkp + c * bkq;
  }
  B[p][p] -= t * apq;
  B[q][q] += t * apq;
  B[p][q] = B[q][p] = T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T vkp = V[k][p], vkq = V[k][q];
    V[k][p] = c * vkp - s * vkq;
    V[k][q] = s * vkp + c * vkq;
  }
}

// Unit-norm-free quaternion (w, x, y, z) of the closest rotation.
template <typename T>
__device__ inline void closest_quat_t(const T F[9], T qt[4]) {
  T B[4][4], V[4][4];
  B[0][0] = F[0] + F[4] + F[8];
  B[1][1] = F[0] - F[4] - F[8];
  B[2][2] = -F[0] + F[4] - F[8];
  B[3][3] = -F[0] - F[4] + F[8];
  B[0][1] = B[1][0] = F[7] - F[5];
  B[0][2] = B[2][0] = F[2] - F[6];
  B[0][3] = B[3][0] = F[3] - F[1];
  B[1][2] = B[2][1] = F[1] + F[3];
  B[1][3] = B[3][1] = F[2] + F[6];
  B[2][3] = B[3][2] = F[5] + F[7];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? T(1) : T(0);
  T nrm = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) nrm += B[i][j] * B[i][j];
  for (int sweep = 0; sweep < 10; ++sweep) {
    const T off = B[0][1] * B[0][1] + B[0][2] * B[0][2] + B[0][3] * B[0][3] +
                  B[1][2] * B[1][2] + B[1][3] * B[1][3] + B[2][3] * B[2][3];
    if (off <= JacobiEps<T>::off * nrm) break;
    jrot(B, V, 0, 1);
    jrot(B, V, 0, 2);
    jrot(B, V, 0, 3);
    jrot(B, V, 1, 2);
    jrot(B, V, 1, 3);
    jrot(B, V, 2, 3);
  }
  int k = 0;
  T best = B[0][0];
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (B[i][i] > best) {
      best = B[i][i];
      k = i;
    }
  qt[0] = T(1);
  qt[1] = qt[2] = qt[3] = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i == k) {
      qt[0] = V[0][i];
      qt[1] = V[1][i];
      qt[2] = V[2][i];
      qt[3] = V[3][i];
    }
}

// Rotation of a (not necessarily normalised) quaternion, in FP64: orthogonal
// to FP64 round-off whatever the precision the quaternion was found in.
__device__ inline void quat_rotation(double w, double x, double y, double z, double R[9]) {
  const double s = 2.0 / (w * w + x * x + y * y + z * z);
  R[0] = 1.0 - s * (y * y + z * z);
  R[1] = s * (x * y - w * z);
  R[2] = s * (x * z + w * y);
  R[3] = s * (x * y + w * z);
  R[4] = 1.0 - s * (x * x + z * z);
  R[5] = s * (y * z - w * x);
  R[6] = s * (x * z - w * y);
  R[7] = s * (y * z + w * x);
  R[8] = 1.0 - s * (x * x + y * y);
}

// Orthogonal polar factor by Newton's iteration X <- (g X + X^{-T} / g) / 2
// (Higham 1986, "Computing the polar decomposition -- with applications"),
// with determinant scaling g = |det X|^{-1/3} while the steps are large.  For
// det F > 0 the factor is the closest proper rotation; the iteration converges
// quadratically, so it stops once a step is below sqrt(eps) and takes that
// iterate.  Returns false (caller falls back to the q-method) when det X <= 0
// or it has not converged within the cap.  With warm = true the iteration
// starts from the X given (an approximate polar factor of F, e.g. from a
// lower precision) instead of from F.
template <typename T>
__device__ inline bool polar_newton(const T F[9], T X[9], bool warm = false) {
  const T stop = sizeof(T) == 8 ? T(1e-18) : T(1e-10);   // squared step norm
  if (!warm) {
#pragma unroll
    for (int i = 0; i < 9; ++i) X[i] = F[i];
  }
  for (int it = 0; it < 12; ++it) {
    // cofactors: X^{-T} = C / det X
    const T c0 = X[4] * X[8] - X[5] * X[7], c1 = X[5] * X[6] - X[3] * X[8], c2 = X[3] * X[7] - X[4] * X[6];
    const T c3 = X[2] * X[7] - X[1] * X[8], c4 = X[0] * X[8] - X[2] * X[6], c5 = X[1] * X[6] - X[0] * X[7];
    const T c6 = X[1] * X[5] - X[2] * X[4], c7 = X[2] * X[3] - X[0] * X[5], c8 = X[0] * X[4] - X[1] * X[3];
    const T det = X[0] * c0 + X[1] * c1 + X[2] * c2;
    if (!(det > T(0))) return false;
    const T g = it < 2 && !warm ? T(1) / cbrt(det) : T(1);
    const T a = T(0.5) * g, b = T(0.5) / (g * det);
    const T C[9] = {c0, c1, c2, c3, c4, c5, c6, c7, c8};
    T d2 = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const T xn = a * X[i] + b * C[i];
      d2 += (xn - X[i]) * (xn - X[i]);
      X[i] = xn;
    }
    if (d2 <= stop) return true;
  }
  return false;
}

__device__ inline void closest_rotation(const double F[9], double R[9]) {
  if (polar_newton<double>(F, R)) return;
  double qt[4];
  closest_quat_t<double>(F, qt);
  quat_rotation(qt[0], qt[1], qt[2], qt[3], R);
}

__device__ inline double det3(const double F[9]) {
  return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// Differential of the closest rotation: dR = R [w]_x with
// (tr(S) I - S) w = axial(R^T dF - dF^T R), S = R^T F (symmetric).  Returns the
// inverse of K = tr(S) I - S as 6 entries (xx, yy, zz, xy, xz, yz); a singular K
// (sigma_i + sigma_j = 0) yields zeros and is reported through the flag.
__device__ inline bool rotation_kinv(const double F[9], const double R[9], double Ki[6]) {
  double S[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = R[i] * F[j] + R[3 + i] * F[3 + j] + R[6 + i] * F[6 + j];
  const double sxy = 0.5 * (S[1] + S[3]), sxz = 0.5 * (S[2] + S[6]), syz = 0.5 * (S[5] + S[7]);
  const double tr = S[0] + S[4] + S[8];
  const double kxx = tr - S[0], kyy = tr - S[4], kzz = tr - S[8];
  const double kxy = -sxy, kxz = -sxz, kyz = -syz;
  const double cxx = kyy * kzz - kyz * kyz, cyy = kxx * kzz - kxz * kxz, czz = kxx * kyy - kxy * kxy;
  const double cxy = kxz * kyz - kxy * kzz, cxz = kxy * kyz - kxz * kyy, cyz = kxy * kxz - kxx * kyz;
  const double det = kxx * cxx + kxy * cxy + kxz * cxz;
  const double scale = fabs(tr) + 1e-300;
  if (!(fabs(det) > 1e-12 * scale * scale * scale)) {
#pragma unroll
    for (int i = 0; i < 6; ++i) Ki[i] = 0.0;
    return false;
  }
  const double id = 1.0 / det;
  Ki[0] = cxx * id;
  Ki[1] = cyy * id;
  Ki[2] = czz * id;
  Ki[3] = cxy * id;
  Ki[4] = cxz * id;
  Ki[5] = cyz * id;
  return true;
}

// One FP64 Newton step of the polar decomposition of F from an orthogonal
// approximation R0: with S = R0^T F, K = tr(sym S) I - sym S and
// a = axial(S - S^T), R = R0 exp([K^{-1} a]_x) (Rodrigues), the same
// linearisation of F = R S as dR/dF.  From an FP32-accurate R0 it leaves an
// error of order eps32^2.  When K is singular R0 is kept.
__device__ inline void polish_rotation(const double F[9], const double R0[9], double R[9]) {
  double Ki[6], S[9];
  if (!rotation_kinv(F, R0, Ki)) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = R0[i];
    return;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = R0[i] * F[j] + R0[3 + i] * F[3 + j] + R0[6 + i] * F[6 + j];
  const double a0 = S[7] - S[5], a1 = S[2] - S[6], a2 = S[3] - S[1];
  const double w0 = Ki[0] * a0 + Ki[3] * a1 + Ki[4] * a2;
  const double w1 = Ki[3] * a0 + Ki[1] * a1 + Ki[5] * a2;
  const double w2 = Ki[4] * a0 + Ki[5] * a1 + Ki[2] * a2;
  const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
  double c1, c2;  // sin(t)/t and (1 - cos(t))/t^2
  if (th2 < 1e-4) {
    c1 = 1.0 - th2 / 6.0 * (1.0 - th2 / 20.0);
    c2 = 0.5 - th2 / 24.0 * (1.0 - th2 / 30.0);
  } else {
    const double t = sqrt(th2);
    c1 = sin(t) / t;
    c2 = (1.0 - cos(t)) / th2;
  }
  // E = I + c1 [w]_x + c2 [w]_x^2
  const double E[9] = {1.0 - c2 * (w1 * w1 + w2 * w2), -c1 * w2 + c2 * w0 * w1, c1 * w1 + c2 * w0 * w2,
                       c1 * w2 + c2 * w0 * w1, 1.0 - c2 * (w0 * w0 + w2 * w2), -c1 * w0 + c2 * w1 * w2,
                       -c1 * w1 + c2 * w0 * w2, c1 * w0 + c2 * w1 * w2, 1.0 - c2 * (w0 * w0 + w1 * w1)};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = R0[3 * i] * E[j] + R0[3 * i + 1] * E[3 + j] + R0[3 * i + 2] * E[6 + j];
}

// Mixed-precision local step: an FP32 rotation (the Newton polar factor, or
// where that iteration does not apply, det F <= 0, the q-method's
// quaternion), made orthogonal in FP64 (Newton steps on the FP32 factor
// itself; the quaternion's rotation formed in FP64), then one FP64 polishing
// step towards the polar factor of F.
__device__ inline void closest_rotation_mixed(const double F[9], double R[9]) {
  float Ff[9], Xf[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Ff[i] = (float)F[i];
  double R0[9];
  bool have = false;
  if (polar_newton<float>(Ff, Xf)) {
    double Xd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Xd[i] = R0[i] = (double)Xf[i];
    have = polar_newton<double>(Xd, R0, true);   // orthogonal polar factor of the FP32 iterate
  }
  if (!have) {
    float qf[4];
    closest_quat_t<float>(Ff, qf);
    quat_rotation(qf[0], qf[1], qf[2], qf[3], R0);
  }
  polish_rotation(F, R0, R);
}

__device__ inline void rotation_apply_diff(const double R[9], const double Ki[6], const double dF[9],
                                           double dR[9]) {
  // M = R^T dF; a = axial(M - M^T) = (M21 - M12, M02 - M20, M10 - M01)
  double M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = R[i] * dF[j] + R[3 + i] * dF[3 + j] + R[6 + i] * dF[6 + j];
  const double a0 = M[7] - M[5], a1 = M[2] - M[6], a2 = M[3] - M[1];
  const double w0 = Ki[0] * a0 + Ki[3] * a1 + Ki[4] * a2;
  const double w1 = Ki[3] * a0 + Ki[1] * a1 + Ki[5] * a2;
  const double w2 = Ki[4] * a0 + Ki[5] * a1 + Ki[2] * a2;
  // R [w]_x, [w]_x = [[0,-w2,w1],[w2,0,-w0],[-w1,w0,0]]
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double r0 = R[3 * i], r1 = R[3 * i + 1], r2 = R[3 * i + 2];
    dR[3 * i + 0] = r1 * w2 - r2 * w1;
    dR[3 * i + 1] = -r0 * w2 + r2 * w0;
    dR[3 * i + 2] = r0 * w1 - r1 * w0;
  }
}

// ------------------------------------------------------------------ volume preservation
//
// Volume-preserving term (supplemental Sec. Energy Definitions): the
// projection D of F onto {det D = 1}.  F = R S with R the closest rotation
// and S = R^T F symmetric; S = V diag(s) V^T (cyclic Jacobi rotations, V a
// proper rotation) gives the signed SVD F = (R V) diag(s) V^T.  With d the
// minimiser of |d|^2 subject to prod(s_i + d_i) = 1, found by Newton's method
// on its KKT conditions d + lam grad c = 0, c = prod(s + d) - 1 from d = 0,
// D = R V diag(s + d) V^T.  Where an eigenvalue of S is not positive (det F
// <= 0) the constraint cannot be met on that branch and D = R (its derivative
// then dR/dF).  For the adjoint, dD[dF] = U B V^T with U = R V, A = U^T dF V,
// B_ii = sum_k G_ik A_kk (G = dD/ds from the differentiated KKT system,
// eq:vol_kkt) and for i != j
//   B_ij = r_ij (A_ij + A_ji)/2 + k_ij (A_ij - A_ji)/2,
// r_ij = (D_i - D_j)/(s_i - s_j) (G_ii - G_ij where s_i = s_j),
// k_ij = (D_i + D_j)/(s_i + s_j).

// Symmetric 3x3 A (row-major, symmetric) = V diag(w) V^T by cyclic Jacobi
// rotations; V is a product of plane rotations (det +1).
__device__ inline void sym3_eigen(const double S[9], double V[9], double w[3]) {
  double a[3][3] = {{S[0], 0.5 * (S[1] + S[3]), 0.5 * (S[2] + S[6])},
                    {0.5 * (S[1] + S[3]), S[4], 0.5 * (S[5] + S[7])},
                    {0.5 * (S[2] + S[6]), 0.5 * (S[5] + S[7]), S[8]}};
  double v[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-34 * dia)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
      // A <- J^T A J with J the rotation in the (p, q) plane
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - sn * akq;
        a[k][q] = sn * akp + c * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - sn * aqk;
        a[q][k] = sn * apk + c * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - sn * vkq;
        v[k][q] = sn * vkp + c * vkq;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    w[i] = a[i][i];
#pragma unroll
    for (int j = 0; j < 3; ++j) V[3 * i + j] = v[i][j];
  }
}

// Solution of the KKT system [[K, g], [g^T, 0]] [x; y] = [b1; b2] with
// K = I + lam H (H: the Hessian of c, zero diagonal, off-diagonal
// h01 = D2, h02 = D1, h12 = D0) by the Schur complement on g.
__device__ inline void kkt_solve(double lam, const double D[3], const double g[3], const double b1[3],
                                 double b2, double x[3], double& y) {
  const double k00 = 1.0, k11 = 1.0, k22 = 1.0, k01 = lam * D[2], k02 = lam * D[1], k12 = lam * D[0];
  const double c00 = k11 * k22 - k12 * k12, c11 = k00 * k22 - k02 * k02, c22 = k00 * k11 - k01 * k01;
  const double c01 = k02 * k12 - k01 * k22, c02 = k01 * k12 - k02 * k11, c12 = k01 * k02 - k00 * k12;
  const double det = k00 * c00 + k01 * c01 + k02 * c02;
  const double id = 1.0 / det;
  auto kinv = [&](const double r[3], double o[3]) {
    o[0] = (c00 * r[0] + c01 * r[1] + c02 * r[2]) * id;
    o[1] = (c01 * r[0] + c11 * r[1] + c12 * r[2]) * id;
    o[2] = (c02 * r[0] + c12 * r[1] + c22 * r[2]) * id;
  };
  double kb[3], kg[3];
  kinv(b1, kb);
  kinv(g, kg);
  y = (g[0] * kb[0] + g[1] * kb[1] + g[2] * kb[2] - b2) / (g[0] * kg[0] + g[1] * kg[1] + g[2] * kg[2]);
  x[0] = kb[0] - kg[0] * y;
  x[1] = kb[1] - kg[1] * y;
  x[2] = kb[2] - kg[2] * y;
}

// Per Gauss point: V (signed SVD F = R V diag(s) V^T), the projected singular
// values Dd = s + d, and whether the projection applies (det F > 0).
struct VolumeProj {
  double V[9], s[3], Dd[3], lam;
  bool ok;
};

__device__ inline void volume_project(const double F[9], const double R[9], VolumeProj& P) {
  double S[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = R[i] * F[j] + R[3 + i] * F[3 + j] + R[6 + i] * F[6 + j];
  sym3_eigen(S, P.V, P.s);
  P.ok = P.s[0] > 0.0 && P.s[1] > 0.0 && P.s[2] > 0.0;
  P.lam = 0.0;
  if (!P.ok) {
    P.Dd[0] = P.Dd[1] = P.Dd[2] = 1.0;
    return;
  }
  double d[3] = {0.0, 0.0, 0.0}, lam = 0.0;
  for (int it = 0; it < 40; ++it) {
    const double D[3] = {P.s[0] + d[0], P.s[1] + d[1], P.s[2] + d[2]};
    const double g[3] = {D[1] * D[2], D[0] * D[2], D[0] * D[1]};
    const double c = D[0] * D[1] * D[2] - 1.0;
    const double r1[3] = {-(d[0] + lam * g[0]), -(d[1] + lam * g[1]), -(d[2] + lam * g[2])};
    double dd[3], dl;
    kkt_solve(lam, D, g, r1, -c, dd, dl);
    d[0] += dd[0];
    d[1] += dd[1];
    d[2] += dd[2];
    lam += dl;
    if (fabs(dd[0]) <= 1e-16 * (1.0 + fabs(P.s[0])) && fabs(dd[1]) <= 1e-16 * (1.0 + fabs(P.s[1])) &&
        fabs(dd[2]) <= 1e-16 * (1.0 + fabs(P.s[2])))
      break;
  }
  P.Dd[0] = P.s[0] + d[0];
  P.Dd[1] = P.s[1] + d[1];
  P.Dd[2] = P.s[2] + d[2];
  P.lam = lam;
}

// D = R V diag(Dd) V^T.
__device__ inline void volume_matrix(const double R[9], const double V[9], const double Dd[3], double D[9]) {
  double M[9];   // V diag(Dd) V^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = V[3 * i] * Dd[0] * V[3 * j] + V[3 * i + 1] * Dd[1] * V[3 * j + 1] +
                     V[3 * i + 2] * Dd[2] * V[3 * j + 2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      D[3 * i + j] = R[3 * i] * M[j] + R[3 * i + 1] * M[3 + j] + R[3 * i + 2] * M[6 + j];
}

// Derivative data of the projection: G = dD/ds (row-major 3x3) from the
// differentiated KKT system, the ratios r (pairs 01, 02, 12) and k.
__device__ inline void volume_derivative_data(const VolumeProj& P, double G[9], double r[3], double k[3]) {
  const double* D = P.Dd;
  const double g[3] = {D[1] * D[2], D[0] * D[2], D[0] * D[1]};
  const double lam = P.lam;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    // right-hand side (-lam H e_j, -g_j)
    double b1[3];
    b1[0] = j == 0 ? 0.0 : -lam * (j == 1 ? D[2] : D[1]);
    b1[1] = j == 1 ? 0.0 : -lam * (j == 0 ? D[2] : D[0]);
    b1[2] = j == 2 ? 0.0 : -lam * (j == 0 ? D[1] : D[0]);
    double x[3], y;
    kkt_solve(lam, D, g, b1, -g[j], x, y);
#pragma unroll
    for (int i = 0; i < 3; ++i) G[3 * i + j] = (i == j ? 1.0 : 0.0) + x[i];
  }
  const int I[3] = {0, 0, 1}, J[3] = {1, 2, 2};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = I[p], j = J[p];
    const double ds = P.s[i] - P.s[j];
    r[p] = fabs(ds) <= 1e-9 * (fabs(P.s[i]) + fabs(P.s[j])) ? G[3 * i + i] - G[3 * i + j] : (D[i] - D[j]) / ds;
    k[p] = (D[i] + D[j]) / (P.s[i] + P.s[j]);
  }
}

// dD[dF] from the cached data (R, V, G, r, k).
__device__ inline void volume_apply_diff(const double R[9], const double V[9], const double G[9], const double r[3],
                                         const double k[3], const double dF[9], double dD[9]) {
  double U[9], T[9], A[9], B[9];
  // U = R V
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) U[3 * i + j] = R[3 * i] * V[j] + R[3 * i + 1] * V[3 + j] + R[3 * i + 2] * V[6 + j];
  // A = U^T dF V
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[3 * i + j] = U[i] * dF[j] + U[3 + i] * dF[3 + j] + U[6 + i] * dF[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = T[3 * i] * V[j] + T[3 * i + 1] * V[3 + j] + T[3 * i + 2] * V[6 + j];
  B[0] = G[0] * A[0] + G[1] * A[4] + G[2] * A[8];
  B[4] = G[3] * A[0] + G[4] * A[4] + G[5] * A[8];
  B[8] = G[6] * A[0] + G[7] * A[4] + G[8] * A[8];
  const int I[3] = {0, 0, 1}, J[3] = {1, 2, 2};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int i = I[p], j = J[p];
    const double sym = 0.5 * (A[3 * i + j] + A[3 * j + i]), skw = 0.5 * (A[3 * i + j] - A[3 * j + i]);
    B[3 * i + j] = r[p] * sym + k[p] * skw;
    B[3 * j + i] = r[p] * sym - k[p] * skw;
  }
  // dD = U B V^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[3 * i + j] = U[3 * i] * B[j] + U[3 * i + 1] * B[3 + j] + U[3 * i + 2] * B[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      dD[3 * i + j] = T[3 * i] * V[3 * j] + T[3 * i + 1] * V[3 * j + 1] + T[3 * i + 2] * V[3 * j + 2];
}

// Element tile: 32 elements x 8 Gauss points per 256-thread block.
template <int kE>
struct ElemTileT {
  double xs[kE][8][3];
  double Ps[kE][8][9];
};
using ElemTile = ElemTileT<kElemsPerBlock>;

__device__ inline void gather_nodes(const DevMesh& M, const double* __restrict__ x, ElemTile& T,
                                    int le, int a, int e, bool valid) {
  if (valid) {
    const int n = M.conn[(int64_t)a * M.E + e];
    T.xs[le][a][0] = x[n];
    T.xs[le][a][1] = x[(int64_t)M.N + n];
    T.xs[le][a][2] = x[2 * (int64_t)M.N + n];
  }
}

template <class Tile>
__device__ inline void deformation_gradient(const Tile& T, int le, int q, const GradTable& G,
                                            double F[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double b0 = bgrad(q, 0, a, G), b1 = bgrad(q, 1, a, G), b2 = bgrad(q, 2, a, G);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double xi = T.xs[le][a][i];
      F[3 * i + 0] += xi * b0;
      F[3 * i + 1] += xi * b1;
      F[3 * i + 2] += xi * b2;
    }
  }
}

// f_a = sum_q P_q gradN_a(xi_q), written to fe[c][8e + a]
template <class Tile>
__device__ inline void corner_force(const Tile& T, int le, int a, const GradTable& G, double& f0,
                                    double& f1, double& f2) {
  f0 = f1 = f2 = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double b0 = bgrad(q, 0, a, G), b1 = bgrad(q, 1, a, G), b2 = bgrad(q, 2, a, G);
    const double* P = T.Ps[le][q];
    f0 += P[0] * b0 + P[1] * b1 + P[2] * b2;
    f1 += P[3] * b0 + P[4] * b1 + P[5] * b2;
    f2 += P[6] * b0 + P[7] * b1 + P[8] * b2;
  }
}

__device__ inline void element_forces_out(const DevMesh& M, const ElemTile& T, int le, int a,
                                          int e, bool valid, const GradTable& G, double* fe) {
  if (!valid) return;
  double f0, f1, f2;
  corner_force(T, le, a, G, f0, f1, f2);
  const int64_t E8 = 8 * (int64_t)M.E, idx = 8 * (int64_t)e + a;
  fe[idx] = f0;
  fe[E8 + idx] = f1;
  fe[2 * E8 + idx] = f2;
}


// Stress differential of the adjoint local step at Gauss point q of an element
// (eq:matrix_split): w (dF - dR[dF]) with dR from the cached rotation and
// inv(tr(S) I - S), plus the muscle term (I - (r/|f|)(I - n n^T)) df m^T.
// dF is formed from the direction staged in T.xs; the result goes to T.Ps.
// cq holds the Gauss point's cache entries: R (9), inv(tr(S) I - S) (6) and,
// with muscles, the unit fibre image n (3) and r/|f| (1).
__device__ inline void hvp_stress_from_dF(const DevMesh& M, double* P, const double dF[9], double w,
                                          const double* cq) {
  double dR[9];
  rotation_apply_diff(cq, cq + 9, dF, dR);
#pragma unroll
  for (int i = 0; i < 9; ++i) P[i] = w * (dF[i] - dR[i]);
  if (M.muscle_k > 0.0) {
    const double m0 = M.fiber[0], m1 = M.fiber[1], m2 = M.fiber[2];
    const double d0 = dF[0] * m0 + dF[1] * m1 + dF[2] * m2;
    const double d1 = dF[3] * m0 + dF[4] * m1 + dF[5] * m2;
    const double d2 = dF[6] * m0 + dF[7] * m1 + dF[8] * m2;
    const double n0 = cq[15], n1 = cq[16], n2 = cq[17], sc = cq[18];
    const double nd = n0 * d0 + n1 * d1 + n2 * d2;
    const double wm = M.muscle_k * M.Vq;
    const double g0 = wm * (d0 - sc * (d0 - n0 * nd));
    const double g1 = wm * (d1 - sc * (d1 - n1 * nd));
    const double g2 = wm * (d2 - sc * (d2 - n2 * nd));
    P[0] += g0 * m0; P[1] += g0 * m1; P[2] += g0 * m2;
    P[3] += g1 * m0; P[4] += g1 * m1; P[5] += g1 * m2;
    P[6] += g2 * m0; P[7] += g2 * m1; P[8] += g2 * m2;
  }
}

// Cache entries of Gauss point q of element e (layout [19][8E]).
__device__ inline void load_gauss_cache(const DevMesh& M, const double* __restrict__ cache, int e, int q,
                                        double cq[19]) {
  const int64_t Q = 8 * (int64_t)M.E, qi = 8 * (int64_t)e + q;
  const int rows = M.muscle_k > 0.0 ? 19 : 15;
#pragma unroll
  for (int i = 0; i < 19; ++i) cq[i] = i < rows ? cache[i * Q + qi] : 0.0;
}

// The volume-preserving term of (A - dA) p at Gauss point q of element e:
// P += w_v (dF - dD[dF]) from the cached projection data.
__device__ inline void hvp_volume(const DevMesh& M, double* P, const double dF[9], int e, int q,
                                  const double* __restrict__ cache, const double cq[19]) {
  const int64_t Q = 8 * (int64_t)M.E, qi = 8 * (int64_t)e + q;
  double dD[9];
  if (cache[kVolOk * Q + qi] != 0.0) {
    double V[9], Gm[9], r[3], k[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      V[i] = cache[(kVolV + i) * Q + qi];
      Gm[i] = cache[(kVolG + i) * Q + qi];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      r[i] = cache[(kVolR + i) * Q + qi];
      k[i] = cache[(kVolK + i) * Q + qi];
    }
    volume_apply_diff(cq, V, Gm, r, k, dF, dD);
  } else {
    rotation_apply_diff(cq, cq + 9, dF, dD);   // D = R where det F <= 0
  }
  const double wv = M.wv_e[e];
#pragma unroll
  for (int i = 0; i < 9; ++i) P[i] += wv * (dF[i] - dD[i]);
}

__device__ inline void hvp_stress(const DevMesh& M, ElemTile& T, int le, int q, int e, const GradTable& G,
                                  const double* __restrict__ cache) {
  double cq[19], dF[9];
  load_gauss_cache(M, cache, e, q, cq);
  deformation_gradient(T, le, q, G, dF);
  hvp_stress_from_dF(M, T.Ps[le][q], dF, M.w_e[e], cq);
  if (M.wv_e) hvp_volume(M, T.Ps[le][q], dF, e, q, cache, cq);
}

// Sum the element forces of every node (fixed order) and form the residual.
__device__ inline void node_force(const DevMesh& M, const double* __restrict__ fe, int n,
                                  double& f0, double& f1, double& f2) {
  if (M.inc_ptr) {   // tetrahedra: [3][4E] corner forces, compressed incidence in (e, a) order
    const int64_t E4 = 4 * (int64_t)M.E;
    f0 = f1 = f2 = 0.0;
    int k = M.inc_ptr[n];
    const int k1 = M.inc_ptr[n + 1];
    // four incidences' loads issued together, added in incidence order
    for (; k + 3 < k1; k += 4) {
      const int p0 = M.inc[k], p1 = M.inc[k + 1], p2 = M.inc[k + 2], p3 = M.inc[k + 3];
      const double a0 = fe[p0], a1 = fe[p1], a2 = fe[p2], a3 = fe[p3];
      const double b0 = fe[E4 + p0], b1 = fe[E4 + p1], b2 = fe[E4 + p2], b3 = fe[E4 + p3];
      const double c0 = fe[2 * E4 + p0], c1 = fe[2 * E4 + p1], c2 = fe[2 * E4 + p2], c3 = fe[2 * E4 + p3];
      f0 += a0;
      f0 += a1;
      f0 += a2;
      f0 += a3;
      f1 += b0;
      f1 += b1;
      f1 += b2;
      f1 += b3;
      f2 += c0;
      f2 += c1;
      f2 += c2;
      f2 += c3;
    }
    for (; k < k1; ++k) {
      const int p = M.inc[k];
      f0 += fe[p];
      f1 += fe[E4 + p];
      f2 += fe[2 * E4 + p];
    }
    return;
  }
  const int64_t E8 = 8 * (int64_t)M.E;
  f0 = f1 = f2 = 0.0;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int p = M.node_inc[(int64_t)s * M.N + n];
    if (p >= 0) {
      f0 += fe[p];
      f1 += fe[E8 + p];
      f2 += fe[2 * E8 + p];
    }
  }
}

}  // namespace dpd
