// Global step with a contact set: kernel launchers (contact.hip, internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device.hpp"

namespace dpd {

constexpr int kContactMaxSet = 120;    // active-set size: the c x c Cholesky stays in LDS
constexpr int kContactThreads = 1024;  // threads of the one-workgroup factorization
constexpr int kContactDenseThreads = 512;   // dense reduced step: 8 waves, a row each in turn
constexpr int kContactDenseMaxRows = 2048;  // its r in LDS: 3 x 2048 doubles (the dense inverse's limit)

size_t contact_factor_lds(int c);
void launch_contact_unit(hipStream_t s, int N, int n_cand, const int32_t* cand, int k0, double* b);
void launch_contact_collect(hipStream_t s, int N, int n_cand, int k0, const double* x, double* B1);
hipError_t launch_contact_factor(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c,
                                 const double* B1, double* Sinv, int* status);
void launch_contact_lam(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c, const double* Sinv,
                        const double* a1, double* lam, const IterState* st = nullptr);
// time step with contact (Alg. 3 / Alg. 5)
void launch_contact_descend(hipStream_t s, int N, const int32_t* set, int c, const double* B1, const double* lam,
                            const double* d, const uint8_t* mask, double* x, const IterState* st);
void launch_contact_detect(hipStream_t s, int N, int n_cand, const int32_t* cand, double h, const double* x,
                           const double* v, double* tgt, int32_t* kind, uint8_t* left);
void launch_contact_mark(hipStream_t s, int n_cand, const int32_t* cand, const int32_t* kind, uint8_t* mask);
void launch_contact_place(hipStream_t s, int N, int n_cand, const int32_t* cand, const int32_t* kind,
                          const double* tgt, double* x);
void launch_contact_active_set(hipStream_t s, int N, int n_cand, const int32_t* cand, const double* x0,
                               const double* xn, const double* r, int32_t* kind, uint8_t* left, double* tgt);
hipError_t launch_contact_reduced_inverse(hipStream_t s, int n, const int32_t* inv, const int32_t* cand,
                                          const int32_t* set, int c, const double* Ainv, const double* Sinv,
                                          double* T, uint8_t* in_c, double* W);
size_t contact_dense_lds(int n);
hipError_t launch_contact_dense_step(hipStream_t s, int n, int N, const int32_t* perm, const double* W,
                                     const double* r, double* x, const IterState* st);
constexpr int kContactBarWords = 64 * 9;    // fused loop's barrier: 8 group counters on own lines, flags, abort
hipError_t launch_contact_fused_cg(hipStream_t s, const DevMesh& Mmask, const DenseCG& D, int blocks,
                                   const double* W, double* z, const double* xbar, const double* cache,
                                   IterState* st, uint32_t* bar, int max_iter);
hipError_t launch_contact_fused(hipStream_t s, const DevMesh& Mmask, const DenseCG& D, int blocks,
                                const double* W, double* x, const double* y, const double* act, const double* cache,
                                IterState* st, uint32_t* bar, int mode, int max_iter);
void launch_contact_target_vjp(hipStream_t s, int N, int n_cand, const int32_t* cand, const int32_t* kind,
                               const double* x, const double* v, const double* r, double* gx, double* gv);
void launch_contact_update(hipStream_t s, int N, const int32_t* set, int c, const double* B1, const double* lam,
                           double* x);
void launch_contact_set(hipStream_t s, int N, const int32_t* cand, const int32_t* set, int c, const double* xstar,
                        double* x);

}  // namespace dpd
