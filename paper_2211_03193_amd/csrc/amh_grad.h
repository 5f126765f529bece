// amh_grad.h -- parameter blocks of the gradient and L-BFGS kernels (amh_grad.hip),
// shared with the C ABI (amh_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "amh_kernels.h"

namespace amh {

constexpr unsigned int kErrGradEnergy = kErrEnergy;
constexpr int kGradThreads = 256;
constexpr int kLbfgsMaxHistory = 64;
constexpr int kLbfgsMaxNonmonotone = 64;
// Fixed L-BFGS workspace of amh_minimize_noalloc: 8 Mi doubles (64 MiB) per device,
// e.g. 499 conformations of 400 residues with m = 8 (16,800 doubles each).
constexpr long long kNoallocScratchDoubles = 8LL << 20;
constexpr int kMaxDevices = 64;

struct GradParams {
  int L;
  const double* s;      // [B][2L]
  const float* table;   // padded -ln p rows
  int stride, nb;
  double d_min, bin_w;
  double* V;            // [B] or null
  double* g;            // [B][2L] or null
  unsigned int* err;
};

struct LbfgsParams {
  int L;
  double* s;            // [B][2L] in/out
  const float* table;
  int stride, nb;
  double d_min, bin_w;
  int n_iter, m, nonmonotone, max_ls;
  double c1, shrink, gtol, step0;
  double* work;         // [B][(5 + 2m) 2L]
  double* V;            // [B] or null
  int32_t* iters;       // [B] or null
  int32_t* status;      // [B] or null
  double* f_trace;      // [B][n_iter + 1] or null
  double* x_trace;      // [B][n_iter + 1][2L] or null (iterates, unwrapped)
  double* v_state;      // [B][2] (current V, best V) or null
  double* s_best;       // [B][2L], updated with v_state
  unsigned int* err;
};

inline size_t grad_lds_bytes(int L, int W) {
  return 8 * (12 * (size_t)L + 6 * ((size_t)L + 1) + 3 * (size_t)W);
}
inline size_t lbfgs_lds_bytes(int L, int W, int m, int M) {
  return grad_lds_bytes(L, W) + 8 * (2 * (size_t)m + (size_t)M);
}
inline size_t lbfgs_work_doubles(int L, int m) { return (5 + 2 * (size_t)m) * 2 * (size_t)L; }

__global__ void grad_kernel(GradParams P);
__global__ void lbfgs_kernel(LbfgsParams P);

}  // namespace amh
