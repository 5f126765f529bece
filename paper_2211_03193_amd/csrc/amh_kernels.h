// amh_kernels.h -- kernel parameter blocks and launch entry points shared by the
// kernels (amh_kernels.hip) and the C ABI (amh_api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace amh {

// bits of the device error word
constexpr unsigned int kErrTable = 1u;   // non-finite distogram entry
constexpr unsigned int kErrEnergy = 2u;  // non-finite energy or energy change
constexpr unsigned int kErrStall = 4u;   // a pipelined localized sweep waited past its bound

struct SweepParams {
  // distogram table, padded rows
  const float* table;     // padded -ln p rows (anchors)
  const float* ydev;      // padded rows minus the no-contact value (sweeps)
  const float* zrow;      // a padded row of zeros (read by pairs beyond the last knot)
  int stride, nb;
  float inv_w, off, tmax, d2far;
  double d_min, bin_w;
  double vfar;            // sum of every row's no-contact value (far_sum_kernel)
  // run
  int L, C, half_window, global_every, n_global, anchor_every;   // n_global >= 1
  int n_cascade, cascade_hw[3];   // extra window half-widths taken in turn with half_window
  double sigma, sigma_end, T0, T1;  // sigma_end > 0: geometric decay of the proposal width
  int64_t S, t0, n_sweeps;
  uint32_t key0, key1, chain_offset;
  int spin_limit;     // polls of a pipelined localized sweep's wait before it gives up
  double target;
  // chain state
  double* s;          // [C][2L]
  double* s_best;     // [C][2L]
  double* atoms;      // [C][L][4][3] N, CA, C, CB (float64)
  double* v;          // [C][2]     V at last anchor, best V
  int64_t* counters;  // [C][4]
  unsigned int* err;
  // trace
  int n_trace;
  int trace_chain[4];
  double* tr_dE;
  double* tr_delta;
  uint8_t* tr_acc;
  int64_t trace_cap, trace_t0;
  double* tr_anchor;
  int64_t trace_anchor_cap, trace_anchor0;
  // executed-work counters of the global sweeps, or null: [0] rectangle tiles that
  // survive the bounding-sphere test, [1] pair tests inside the rectangle in those
  // tiles, [2] near pairs evaluated (one stencil each); added to at the end of a launch
  unsigned long long* work;
};

struct ConfParams {
  int L;
  const double* s_in;   // [B][2L] or null (extended chain)
  // energy (optional: table == null skips it)
  const float* table;
  int stride, nb;
  double d_min, bin_w;
  double vfar;          // sum of every row's no-contact value (far_sum_kernel)
  double* V_out;        // [B]
  double* s_out;        // [B][2L]
  float* cb_out;        // [B][L][3]
  float* atoms_out;     // [B][L][4][3]
  double* atoms64_out;  // [B][L][4][3]
  // context initialisation (optional)
  double* v_state;      // [B][2]
  int64_t* counters;    // [B][4]
  double* s_best;       // [B][2L]
  int keep_best;        // v_state: set V as current, lower the best (and s_best) only if V is lower
  unsigned int* err;
};

size_t sweep_lds_bytes(int G, int L, int W);
size_t sweep_lds_bytes_local(int G, int L, int W);

// Sweep t is global iff it is one of the last n_global sweeps of its cycle of
// global_every sweeps (Algorithm 1's alternation, localized sweeps first).
__host__ __device__ inline bool is_global(const SweepParams& P, int64_t t) {
  return P.global_every > 0 && (int)((uint32_t)t % (uint32_t)P.global_every) >= P.global_every - P.n_global;
}

// kinds of sweep a sweep kernel instance runs
constexpr int kSweepMixed = 0, kSweepLocal = 1, kSweepGlobal = 2;
// virtual wavefronts of the float64 energy reduction (fixed, so that the energy
// does not depend on the launch shape)
constexpr int kVirtWaves = 8;
inline size_t conf_lds_bytes(int L, int W) {
  (void)W;
  return 8 * (2 * (size_t)L + 12 * (size_t)L + 2 * (size_t)kVirtWaves + 2) + 16 * (size_t)((L + 7) / 8) + 32;
}

__global__ void ingest_kernel(const float* y, int64_t P, int nb, int stride, float* out,
                              float* dev, unsigned int* err);
__global__ void conf_energy_kernel(ConfParams P);
__global__ void far_sum_kernel(const float* table, int64_t P, int stride, int nb, double* out);
__global__ void philox_kernel(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t* out);
__global__ void perturb_kernel(double* s, int64_t n_total, int n, uint32_t chain_offset, uint32_t tag,
                               uint32_t k0, uint32_t k1, double amplitude);
template <int G, int MODE>
__global__ void sweep_kernel(SweepParams P);
template <int G, int MODE>
__global__ void sweep_batch_kernel(const SweepParams* descs, const int2* map);

}  // namespace amh
