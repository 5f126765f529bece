// amh_kernels.hip -- HIP kernels of the Alternating Metropolis-Hastings sampler
// for MI355X (gfx950, wave64).
//
// Method (Ghantasala, Jaiswal, Datta, arXiv 2211.03193): single-torsion Gaussian
// proposals swept over k = 0 .. 2L-1 (Sec. 2.1, Algorithm 1), judged either by the
// full distogram energy V (global MH) or by the energy of the window of residues
// within d/2 of residue k/2 (localized MH, Sec. 2.3); global and localized sweeps
// alternate (Algorithm 1, Fig. 1); acceptance min(1, exp(-beta dE)) (Sec. 2.1).
//
// Mapping to the GPU (our design, not the paper's block-per-chain layout):
//   * a workgroup owns G chains that walk the same proposal index k in lockstep,
//     so every table row a global proposal needs is fetched once per workgroup
//     from L2 and shared by the G chains;
//   * localized sweeps are run by one wavefront per chain with no workgroup
//     barrier; residues beyond the window are brought up to date lazily with one
//     accumulated rigid transform (float64) when they enter the window;
//   * pair energies are handled as deviations from the pair's no-contact value
//     (a second copy of the table with that value subtracted), which are exactly
//     zero beyond the last knot: a pair farther apart than 20.25 A costs a
//     distance and a compare, no table access;
//   * global proposals use every wavefront of the workgroup; dE of pivot p is
//     D_new(p) - D(p), where D(p), the deviation energy of the pair rectangle
//     i < p <= j of the current conformation, is carried from proposal to
//     proposal (the new rectangle sum on accept, an O(L) row/column update when
//     p advances), so each global proposal evaluates one spline per changed near
//     pair instead of two;
//   * the rectangle is walked in 8 x 8 tiles (blocks of 8 residues); a tile whose
//     two bounding spheres lie farther apart than the last knot holds only pairs
//     that add zero and is skipped whole, a decision uniform over the wavefront;
//   * the proposal randoms come from Philox4x32-10 at counter (k, t, chain, 0),
//     the same stream the oracle replays, drawn 64 proposals at a time, one per lane;
//   * the master coordinates (N, CA, C, C-beta) live in LDS in float64 and are
//     rotated in float64; the O(L^2) pair loop reads float32 C-beta positions taken
//     relative to the pivot point, rounded once per proposal, so float32 never
//     accumulates error in the state (an extended 300-residue chain spans ~1000 A,
//     where float32 resolves only ~6e-5 A);
//   * after every anchor sweep the coordinates are rebuilt from the float64
//     torsions by NeRF and V is re-anchored in float64 with Neumaier summation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "amh_device.h"
#include "amh_geom.h"
#include "amh_kernels.h"

namespace amh {

// ---------------------------------------------------------------------------
// Table ingest: repack [P][nb] rows into padded rows [y1, y0..y_{nb-1}, y_{nb-2}, 0...]
// (`out`) and the same rows minus the row's no-contact value y_{nb-1} (`dev`, rounded
// once from float64), and flag non-finite entries.
__global__ void ingest_kernel(const float* __restrict__ y, int64_t P, int nb, int stride,
                              float* __restrict__ out, float* __restrict__ dev, unsigned int* err) {
  const int64_t n = P * (int64_t)stride;
  bool bad = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / stride;
    const int c = (int)(e - r * stride);
    float v = 0.0f;
    if (c == 0) v = y[r * nb + 1];
    else if (c <= nb) v = y[r * nb + (c - 1)];
    else if (c == nb + 1) v = y[r * nb + (nb - 2)];
    if (c <= nb && !isfinite(v)) bad = true;
    out[e] = v;
    dev[e] = c <= nb + 1 ? (float)((double)v - (double)y[r * nb + (nb - 1)]) : 0.0f;
  }
  if (bad) atomicOr(err, kErrTable);
}

// Noisy restart: s_k += amplitude (2u - 1) with u from Philox at (k, tag, chain, 1),
// wrapped into (-pi, pi]; one thread per torsion of every chain.
__global__ void perturb_kernel(double* __restrict__ s, int64_t n_total, int n, uint32_t chain_offset,
                               uint32_t tag, uint32_t k0, uint32_t k1, double amplitude) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / n), k = (int)(e - (int64_t)c * n);
    const U4 r = philox10(U4{(uint32_t)k, tag, chain_offset + (uint32_t)c, 1u}, k0, k1);
    const double u = ((double)r.x + 0.5) * (1.0 / 4294967296.0);
    s[e] = wrap_angle(s[e] + amplitude * (2.0 * u - 1.0));
  }
}

__global__ void philox_kernel(const uint32_t* __restrict__ ctr, int64_t n, uint32_t k0, uint32_t k1,
                              uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const U4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    const U4 r = philox10(c, k0, k1);
    out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
  }
}

// Float64 energies V = sum_{i<j} E_ij(|CB_i - CB_j|) of nact <= G conformations of
// one protein (C-beta of conformation g read from x0 + g xstride).  Beyond the last
// knot E_ij is the row's no-contact value E_ij(inf), so V = vfar + sum over the pairs
// inside it of (E_ij - E_ij(inf)), vfar the sum of every row's no-contact value.
// The pairs inside are found as in a global proposal: bounding spheres of blocks of
// 8 residues (float32 centre and radius in sph0 + g sstride) cull the 8 x 8 tiles
// whose spheres lie farther apart than the last knot plus 0.05 A; a surviving tile
// is one wavefront step, a pair per lane, tested in float64.  Each pair term is
// rounded to a multiple of 2^-40 (error < 5e-13 per pair) and summed as an integer,
// exactly and so in any order: V does not depend on the launch shape.  acc holds G
// 64-bit integers; V_out[g] is written by thread g, visible after the last barrier.
template <int G>
__device__ void energy64(const float* __restrict__ table, int stride, int nb, double d_min, double w,
                         double vfar, int L, const double* __restrict__ x0, size_t xstride,
                         float4* __restrict__ sph0, size_t sstride, int nact, long long* acc,
                         double* V_out) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63;
  const double dfar = d_min + w * ((double)nb - 0.5), d2far = dfar * dfar;   // the last knot
  const double inv_w = 1.0 / w;
  const float rcut = (float)dfar + 0.05f;
  const int nb8 = (L + 7) >> 3, nres8 = 8 * nb8;
  if (tid < G) acc[tid] = 0;
  // spheres: the 8 residues of a block in 8 aligned lanes of one wavefront
  const float inv_nres8 = 1.0f / (float)nres8;
  for (int e0 = 0; e0 < nact * nres8; e0 += T) {
    const int e = e0 + tid, g = (int)(((float)e + 0.5f) * inv_nres8), r = e - g * nres8;
    const bool real = g < nact && r < L;
    float vx = 0.0f, vy = 0.0f, vz = 0.0f;
    if (real) {
      const double* q = atom(x0 + g * xstride, r, 3);
      vx = (float)q[0]; vy = (float)q[1]; vz = (float)q[2];
    }
    const float cnt = sum8(real ? 1.0f : 0.0f), inv = __builtin_amdgcn_rcpf(cnt > 1.0f ? cnt : 1.0f);
    const float cx = sum8(vx) * inv, cy = sum8(vy) * inv, cz = sum8(vz) * inv;
    const float rad = max8(real ? __builtin_amdgcn_sqrtf((vx - cx) * (vx - cx) + (vy - cy) * (vy - cy) +
                                                         (vz - cz) * (vz - cz))
                                : 0.0f);
    if (g < nact && (r & 7) == 0) sph0[g * sstride + (r >> 3)] = make_float4(cx, cy, cz, rad);
  }
  __syncthreads();
  // candidate tiles (chain, row block I, column block J), I <= J, one per thread
  long long part[G];
#pragma unroll
  for (int g = 0; g < G; ++g) part[g] = 0;
  const int lr = lane >> 3, lc = lane & 7, per = nb8 * nb8;
  const float inv_per = 1.0f / (float)per, inv_nb8 = 1.0f / (float)nb8;
  for (int base = 0; base < nact * per; base += T) {
    const int cand = base + tid;
    int code = 0;
    bool keep = false;
    if (cand < nact * per) {
      const int g = (int)(((float)cand + 0.5f) * inv_per), rem = cand - g * per;
      const int I = (int)(((float)rem + 0.5f) * inv_nb8), J = rem - I * nb8;
      if (I <= J) {
        const float4 u = sph0[g * sstride + I], v = sph0[g * sstride + J];
        const float dx = u.x - v.x, dy = u.y - v.y, dz = u.z - v.z, lim = rcut + u.w + v.w;
        keep = dx * dx + dy * dy + dz * dz <= lim * lim;
      }
      code = (g << 20) | (I << 10) | J;
    }
    unsigned long long m = __ballot(keep);
    while (m) {
      const int l = __builtin_ctzll(m);
      m &= m - 1;
      const int cd = __builtin_amdgcn_readlane(code, l);
      const int g = cd >> 20, i = 8 * ((cd >> 10) & 1023) + lr, j = 8 * (cd & 1023) + lc;
      if (i < j && j < L) {
        const double* pa = atom(x0 + g * xstride, i, 3);
        const double* pb = atom(x0 + g * xstride, j, 3);
        const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < d2far) {
          const float* row = table + (size_t)pair_row(i, j, L) * stride;
          // distance through the hardware reciprocal square root and two Newton steps
          const double e = spline64(row, d2 * rsqrt64(d2), nb, d_min, w, inv_w) - (double)row[nb];
          const long long q = (long long)rint(e * 1099511627776.0);   // e 2^40
#pragma unroll
          for (int gg = 0; gg < G; ++gg)
            if (gg == g) part[gg] += q;
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    long long v = part[g];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0 && g < nact && v != 0) atomicAdd(reinterpret_cast<unsigned long long*>(acc + g),
                                                 (unsigned long long)v);
  }
  __syncthreads();
  if (tid < nact) V_out[tid] = vfar + (double)acc[tid] * (1.0 / 1099511627776.0);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Sum over the P rows of the table of their no-contact value row[nb] (the energy of
// a conformation whose pairs all lie beyond the last knot), float64 Neumaier in a
// fixed order: one workgroup; thread t takes rows t, t + T, ...; the partials are
// combined in thread order by thread 0.
__global__ void far_sum_kernel(const float* __restrict__ table, int64_t P, int stride, int nb,
                               double* __restrict__ out) {
  __shared__ double part[2 * 1024];
  const int tid = threadIdx.x, T = blockDim.x;
  double s = 0.0, c = 0.0;
  for (int64_t r = tid; r < P; r += T) neumaier_add(s, c, (double)table[r * stride + nb]);
  part[2 * tid] = s;
  part[2 * tid + 1] = c;
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int t = 0; t < T; ++t) { neumaier_add(a, b, part[2 * t]); b += part[2 * t + 1]; }
    *out = a + b;
  }
}

// Conformation / energy kernel: one workgroup per conformation.
__global__ void conf_energy_kernel(ConfParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int L = P.L, tid = threadIdx.x, lane = tid & 63;
  const int b = blockIdx.x;
  double* s = reinterpret_cast<double*>(lds);   // [2L]
  double* x64 = s + 2 * L;                      // [12L]
  double* red64 = x64 + 12 * L;                 // [2 kVirtWaves]
  double* Vs = red64 + 2 * kVirtWaves;          // [1]
  float4* sph = reinterpret_cast<float4*>(Vs + 2);   // [(L + 7) / 8] (16-byte aligned)
  const double* src = P.s_in ? P.s_in + (size_t)b * 2 * L : nullptr;
  int bad = 0;   // a non-finite torsion: V(s) is undefined and returned as NaN
  for (int m = tid; m < 2 * L; m += blockDim.x) {
    s[m] = src ? src[m] : kPi;
    bad |= !isfinite(s[m]);
  }
  bad = __syncthreads_or(bad);
  if (tid < 64) nerf_chain(s, L, x64, lane);
  __syncthreads();
  if (P.atoms_out) {
    float* o = P.atoms_out + (size_t)b * L * 12;
    for (int e = tid; e < L * 12; e += blockDim.x) o[e] = (float)x64[e];
  }
  if (P.atoms64_out) {
    double* o = P.atoms64_out + (size_t)b * L * 12;
    for (int e = tid; e < L * 12; e += blockDim.x) o[e] = x64[e];
  }
  if (P.cb_out) {
    float* o = P.cb_out + (size_t)b * L * 3;
    for (int e = tid; e < L * 3; e += blockDim.x) o[e] = (float)atom(x64, e / 3, 3)[e % 3];
  }
  if (P.s_out)
    for (int m = tid; m < 2 * L; m += blockDim.x) P.s_out[(size_t)b * 2 * L + m] = s[m];
  if (P.table) {
    energy64<1>(P.table, P.stride, P.nb, P.d_min, P.bin_w, P.vfar, L, x64, 0, sph, 0, 1,
                reinterpret_cast<long long*>(red64), Vs);
    const double V = bad ? __builtin_nan("") : Vs[0];
    // keep_best: V becomes the current energy and replaces the best one only if lower
    // (every thread decides from the old best before it is overwritten)
    const bool better = !(P.v_state && P.keep_best) || V < P.v_state[2 * b + 1];
    __syncthreads();
    if (tid == 0) {
      if (!isfinite(V)) atomicOr(P.err, kErrEnergy);
      if (P.V_out) P.V_out[b] = V;
      if (P.v_state) {
        P.v_state[2 * b] = V;
        if (better) P.v_state[2 * b + 1] = V;
      }
      if (P.counters) {
        P.counters[4 * b + 0] = 0; P.counters[4 * b + 1] = 0;
        P.counters[4 * b + 2] = -1; P.counters[4 * b + 3] = 0;
      }
    }
    if (P.s_best && better)
      for (int m = tid; m < 2 * L; m += blockDim.x) P.s_best[(size_t)b * 2 * L + m] = s[m];
  }
}

// ---------------------------------------------------------------------------
// LDS layout of a sweep workgroup: per chain (stride 128 L bytes) the float64
// atoms [L][4][3], the float32 C-beta work array of global sweeps [L] and the
// torsions [2L]; then the rotation slots of the current and next proposal per
// chain, the wavefront partials, the anchor scratch, the near-pair queues, the
// bounding spheres of the rectangle's tiles and the work arrays' origins.
__host__ __device__ inline size_t chain_stride(int L) {
  const size_t b = 128 * (size_t)L;
  return b + ((64 + 256 - (b & 255)) & 255);
}

struct Lds {
  unsigned char* base;
  int L, G;
  // per-chain stride: 128 L bytes padded to 64 mod 256, so that the same residue of
  // the G chains (read together by the localized sweeps) falls in different banks
  __device__ size_t per() const { return chain_stride(L); }
  __device__ double* x64(int g) const { return reinterpret_cast<double*>(base + g * per()); }
  __device__ float4* w32(int g) const { return reinterpret_cast<float4*>(base + g * per() + 96 * (size_t)L); }
  __device__ double* s(int g) const { return reinterpret_cast<double*>(base + g * per() + 112 * (size_t)L); }
  __device__ Rot* par() const { return reinterpret_cast<Rot*>(base + G * per()); }
  __device__ double* red() const { return reinterpret_cast<double*>(par() + 2 * G); }
  __device__ double* red64(int W) const { return red() + 2 * W * G; }
  __device__ double* Vtmp(int W) const { return red64(W) + 2 * kVirtWaves * G; }
  // progress of the pipelined localized sweeps: [W] ints, then [W][G] int64 accept counts
  __device__ int* prog(int W) const { return reinterpret_cast<int*>(Vtmp(W) + G); }
  __device__ long long* nacc(int W) const {
    return reinterpret_cast<long long*>(prog(W) + ((W + 1) & ~1));
  }
  // per-wavefront queue of 64 near pairs of a global proposal (row, column, chain, d^2)
  // (offsets from base, not integer addresses, so that the compiler keeps LDS accesses)
  __device__ uint2* qbuf(int W, int wave) const {
    const size_t o = (size_t)(reinterpret_cast<unsigned char*>(nacc(W) + W * G) - base);
    return reinterpret_cast<uint2*>(base + ((o + 15) & ~(size_t)15)) + 64 * wave;
  }
  // bounding spheres (centroid, radius) of the blocks of 8 residues of chain g
  __device__ float4* sph(int W, int g) const {
    return reinterpret_cast<float4*>(qbuf(W, W)) + g * ((L + 7) >> 3);
  }
  // origin of chain g's float32 work array during a global sweep (3 doubles)
  __device__ double* orig(int W, int g) const { return reinterpret_cast<double*>(sph(W, G)) + 3 * g; }
};

size_t sweep_lds_bytes(int G, int L, int W) {
  return (size_t)G * chain_stride(L) + sizeof(Rot) * 2 * G + 16 * (size_t)W * G + 16 * (size_t)kVirtWaves * G +
         8 * (size_t)G + 4 * (size_t)((W + 1) & ~1) + 8 * (size_t)W * G + 64 + 16 +
         8 * 64 * (size_t)W + 16 * (size_t)G * ((L + 7) / 8) + 24 * (size_t)G;
}

// a localized-only launch does not use the near-pair queues, spheres and origins
size_t sweep_lds_bytes_local(int G, int L, int W) {
  return sweep_lds_bytes(G, L, W) - 8 * 64 * (size_t)W - 16 * (size_t)G * ((L + 7) / 8) - 24 * (size_t)G;
}

__device__ __forceinline__ void axis_atoms(const double* x64, int k, D3& A, D3& B) {
  const int c = k >> 1;
  if (k & 1) { A = ld3(atom(x64, c, 1)); B = ld3(atom(x64, c, 2)); }  // psi_c: CA_c -> C_c
  else { A = ld3(atom(x64, c, 0)); B = ld3(atom(x64, c, 1)); }        // phi_c: N_c -> CA_c
}

struct Batch {  // proposal randoms of 64 consecutive proposals, one per lane
  double delta, log_u, cd, sd;
};

// Proposal width of sweep t: constant, or reduced geometrically from sigma to
// sigma_end over the schedule (Sec. 2.3 and Sec. 3 reduce it from 10 to 4 degrees).
__device__ __forceinline__ double sigma_at(const SweepParams& P, int64_t t) {
  if (P.sigma_end > 0.0 && P.sigma > 0.0 && P.S > 1)
    return P.sigma * pow(P.sigma_end / P.sigma, (double)t / (double)(P.S - 1));
  return P.sigma;
}


// Window half-width of localized sweep t: window_d, then the cascade radii in turn
// (Sec. 2.2 allows several localization ranges).
__device__ __forceinline__ int half_window_at(const SweepParams& P, int64_t t) {
  if (P.n_cascade == 0) return P.half_window;
  const int r = (int)((uint32_t)t % (uint32_t)(1 + P.n_cascade));   // t < 2^32
  return r == 0 ? P.half_window : r == 1 ? P.cascade_hw[0] : r == 2 ? P.cascade_hw[1] : P.cascade_hw[2];
}

__device__ __forceinline__ Batch fill_batch(const SweepParams& P, int kb, uint32_t t,
                                            uint32_t chain, int lane) {
  const int k = kb + lane;
  Batch b{0.0, 0.0, 1.0, 0.0};
  if (k < 2 * P.L) {
    const Draw d = proposal_draw((uint32_t)k, t, chain, P.key0, P.key1, sigma_at(P, t));
    b.delta = d.delta; b.log_u = d.log_u; b.cd = d.cd; b.sd = d.sd;
  }
  return b;
}

__device__ __forceinline__ int trace_slot(const SweepParams& P, int chain) {
  int slot = -1;
#pragma unroll
  for (int m = 0; m < 4; ++m)
    if (m < P.n_trace && P.trace_chain[m] == chain) slot = m;
  return slot;
}

__device__ __forceinline__ void trace_step(const SweepParams& P, int slot, int64_t t, int k,
                                           double dE, double delta, int acc) {
  if (slot < 0) return;
  const int64_t idx = (t - P.trace_t0) * (int64_t)(2 * P.L) + k;
  if (idx < 0 || idx >= P.trace_cap) return;
  P.tr_dE[slot * P.trace_cap + idx] = dE;
  P.tr_delta[slot * P.trace_cap + idx] = delta;
  P.tr_acc[slot * P.trace_cap + idx] = (uint8_t)acc;
}

// Localized sweeps run all chains of a workgroup side by side in one wavefront:
// chain q owns the LW = 64 / G lanes [q LW, (q + 1) LW), and every chain is at the
// same proposal k of the same sweep, so the window bounds are uniform and only the
// geometry differs between the lane groups.  The wavefronts of a workgroup are
// consecutive sweeps of a block, pipelined.
//
// Pipelining: the m-th sweep of a block of consecutive localized sweeps publishes
// m * 4096 + (proposals done) in `publish`; sweep m+1 waits on that counter so that
// it runs proposal k' (residue c') only once sweep m stands at residue c'+2h+1 or
// beyond.  A localized dE depends only on the geometry of its window, and a
// rotation moves only residues downstream of its bond, so the two sweeps never
// touch the same residues and the results equal those of running them in turn.
struct Pipe {
  const int* wait_on;   // progress counter of the previous sweep, or null
  int* publish;         // this sweep's progress counter
  int m;                // index of the sweep in its block
};

// Waits until *ctr >= target and returns the value seen (bounded: on a stall the
// error word is flagged and the sweep goes on rather than hang).
__device__ __forceinline__ int wait_progress(const SweepParams& P, const int* ctr, int target,
                                             bool& stalled) {
  if (stalled) return 0x7fffffff;
  for (int spin = 0; spin < P.spin_limit; ++spin) {
    const int v = __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (v >= target) return v;
    __builtin_amdgcn_s_sleep(2);
  }
  stalled = true;
  atomicOr(P.err, kErrStall);
  return 0x7fffffff;
}

// Value of lane (q LW + kl) for the lanes of chain group q (kl uniform).
template <int LW>
__device__ __forceinline__ double group_bcast(double v, int lane, int kl) {
  if constexpr (LW == 64) {
    return readlane_d(v, kl);
  } else {
    const int src = ((lane & ~(LW - 1)) + kl) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
    return __hiloint2double(hi, lo);
  }
}

// Sum over the LW lanes of each chain group; every lane of a group gets its group's
// sum.  The addends are multiples of 2^-30 below 2^23 in magnitude, so every partial
// sum is exact and the result does not depend on LW or on the order.
template <int LW>
__device__ __forceinline__ double group_sum(double v, int lane) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppRor4>(v);
  v += dpp_d<kDppRor8>(v);   // every lane: the sum of its row of 16
  if constexpr (LW == 16) {
    return v;
  } else if constexpr (LW == 32) {
    const double a = readlane_d(v, 0) + readlane_d(v, 16), b = readlane_d(v, 32) + readlane_d(v, 48);
    return lane < 32 ? a : b;
  } else {
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
  }
}

// A pair's deviation energy rounded to a multiple of 2^-30: sums of such terms
// (|sum| < 2^23) are exact in float64 whatever the order of the additions, so every
// launch shape, batch and lane assignment gives the same value (the rounding,
// < 1e-9 per pair, is far inside the parity tolerance).
__device__ __forceinline__ double fixed30(float x) {
  return rint((double)x * 1073741824.0) * (1.0 / 1073741824.0);
}

// One localized sweep of the workgroup's chains (G of them, nact active) by one
// wavefront, with no workgroup barrier inside.
template <int G>
__device__ void local_sweep(const SweepParams& P, const Lds& S, int nact, int c0, int64_t t,
                            double beta, int h, int h_prev, int lane, int slot, int64_t& n_acc,
                            const Pipe& pipe, bool& stalled) {
  constexpr int LW = 64 / G;   // lanes per chain
  constexpr int R = G > 2 ? 3 : G;   // pair slots per lane: LW R pairs per pass (48 at G = 4)
  const int L = P.L, n = 2 * L;
  const int q = lane / LW, ll = lane - q * LW;
  const bool act = q < nact;
  double* __restrict__ x64 = S.x64(q);
  double* __restrict__ s = S.s(q);
  const uint32_t chain = (uint32_t)(P.chain_offset + c0 + q);
  const Spline32 sp{P.inv_w, P.off, P.tmax};
  // accumulated rigid transform x -> A x + b of the residues that have not yet
  // entered the window (float64, uniform over the chain's lanes)
  double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tb[3] = {0, 0, 0};
  bool moved = false;
  int entered = h < L - 1 ? h : L - 1;
  int seen = -1;   // progress of the previous sweep last read
  Batch bt{};
  for (int k = 0; k < n; ++k) {
    const int kl = k & (LW - 1);
    if (kl == 0) bt = fill_batch(P, k, (uint32_t)t, chain, ll);
    // this proposal's randoms from the lane of the chain that drew them
    const double cd = group_bcast<LW>(bt.cd, lane, kl), sd = group_bcast<LW>(bt.sd, lane, kl);
    const double log_u = group_bcast<LW>(bt.log_u, lane, kl), delta = group_bcast<LW>(bt.delta, lane, kl);
    const int c = k >> 1, p = (k & 1) ? c + 1 : c;
    const int lo = c - h > 0 ? c - h : 0, hi = c + h < L - 1 ? c + h : L - 1;
    if (pipe.wait_on) {
      // the previous sweep (half-width h_prev) must be done with every proposal whose
      // window reaches residue c + h, i.e. with all proposals up to c' = c + h + h_prev
      const int need = (pipe.m - 1) * 4096 +
                       (2 * (c + h + h_prev) + 2 < n ? 2 * (c + h + h_prev) + 2 : n);
      if (seen < need) seen = wait_progress(P, pipe.wait_on, need, stalled);
    }
    // residues entering the window take the transform accumulated so far
    while (entered < hi) {
      ++entered;
      if (moved && ll < 4) {
        double* qa = atom(x64, entered, ll);
        const double X = qa[0], Y = qa[1], Z = qa[2];
        qa[0] = A[0] * X + A[1] * Y + A[2] * Z + tb[0];
        qa[1] = A[3] * X + A[4] * Y + A[5] * Z + tb[1];
        qa[2] = A[6] * X + A[7] * Y + A[8] * Z + tb[2];
      }
      wave_sync();
    }
    const bool live = k != 0 && k != n - 1;
    const int nF = p - lo > 0 ? p - lo : 0, nM = hi - p + 1 > 0 ? hi - p + 1 : 0;
    const int npair = live ? nF * nM : 0;
    // hardware reciprocal (1 ulp): floor((x + 1/2) inv_nM) stays exact for x < 2^22
    const float inv_nM = __builtin_amdgcn_rcpf((float)(nM > 0 ? nM : 1));
    double part = 0.0;
    Rot Rk;
    // the changed pairs (lo + a, p + b), a in [0, nF), b in [0, nM), in passes of LW R:
    // pair x = a nM + b sits in slot (x mod LW R) / LW of lane x mod LW.  The stencils
    // of the current distances are fetched before the rotation is set up; only the
    // stencils stay in registers, the coordinates are read again afterwards
    for (int x0 = 0; x0 < npair || x0 == 0; x0 += LW * R) {
      // branch-free over the slots, so that all their loads are in flight together:
      // an unused slot reads atoms of the window and the zero row
      int pr[R];   // (row residue << 16) | column residue of the slot's pair
      float4 q0[R];
      float f0[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = x0 + r * LW + ll;
        // floor((x + 1/2) / nM) is exact through the float reciprocal for x < 2^22
        const int a = (int)(((float)x + 0.5f) * inv_nM);
        const bool use = x < npair;
        const int ii = use ? lo + a : lo, j = use ? p + (x - a * nM) : p;
        pr[r] = (ii << 16) | j;
        const float d2 = use ? dist2_64(ld3(atom(x64, ii, 3)), ld3(atom(x64, j, 3))) : __builtin_inff();
        const float* row = P.ydev + (size_t)pair_row(ii, j, L) * P.stride;
        q0[r] = ld_stencil(stencil_addr(row, P.zrow, d2, sp, P.d2far, f0[r]));
      }
      if (x0 == 0 && live) {
        D3 a, b;
        axis_atoms(x64, k, a, b);
        make_rot(a, b, cd, sd, Rk);
      }
      float4 q1[R];
      float f1[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int ii = pr[r] >> 16, j = pr[r] & 0xffff;
        const float d2 = x0 + r * LW + ll < npair
                             ? dist2_64(ld3(atom(x64, ii, 3)), apply_rot(Rk, ld3(atom(x64, j, 3))))
                             : __builtin_inff();
        const float* row = P.ydev + (size_t)pair_row(ii, j, L) * P.stride;
        q1[r] = ld_stencil(stencil_addr(row, P.zrow, d2, sp, P.d2far, f1[r]));
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        part += fixed30_units(catmull_rom(q1[r].x, q1[r].y, q1[r].z, q1[r].w, f1[r])) -
                fixed30_units(catmull_rom(q0[r].x, q0[r].y, q0[r].z, q0[r].w, f0[r]));
    }
    const double dE = npair > 0 ? group_sum<LW>(act ? part : 0.0, lane) * (1.0 / 1073741824.0) : 0.0;
    const int acc = (dE <= 0.0) || (log_u < -beta * dE);
    if (act && ll == 0 && !isfinite(dE)) atomicOr(P.err, kErrEnergy);
    trace_step(P, act && ll == 0 ? slot : -1, t, k, dE, delta, acc);
    if (act && acc) {
      if (ll == 0) s[k] = wrap_angle(s[k] + delta);
      ++n_acc;
      if (live) {
        // rotate the atoms of the entered residues p..entered that the torsion moves,
        // two per lane at a time (both read before either is written)
        const int nat = 4 * (entered - p + 1);
        for (int x0 = 0; x0 < nat; x0 += 2 * LW) {
          const int xa = x0 + ll, xb = xa + LW;
          const int ya = xa < nat ? xa : nat - 1, yb = xb < nat ? xb : nat - 1;
          // phi_c leaves N_c and CA_c in place
          const bool va = xa < nat && ((k & 1) || xa >= 2), vb = xb < nat && ((k & 1) || xb >= 2);
          double* qa = atom(x64, p + (ya >> 2), ya & 3);
          double* qb = atom(x64, p + (yb >> 2), yb & 3);
          const D3 ra = apply_rot(Rk, ld3(qa)), rb = apply_rot(Rk, ld3(qb));
          if (va) st3(qa, ra);
          if (vb) st3(qb, rb);
        }
        // compose the pending transform: x -> R (x - a) + a after (A, b)
        double nA[9], nb[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int qq = 0; qq < 3; ++qq)
            nA[3 * r + qq] = Rk.r[3 * r] * A[qq] + Rk.r[3 * r + 1] * A[3 + qq] + Rk.r[3 * r + 2] * A[6 + qq];
          nb[r] = Rk.r[3 * r] * (tb[0] - Rk.a[0]) + Rk.r[3 * r + 1] * (tb[1] - Rk.a[1]) +
                  Rk.r[3 * r + 2] * (tb[2] - Rk.a[2]) + Rk.a[r];
        }
#pragma unroll
        for (int qq = 0; qq < 9; ++qq) A[qq] = nA[qq];
        tb[0] = nb[0]; tb[1] = nb[1]; tb[2] = nb[2];
        moved = true;
      }
    }
    wave_sync();
    if (pipe.publish && lane == 0)
      __hip_atomic_store(pipe.publish, pipe.m * 4096 + k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Anchor: rebuild every chain's coordinates from its float64 torsions (NeRF),
// re-anchor V in float64 and update the best state and the time-to-target.
template <int G>
__device__ void anchor(const SweepParams& P, const Lds& S, int c0, int nact, int64_t t,
                       double* vbest_own, int64_t* ttt, int64_t* nanchor) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, L = P.L, W = blockDim.x >> 6;
  __syncthreads();
  if (wave < nact) nerf_chain(S.s(wave), L, S.x64(wave), lane);
  __syncthreads();
  // (the float32 work arrays hold the spheres: a global sweep no longer needs them)
  energy64<G>(P.table, P.stride, P.nb, P.d_min, P.bin_w, P.vfar, L, S.x64(0), S.per() / sizeof(double),
              S.w32(0), S.per() / sizeof(float4), nact, reinterpret_cast<long long*>(S.red64(W)),
              S.Vtmp(W));
  if (wave < nact) {
    const int g = wave, chain = c0 + g;
    const double v = S.Vtmp(W)[g];
    const bool better = v < *vbest_own;
    if (lane == 0) {
      if (!isfinite(v)) atomicOr(P.err, kErrEnergy);
      P.v[2 * chain] = v;
      if (better) P.v[2 * chain + 1] = v;
      const int slot = trace_slot(P, chain);
      if (slot >= 0) {
        const int64_t ai = (t + 1) / P.anchor_every - P.trace_anchor0;
        if (ai >= 0 && ai < P.trace_anchor_cap) P.tr_anchor[slot * P.trace_anchor_cap + ai] = v;
      }
    }
    if (better) {
      const double* sg = S.s(g);
      for (int m = lane; m < 2 * L; m += 64) P.s_best[(size_t)chain * 2 * L + m] = sg[m];
      *vbest_own = v;
    }
    if (*ttt < 0 && v <= P.target) *ttt = t + 1;
    *nanchor += 1;
  }
  __syncthreads();
}

// acc[g] += v for a lane-varying chain index g (kept in registers).
template <int G>
__device__ __forceinline__ void add_chain(double* acc, int g, double v) {
#pragma unroll
  for (int q = 0; q < G; ++q)
    if (q == g) acc[q] += v;
}

// The sweeps of one workgroup: chains group*G .. group*G + G-1 of the protein that P
// describes, over sweeps [P.t0, P.t0 + P.n_sweeps).
template <int G, int MODE>
__device__ __forceinline__ void sweep_body(const SweepParams& P, const int group) {
  extern __shared__ __align__(16) unsigned char lds[];
  // (the localized-only instance holds the wavefront index in a scalar register)
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, W = T >> 6;
  const int wave = MODE == kSweepLocal ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  const int L = P.L, n = 2 * L;
  const int c0 = group * G;
  const int nact = P.C - c0 < G ? P.C - c0 : G;
  const Lds S{lds, L, G};
  const Spline32 sp{P.inv_w, P.off, P.tmax};

  // load chain state
  for (int e = tid; e < nact * L * 12; e += T) {
    const int g = e / (12 * L), q = e - g * 12 * L;
    S.x64(g)[q] = P.atoms[(size_t)(c0 + g) * L * 12 + q];
  }
  for (int e = tid; e < nact * n; e += T) {
    const int g = e / n, m = e % n;
    S.s(g)[m] = P.s[(size_t)(c0 + g) * n + m];
  }
  // the slots of absent chains (a last workgroup with nact < G) hold zeros: their
  // lanes of the localized sweeps compute on them without any effect
  for (int e = tid; e < (G - nact) * L * 12; e += T) {
    const int g = nact + e / (12 * L);
    S.x64(g)[e - (g - nact) * 12 * L] = 0.0;
  }
  // per-chain registers of the owner wavefront
  int64_t acc_local = 0, acc_global = 0, ttt = -1, nanchor = 0;
  const bool owner = wave < nact;
  double vbest_own = owner ? P.v[2 * (c0 + wave) + 1] : 0.0;
  const int my_chain = c0 + wave;
  const int slot = owner ? trace_slot(P, my_chain) : -1;
  if (owner) {
    acc_local = P.counters[4 * my_chain + 0];
    acc_global = P.counters[4 * my_chain + 1];
    ttt = P.counters[4 * my_chain + 2];
    nanchor = P.counters[4 * my_chain + 3];
  }
  __syncthreads();

  // every wavefront runs all chains of the workgroup (LW lanes each); the W wavefronts
  // run the consecutive localized sweeps of a block in turn, pipelined
  const int nstage = W, stage = wave;
  const int lslot = (lane / (64 / G)) < nact ? trace_slot(P, c0 + lane / (64 / G)) : -1;
  int64_t acc_local_stage = 0;   // accepted localized proposals of this lane's chain
  // executed work of this wavefront's share of the global sweeps (uniform)
  unsigned int wk_tiles = 0, wk_tests = 0, wk_near = 0;
  bool stalled = false;
  const int64_t t_end = P.t0 + P.n_sweeps;
  for (int64_t t = P.t0; t < t_end;) {
    const bool global = MODE == kSweepLocal ? false : MODE == kSweepGlobal ? true : is_global(P, t);
    double T_t = P.T0;
    if (P.S > 1) T_t = P.T0 * pow(P.T1 / P.T0, (double)t / (double)(P.S - 1));
    const double beta = 1.0 / T_t;
    if (!global) {
      // block [t, tb) of localized sweeps, ended by a global sweep, an anchor sweep,
      // the end of the launch or 4096 sweeps
      int64_t tb = t;
      while (tb < t_end && tb - t < 4096 &&
             !is_global(P, tb)) {
        ++tb;
        if ((tb % P.anchor_every) == 0) break;
      }
      const int nblk = (int)(tb - t);
      for (int e = tid; e < W; e += T) S.prog(W)[e] = 0;
      __syncthreads();
      for (int m = stage; m < nblk; m += nstage) {
        const int64_t tm = t + m;
        double Tm = P.T0;
        if (P.S > 1) Tm = P.T0 * pow(P.T1 / P.T0, (double)tm / (double)(P.S - 1));
        Pipe pipe;
        pipe.m = m;
        pipe.publish = S.prog(W) + stage;
        pipe.wait_on = m > 0 ? S.prog(W) + ((m - 1) % nstage) : nullptr;
        local_sweep<G>(P, S, nact, c0, tm, 1.0 / Tm, half_window_at(P, tm),
                       tm > 0 ? half_window_at(P, tm - 1) : 0, lane, lslot, acc_local_stage, pipe,
                       stalled);
      }
      __syncthreads();
      t = tb;
      if ((t % P.anchor_every) == 0) anchor<G>(P, S, c0, nact, t - 1, &vbest_own, &ttt, &nanchor);
      continue;
    } else {
      // ---------------- global sweep, all wavefronts ----------------
      double Rp[G];
#pragma unroll
      for (int g = 0; g < G; ++g) Rp[g] = 0.0;
      double rp = 0.0;   // W = 4 or 8: chain g's carried rectangle energy in lane ls(g)
      Batch bt{};
      D3 nA{0, 0, 0}, nU{0, 0, 1};   // owner: pivot point and axis of proposal k+1
      // blocks of 8 residues for the rectangle's tiles; a tile is skipped when its
      // spheres are more than rcut apart (the last knot + 0.05 A)
      const int nb8 = (L + 7) >> 3, nres8 = 8 * nb8;
      const float rcut = __builtin_amdgcn_sqrtf(P.d2far) + 0.05f;
      int pprev = 0;   // pivot of the previous proposal (0: refresh every residue)
      if (owner) {
        // origin of the chain's float32 work array for this sweep: its middle C-beta
        if (lane < 3) S.orig(W, wave)[lane] = atom(S.x64(wave), L / 2, 3)[lane];
        bt = fill_batch(P, 0, (uint32_t)t, (uint32_t)(P.chain_offset + my_chain), lane);
        D3 a, b;
        axis_atoms(S.x64(wave), 0, a, b);
        Rot R;
        make_rot(a, b, readlane_d(bt.cd, 0), readlane_d(bt.sd, 0), R);
        R.log_u = readlane_d(bt.log_u, 0);
        if (lane == 0) S.par()[wave] = R;
      }
      __syncthreads();
      for (int k = 0; k < n; ++k) {
        const int c = k >> 1, p = (k & 1) ? c + 1 : c, M = L - p;
        const Rot* pr = S.par() + (k & 1) * G;
        // [T] for odd k, the row and column that carry the rectangle energy from pivot
        // p-1 to p (current conformation): pair x is (x, p-1) for x < p-1, else
        // (p-1, p + x - (p-1)); the G chains' stencils are loaded together (absent
        // chains read the zero row).  A thread's first pair is loaded here and evaluated
        // after [B], so that the loads overlap it.
        double tr[G];
#pragma unroll
        for (int g = 0; g < G; ++g) tr[g] = 0.0;
        float4 tq[G];
        float tf[G];
        double tsgn = 0.0;
        auto transition_load = [&](int x) {
          int i, j;
          if (x < p - 1) { i = x; j = p - 1; tsgn = -1.0; }
          else { i = p - 1; j = p + (x - (p - 1)); tsgn = 1.0; }
          const float* row = P.ydev + (size_t)pair_row(i, j, L) * P.stride;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const float d2 = g < nact ? dist2_64(ld3(atom(S.x64(g), i, 3)), ld3(atom(S.x64(g), j, 3)))
                                      : __builtin_inff();
            tq[g] = ld_stencil(stencil_addr(row, P.zrow, d2, sp, P.d2far, tf[g]));
          }
        };
        auto transition_add = [&]() {
#pragma unroll
          for (int g = 0; g < G; ++g)
            tr[g] += tsgn * fixed30(catmull_rom(tq[g].x, tq[g].y, tq[g].z, tq[g].w, tf[g]));
        };
        auto transition = [&](int x) {
          transition_load(x);
          transition_add();
        };
        const bool tfirst = (k & 1) && tid < L - 1;
        if (tfirst) transition_load(tid);
        // [B] float32 C-beta of the trial conformation relative to the chain's origin
        // for this global sweep (the fixed residues i < p as they are, the moved ones
        // rotated) and a bounding sphere (centroid, radius) of every block of 8
        // consecutive residues; the 8 residues of a block sit in 8 aligned lanes of one
        // wavefront.  Residues below the previous pivot hold their committed position
        // already (a proposal moves only residues from its pivot on), so only the blocks
        // from that of the previous pivot are refreshed.
        const int rb = 8 * (pprev >> 3), nrb = nres8 - rb;
        const float inv_nrb = 1.0f / (float)nrb;
        for (int e0 = 0; e0 < nact * nrb; e0 += T) {
          // floor((e + 1/2) / nrb) through the float reciprocal (exact for e < 2^21)
          const int e = e0 + tid, g = (int)(((float)e + 0.5f) * inv_nrb), r = rb + (e - g * nrb);
          const bool real = g < nact && r < L;
          float vx = 0.0f, vy = 0.0f, vz = 0.0f;
          if (real) {
            if (r < pprev) {
              const float4 v = S.w32(g)[r];
              vx = v.x; vy = v.y; vz = v.z;
            } else {
              const double* const o = S.orig(W, g);
              D3 x = ld3(atom(S.x64(g), r, 3));
              if (r >= p) x = apply_rot(pr[g], x);
              vx = (float)(x.x - o[0]); vy = (float)(x.y - o[1]); vz = (float)(x.z - o[2]);
              S.w32(g)[r] = make_float4(vx, vy, vz, 0.0f);
            }
          }
          // any centre will do (the radius is measured from it); the 0.05 A margin of the
          // tile test covers the 1-ulp hardware square root
          const float cnt = sum8(real ? 1.0f : 0.0f), inv = __builtin_amdgcn_rcpf(cnt > 1.0f ? cnt : 1.0f);
          const float cx = sum8(vx) * inv, cy = sum8(vy) * inv, cz = sum8(vz) * inv;
          const float rad = max8(real ? __builtin_amdgcn_sqrtf((vx - cx) * (vx - cx) + (vy - cy) * (vy - cy) +
                                                               (vz - cz) * (vz - cz))
                                      : 0.0f);
          if (g < nact && (r & 7) == 0) S.sph(W, g)[r >> 3] = make_float4(cx, cy, cz, rad);
        }
        pprev = p;
        if (tfirst) transition_add();
        if (owner && k + 1 < n) {
          D3 nB;
          axis_atoms(S.x64(wave), k + 1, nA, nB);
          nU = unit(nA, nB);
        }
        __syncthreads();
        // [C] rectangle i < p <= j (trial), and for odd k the row and column that
        // carry the rectangle energy from pivot p-1 to p (current conformation)
        double acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0.0;
        const int npairs = p * M;
        if (npairs > 0) {
          // The rectangle is cut into tiles of 8 rows (blocks I up to that of p - 1) by 8
          // columns (blocks J from that of p) of every chain.  A tile whose bounding
          // spheres lie farther apart than the last knot (plus a margin far above
          // float32 rounding) holds only pairs beyond it, which add exactly 0, and is
          // skipped whole.  Candidate tiles are dealt to the wavefronts round-robin; a
          // surviving tile is one wavefront step, a pair per lane.  Pairs inside the
          // last knot are queued in a per-wavefront LDS buffer (ballot and lane rank
          // give each its slot) and evaluated 64 at a time, one per lane.
          uint2* const qb = S.qbuf(W, wave);
          int fill = 0;   // entries in the wavefront's buffer (uniform over the wave)
          // evaluate the first n queued pairs, one per lane
          auto flush = [&](int nq) {
            wave_sync();
            if (lane < nq) {
              const uint2 e = qb[lane];
              const int qi = (int)(e.x & 1023u), qj = (int)((e.x >> 10) & 1023u), qg = (int)(e.x >> 20);
              int bin;
              float f;
              spline_pos(__builtin_amdgcn_sqrtf(__uint_as_float(e.y)), sp, bin, f);
              const float* row = P.ydev + (size_t)pair_row(qi, qj, L) * P.stride + bin;
              add_chain<G>(acc, qg, fixed30(catmull_rom(row[0], row[1], row[2], row[3], f)));
            }
            wave_sync();
          };
          const int Ip = (p - 1) >> 3, Jp = p >> 3, nJ = nb8 - Jp, per = (Ip + 1) * nJ;
          const int ncand = nact * per;
          const float inv_per = 1.0f / (float)per, inv_nJ = 1.0f / (float)nJ;
          const int lr = lane >> 3, lc = lane & 7;
          for (int base = 0; base < ncand; base += T) {
            const int cand = base + lane * W + wave;
            int code = 0;
            bool keep = false;
            if (cand < ncand) {
              // quotients through the float reciprocal, exact for operands below 2^21
              const int g = (int)(((float)cand + 0.5f) * inv_per), rem = cand - g * per;
              const int I = (int)(((float)rem + 0.5f) * inv_nJ), J = Jp + (rem - I * nJ);
              const float4 a = S.sph(W, g)[I], b = S.sph(W, g)[J];
              const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
              const float lim = rcut + a.w + b.w;
              keep = dx * dx + dy * dy + dz * dz <= lim * lim;
              code = (g << 16) | (I << 8) | J;
            }
            unsigned long long m = __ballot(keep);
            while (m) {
              const int l = __builtin_ctzll(m);
              m &= m - 1;
              ++wk_tiles;
              const int cd = __builtin_amdgcn_readlane(code, l);
              const int g = cd >> 16, i = 8 * ((cd >> 8) & 255) + lr, j = 8 * (cd & 255) + lc;
              const bool ok = i < p && j >= p && j < L;
              const float4 xi = S.w32(g)[i < L ? i : L - 1], xj = S.w32(g)[j < L ? j : L - 1];
              const float dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
              const float q = dx * dx + dy * dy + dz * dz;
              const float d2 = ok ? q : 3.0e38f;
              const bool near = d2 < P.d2far;
              wk_tests += (unsigned int)__popcll(__ballot(ok));
              const unsigned long long bal = __ballot(near);
              if (bal == 0ull) continue;
              const int cs = (int)__popcll(bal);
              wk_near += (unsigned int)cs;
              const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                  (unsigned int)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned int)bal, 0u));
              const uint2 e = make_uint2((unsigned int)i | ((unsigned int)j << 10) | ((unsigned int)g << 20),
                                         __float_as_uint(d2));
              const int room = 64 - fill;
              if (near && rank < room) qb[fill + rank] = e;
              if (cs >= room) {          // the buffer is full: evaluate it, keep the rest
                flush(64);
                if (near && rank >= room) qb[rank - room] = e;
                fill = cs - room;
              } else {
                fill += cs;
              }
            }
          }
          if (fill > 0) flush(fill);
        }
        if (k & 1)
          for (int x = tid + T; x < L - 1; x += T) transition(x);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (g < nact) {
            const double a = wave_sum_dpp(acc[g]), b = (k & 1) ? wave_sum_dpp(tr[g]) : 0.0;
            // wave-major partials: one base address per wavefront, constant offsets
            if (lane == 0) { S.red()[wave * 2 * G + 2 * g] = a; S.red()[wave * 2 * G + 2 * g + 1] = b; }
          }
        }
        __syncthreads();
        // [D] every wavefront takes the same decisions from the same partials: lane
        // l < 2 W G holds partial (wave v, chain g, kind c) and the W waves of each
        // (g, c) are summed in a fixed order
        double part = lane < 2 * W * G ? S.red()[(lane % W) * 2 * G + lane / W] : 0.0;
        // sum each aligned group of W lanes: quad sums by DPP butterflies, then the
        // quads of a group in lane order (W = 4 or 8; other W lane by lane)
        if (W == 4 || W == 8) {
          part += dpp_d<kDppXor1>(part);
          part += dpp_d<kDppXor2>(part);
        }
        unsigned int accmask = 0;
        double dE_own = 0.0;
        if (W == 4 || W == 8) {
          // the chains' decisions side by side: lane ls(g) = off + 2 W g gathers chain
          // g's new rectangle sum and transition term by DPP (the same additions, in
          // the same order up to commutation, as summing the W partials in turn) and
          // takes the decision; a ballot collects them
          const int off = W == 8 ? 4 : 0, stride = 2 * W;
          double snew = part, trn;
          if (W == 8) {
            snew += dpp_d<kDppShr4>(part);   // lane 16g+4: waves 4-7 + waves 0-3
            trn = dpp_d<kDppShl8>(snew);     // from lane 16g+12
          } else {
            trn = dpp_d<kDppShl4>(part);     // from lane 8g+4
          }
          const int gl = (lane - off) / stride;
          const bool dec = lane >= off && ((lane - off) % stride) == 0 && gl < nact;
          const double lu = dec ? pr[gl].log_u : 0.0;
          if (dec) rp += trn;
          const double dE = npairs > 0 ? snew - rp : 0.0;
          const bool a = dec && ((dE <= 0.0) || (lu < -beta * dE));
          if (a) rp = npairs > 0 ? snew : 0.0;
          const unsigned long long bal = __ballot(a);
#pragma unroll
          for (int g = 0; g < G; ++g) accmask |= (unsigned int)((bal >> (off + stride * g)) & 1ull) << g;
          if (owner) dE_own = readlane_d(dE, off + stride * wave);
        } else {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (g < nact) {
              double Snew = 0.0, Tr = 0.0;
              for (int v = 0; v < W; ++v) {
                Snew += readlane_d(part, (2 * g) * W + v);
                Tr += readlane_d(part, (2 * g + 1) * W + v);
              }
              Rp[g] += Tr;
              const double dE = npairs > 0 ? Snew - Rp[g] : 0.0;
              const int a = (dE <= 0.0) || (pr[g].log_u < -beta * dE);
              if (a) { accmask |= 1u << g; Rp[g] = npairs > 0 ? Snew : 0.0; }
              if (g == wave) dE_own = dE;
            }
          }
        }
        if (owner) {
          const int kl = k & 63;
          const double delta = readlane_d(bt.delta, kl);
          const int a = (accmask >> wave) & 1;
          if (lane == 0) {
            if (a) S.s(wave)[k] = wrap_angle(S.s(wave)[k] + delta);
            if (!isfinite(dE_own)) atomicOr(P.err, kErrEnergy);
          }
          trace_step(P, lane == 0 ? slot : -1, t, k, dE_own, delta, a);
          acc_global += a;
        }
        // [E] commit accepted moves: rotate (float64) every atom the torsion moves
        if (accmask) {
          const int per = 4 * M;
          const float inv_per = 1.0f / (float)per;
          for (int e = tid; e < nact * per; e += T) {
            const int g = (int)(((float)e + 0.5f) * inv_per);   // e / per, exact for e < 2^22
            if (!((accmask >> g) & 1)) continue;
            const int x = e - g * per, r = p + (x >> 2), at = x & 3;
            if (!(k & 1) && r == c && at < 2) continue;   // phi_c leaves N_c and CA_c in place
            double* q = atom(S.x64(g), r, at);
            st3(q, apply_rot(pr[g], ld3(q)));
          }
        }
        // owner: rotation of proposal k+1 from the post-commit pivot bond
        if (owner && k + 1 < n) {
          const int kn = k + 1;
          if ((kn & 63) == 0) bt = fill_batch(P, kn, (uint32_t)t, (uint32_t)(P.chain_offset + my_chain), lane);
          if ((accmask >> wave) & 1) {
            // the accepted rotation turned the next pivot bond rigidly: psi_c moved
            // residue c+1 (both atoms of the phi_{c+1} bond), phi_c moved C_c (the far
            // atom of the psi_c bond, whose near atom CA_c lies on the phi_c axis)
            if (k & 1) nA = apply_rot(pr[wave], nA);
            nU = rot_dir(pr[wave], nU);
          }
          const int kl = kn & 63;
          Rot R;
          make_rot_u(nA, nU, readlane_d(bt.cd, kl), readlane_d(bt.sd, kl), R);
          R.log_u = readlane_d(bt.log_u, kl);
          if (lane == 0) S.par()[(kn & 1) * G + wave] = R;
        }
        __syncthreads();
      }
    }
    if (((t + 1) % P.anchor_every) == 0) anchor<G>(P, S, c0, nact, t, &vbest_own, &ttt, &nanchor);
    ++t;
  }

  if (P.work && lane == 0) {
    atomicAdd(P.work + 0, (unsigned long long)wk_tiles);
    atomicAdd(P.work + 1, (unsigned long long)wk_tests);
    atomicAdd(P.work + 2, (unsigned long long)wk_near);
  }
  // store chain state; the localized-sweep accept counts of a chain's waves are summed
  __syncthreads();
  if ((lane & (64 / G - 1)) == 0) S.nacc(W)[wave * G + lane / (64 / G)] = acc_local_stage;
  __syncthreads();
  if (owner)
    for (int v = 0; v < W; ++v) acc_local += S.nacc(W)[v * G + wave];
  for (int e = tid; e < nact * L * 12; e += T) {
    const int g = e / (12 * L), q = e - g * 12 * L;
    P.atoms[(size_t)(c0 + g) * L * 12 + q] = S.x64(g)[q];
  }
  for (int e = tid; e < nact * n; e += T) {
    const int g = e / n, m = e % n;
    P.s[(size_t)(c0 + g) * n + m] = S.s(g)[m];
  }
  if (owner && lane == 0) {
    P.counters[4 * my_chain + 0] = acc_local;
    P.counters[4 * my_chain + 1] = acc_global;
    P.counters[4 * my_chain + 2] = ttt;
    P.counters[4 * my_chain + 3] = nanchor;
  }
}

// MODE kSweepLocal / kSweepGlobal: every sweep of [t0, t0 + n_sweeps) is localized /
// global (the caller splits a range where the kind changes); each instance holds
// only its kind of sweep, and so its own register allocation.
template <int G, int MODE>
__global__ __launch_bounds__(MODE == kSweepLocal ? 768 : 512) void sweep_kernel(SweepParams P) {
  sweep_body<G, MODE>(P, blockIdx.x);
}

// Several proteins in one launch: workgroup b runs chain group map[b].y of the
// protein described by descs[map[b].x] (the grid is ordered by decreasing work).
// MODE as for sweep_kernel (kSweepMixed: any sweeps).
template <int G, int MODE>
__global__ __launch_bounds__(MODE == kSweepLocal ? 768 : 512) void sweep_batch_kernel(
    const SweepParams* __restrict__ descs, const int2* __restrict__ map) {
  const int2 wm = map[blockIdx.x];
  sweep_body<G, MODE>(descs[wm.x], wm.y);
}

template __global__ void sweep_kernel<1, kSweepLocal>(SweepParams);
template __global__ void sweep_kernel<2, kSweepLocal>(SweepParams);
template __global__ void sweep_kernel<4, kSweepLocal>(SweepParams);
template __global__ void sweep_kernel<1, kSweepGlobal>(SweepParams);
template __global__ void sweep_kernel<2, kSweepGlobal>(SweepParams);
template __global__ void sweep_kernel<4, kSweepGlobal>(SweepParams);
template __global__ void sweep_batch_kernel<1, kSweepMixed>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<2, kSweepMixed>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<4, kSweepMixed>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<1, kSweepLocal>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<2, kSweepLocal>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<4, kSweepLocal>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<1, kSweepGlobal>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<2, kSweepGlobal>(const SweepParams*, const int2*);
template __global__ void sweep_batch_kernel<4, kSweepGlobal>(const SweepParams*, const int2*);

}  // namespace amh
