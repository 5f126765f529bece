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
//   * global proposals use every wavefront of the workgroup; dE of pivot p is
//     S_new(p) - R(p), where R(p), the energy of the pair rectangle i < p <= j of
//     the current conformation, is carried from proposal to proposal (the new
//     rectangle sum on accept, an O(L) row/column update when p advances), so
//     each global proposal evaluates one spline per changed pair instead of two;
//   * the proposal randoms come from Philox4x32-10 at counter (k, t, chain, 0),
//     the same stream the oracle replays, drawn 64 proposals at a time, one per lane;
//   * after every anchor sweep the coordinates are rebuilt from the float64
//     torsions by NeRF and V is re-anchored in float64 with Neumaier summation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "amh_device.h"
#include "amh_kernels.h"

namespace amh {

constexpr double kDeg = kPi / 180.0;

// ---------------------------------------------------------------------------
// Table ingest: repack [P][nb] rows into padded rows [y1, y0..y_{nb-1}, y_{nb-2}, 0...]
// and flag non-finite entries.
__global__ void ingest_kernel(const float* __restrict__ y, int64_t P, int nb, int stride,
                              float* __restrict__ out, unsigned int* err) {
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
  }
  if (bad) atomicOr(err, kErrTable);
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

// ---------------------------------------------------------------------------
// Serial float64 NeRF of one chain, executed in lockstep by a whole wavefront
// (all lanes hold the same values; the torsion cosines and sines are computed
// 64 at a time, one per lane).  Writes float32 N/CA/C and C-beta and, if cb64 is
// given, float64 C-beta.
__device__ void nerf_chain(const double* __restrict__ s, int L, float4* __restrict__ bb,
                           float4* __restrict__ cb, double* __restrict__ cb64, int lane) {
  const double ct_cacn = cos(kAngCACN * kDeg), st_cacn = sin(kAngCACN * kDeg);
  const double ct_cnca = cos(kAngCNCA * kDeg), st_cnca = sin(kAngCNCA * kDeg);
  const double ct_ncac = cos(kAngNCAC * kDeg), st_ncac = sin(kAngNCAC * kDeg);
  const double ct_ncacb = cos(kAngNCACB * kDeg), st_ncacb = sin(kAngNCACB * kDeg);
  const double co = cos(kTorOmega * kDeg), so = sin(kTorOmega * kDeg);
  const double ccb = cos(kTorCB * kDeg), scb = sin(kTorCB * kDeg);
  double N[3] = {0.0, 0.0, 0.0};
  double CA[3] = {kBondNCA, 0.0, 0.0};
  double C[3] = {kBondNCA - kBondCAC * ct_ncac, kBondCAC * st_ncac, 0.0};
  const int n = 2 * L;
  double cs = 1.0, sn = 0.0;
  for (int c = 0; c < L; ++c) {
    if (c > 0) {
      // torsions 2c-1 (psi_{c-1}) and 2c (phi_c)
      const int m0 = 2 * c - 1;
      double cpsi, spsi, cphi, sphi;
      {
        const int b = m0 & ~63;
        if (m0 == b || c == 1) {
          const int m = b + lane;
          const double a = m < n ? s[m] : 0.0;
          sincos(a, &sn, &cs);
        }
        cpsi = readlane_d(cs, m0 - b);
        spsi = readlane_d(sn, m0 - b);
        const int m1 = m0 + 1;
        if ((m1 & 63) == 0) {
          const int m = m1 + lane;
          const double a = m < n ? s[m] : 0.0;
          sincos(a, &sn, &cs);
        }
        cphi = readlane_d(cs, m1 & 63);
        sphi = readlane_d(sn, m1 & 63);
      }
      double Nn[3], CAn[3], Cn[3];
      nerf_place(N, CA, C, kBondCN, ct_cacn, st_cacn, cpsi, spsi, Nn);
      nerf_place(CA, C, Nn, kBondNCA, ct_cnca, st_cnca, co, so, CAn);
      nerf_place(C, Nn, CAn, kBondCAC, ct_ncac, st_ncac, cphi, sphi, Cn);
#pragma unroll
      for (int a = 0; a < 3; ++a) { N[a] = Nn[a]; CA[a] = CAn[a]; C[a] = Cn[a]; }
    }
    double B[3];
    nerf_place(C, N, CA, kBondCACB, ct_ncacb, st_ncacb, ccb, scb, B);
    if (lane == 0) {
      bb[3 * c + 0] = make_float4((float)N[0], (float)N[1], (float)N[2], 0.0f);
      bb[3 * c + 1] = make_float4((float)CA[0], (float)CA[1], (float)CA[2], 0.0f);
      bb[3 * c + 2] = make_float4((float)C[0], (float)C[1], (float)C[2], 0.0f);
      cb[c] = make_float4((float)B[0], (float)B[1], (float)B[2], 0.0f);
      if (cb64) { cb64[3 * c] = B[0]; cb64[3 * c + 1] = B[1]; cb64[3 * c + 2] = B[2]; }
    }
  }
}

// Float64 energy sum over all pairs i < j of `nchain` conformations held as
// float64 C-beta in LDS (cb64[g] = base + g * 3L).  Each thread accumulates a
// Neumaier pair (sum, compensation) per chain; the wavefronts' partials are
// combined in a fixed order by wave 0.  red64 needs 2 * nwaves * nchain doubles.
template <int G>
__device__ void energy64(const float* __restrict__ table, int stride, int nb, double d_min,
                         double w, int L, const double* __restrict__ cb64, int nchain,
                         double* red64, double* V_out /*[G] in LDS*/) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wave = tid >> 6, W = T >> 6;
  double sum[G], cmp[G];
#pragma unroll
  for (int g = 0; g < G; ++g) { sum[g] = 0.0; cmp[g] = 0.0; }
  // walk the strict upper triangle row by row with stride T
  int i = 0, j = 1 + tid;
  while (i < L - 1) {
    if (j < L) {
      const float* row = table + (size_t)pair_row(i, j, L) * stride;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g < nchain) {
          const double* p = cb64 + (size_t)g * 3 * L;
          const double dx = p[3 * j] - p[3 * i], dy = p[3 * j + 1] - p[3 * i + 1],
                       dz = p[3 * j + 2] - p[3 * i + 2];
          neumaier_add(sum[g], cmp[g], spline64(row, sqrt(dx * dx + dy * dy + dz * dz), nb, d_min, w));
        }
      }
      j += T;
    }
    while (j >= L && i < L - 1) { j = j - L + i + 2; ++i; }
  }
  // combine: within a wave (fixed butterfly order), then across waves in wave order
#pragma unroll
  for (int g = 0; g < G; ++g) {
    double s = sum[g], c = cmp[g];
    for (int o = 32; o > 0; o >>= 1) {
      const double so = __shfl_down(s, o, 64), co = __shfl_down(c, o, 64);
      if (lane < o) { neumaier_add(s, c, so); c += co; }
    }
    if (lane == 0) { red64[2 * (wave * G + g)] = s; red64[2 * (wave * G + g) + 1] = c; }
  }
  __syncthreads();
  if (tid < G && tid < nchain) {
    double s = 0.0, c = 0.0;
    for (int v = 0; v < W; ++v) {
      neumaier_add(s, c, red64[2 * (v * G + tid)]);
      c += red64[2 * (v * G + tid) + 1];
    }
    V_out[tid] = s + c;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Conformation / energy kernel: one workgroup per conformation.
__global__ void conf_energy_kernel(ConfParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int L = P.L, tid = threadIdx.x, lane = tid & 63;
  const int b = blockIdx.x;
  double* s = reinterpret_cast<double*>(lds);                 // [2L]
  double* cb64 = s + 2 * L;                                   // [3L]
  double* red64 = cb64 + 3 * L;                               // [2 * W]
  double* Vs = red64 + 2 * (blockDim.x >> 6);                 // [1]
  float4* bb = reinterpret_cast<float4*>((reinterpret_cast<uintptr_t>(Vs + 2) + 15) & ~uintptr_t(15));  // [3L]
  float4* cb = bb + 3 * L;                                    // [L]
  const double* src = P.s_in ? P.s_in + (size_t)b * 2 * L : nullptr;
  for (int m = tid; m < 2 * L; m += blockDim.x) s[m] = src ? src[m] : kPi;
  __syncthreads();
  if (tid < 64) nerf_chain(s, L, bb, cb, cb64, lane);
  __syncthreads();
  if (P.atoms_out) {
    float* o = P.atoms_out + (size_t)b * L * 12;
    for (int e = tid; e < L * 12; e += blockDim.x) {
      const int r = e / 12, a = (e % 12) / 3, x = e % 3;
      const float4 v = a < 3 ? bb[3 * r + a] : cb[r];
      o[e] = x == 0 ? v.x : (x == 1 ? v.y : v.z);
    }
  }
  if (P.atoms4_out) {
    float4* o = P.atoms4_out + (size_t)b * L * 4;
    for (int e = tid; e < L * 4; e += blockDim.x) {
      const int r = e >> 2, a = e & 3;
      o[e] = a < 3 ? bb[3 * r + a] : cb[r];
    }
  }
  if (P.cb_out) {
    float* o = P.cb_out + (size_t)b * L * 3;
    for (int e = tid; e < L * 3; e += blockDim.x) {
      const float4 v = cb[e / 3];
      const int x = e % 3;
      o[e] = x == 0 ? v.x : (x == 1 ? v.y : v.z);
    }
  }
  if (P.s_out)
    for (int m = tid; m < 2 * L; m += blockDim.x) P.s_out[(size_t)b * 2 * L + m] = s[m];
  if (P.table) {
    energy64<1>(P.table, P.stride, P.nb, P.d_min, P.bin_w, L, cb64, 1, red64, Vs);
    if (tid == 0) {
      const double V = Vs[0];
      if (!isfinite(V)) atomicOr(P.err, kErrEnergy);
      if (P.V_out) P.V_out[b] = V;
      if (P.v_state) { P.v_state[2 * b] = V; P.v_state[2 * b + 1] = V; }
      if (P.counters) {
        P.counters[4 * b + 0] = 0; P.counters[4 * b + 1] = 0;
        P.counters[4 * b + 2] = -1; P.counters[4 * b + 3] = 0;
      }
    }
    if (P.s_best)
      for (int m = tid; m < 2 * L; m += blockDim.x) P.s_best[(size_t)b * 2 * L + m] = s[m];
  }
}

// ---------------------------------------------------------------------------
// The sweep kernel.
// LDS layout of a sweep workgroup: per chain (stride `per` bytes) the current
// C-beta [L], the trial C-beta [L] (which also holds 3L float64 C-beta at anchors),
// N/CA/C [3L] and the torsions [2L]; then the shared rotation slots and partials.
__host__ __device__ inline int off_bb(int L) { return 16 * L + ((24 * L + 15) & ~15); }
__host__ __device__ inline int lds_per_chain(int L) { return off_bb(L) + 64 * L; }

struct Lds {
  unsigned char* base;
  int L, per, G;
  unsigned char* tail;
  __device__ float4* cb(int g) const { return reinterpret_cast<float4*>(base + (size_t)g * per); }
  __device__ float4* cbt(int g) const { return reinterpret_cast<float4*>(base + (size_t)g * per + 16 * L); }
  __device__ double* cb64(int g) const { return reinterpret_cast<double*>(cbt(g)); }
  __device__ float4* bb(int g) const { return reinterpret_cast<float4*>(base + (size_t)g * per + off_bb(L)); }
  __device__ double* s(int g) const { return reinterpret_cast<double*>(base + (size_t)g * per + off_bb(L) + 48 * L); }
  __device__ Rot* par() const { return reinterpret_cast<Rot*>(tail); }
  __device__ double* red() const { return reinterpret_cast<double*>(tail + sizeof(Rot) * 2 * G); }
  __device__ double* red64(int W) const { return red() + 2 * W * G; }
  __device__ double* Vtmp(int W) const { return red64(W) + 2 * W * G; }
};

__device__ __forceinline__ Lds carve(unsigned char* base, int L, int G) {
  Lds d;
  d.base = base;
  d.L = L;
  d.G = G;
  d.per = lds_per_chain(L);
  d.tail = base + (size_t)G * d.per;
  return d;
}

size_t sweep_lds_bytes(int G, int L, int W) {
  return (size_t)G * lds_per_chain(L) + sizeof(Rot) * 2 * G + 16 * (size_t)W * G * 2 +
         8 * (size_t)G + 64;
}

// Rotation of the proposal k of one chain (the owner wavefront computes it from
// the pivot bond of residue k/2 and the drawn increment).
__device__ __forceinline__ void axis_atoms(const float4* bb, int k, float4& A, float4& B) {
  const int c = k >> 1;
  if (k & 1) { A = bb[3 * c + 1]; B = bb[3 * c + 2]; }   // psi_c: CA_c -> C_c
  else { A = bb[3 * c + 0]; B = bb[3 * c + 1]; }         // phi_c: N_c -> CA_c
}

struct Batch {  // proposal randoms of 64 consecutive proposals, one per lane
  double delta, log_u;
  float cd, sd;
};

__device__ __forceinline__ Batch fill_batch(const SweepParams& P, int kb, uint32_t t,
                                            uint32_t chain, int lane) {
  const int k = kb + lane;
  Batch b;
  if (k < 2 * P.L) {
    const Draw d = proposal_draw((uint32_t)k, t, chain, P.key0, P.key1, P.sigma);
    b.delta = d.delta; b.log_u = d.log_u; b.cd = d.cd; b.sd = d.sd;
  } else {
    b.delta = 0.0; b.log_u = 0.0; b.cd = 1.0f; b.sd = 0.0f;
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

// Localized sweep of chain g by its owner wavefront (no workgroup barrier inside).
__device__ void local_sweep(const SweepParams& P, const Lds& S, int g, int chain, int64_t t,
                            double beta, int lane, int slot, int64_t& n_acc) {
  const int L = P.L, n = 2 * L, h = P.half_window;
  float4* __restrict__ cb = S.cb(g);
  float4* __restrict__ bb = S.bb(g);
  double* __restrict__ s = S.s(g);
  const Spline32 sp{P.inv_w, P.off, P.tmax};
  // accumulated rigid transform x -> A x + b of the residues that have not yet
  // entered the window (float64, uniform over the wave)
  double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tb[3] = {0, 0, 0};
  bool moved = false;
  int entered = h < L - 1 ? h : L - 1;
  Batch bt{};
  for (int k = 0; k < n; ++k) {
    if ((k & 63) == 0) bt = fill_batch(P, k, (uint32_t)t, (uint32_t)(P.chain_offset + chain), lane);
    const int c = k >> 1, p = (k & 1) ? c + 1 : c;
    const int lo = c - h > 0 ? c - h : 0, hi = c + h < L - 1 ? c + h : L - 1;
    // residues entering the window take the transform accumulated so far
    while (entered < hi) {
      ++entered;
      if (moved && lane < 4) {
        const float4 x = lane < 3 ? bb[3 * entered + lane] : cb[entered];
        const double X = x.x, Y = x.y, Z = x.z;
        const float4 o = make_float4((float)(A[0] * X + A[1] * Y + A[2] * Z + tb[0]),
                                     (float)(A[3] * X + A[4] * Y + A[5] * Z + tb[1]),
                                     (float)(A[6] * X + A[7] * Y + A[8] * Z + tb[2]), 0.0f);
        if (lane < 3) bb[3 * entered + lane] = o; else cb[entered] = o;
      }
      wave_sync();
    }
    const int kl = k & 63;
    const double delta = readlane_d(bt.delta, kl), log_u = readlane_d(bt.log_u, kl);
    const bool live = k != 0 && k != n - 1;
    const int nF = p - lo > 0 ? p - lo : 0, nM = hi - p + 1 > 0 ? hi - p + 1 : 0;
    const int npair = nF * nM;
    double dE = 0.0;
    Rot R;
    if (live) {
      float4 a, b;
      axis_atoms(bb, k, a, b);
      make_rot(a.x, a.y, a.z, b.x, b.y, b.z, readlane_f(bt.cd, kl), readlane_f(bt.sd, kl), R);
      if (npair > 0) {
        double part = 0.0;
        for (int x = lane; x < npair; x += 64) {
          const int ii = lo + x / nM, j = p + x % nM;
          const float4 xi = cb[ii], xj = cb[j];
          const float4 xt = apply_rot(R, xj);
          const float* row = P.table + (size_t)pair_row(ii, j, L) * P.stride;
          const float dx0 = xj.x - xi.x, dy0 = xj.y - xi.y, dz0 = xj.z - xi.z;
          const float dx1 = xt.x - xi.x, dy1 = xt.y - xi.y, dz1 = xt.z - xi.z;
          const float e0 = spline32(row, sqrtf(dx0 * dx0 + dy0 * dy0 + dz0 * dz0), sp);
          const float e1 = spline32(row, sqrtf(dx1 * dx1 + dy1 * dy1 + dz1 * dz1), sp);
          part += (double)e1 - (double)e0;
        }
        dE = wave_sum(part);
      }
    }
    const int acc = (dE <= 0.0) || (log_u < -beta * dE);
    if (lane == 0) {
      if (!isfinite(dE)) atomicOr(P.err, kErrEnergy);
    }
    trace_step(P, lane == 0 ? slot : -1, t, k, dE, delta, acc);
    if (acc) {
      if (lane == 0) s[k] = wrap_angle(s[k] + delta);
      ++n_acc;
      if (live) {
        // rotate the atoms of the entered residues p..entered that the torsion moves
        const int nres = entered - p + 1;
        for (int x = lane; x < 4 * nres; x += 64) {
          const int r = p + (x >> 2), at = x & 3;
          if (!(k & 1) && r == c && at < 2) continue;   // phi_c leaves N_c and CA_c in place
          if (at < 3) bb[3 * r + at] = apply_rot(R, bb[3 * r + at]);
          else cb[r] = apply_rot(R, cb[r]);
        }
        // compose the pending transform: x -> R (x - a) + a after (A, b)
        double nA[9], nb[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int q = 0; q < 3; ++q)
            nA[3 * r + q] = (double)R.r[3 * r] * A[q] + (double)R.r[3 * r + 1] * A[3 + q] +
                            (double)R.r[3 * r + 2] * A[6 + q];
          nb[r] = (double)R.r[3 * r] * (tb[0] - R.a[0]) + (double)R.r[3 * r + 1] * (tb[1] - R.a[1]) +
                  (double)R.r[3 * r + 2] * (tb[2] - R.a[2]) + (double)R.a[r];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) A[q] = nA[q];
        tb[0] = nb[0]; tb[1] = nb[1]; tb[2] = nb[2];
        moved = true;
      }
    }
    wave_sync();
  }
}

template <int G>
__device__ void anchor(const SweepParams& P, const Lds& S, int c0, int nact, int64_t t,
                       double* vbest_own, int64_t* ttt, int64_t* nanchor) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, L = P.L, W = blockDim.x >> 6;
  __syncthreads();
  if (wave < nact) nerf_chain(S.s(wave), L, S.bb(wave), S.cb(wave), S.cb64(wave), lane);
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (g < nact)
      energy64<1>(P.table, P.stride, P.nb, P.d_min, P.bin_w, L, S.cb64(g), 1, S.red64(W),
                  S.Vtmp(W) + g);
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

template <int G>
__global__ __launch_bounds__(512) void sweep_kernel(SweepParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int tid = threadIdx.x, T = blockDim.x, wave = tid >> 6, lane = tid & 63, W = T >> 6;
  const int L = P.L, n = 2 * L;
  const int c0 = blockIdx.x * G;
  const int nact = P.C - c0 < G ? P.C - c0 : G;
  const Lds S = carve(lds, L, G);
  const Spline32 sp{P.inv_w, P.off, P.tmax};

  // load chain state
  for (int e = tid; e < nact * L * 4; e += T) {
    const int g = e / (4 * L), r = (e >> 2) % L, a = e & 3;
    const float4 v = P.atoms[((size_t)(c0 + g) * L + r) * 4 + a];
    if (a < 3) S.bb(g)[3 * r + a] = v; else S.cb(g)[r] = v;
  }
  for (int e = tid; e < nact * n; e += T) {
    const int g = e / n, m = e % n;
    S.s(g)[m] = P.s[(size_t)(c0 + g) * n + m];
  }
  // per-chain registers of the owner wavefront
  int64_t acc_local = 0, acc_global = 0, ttt = -1, nanchor = 0;
  const bool owner = wave < nact;
  double vbest_own = owner ? P.v[2 * (c0 + wave) + 1] : 0.0;
  const int my_chain = c0 + wave;
  const int slot = owner ? trace_slot(P, my_chain) : -1;
  if (owner) {
    ttt = P.counters[4 * my_chain + 2];
    acc_local = P.counters[4 * my_chain + 0];
    acc_global = P.counters[4 * my_chain + 1];
    nanchor = P.counters[4 * my_chain + 3];
  }
  __syncthreads();

  for (int64_t t = P.t0; t < P.t0 + P.n_sweeps; ++t) {
    const bool global = P.global_every > 0 && ((t + 1) % P.global_every) == 0;
    double T_t = P.T0;
    if (P.S > 1) T_t = P.T0 * pow(P.T1 / P.T0, (double)t / (double)(P.S - 1));
    const double beta = 1.0 / T_t;
    if (!global) {
      if (owner) local_sweep(P, S, wave, my_chain, t, beta, lane, slot, acc_local);
      __syncthreads();
    } else {
      // ---------------- global sweep, all wavefronts ----------------
      double Rp[G];
#pragma unroll
      for (int g = 0; g < G; ++g) Rp[g] = 0.0;
      Batch bt{};
      float4 nA = make_float4(0, 0, 0, 0), nB = nA;   // owner: raw axis atoms of k+1
      if (owner) {
        bt = fill_batch(P, 0, (uint32_t)t, (uint32_t)(P.chain_offset + my_chain), lane);
        float4 a, b;
        axis_atoms(S.bb(wave), 0, a, b);
        Rot R;
        make_rot(a.x, a.y, a.z, b.x, b.y, b.z, readlane_f(bt.cd, 0), readlane_f(bt.sd, 0), R);
        R.log_u = readlane_d(bt.log_u, 0);
        if (lane == 0) S.par()[wave] = R;
      }
      __syncthreads();
      for (int k = 0; k < n; ++k) {
        const int c = k >> 1, p = (k & 1) ? c + 1 : c, M = L - p;
        const Rot* pr = S.par() + (k & 1) * G;
        // [B] trial positions of the moved C-beta
        for (int e = tid; e < nact * M; e += T) {
          const int g = e / M, j = p + (e - g * M);
          S.cbt(g)[j] = apply_rot(pr[g], S.cb(g)[j]);
        }
        if (owner && k + 1 < n) axis_atoms(S.bb(wave), k + 1, nA, nB);
        __syncthreads();
        // [C] rectangle i < p <= j with the trial positions, and (odd k) the row and
        // column that move the rectangle from pivot p-1 to p, with the current ones
        double acc[G], tr[G];
#pragma unroll
        for (int g = 0; g < G; ++g) { acc[g] = 0.0; tr[g] = 0.0; }
        const int npairs = p * M;
        if (npairs > 0) {
          int i = tid / M, jj = tid - (tid / M) * M;
          const int di = T / M, dj = T - (T / M) * M;
          while (i < p) {
            const int j = p + jj;
            const float* row = P.table + (size_t)pair_row(i, j, L) * P.stride;
#pragma unroll
            for (int g = 0; g < G; ++g) {
              if (g < nact) {
                const float4 xi = S.cb(g)[i], xj = S.cbt(g)[j];
                const float dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
                acc[g] += (double)spline32(row, sqrtf(dx * dx + dy * dy + dz * dz), sp);
              }
            }
            jj += dj; i += di;
            if (jj >= M) { jj -= M; ++i; }
          }
        }
        if (k & 1) {
          for (int x = tid; x < L - 1; x += T) {
            int i, j;
            double sgn;
            if (x < p - 1) { i = x; j = p - 1; sgn = -1.0; }
            else { i = p - 1; j = p + (x - (p - 1)); sgn = 1.0; }
            const float* row = P.table + (size_t)pair_row(i, j, L) * P.stride;
#pragma unroll
            for (int g = 0; g < G; ++g) {
              if (g < nact) {
                const float4 xi = S.cb(g)[i], xj = S.cb(g)[j];
                const float dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
                tr[g] += sgn * (double)spline32(row, sqrtf(dx * dx + dy * dy + dz * dz), sp);
              }
            }
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (g < nact) {
            const double a = wave_sum(acc[g]), b = wave_sum(tr[g]);
            if (lane == 0) { S.red()[2 * (wave * G + g)] = a; S.red()[2 * (wave * G + g) + 1] = b; }
          }
        }
        __syncthreads();
        // [D] every wavefront takes the same decisions from the same partials
        unsigned int accmask = 0;
        double dE_own = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (g < nact) {
            double Snew = 0.0, Tr = 0.0;
            for (int v = 0; v < W; ++v) { Snew += S.red()[2 * (v * G + g)]; Tr += S.red()[2 * (v * G + g) + 1]; }
            Rp[g] += Tr;
            const double dE = npairs > 0 ? Snew - Rp[g] : 0.0;
            const int a = (dE <= 0.0) || (pr[g].log_u < -beta * dE);
            if (a) { accmask |= 1u << g; Rp[g] = npairs > 0 ? Snew : 0.0; }
            if (g == wave) dE_own = dE;
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
        // [E] commit accepted moves
        if (accmask) {
          const int per = 4 * M;
          for (int e = tid; e < nact * per; e += T) {
            const int g = e / per;
            if (!((accmask >> g) & 1)) continue;
            const int x = e - g * per, r = p + (x >> 2), at = x & 3;
            if (at == 3) { S.cb(g)[r] = S.cbt(g)[r]; continue; }
            if (!(k & 1) && r == c && at < 2) continue;   // phi_c leaves N_c and CA_c in place
            S.bb(g)[3 * r + at] = apply_rot(pr[g], S.bb(g)[3 * r + at]);
          }
        }
        // owner: rotation of proposal k+1 from the post-commit pivot bond
        if (owner && k + 1 < n) {
          const int kn = k + 1;
          if ((kn & 63) == 0) bt = fill_batch(P, kn, (uint32_t)t, (uint32_t)(P.chain_offset + my_chain), lane);
          if ((accmask >> wave) & 1) {
            if (k & 1) { nA = apply_rot(pr[wave], nA); nB = apply_rot(pr[wave], nB); }  // psi_c moved residue c+1
            else nB = apply_rot(pr[wave], nB);                                         // phi_c moved C_c
          }
          const int kl = kn & 63;
          Rot R;
          make_rot(nA.x, nA.y, nA.z, nB.x, nB.y, nB.z, readlane_f(bt.cd, kl), readlane_f(bt.sd, kl), R);
          R.log_u = readlane_d(bt.log_u, kl);
          if (lane == 0) S.par()[(kn & 1) * G + wave] = R;
        }
        __syncthreads();
      }
    }
    if (((t + 1) % P.anchor_every) == 0) anchor<G>(P, S, c0, nact, t, &vbest_own, &ttt, &nanchor);
  }

  // store chain state
  __syncthreads();
  for (int e = tid; e < nact * L * 4; e += T) {
    const int g = e / (4 * L), r = (e >> 2) % L, a = e & 3;
    P.atoms[((size_t)(c0 + g) * L + r) * 4 + a] = a < 3 ? S.bb(g)[3 * r + a] : S.cb(g)[r];
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

template __global__ void sweep_kernel<1>(SweepParams);
template __global__ void sweep_kernel<2>(SweepParams);
template __global__ void sweep_kernel<4>(SweepParams);

}  // namespace amh
