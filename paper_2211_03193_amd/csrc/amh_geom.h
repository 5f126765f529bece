// amh_geom.h -- float64 chain geometry shared by the sweep, energy and gradient
// kernels: the atom layout [L][4][3] (N, CA, C, C-beta) and the NeRF build of a
// chain from its torsions.
#pragma once
#include <hip/hip_runtime.h>

#include "amh_device.h"

namespace amh {

constexpr double kDeg = kPi / 180.0;

__device__ __forceinline__ double* atom(double* x64, int r, int a) { return x64 + (4 * r + a) * 3; }
__device__ __forceinline__ const double* atom(const double* x64, int r, int a) {
  return x64 + (4 * r + a) * 3;
}

// ---------------------------------------------------------------------------
// Serial float64 NeRF of one chain, executed in lockstep by a whole wavefront (all
// lanes hold the same values; the torsion cosines and sines are computed 64 at a
// time, one per lane).  Lane 0 writes the float64 atoms x64 [L][4][3].
static __device__ void nerf_chain(const double* __restrict__ s, int L, double* __restrict__ x64, int lane) {
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
  {
    const double a = lane < n ? s[lane] : 0.0;
    sincos(a, &sn, &cs);
  }
  for (int c = 0; c < L; ++c) {
    if (c > 0) {
      const int m0 = 2 * c - 1, m1 = 2 * c;   // psi_{c-1}, phi_c
      const double cpsi = readlane_d(cs, m0 & 63), spsi = readlane_d(sn, m0 & 63);
      if ((m1 & 63) == 0) {
        const int m = m1 + lane;
        const double a = m < n ? s[m] : 0.0;
        sincos(a, &sn, &cs);
      }
      const double cphi = readlane_d(cs, m1 & 63), sphi = readlane_d(sn, m1 & 63);
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
      double* o = atom(x64, c, 0);
      o[0] = N[0]; o[1] = N[1]; o[2] = N[2];
      o[3] = CA[0]; o[4] = CA[1]; o[5] = CA[2];
      o[6] = C[0]; o[7] = C[1]; o[8] = C[2];
      o[9] = B[0]; o[10] = B[1]; o[11] = B[2];
    }
  }
}

}  // namespace amh
