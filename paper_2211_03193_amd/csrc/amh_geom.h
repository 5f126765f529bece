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
// Float64 NeRF of one chain by a whole wavefront, in parallel over the atoms
// (Parsons et al. 2005 placement; the parallel form of AlQuraishi's pNeRF).  Backbone
// atom a_k (k >= 3: N, CA, C of residue k/3) is placed from a_{k-3}, a_{k-2}, a_{k-1}
// in the frame (e1 = unit(a_{k-1} - a_{k-2}), n = unit((a_{k-2} - a_{k-3}) x e1),
// m = n x e1) at a_{k-1}: a_k = a_{k-1} + F (l (-cos t, sin t cos x, sin t sin x)),
// F = [e1 m n], with bond l, angle t and torsion x of atom k.  The frame of atom k+1
// is then F R_k with
//   R_k = [[-cos t, -sin t, 0], [sin t cos x, -cos t cos x, -sin x],
//          [sin t sin x, -cos t sin x, cos x]],
// which depends only on (t, x), so every frame is a prefix product of the rigid
// transforms (R_k, l R_k e_1) (composition (R, u) o (R', u') = (R R', u + R u')).  The
// wavefront takes the transforms 64 at a time (one per lane), scans them across the
// lanes (Hillis-Steele, six steps) and applies the frame carried from the previous
// 64; C-beta then follows per residue from its N, CA, C.  The rounding differs from
// a serial build only at the last bits (about 1e-13 of the chain's extent).
static __device__ void nerf_chain(const double* __restrict__ s, int L, double* __restrict__ x64, int lane) {
  const double ct_cacn = cos(kAngCACN * kDeg), st_cacn = sin(kAngCACN * kDeg);
  const double ct_cnca = cos(kAngCNCA * kDeg), st_cnca = sin(kAngCNCA * kDeg);
  const double ct_ncac = cos(kAngNCAC * kDeg), st_ncac = sin(kAngNCAC * kDeg);
  const double ct_ncacb = cos(kAngNCACB * kDeg), st_ncacb = sin(kAngNCACB * kDeg);
  const double co = cos(kTorOmega * kDeg), so = sin(kTorOmega * kDeg);
  const double ccb = cos(kTorCB * kDeg), scb = sin(kTorCB * kDeg);
  // residue 0: N at the origin, CA on +x, C in the xy-plane
  const double N0[3] = {0.0, 0.0, 0.0};
  const double CA0[3] = {kBondNCA, 0.0, 0.0};
  const double C0[3] = {kBondNCA - kBondCAC * ct_ncac, kBondCAC * st_ncac, 0.0};
  if (lane < 9) atom(x64, 0, lane / 3)[lane % 3] = lane < 3 ? N0[lane] : lane < 6 ? CA0[lane - 3] : C0[lane - 6];
  // frame of atom 3 (N_1): from N_0, CA_0, C_0, origin C_0 (uniform over the lanes)
  double F[9], o[3];
  {
    double bx = C0[0] - CA0[0], by = C0[1] - CA0[1], bz = C0[2] - CA0[2];
    const double ib = 1.0 / sqrt(bx * bx + by * by + bz * bz);
    bx *= ib; by *= ib; bz *= ib;
    const double ax = CA0[0] - N0[0], ay = CA0[1] - N0[1], az = CA0[2] - N0[2];
    double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const double in = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
    nx *= in; ny *= in; nz *= in;
    const double mx = ny * bz - nz * by, my = nz * bx - nx * bz, mz = nx * by - ny * bx;
    F[0] = bx; F[1] = mx; F[2] = nx;
    F[3] = by; F[4] = my; F[5] = ny;
    F[6] = bz; F[7] = mz; F[8] = nz;
    o[0] = C0[0]; o[1] = C0[1]; o[2] = C0[2];
  }
  const int nt = 3 * (L - 1);   // placed backbone atoms
  for (int k0 = 0; k0 < nt; k0 += 64) {
    const int j = k0 + lane, k = 3 + j, kind = k % 3, c = k / 3;
    // this lane's transform (absent lanes: the identity)
    double ct = 1.0, st = 0.0, l = 0.0, cx = 1.0, sx = 0.0;
    if (j < nt) {
      if (kind == 0) { ct = ct_cacn; st = st_cacn; l = kBondCN; sincos(s[2 * c - 1], &sx, &cx); }
      else if (kind == 1) { ct = ct_cnca; st = st_cnca; l = kBondNCA; cx = co; sx = so; }
      else { ct = ct_ncac; st = st_ncac; l = kBondCAC; sincos(s[2 * c], &sx, &cx); }
    }
    double R[9], u[3];
    if (j < nt) {
      R[0] = -ct;      R[1] = -st;      R[2] = 0.0;
      R[3] = st * cx;  R[4] = -ct * cx; R[5] = -sx;
      R[6] = st * sx;  R[7] = -ct * sx; R[8] = cx;
    } else {
      R[0] = 1.0; R[1] = 0.0; R[2] = 0.0; R[3] = 0.0; R[4] = 1.0; R[5] = 0.0; R[6] = 0.0; R[7] = 0.0; R[8] = 1.0;
    }
    u[0] = l * R[0]; u[1] = l * R[3]; u[2] = l * R[6];
    // inclusive scan over the lanes: (R, u) <- (R, u) of lane - off  o  (R, u)
    for (int off = 1; off < 64; off <<= 1) {
      double Rp[9], up[3];
#pragma unroll
      for (int q = 0; q < 9; ++q) Rp[q] = __shfl_up(R[q], off, 64);
#pragma unroll
      for (int q = 0; q < 3; ++q) up[q] = __shfl_up(u[q], off, 64);
      if (lane >= off) {
        double Rn[9], un[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int q = 0; q < 3; ++q) Rn[3 * r + q] = Rp[3 * r] * R[q] + Rp[3 * r + 1] * R[3 + q] + Rp[3 * r + 2] * R[6 + q];
          un[r] = up[r] + Rp[3 * r] * u[0] + Rp[3 * r + 1] * u[1] + Rp[3 * r + 2] * u[2];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) R[q] = Rn[q];
        u[0] = un[0]; u[1] = un[1]; u[2] = un[2];
      }
    }
    // atom k = origin of the frame after this lane's transform
    if (j < nt) {
      double* x = atom(x64, c, kind);
#pragma unroll
      for (int r = 0; r < 3; ++r) x[r] = o[r] + F[3 * r] * u[0] + F[3 * r + 1] * u[1] + F[3 * r + 2] * u[2];
    }
    // carry the frame past the last transform of these 64 (uniform)
    const int last = nt - k0 < 64 ? nt - k0 - 1 : 63;
    double Rl[9], ul[3];
#pragma unroll
    for (int q = 0; q < 9; ++q) Rl[q] = readlane_d(R[q], last);
#pragma unroll
    for (int q = 0; q < 3; ++q) ul[q] = readlane_d(u[q], last);
    double Fn[9], on[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int q = 0; q < 3; ++q) Fn[3 * r + q] = F[3 * r] * Rl[q] + F[3 * r + 1] * Rl[3 + q] + F[3 * r + 2] * Rl[6 + q];
      on[r] = o[r] + F[3 * r] * ul[0] + F[3 * r + 1] * ul[1] + F[3 * r + 2] * ul[2];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) F[q] = Fn[q];
    o[0] = on[0]; o[1] = on[1]; o[2] = on[2];
  }
  wave_sync();
  // C-beta of residue c from C_c, N_c, CA_c (one residue per lane)
  for (int c = lane; c < L; c += 64) {
    const double* pN = atom(x64, c, 0);
    const double* pCA = atom(x64, c, 1);
    const double* pC = atom(x64, c, 2);
    const double Nc[3] = {pN[0], pN[1], pN[2]}, CAc[3] = {pCA[0], pCA[1], pCA[2]}, Cc[3] = {pC[0], pC[1], pC[2]};
    double B[3];
    nerf_place(Cc, Nc, CAc, kBondCACB, ct_ncacb, st_ncacb, ccb, scb, B);
    double* pB = atom(x64, c, 3);
    pB[0] = B[0]; pB[1] = B[1]; pB[2] = B[2];
  }
  wave_sync();
}

}  // namespace amh
