// amh_device.h -- device-side building blocks of the AMH sampler for gfx950.
//
// Philox4x32-10 (Salmon et al., SC'11), the Box-Muller proposal increment, the
// NeRF placement step and Rodrigues rotation about a bond axis in float64,
// and the Catmull-Rom distogram spline in float32 (hot loop) and float64 (anchors).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amh {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;

// Ideal backbone geometry (Angstrom, degrees): N-CA, CA-C, C-N, CA-CB bonds; the
// N-CA-C, CA-C-N, C-N-CA and N-CA-CB angles; omega and the C-N-CA-CB torsion.
constexpr double kBondNCA = 1.458, kBondCAC = 1.525, kBondCN = 1.329, kBondCACB = 1.53;
constexpr double kAngNCAC = 111.2, kAngCACN = 116.2, kAngCNCA = 121.7, kAngNCACB = 110.5;
constexpr double kTorOmega = 180.0, kTorCB = -122.5;

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of two 32x32->64 multiplies and xors, the key bumped
// by the golden-ratio Weyl constants between rounds.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ double open_unit(uint32_t x) {
  return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

// Randoms of proposal k of sweep t of chain `chain`: counter (k, t, chain, 0).
struct Draw { double delta, log_u, cd, sd; };

__device__ __forceinline__ Draw proposal_draw(uint32_t k, uint32_t t, uint32_t chain, uint32_t k0,
                                              uint32_t k1, double sigma) {
  U4 x = philox10(U4{k, t, chain, 0u}, k0, k1);
  double u0 = open_unit(x.x), u1 = open_unit(x.y), u2 = open_unit(x.z);
  Draw d;
  d.delta = sigma * sqrt(-2.0 * log(u0)) * cos(kTwoPi * u1);
  d.log_u = log(u2);
  sincos(d.delta, &d.sd, &d.cd);
  return d;
}

__device__ __forceinline__ double wrap_angle(double a) {
  if (a > kPi) a -= kTwoPi;
  else if (a <= -kPi) a += kTwoPi;
  return a;
}

// ---------------------------------------------------------------------------
// Float64 coordinates: atom a of residue r at x[(4 r + a) * 3 .. +2] (N, CA, C, CB).
struct D3 { double x, y, z; };

__device__ __forceinline__ D3 ld3(const double* p) { return D3{p[0], p[1], p[2]}; }
__device__ __forceinline__ void st3(double* p, D3 v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }

// Rotation by angle (c, s) about the unit axis through `a` along B - A (float64).
struct Rot {
  double r[9];
  double a[3];
  double log_u;  // acceptance log-uniform of the proposal the rotation belongs to
};

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps (float64).
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}

__device__ __forceinline__ void make_rot(D3 A, D3 B, double c, double s, Rot& R) {
  double ux = B.x - A.x, uy = B.y - A.y, uz = B.z - A.z;
  const double inv = rsqrt64(ux * ux + uy * uy + uz * uz);
  ux *= inv; uy *= inv; uz *= inv;
  const double t = 1.0 - c;
  R.r[0] = c + t * ux * ux;      R.r[1] = t * ux * uy - s * uz; R.r[2] = t * ux * uz + s * uy;
  R.r[3] = t * uy * ux + s * uz; R.r[4] = c + t * uy * uy;      R.r[5] = t * uy * uz - s * ux;
  R.r[6] = t * uz * ux - s * uy; R.r[7] = t * uz * uy + s * ux; R.r[8] = c + t * uz * uz;
  R.a[0] = A.x; R.a[1] = A.y; R.a[2] = A.z;
}

// Rotation by angle (c, s) about the unit axis u through the point A.
__device__ __forceinline__ void make_rot_u(D3 A, D3 u, double c, double s, Rot& R) {
  const double t = 1.0 - c;
  R.r[0] = c + t * u.x * u.x;       R.r[1] = t * u.x * u.y - s * u.z; R.r[2] = t * u.x * u.z + s * u.y;
  R.r[3] = t * u.y * u.x + s * u.z; R.r[4] = c + t * u.y * u.y;       R.r[5] = t * u.y * u.z - s * u.x;
  R.r[6] = t * u.z * u.x - s * u.y; R.r[7] = t * u.z * u.y + s * u.x; R.r[8] = c + t * u.z * u.z;
  R.a[0] = A.x; R.a[1] = A.y; R.a[2] = A.z;
}

__device__ __forceinline__ D3 unit(D3 A, D3 B) {
  const double ux = B.x - A.x, uy = B.y - A.y, uz = B.z - A.z;
  const double inv = rsqrt64(ux * ux + uy * uy + uz * uz);
  return D3{ux * inv, uy * inv, uz * inv};
}

// R v for a direction v (no translation).
__device__ __forceinline__ D3 rot_dir(const Rot& R, D3 v) {
  return D3{R.r[0] * v.x + R.r[1] * v.y + R.r[2] * v.z, R.r[3] * v.x + R.r[4] * v.y + R.r[5] * v.z,
            R.r[6] * v.x + R.r[7] * v.y + R.r[8] * v.z};
}

// R (x - a): the rotated position relative to the pivot point.
__device__ __forceinline__ D3 rot_rel(const Rot& R, D3 x) {
  const double vx = x.x - R.a[0], vy = x.y - R.a[1], vz = x.z - R.a[2];
  return D3{R.r[0] * vx + R.r[1] * vy + R.r[2] * vz, R.r[3] * vx + R.r[4] * vy + R.r[5] * vz,
            R.r[6] * vx + R.r[7] * vy + R.r[8] * vz};
}

__device__ __forceinline__ D3 apply_rot(const Rot& R, D3 x) {
  const D3 v = rot_rel(R, x);
  return D3{R.a[0] + v.x, R.a[1] + v.y, R.a[2] + v.z};
}

// float32 squared distance of two float64 points (difference taken in float64).
__device__ __forceinline__ float dist2_64(D3 a, D3 b) {
  const float dx = (float)(b.x - a.x), dy = (float)(b.y - a.y), dz = (float)(b.z - a.z);
  return dx * dx + dy * dy + dz * dz;
}

// ---------------------------------------------------------------------------
// Catmull-Rom spline of -ln p over the bin centres.  A padded row holds
// [y1, y0, y1, ..., y_{nb-1}, y_{nb-2}, pad...]: entry b+1 is y_b and the two
// mirrored ghosts sit at both ends, so the 4-tap stencil of interval b is
// row[b .. b+3] for every b in [0, nb-2].
struct Spline32 {
  float inv_w;  // 1 / bin width
  float off;    // (d_min + w/2) / w
  float tmax;   // nb - 1
};

// Knot interval b and fraction f of a distance: t = (d - first knot) / w clamped to
// [0, nb-1], b = min(floor t, nb-2), f = t - b (f = 1 at the far clamp).
__device__ __forceinline__ void spline_pos(float d, const Spline32& S, int& b, float& f) {
  float t = fmaf(d, S.inv_w, -S.off);
  t = fminf(fmaxf(t, 0.0f), S.tmax);
  const float bf = fminf(floorf(t), S.tmax - 1.0f);
  f = t - bf;
  b = (int)bf;
}

// Uniform Catmull-Rom cubic through (y0, y1, y2, y3) at fraction f of [y1, y2].
__device__ __forceinline__ float catmull_rom(float y0, float y1, float y2, float y3, float f) {
  const float a1 = y2 - y0;
  const float a2 = 2.0f * y0 - 5.0f * y1 + 4.0f * y2 - y3;
  const float a3 = 3.0f * (y1 - y2) + y3 - y0;
  return fmaf(0.5f * f, fmaf(f, fmaf(f, a3, a2), a1), y1);
}

__device__ __forceinline__ float spline32(const float* __restrict__ row, float d, const Spline32& S) {
  int b;
  float f;
  spline_pos(d, S, b, f);
  const float* q = row + b;
  return catmull_rom(q[0], q[1], q[2], q[3], f);
}

// Pair energy minus the pair's no-contact value, from a row of the deviation table:
// exactly zero beyond the last knot (squared distance d2far), where the spline is flat.
__device__ __forceinline__ float edev32(const float* __restrict__ dev_row, float d2, const Spline32& S,
                                        float d2far) {
  return d2 < d2far ? spline32(dev_row, __builtin_amdgcn_sqrtf(d2), S) : 0.0f;
}

// The same, split in two so that the loads can be issued well before the value is
// needed: the stencil of a squared distance (zeros beyond the last knot, which
// evaluate to exactly 0), then its evaluation.
struct Stencil {
  float y0, y1, y2, y3, f;
};
__device__ __forceinline__ Stencil fetch_dev(const float* __restrict__ dev_row, float d2,
                                             const Spline32& S, float d2far) {
  Stencil s{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (d2 < d2far) {
    int b;
    spline_pos(__builtin_amdgcn_sqrtf(d2), S, b, s.f);
    const float* q = dev_row + b;
    s.y0 = q[0]; s.y1 = q[1]; s.y2 = q[2]; s.y3 = q[3];
  }
  return s;
}
__device__ __forceinline__ float eval_dev(const Stencil& s) {
  return catmull_rom(s.y0, s.y1, s.y2, s.y3, s.f);
}

// Branch-free form for several pairs in flight: the address of the stencil of a
// squared distance in `dev_row`, or of the same taps of the zero row beyond the last
// knot (d2 = +inf marks an unused slot), and the fraction.  Loads from the returned
// address can be issued for all slots before any is used.
__device__ __forceinline__ const float* stencil_addr(const float* __restrict__ dev_row,
                                                     const float* __restrict__ zrow, float d2,
                                                     const Spline32& S, float d2far, float& f) {
  int b;
  spline_pos(__builtin_amdgcn_sqrtf(fminf(d2, d2far)), S, b, f);
  return (d2 < d2far ? dev_row : zrow) + b;
}
__device__ __forceinline__ float4 ld_stencil(const float* q) {
  return make_float4(q[0], q[1], q[2], q[3]);
}

// rint(x 2^30) as a float64 integer: x 2^30 is exact in float32 and rounding it to an
// integer there equals rounding the exact value, so sums of these integers (below
// 2^53) are exact in float64 in any order; the energy is the sum times 2^-30.
__device__ __forceinline__ double fixed30_units(float x) {
  return (double)rintf(x * 1073741824.0f);
}

// Catmull-Rom value of a padded row at distance d in float64 (inv_w = 1 / bin width).
__device__ __forceinline__ double spline64(const float* __restrict__ row, double d, int nb,
                                           double d_min, double w, double inv_w) {
  const double t = (d - (d_min + 0.5 * w)) * inv_w;
  if (t <= 0.0) return (double)row[1];
  if (t >= (double)(nb - 1)) return (double)row[nb];
  const int b = (int)floor(t);
  const double f = t - (double)b;
  const double q0 = row[b], q1 = row[b + 1], q2 = row[b + 2], q3 = row[b + 3];
  const double a0 = 2.0 * q1;
  const double a1 = -q0 + q2;
  const double a2 = 2.0 * q0 - 5.0 * q1 + 4.0 * q2 - q3;
  const double a3 = -q0 + 3.0 * q1 - 3.0 * q2 + q3;
  return 0.5 * (a0 + a1 * f + a2 * f * f + a3 * f * f * f);
}

// Packed row of the pair i < j.
__device__ __forceinline__ int pair_row(int i, int j, int L) {
  return i * L - ((i * (i + 1)) >> 1) + (j - i - 1);
}

// ---------------------------------------------------------------------------
// NeRF placement in float64 (Parsons et al. 2005): D from A, B, C with bond l,
// angle BCD (cos ct, sin st) and dihedral ABCD (cos cc, sin sc).
__device__ __forceinline__ void nerf_place(const double* A, const double* B, const double* C,
                                           double l, double ct, double st, double cc, double sc,
                                           double* D) {
  double bx = C[0] - B[0], by = C[1] - B[1], bz = C[2] - B[2];
  double ib = 1.0 / sqrt(bx * bx + by * by + bz * bz);
  bx *= ib; by *= ib; bz *= ib;
  const double ax = B[0] - A[0], ay = B[1] - A[1], az = B[2] - A[2];
  double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  double in = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
  nx *= in; ny *= in; nz *= in;
  const double mx = ny * bz - nz * by, my = nz * bx - nx * bz, mz = nx * by - ny * bx;
  const double d0 = -l * ct, d1 = l * st * cc, d2 = l * st * sc;
  D[0] = C[0] + bx * d0 + mx * d1 + nx * d2;
  D[1] = C[1] + by * d0 + my * d1 + ny * d2;
  D[2] = C[2] + bz * d0 + mz * d1 + nz * d2;
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).

// DPP move of both halves of a double (row_mask, bank_mask all set, bound_ctrl on).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRor4 = 0x124;  // row_ror:4 (lane i of a row reads lane i-4 mod 16)
constexpr int kDppRor8 = 0x128;  // row_ror:8
constexpr int kDppShl4 = 0x104;  // row_shl:4 (lane i of a row reads lane i+4; 0 past the row's end)
constexpr int kDppShl8 = 0x108;  // row_shl:8
constexpr int kDppShr4 = 0x114;  // row_shr:4 (lane i of a row reads lane i-4; 0 before its start)
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: lane i of each 8 reads lane 7 - i

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum and maximum over each aligned group of 8 lanes; every lane of a group gets the
// same value (the two operands of each addition are the same in both partners).
__device__ __forceinline__ float sum8(float v) {
  v += dpp_f<kDppXor1>(v);
  v += dpp_f<kDppXor2>(v);
  return v + dpp_f<kDppHalfMirror>(v);
}
__device__ __forceinline__ float max8(float v) {
  v = fmaxf(v, dpp_f<kDppXor1>(v));
  v = fmaxf(v, dpp_f<kDppXor2>(v));
  return fmaxf(v, dpp_f<kDppHalfMirror>(v));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Sum over the 64 lanes without LDS traffic: quad butterflies and row rotations by
// DPP, then the four row totals in a fixed order; every lane gets the same value.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppRor4>(v);
  v += dpp_d<kDppRor8>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Neumaier step: add x into (s, c).
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

}  // namespace amh
