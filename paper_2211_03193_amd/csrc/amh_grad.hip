// amh_grad.hip -- gradient of the distogram energy with respect to the torsions,
// and a per-chain L-BFGS minimiser built on it, for MI355X (gfx950, wave64).
//
// The energy is V(s) = sum_{i<j} E_ij(|CB_i - CB_j|) over the conformation G(s)
// (the AlphaFold1 distogram term the paper samples, Sec. 2.3).  Turning torsion k
// by eps rotates every residue from the pivot p on about the bond axis u through
// the point a (N_c -> CA_c for phi_c, CA_c -> C_c for psi_c), so with the C-beta
// forces F_j = dV/dx_j
//     dV/ds_k = sum_{j >= p} F_j . (u x (x_j - a)) = u . (T_p - a x S_p),
// where S_p = sum_{j >= p} F_j and T_p = sum_{j >= p} x_j x F_j are suffix sums
// along the chain (pairs with both ends at or after p move rigidly and cancel).
// One O(L^2) force pass and an O(L) scan give the whole gradient.
//
// Everything here is float64 (coordinates, distances, spline and its derivative of
// the float32 table values, sums); this is not the sampling hot loop.
//
// The minimiser is L-BFGS (Liu and Nocedal 1989; two-loop recursion) with a
// backtracking Armijo line search against the largest of the last M accepted
// values (Grippo, Lampariello and Lucidi 1986), the minimiser the paper pairs with
// its sampler (Sec. 3, the L-BFGS columns of Fig. 3).  One workgroup runs one
// chain's whole minimisation; the vectors and the curvature history live in a
// global workspace (resident in L2 for a few hundred chains), the geometry in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "amh_device.h"
#include "amh_geom.h"
#include "amh_grad.h"

namespace amh {

// Pair energy and its derivative dE/dd from a padded row [y1, y0 .. y_{nb-1}, y_{nb-2}]:
// uniform Catmull-Rom on the bin centres, flat (zero derivative) outside the knots.
// t is the position in bin widths from the first centre; the four taps row[b .. b+3]
// are gathered beforehand at b = stencil_base(t): b = 0 below the first knot (q1 =
// row[1] is the value there) and for a NaN position, b = nb - 3 at or beyond the last
// knot (q3 = row[nb]), else the interval of t.
__device__ __forceinline__ int stencil_base(double t, int nb) {
  return !(t > 0.0) ? 0 : t >= (double)(nb - 1) ? nb - 3 : (int)floor(t);
}

__device__ __forceinline__ void spline64_ed(double q0, double q1, double q2, double q3, double t, int b,
                                            int nb, double inv_w, double& E, double& dE) {
  if (t != t) { E = t; dE = t; return; }   // a NaN distance: V turns NaN
  if (t <= 0.0) { E = q1; dE = 0.0; return; }
  if (t >= (double)(nb - 1)) { E = q3; dE = 0.0; return; }
  const double f = t - (double)b;
  const double a1 = -q0 + q2;
  const double a2 = 2.0 * q0 - 5.0 * q1 + 4.0 * q2 - q3;
  const double a3 = -q0 + 3.0 * q1 - 3.0 * q2 + q3;
  E = 0.5 * (2.0 * q1 + a1 * f + a2 * f * f + a3 * f * f * f);
  dE = 0.5 * (a1 + 2.0 * a2 * f + 3.0 * a3 * f * f) * inv_w;
}

typedef __attribute__((address_space(1))) const float gfloat;

// integer add to an LDS word through an LDS pointer (a generic-pointer atomic would be a
// flat operation, which the compiler then waits on together with the table gathers)
__device__ __forceinline__ void lds_add(long long* p, long long v) {
  __hip_atomic_fetch_add((__attribute__((address_space(3))) long long*)p, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}

// x rounded to a multiple of 2^-44, as an integer count of 2^-44 (|x| < 2^19)
__device__ __forceinline__ long long fixed44(double x) { return (long long)rint(x * 0x1p44); }

// Sum over the 64 lanes by a fixed butterfly: every lane gets the same value.
__device__ __forceinline__ double wave_allsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_allmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide reductions; every thread returns the same value, summed in a fixed
// order (per-thread strided partials, the lane butterfly, the waves in order).
// `red` holds 3 W doubles.  Each call begins and ends with a barrier.
__device__ void block_sum3(double& a, double& b, double& c, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  a = wave_allsum(a); b = wave_allsum(b); c = wave_allsum(c);
  __syncthreads();
  if (lane == 0) { red[3 * wave] = a; red[3 * wave + 1] = b; red[3 * wave + 2] = c; }
  __syncthreads();
  a = 0.0; b = 0.0; c = 0.0;
  for (int v = 0; v < W; ++v) { a += red[3 * v]; b += red[3 * v + 1]; c += red[3 * v + 2]; }
  __syncthreads();
}

__device__ double block_dot(const double* __restrict__ x, const double* __restrict__ y, int n,
                            double* red) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) a += x[e] * y[e];
  block_sum3(a, b, c, red);
  return a;
}

__device__ double block_maxabs(const double* __restrict__ x, int n, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
  double m = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) m = fmax(m, fabs(x[e]));
  m = wave_allmax(m);
  __syncthreads();
  if (lane == 0) red[wave] = m;
  __syncthreads();
  m = 0.0;
  for (int v = 0; v < W; ++v) m = fmax(m, red[v]);
  __syncthreads();
  return m;
}

// V(s) and, if g != null, dV/ds of one conformation, by the whole workgroup.
// x64 [12 L] and ft [6 (L + 1)] are LDS scratch, red [3 W] the reduction slots.
// Returns V in every thread; g is complete after the closing barrier.
__device__ double value_grad(const double* __restrict__ s, int L, const float* __restrict__ table,
                             int stride, int nb, double d_min, double w, double* x64, double* ft,
                             double* red, double* __restrict__ g) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wave = tid >> 6, W = T >> 6;
  const double dfar = d_min + w * ((double)nb - 0.5), d2far = dfar * dfar;   // the last knot
  const double inv_w = 1.0 / w;
  // the table through a global-memory pointer, so that its gathers wait only on their own
  // counter and not on the LDS traffic of the same steps
  const gfloat* gtable = (const gfloat*)table;
  // the C-beta forces F_k accumulate as integers (multiples of 2^-44) in the first
  // three slots of ft[6k .. 6k+5]
  long long* facc = reinterpret_cast<long long*>(ft);
  for (int k = tid; k < L; k += T) facc[6 * k] = facc[6 * k + 1] = facc[6 * k + 2] = 0;
  if (wave == 0) nerf_chain(s, L, x64, lane);
  __syncthreads();
  // forces: every pair i < j once, in tiles of 64 rows (block I) by 64 columns (block
  // J >= I) dealt to the wavefronts in turn.  Lane l holds row i = 64 I + l and at step
  // u the column j = 64 J + ((l + u) & 63); the row's force accumulates in registers,
  // and each column's travels with it (every step a lane takes the column sum of the
  // lane above), so that after 64 steps lane l holds column 64 J + l's.  The tile's
  // row and column sums, rounded to multiples of 2^-44, are added as integers: the
  // totals do not depend on the order in which the wavefronts add them.
  double vs = 0.0, vc = 0.0;
  bool wide = false;   // a tile sum beyond the integer range (or NaN): V is returned NaN
  const int nb64 = (L + 63) >> 6, ntile = nb64 * (nb64 + 1) / 2;
  // retire every memory operation before the tiles (the NeRF's spill stores among them),
  // so that inside the tiles only the table gathers are counted and each step waits for
  // the gather of the pair it evaluates, not for the one issued for the next step
  __builtin_amdgcn_s_waitcnt(0);
  for (int tile = wave; tile < ntile; tile += W) {
    int I = 0, rem = tile;
    while (rem >= nb64 - I) { rem -= nb64 - I; ++I; }
    const int J = I + rem, i = 64 * I + lane;
    const double* xi = atom(x64, i < L ? i : 0, 3);
    const double ix = xi[0], iy = xi[1], iz = xi[2];
    double rx = 0.0, ry = 0.0, rz = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    // step u's partner, distance, stencil base and taps; issued one step ahead of its
    // evaluation so that the table gather overlaps the previous pair (an absent pair
    // reads row 0, a far one the taps ending at its no-contact value)
    struct Pair {
      double ex, ey, ez, inv_d, t;
      int b;
      bool real, near;
      float q0, q1, q2, q3;
    };
    auto prep = [&](int u) {
      Pair a;
      const int j = 64 * J + ((lane + u) & 63);
      a.real = i < j && j < L;
      const double* xj = atom(x64, a.real ? j : 0, 3);
      a.ex = xj[0] - ix; a.ey = xj[1] - iy; a.ez = xj[2] - iz;
      const double d2 = a.ex * a.ex + a.ey * a.ey + a.ez * a.ez;
      a.near = a.real && !(d2 >= d2far);   // a NaN distance is evaluated, so V turns NaN
      // distance through the hardware reciprocal square root and two Newton steps
      a.inv_d = a.near && d2 > 0.0 ? rsqrt64(d2) : 0.0;
      a.t = a.near ? (d2 * a.inv_d - (d_min + 0.5 * w)) * inv_w : (double)nb;
      a.b = stencil_base(a.t, nb);
      const gfloat* row = gtable + (size_t)(a.real ? pair_row(i, j, L) : 0) * stride + a.b;
      a.q0 = row[0]; a.q1 = row[1]; a.q2 = row[2]; a.q3 = row[3];
      return a;
    };
    auto eval = [&](const Pair& a) {
      if (a.real) {
        double E = (double)a.q3, dE = 0.0;   // beyond the last knot: the no-contact value
        if (a.near)
          spline64_ed((double)a.q0, (double)a.q1, (double)a.q2, (double)a.q3, a.t, a.b, nb, inv_w, E, dE);
        neumaier_add(vs, vc, E);
        if (a.inv_d > 0.0) {   // dV/dx_j = +q e, dV/dx_i = -q e
          const double q = dE * a.inv_d, qx = q * a.ex, qy = q * a.ey, qz = q * a.ez;
          cx += qx; cy += qy; cz += qz;
          rx -= qx; ry -= qy; rz -= qz;
        }
      }
      const int up = (lane + 1) & 63;
      cx = __shfl(cx, up, 64); cy = __shfl(cy, up, 64); cz = __shfl(cz, up, 64);
    };
    // two records in turn, so that no gathered value is copied (u = 64 prepares a pair
    // that is not evaluated)
    Pair A = prep(0);
    for (int u = 0; u < 64; u += 2) {
      const Pair B = prep(u + 1);
      eval(A);
      A = prep(u + 2);
      eval(B);
    }
    const double lim = 0x1p13;   // |tile sum| < 2^13: a residue's total stays below 2^19
    wide = wide || !(fabs(rx) < lim && fabs(ry) < lim && fabs(rz) < lim && fabs(cx) < lim &&
                     fabs(cy) < lim && fabs(cz) < lim);
    if (!wide) {
      if (i < L) {
        lds_add(facc + 6 * i, fixed44(rx));
        lds_add(facc + 6 * i + 1, fixed44(ry));
        lds_add(facc + 6 * i + 2, fixed44(rz));
      }
      const int jc = 64 * J + lane;
      if (jc < L) {
        lds_add(facc + 6 * jc, fixed44(cx));
        lds_add(facc + 6 * jc + 1, fixed44(cy));
        lds_add(facc + 6 * jc + 2, fixed44(cz));
      }
    }
  }
  __syncthreads();
  // force and torque x_k x F_k of every residue, in place
  for (int k = tid; k < L; k += T) {
    const double fx = (double)facc[6 * k] * 0x1p-44, fy = (double)facc[6 * k + 1] * 0x1p-44,
                 fz = (double)facc[6 * k + 2] * 0x1p-44;
    const double* xk = atom(x64, k, 3);
    const double kx = xk[0], ky = xk[1], kz = xk[2];
    double* o = ft + 6 * k;
    o[0] = fx; o[1] = fy; o[2] = fz;
    o[3] = ky * fz - kz * fy;
    o[4] = kz * fx - kx * fz;
    o[5] = kx * fy - ky * fx;
  }
  if (wide) vs = __builtin_nan("");
  double V = vs + vc, z1 = 0.0, z2 = 0.0;
  block_sum3(V, z1, z2, red);   // also the barrier that publishes ft
  // suffix sums S_p, T_p (six components, one lane each, in chain order)
  if (wave == 0 && lane < 6) {
    double acc = 0.0;
    ft[6 * L + lane] = 0.0;
    for (int j = L - 1; j >= 0; --j) {
      acc += ft[6 * j + lane];
      ft[6 * j + lane] = acc;
    }
  }
  __syncthreads();
  if (g) {
    for (int k = tid; k < 2 * L; k += T) {
      double gk = 0.0;
      if (k != 0 && k != 2 * L - 1) {   // phi_0 and psi_{L-1} move no C-beta
        const int c = k >> 1, p = (k & 1) ? c + 1 : c;
        const double* A = atom(x64, c, (k & 1) ? 1 : 0);
        const double* B = atom(x64, c, (k & 1) ? 2 : 1);
        double ux = B[0] - A[0], uy = B[1] - A[1], uz = B[2] - A[2];
        const double iu = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
        ux *= iu; uy *= iu; uz *= iu;
        const double* S = ft + 6 * p;
        const double tx = S[3] - (A[1] * S[2] - A[2] * S[1]);
        const double ty = S[4] - (A[2] * S[0] - A[0] * S[2]);
        const double tz = S[5] - (A[0] * S[1] - A[1] * S[0]);
        gk = ux * tx + uy * ty + uz * tz;
      }
      g[k] = gk;
    }
  }
  __syncthreads();
  return V;
}

// ---------------------------------------------------------------------------
// Both kernels are held to two wavefronts per SIMD (at most 256 registers a lane).
// Left free, the compiler gives the parallel NeRF scan, which one wavefront runs once
// per evaluation, 271 registers and every kernel one wavefront per SIMD; under the
// cap it spills a little inside that scan, and two workgroups share each CU (the
// most their LDS allows at 400 residues), hiding the force pass's table gathers.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) grad_kernel(GradParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int L = P.L;
  double* x64 = reinterpret_cast<double*>(lds);
  double* ft = x64 + 12 * L;
  double* red = ft + 6 * (L + 1);
  const int b = blockIdx.x;
  const double V = value_grad(P.s + (size_t)b * 2 * L, L, P.table, P.stride, P.nb, P.d_min,
                              P.bin_w, x64, ft, red, P.g ? P.g + (size_t)b * 2 * L : nullptr);
  if (threadIdx.x == 0) {
    if (!isfinite(V)) atomicOr(P.err, kErrGradEnergy);
    if (P.V) P.V[b] = V;
  }
}

// ---------------------------------------------------------------------------
// One chain's L-BFGS.  Workspace rows (n = 2L doubles each): x, g, d, xn, gn, then
// the curvature pairs S[m], Y[m] kept as a ring (oldest at `head`).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) lbfgs_kernel(LbfgsParams P) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int L = P.L, n = 2 * L, tid = threadIdx.x, T = blockDim.x, W = T >> 6;
  const int m = P.m, M = P.nonmonotone;
  double* x64 = reinterpret_cast<double*>(lds);
  double* ft = x64 + 12 * L;
  double* red = ft + 6 * (L + 1);
  double* rho = red + 3 * W;     // [m]
  double* alp = rho + m;         // [m]
  double* fh = alp + m;          // [M]
  const int b = blockIdx.x;
  double* ws = P.work + (size_t)b * (5 + 2 * (size_t)m) * n;
  double* x = ws;
  double* g = ws + n;
  double* d = ws + 2 * (size_t)n;
  double* xn = ws + 3 * (size_t)n;
  double* gn = ws + 4 * (size_t)n;
  double* Sh = ws + 5 * (size_t)n;
  double* Yh = Sh + (size_t)m * n;
  double* sb = P.s + (size_t)b * n;
  double* trace = P.f_trace ? P.f_trace + (size_t)b * (P.n_iter + 1) : nullptr;
  double* xtr = P.x_trace ? P.x_trace + (size_t)b * (P.n_iter + 1) * n : nullptr;

  for (int e = tid; e < n; e += T) {
    x[e] = sb[e];
    if (xtr) xtr[e] = sb[e];
  }
  __syncthreads();
  double f = value_grad(x, L, P.table, P.stride, P.nb, P.d_min, P.bin_w, x64, ft, red, g);
  if (trace && tid == 0) trace[0] = f;
  if (tid == 0) fh[0] = f;
  int k = 0, head = 0, nf = 1, it = 0, status = 1;
  for (it = 0; it < P.n_iter; ++it) {
    const double gmax = block_maxabs(g, n, red);
    if (gmax <= P.gtol) { status = 0; break; }
    // direction: two-loop recursion, newest pair first, then oldest first
    double gamma = P.step0 / gmax;
    if (k > 0) {
      const int r = (head + k - 1) % m;
      double sy = 0.0, yy = 0.0, z = 0.0;
      for (int e = tid; e < n; e += T) {
        const double ye = Yh[(size_t)r * n + e];
        sy += Sh[(size_t)r * n + e] * ye;
        yy += ye * ye;
      }
      block_sum3(sy, yy, z, red);
      gamma = sy / yy;
    }
    for (int e = tid; e < n; e += T) d[e] = g[e];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
      const int r = (head + i) % m;
      const double* sr = Sh + (size_t)r * n;
      const double* yr = Yh + (size_t)r * n;
      const double a = rho[r] * block_dot(sr, d, n, red);
      if (tid == 0) alp[r] = a;
      for (int e = tid; e < n; e += T) d[e] -= a * yr[e];
      __syncthreads();
    }
    for (int e = tid; e < n; e += T) d[e] *= gamma;
    __syncthreads();
    for (int i = 0; i < k; ++i) {
      const int r = (head + i) % m;
      const double* sr = Sh + (size_t)r * n;
      const double* yr = Yh + (size_t)r * n;
      const double bb = rho[r] * block_dot(yr, d, n, red);
      const double a = alp[r];
      for (int e = tid; e < n; e += T) d[e] += (a - bb) * sr[e];
      __syncthreads();
    }
    for (int e = tid; e < n; e += T) d[e] = -d[e];
    __syncthreads();
    double gd = block_dot(g, d, n, red);
    if (!(gd < 0.0)) {   // not a descent direction: drop the history, scaled steepest descent
      k = 0;
      head = 0;
      const double g0 = P.step0 / gmax;
      for (int e = tid; e < n; e += T) d[e] = -g0 * g[e];
      __syncthreads();
      gd = block_dot(g, d, n, red);
    }
    double fref = fh[0];
    for (int i = 1; i < (nf < M ? nf : M); ++i) fref = fmax(fref, fh[i]);
    // Armijo backtracking
    double alpha = 1.0, fnew = 0.0;
    bool ok = false;
    for (int ls = 0; ls < P.max_ls; ++ls) {
      for (int e = tid; e < n; e += T) xn[e] = x[e] + alpha * d[e];
      __syncthreads();
      fnew = value_grad(xn, L, P.table, P.stride, P.nb, P.d_min, P.bin_w, x64, ft, red, gn);
      if (fnew <= fref + P.c1 * alpha * gd) { ok = true; break; }
      alpha *= P.shrink;
    }
    if (!ok) { status = 2; break; }
    // curvature pair, kept only when s.y is clearly positive
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int e = tid; e < n; e += T) {
      const double se = xn[e] - x[e], ye = gn[e] - g[e];
      sy += se * ye; ss += se * se; yy += ye * ye;
    }
    block_sum3(sy, ss, yy, red);
    if (sy > 1e-8 * sqrt(ss * yy)) {
      if (k == m) { head = (head + 1) % m; --k; }
      const int r = (head + k) % m;
      for (int e = tid; e < n; e += T) {
        Sh[(size_t)r * n + e] = xn[e] - x[e];
        Yh[(size_t)r * n + e] = gn[e] - g[e];
      }
      if (tid == 0) rho[r] = 1.0 / sy;
      ++k;
    }
    __syncthreads();
    // accept: swap the roles of (x, g) and (xn, gn)
    double* t0 = x; x = xn; xn = t0;
    double* t1 = g; g = gn; gn = t1;
    f = fnew;
    if (tid == 0) fh[nf % M] = f;
    ++nf;
    if (trace && tid == 0) trace[it + 1] = f;
    if (xtr)
      for (int e = tid; e < n; e += T) xtr[(size_t)(it + 1) * n + e] = x[e];
    __syncthreads();
  }
  for (int e = tid; e < n; e += T) sb[e] = wrap_angle(x[e]);
  if (P.v_state) {
    const bool better = f < P.v_state[2 * b + 1];
    __syncthreads();
    if (better)
      for (int e = tid; e < n; e += T) P.s_best[(size_t)b * n + e] = wrap_angle(x[e]);
    __syncthreads();
    if (tid == 0) {
      P.v_state[2 * b] = f;
      if (better) P.v_state[2 * b + 1] = f;
    }
  }
  if (tid == 0) {
    if (!isfinite(f)) atomicOr(P.err, kErrGradEnergy);
    if (P.V) P.V[b] = f;
    if (P.iters) P.iters[b] = it;
    if (P.status) P.status[b] = status;
  }
}

}  // namespace amh
