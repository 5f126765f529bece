/*
 * oracle.c -- FP64 CPU oracle for Alternating Metropolis-Hastings (AMH).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct reference that the
 * HIP path is checked against (tests, smoke check, benchmark CPU baseline).  It
 * shares no code with the HIP path.
 *
 * Every function follows a passage of the paper (Ghantasala, Jaiswal, Datta,
 * "An Efficient MCMC Approach to Energy Function Optimization in Protein
 * Structure Prediction", arXiv 2211.03193):
 *   - state vector and single-flip Gaussian proposal: Sec. 2.1 and the
 *     transition-probability equation;
 *   - Metropolis acceptance min(1, e^{-beta (V(s')-V(s))}): the MH and marginal
 *     equations of Sec. 2.1 (Algorithm 1 prints the ratio inverted; the
 *     equations are followed);
 *   - localized energy over residues floor(k/2) +- floor(d/2): the localized-MH
 *     equations and the local AlphaFold1 energy of Sec. 2.3;
 *   - distogram energy V(x) = -sum log P(|x_i - x_j|): Sec. 2.3;
 *   - alternation of global and local sweeps: Algorithm 1, Fig. 1;
 *   - extended-chain start s^0 = 180 deg: Algorithm 1 input, Sec. 2.3;
 *   - coordinates x = G(s) from torsions: Sec. 2.1, rotation of the atoms
 *     downstream of the bond: Sec. 2.4 (proposal generation).
 * Points the paper leaves open (bins, spline, geometry constants, RNG, the
 * local/global order) follow the readings listed in the design notes.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846
#define TWO_PI_D (2.0 * PI_D)
#define DEG (PI_D / 180.0)

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
/* Round: (hi0,lo0)=M0*x0, (hi1,lo1)=M1*x2; x <- (hi1^x1^k0, lo1, hi0^x3^k1, lo0);
 * the key is bumped by the Weyl constants between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void oracle_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out) {
  for (int64_t i = 0; i < n; ++i) oracle_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* u = (x + 1/2) 2^-32, strictly inside (0, 1). */
static double unit_open(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* Proposal randoms of proposal k in sweep t: counter (k, t, chain, 0), key = seed.
 * The Gaussian increment is Box-Muller's cosine branch (Sec. 2.4, RNG step). */
void oracle_proposal(uint64_t seed, uint32_t chain, int64_t t, int32_t k, double sigma,
                     double *delta, double *log_u2) {
  uint32_t ctr[4] = {(uint32_t)k, (uint32_t)t, chain, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  oracle_philox4x32_10(ctr, key, x);
  double u0 = unit_open(x[0]), u1 = unit_open(x[1]), u2 = unit_open(x[2]);
  *delta = sigma * sqrt(-2.0 * log(u0)) * cos(TWO_PI_D * u1);
  *log_u2 = log(u2);
}

/* ------------------------------------------------------------------------- */
/* Schedule: inverse temperature beta_t = 1/T_t with T_t geometric T0 -> T1
 * over the run, and the alternation of global and localized sweeps. */
double oracle_beta(const oracle_cfg *cfg, int64_t t) {
  double T = cfg->T0;
  if (cfg->total_sweeps > 1)
    T = cfg->T0 * pow(cfg->T1 / cfg->T0, (double)t / (double)(cfg->total_sweeps - 1));
  return 1.0 / T;
}

/* The last n_global sweeps of every cycle of global_every sweeps are global
 * (Algorithm 1 alternates N_global global and N_local localized sweeps; here the
 * localized ones come first); n_global = 0 means 1. */
int32_t oracle_is_global(const oracle_cfg *cfg, int64_t t) {
  if (cfg->global_every <= 0) return 0;
  int32_t ng = cfg->n_global < 1 ? 1 : cfg->n_global;
  return (int32_t)(t % cfg->global_every) >= cfg->global_every - ng;
}

/* Proposal width of sweep t: constant, or reduced geometrically from sigma to
 * sigma_end over the schedule (Sec. 2.3: 10 to 4 degrees over a run). */
double oracle_sigma(const oracle_cfg *cfg, int64_t t) {
  if (cfg->sigma_end > 0.0 && cfg->sigma > 0.0 && cfg->total_sweeps > 1)
    return cfg->sigma * pow(cfg->sigma_end / cfg->sigma, (double)t / (double)(cfg->total_sweeps - 1));
  return cfg->sigma;
}

/* Localization radius of (localized) sweep t: window_d, then the cascade radii in
 * turn (Sec. 2.2: several localization ranges may be cascaded). */
int32_t oracle_window_d(const oracle_cfg *cfg, int64_t t) {
  int32_t r = (int32_t)(t % (1 + cfg->n_cascade));
  return r == 0 ? cfg->window_d : cfg->cascade_d[r - 1];
}

/* Noisy restart (the second scheme of Sec. 3): every torsion moves by a uniform
 * amount in [-amplitude, amplitude], drawn from Philox at counter (k, tag, chain, 1),
 * and is wrapped into (-pi, pi]. */
void oracle_perturb(uint64_t seed, uint32_t chain, uint32_t tag, double amplitude, int32_t n,
                    double *s) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int32_t k = 0; k < n; ++k) {
    uint32_t ctr[4] = {(uint32_t)k, tag, chain, 1u}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    double u = unit_open(out[0]);
    double a = s[k] + amplitude * (2.0 * u - 1.0);
    if (a > PI_D) a -= TWO_PI_D;
    else if (a <= -PI_D) a += TWO_PI_D;
    s[k] = a;
  }
}

/* ------------------------------------------------------------------------- */
/* Geometry G(s) by NeRF (Parsons et al., J. Comput. Chem. 26, 2005):
 * D is placed from A, B, C with |CD| = l, angle BCD = theta, dihedral ABCD = chi:
 * D = C + [bc, n x bc, n] (-l cos theta, l sin theta cos chi, l sin theta sin chi),
 * bc = unit(C - B), n = unit((B - A) x bc). */
static const double B_NCA = 1.458, B_CAC = 1.525, B_CN = 1.329, B_CACB = 1.53;
static const double A_NCAC = 111.2, A_CACN = 116.2, A_CNCA = 121.7, A_NCACB = 110.5;
static const double T_OMEGA = 180.0, T_CB = -122.5;

void oracle_geometry_constants(double *out) {
  out[0] = B_NCA; out[1] = B_CAC; out[2] = B_CN; out[3] = B_CACB;
  out[4] = A_NCAC; out[5] = A_CACN; out[6] = A_CNCA; out[7] = A_NCACB;
  out[8] = T_OMEGA; out[9] = T_CB;
}

/* Geometry G(s) by NeRF (Parsons et al., J. Comput. Chem. 26, 2005): place D from
 * A, B, C with |CD| = l, angle BCD = theta and dihedral ABCD = chi. */
static void place(const double *A, const double *B, const double *C, double l,
                  double theta_deg, double cchi, double schi, double *D) {
  double bc[3] = {C[0] - B[0], C[1] - B[1], C[2] - B[2]};
  double nb = sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  bc[0] /= nb; bc[1] /= nb; bc[2] /= nb;
  double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double n[3] = {ab[1] * bc[2] - ab[2] * bc[1], ab[2] * bc[0] - ab[0] * bc[2],
                 ab[0] * bc[1] - ab[1] * bc[0]};
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  n[0] /= nn; n[1] /= nn; n[2] /= nn;
  double m[3] = {n[1] * bc[2] - n[2] * bc[1], n[2] * bc[0] - n[0] * bc[2],
                 n[0] * bc[1] - n[1] * bc[0]};
  double th = theta_deg * DEG;
  double d0 = -l * cos(th), d1 = l * sin(th) * cchi, d2 = l * sin(th) * schi;
  for (int a = 0; a < 3; ++a) D[a] = C[a] + bc[a] * d0 + m[a] * d1 + n[a] * d2;
}

#define AT(atoms, c, a) ((atoms) + ((size_t)(c) * 4 + (a)) * 3)
enum { AN = 0, ACA = 1, AC = 2, ACB = 3 };

/* (Re)build residues from..to (inclusive); residues before `from` must already hold
 * G(s).  Residue 0 carries the fixed frame: N_0 at the origin, CA_0 on +x, C_0 in
 * the xy-plane.  Residue c+1's N, CA, C follow from residue c through psi_c,
 * omega and phi_{c+1}; C-beta_c from C_c, N_c, CA_c. */
static void nerf_range(int32_t L, const double *s, double *atoms, int32_t from, int32_t to) {
  if (to > L - 1) to = L - 1;
  for (int32_t c = from; c <= to; ++c) {
    if (c == 0) {
      double *N0 = AT(atoms, 0, AN), *CA0 = AT(atoms, 0, ACA), *C0 = AT(atoms, 0, AC);
      N0[0] = 0.0; N0[1] = 0.0; N0[2] = 0.0;
      CA0[0] = B_NCA; CA0[1] = 0.0; CA0[2] = 0.0;
      C0[0] = B_NCA - B_CAC * cos(A_NCAC * DEG);
      C0[1] = B_CAC * sin(A_NCAC * DEG);
      C0[2] = 0.0;
    } else {
      double psi = s[2 * (c - 1) + 1], phi = s[2 * c], om = T_OMEGA * DEG;
      place(AT(atoms, c - 1, AN), AT(atoms, c - 1, ACA), AT(atoms, c - 1, AC), B_CN, A_CACN,
            cos(psi), sin(psi), AT(atoms, c, AN));
      place(AT(atoms, c - 1, ACA), AT(atoms, c - 1, AC), AT(atoms, c, AN), B_NCA, A_CNCA,
            cos(om), sin(om), AT(atoms, c, ACA));
      place(AT(atoms, c - 1, AC), AT(atoms, c, AN), AT(atoms, c, ACA), B_CAC, A_NCAC, cos(phi),
            sin(phi), AT(atoms, c, AC));
    }
    place(AT(atoms, c, AC), AT(atoms, c, AN), AT(atoms, c, ACA), B_CACB, A_NCACB,
          cos(T_CB * DEG), sin(T_CB * DEG), AT(atoms, c, ACB));
  }
}

void oracle_nerf(int32_t L, const double *s, double *atoms) { nerf_range(L, s, atoms, 0, L - 1); }

/* ------------------------------------------------------------------------- */
/* Pair energy: -ln p interpolated by the uniform Catmull-Rom cubic through the
 * values at the bin centres; mirrored ghost values at both ends and constant
 * values outside the first and last knots. */
static void spline_stencil(const double *y, int32_t nb, double d_min, double bin_w, double d,
                           int *region, int *b, double *f, double *q) {
  double t = (d - (d_min + 0.5 * bin_w)) / bin_w;
  if (t <= 0.0) { *region = -1; return; }
  if (t >= (double)(nb - 1)) { *region = 1; return; }
  *region = 0;
  int bb = (int)floor(t);
  *b = bb;
  *f = t - (double)bb;
  q[0] = (bb == 0) ? y[1] : y[bb - 1];
  q[1] = y[bb];
  q[2] = y[bb + 1];
  q[3] = (bb + 2 <= nb - 1) ? y[bb + 2] : y[nb - 2];
}

double oracle_pair_energy(const double *y, int32_t nb, double d_min, double bin_w, double d) {
  int region, b;
  double f, q[4];
  spline_stencil(y, nb, d_min, bin_w, d, &region, &b, &f, q);
  if (region < 0) return y[0];
  if (region > 0) return y[nb - 1];
  double a0 = 2.0 * q[1];
  double a1 = -q[0] + q[2];
  double a2 = 2.0 * q[0] - 5.0 * q[1] + 4.0 * q[2] - q[3];
  double a3 = -q[0] + 3.0 * q[1] - 3.0 * q[2] + q[3];
  return 0.5 * (a0 + a1 * f + a2 * f * f + a3 * f * f * f);
}

double oracle_pair_energy_deriv(const double *y, int32_t nb, double d_min, double bin_w, double d) {
  int region, b;
  double f, q[4];
  spline_stencil(y, nb, d_min, bin_w, d, &region, &b, &f, q);
  if (region != 0) return 0.0;
  double a1 = -q[0] + q[2];
  double a2 = 2.0 * q[0] - 5.0 * q[1] + 4.0 * q[2] - q[3];
  double a3 = -q[0] + 3.0 * q[1] - 3.0 * q[2] + q[3];
  return 0.5 * (a1 + 2.0 * a2 * f + 3.0 * a3 * f * f) / bin_w;
}

static int64_t row_of(int32_t L, int32_t i, int32_t j) {
  return (int64_t)i * L - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

static double dist(const double *a, const double *b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

static double pair_E(const oracle_cfg *cfg, const double *y, const double *atoms, int32_t i,
                     int32_t j) {
  const double *row = y + row_of(cfg->L, i, j) * cfg->n_bins;
  return oracle_pair_energy(row, cfg->n_bins, cfg->d_min, cfg->bin_w,
                            dist(AT(atoms, i, ACB), AT(atoms, j, ACB)));
}

double oracle_neumaier_sum(int64_t n, const double *x) {
  double s = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = s + x[i];
    if (fabs(s) >= fabs(x[i]))
      c += (s - t) + x[i];
    else
      c += (x[i] - t) + s;
    s = t;
  }
  return s + c;
}

/* Neumaier sum of E_ij over lo <= i < j <= hi. */
static double energy_range(const oracle_cfg *cfg, const double *y, const double *atoms,
                           int32_t lo, int32_t hi) {
  double s = 0.0, c = 0.0;
  for (int32_t i = lo; i <= hi; ++i)
    for (int32_t j = i + 1; j <= hi; ++j) {
      double x = pair_E(cfg, y, atoms, i, j);
      double t = s + x;
      if (fabs(s) >= fabs(x))
        c += (s - t) + x;
      else
        c += (x - t) + s;
      s = t;
    }
  return s + c;
}

double oracle_energy_full(const oracle_cfg *cfg, const double *y, const double *atoms) {
  return energy_range(cfg, y, atoms, 0, cfg->L - 1);
}

static void window_of(const oracle_cfg *cfg, int32_t k, int32_t global, int32_t *lo, int32_t *hi) {
  int32_t c = k / 2, h = cfg->window_d / 2;
  if (global) { *lo = 0; *hi = cfg->L - 1; return; }
  *lo = c - h < 0 ? 0 : c - h;
  *hi = c + h > cfg->L - 1 ? cfg->L - 1 : c + h;
}

double oracle_energy_window(const oracle_cfg *cfg, const double *y, const double *atoms, int32_t k) {
  int32_t lo, hi;
  window_of(cfg, k, 0, &lo, &hi);
  return energy_range(cfg, y, atoms, lo, hi);
}

/* First moved residue when torsion k turns: phi_c moves C_c (hence CB_c) and
 * everything after; psi_c moves N_{c+1} and everything after. */
static int32_t pivot_of(int32_t k) { return (k % 2) ? k / 2 + 1 : k / 2; }

static double wrap_angle(double a) {
  if (a > PI_D) a -= TWO_PI_D;
  else if (a <= -PI_D) a += TWO_PI_D;
  return a;
}

/* dE between two conformations (atoms, atoms_t) for proposal k.  Brute mode
 * differences the windowed (or full) energies; incremental mode sums only the
 * pairs i < p <= j, the only ones whose distance changes (rigid motion of the
 * residues from the pivot on). */
static double delta_e_atoms(const oracle_cfg *cfg, const double *y, const double *atoms,
                            const double *atoms_t, int32_t k, int32_t global, int32_t mode,
                            double *S_out) {
  int32_t lo, hi, p = pivot_of(k);
  window_of(cfg, k, global, &lo, &hi);
  double dE = 0.0, S = 0.0;
  for (int32_t i = lo; i < p && i <= hi; ++i)
    for (int32_t j = p; j <= hi; ++j) {
      if (j <= i) continue;
      double e0 = pair_E(cfg, y, atoms, i, j), e1 = pair_E(cfg, y, atoms_t, i, j);
      dE += e1 - e0;
      S += fabs(e0) + fabs(e1);
    }
  if (mode == 0) dE = energy_range(cfg, y, atoms_t, lo, hi) - energy_range(cfg, y, atoms, lo, hi);
  if (S_out) *S_out = S;
  return dE;
}

double oracle_delta_e(const oracle_cfg *cfg, const double *y, const double *s, int32_t k,
                      double delta, int32_t global, int32_t mode, double *S_out) {
  int32_t L = cfg->L;
  double *sp = (double *)malloc(sizeof(double) * 2 * L);
  double *a0 = (double *)malloc(sizeof(double) * 12 * L);
  double *a1 = (double *)malloc(sizeof(double) * 12 * L);
  memcpy(sp, s, sizeof(double) * 2 * L);
  sp[k] = wrap_angle(s[k] + delta);
  oracle_nerf(L, s, a0);
  oracle_nerf(L, sp, a1);
  double dE = delta_e_atoms(cfg, y, a0, a1, k, global, mode, S_out);
  free(sp); free(a0); free(a1);
  return dE;
}

/* ------------------------------------------------------------------------- */
/* Gradient: turning torsion k by eps rotates residues p.. about the bond axis u
 * through point a, so dx_j/deps = u x (x_j - a) and
 * dV/ds_k = sum_{i<p<=j} E'_ij(d_ij) (x_j - x_i).(u x (x_j - a)) / d_ij. */
void oracle_grad(const oracle_cfg *cfg, const double *y, const double *s, double *V_out,
                 double *g) {
  int32_t L = cfg->L;
  double *at = (double *)malloc(sizeof(double) * 12 * L);
  oracle_nerf(L, s, at);
  if (V_out) *V_out = oracle_energy_full(cfg, y, at);
  for (int32_t k = 0; k < 2 * L; ++k) {
    int32_t c = k / 2, p = pivot_of(k);
    g[k] = 0.0;
    if (k == 0 || k == 2 * L - 1) continue; /* phi_0 and psi_{L-1} move nothing */
    const double *A = (k % 2) ? AT(at, c, ACA) : AT(at, c, AN);
    const double *B = (k % 2) ? AT(at, c, AC) : AT(at, c, ACA);
    double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    u[0] /= nu; u[1] /= nu; u[2] /= nu;
    double acc = 0.0;
    for (int32_t j = p; j < L; ++j) {
      const double *xj = AT(at, j, ACB);
      double r[3] = {xj[0] - A[0], xj[1] - A[1], xj[2] - A[2]};
      double v[3] = {u[1] * r[2] - u[2] * r[1], u[2] * r[0] - u[0] * r[2], u[0] * r[1] - u[1] * r[0]};
      for (int32_t i = 0; i < p; ++i) {
        const double *xi = AT(at, i, ACB);
        double e[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
        double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        const double *row = y + row_of(L, i, j) * cfg->n_bins;
        double dEdd = oracle_pair_energy_deriv(row, cfg->n_bins, cfg->d_min, cfg->bin_w, d);
        acc += dEdd * (e[0] * v[0] + e[1] * v[1] + e[2] * v[2]) / d;
      }
    }
    g[k] = acc;
  }
  free(at);
}

/* ------------------------------------------------------------------------- */
/* Chains. */
static int cfg_ok(const oracle_cfg *cfg) {
  return cfg && cfg->L >= 2 && cfg->n_bins >= 4 && cfg->bin_w > 0.0 && cfg->window_d >= 0 &&
         cfg->global_every >= 0 && cfg->anchor_every >= 1 && cfg->T0 > 0.0 && cfg->T1 > 0.0 &&
         cfg->n_global >= 0 && (cfg->global_every == 0 || cfg->n_global <= cfg->global_every) &&
         cfg->total_sweeps >= 1 && cfg->sigma >= 0.0 && cfg->sigma_end >= 0.0 &&
         cfg->n_cascade >= 0 && cfg->n_cascade <= 3 &&
         (cfg->n_cascade < 1 || cfg->cascade_d[0] >= 0) &&
         (cfg->n_cascade < 2 || cfg->cascade_d[1] >= 0) &&
         (cfg->n_cascade < 3 || cfg->cascade_d[2] >= 0);
}

void oracle_chain_init(const oracle_cfg *cfg, const double *y, int32_t n_chains,
                       const double *s, double *s_best, double *v) {
  int32_t L = cfg->L;
  double *at = (double *)malloc(sizeof(double) * 12 * L);
  for (int32_t c = 0; c < n_chains; ++c) {
    oracle_nerf(L, s + (size_t)c * 2 * L, at);
    double V = oracle_energy_full(cfg, y, at);
    v[2 * c] = V;
    v[2 * c + 1] = V;
    memcpy(s_best + (size_t)c * 2 * L, s + (size_t)c * 2 * L, sizeof(double) * 2 * L);
  }
  free(at);
}

static int64_t anchors_in(const oracle_cfg *cfg, int64_t t_begin, int64_t n) {
  int64_t A = cfg->anchor_every;
  return (t_begin + n) / A - t_begin / A;
}

/* Working state of one chain: `cur` holds G(s) for residues 0..valid (residues
 * past the end of a localized window are brought up to date when needed);
 * `trial` receives G(s') for the residues a proposal moves. */
typedef struct {
  int32_t L;
  double *s, *sp, *cur, *trial;
  int32_t valid;
} chain_ws;

static void ws_init(chain_ws *w, int32_t L, double *s) {
  w->L = L;
  w->s = s;
  w->sp = (double *)malloc(sizeof(double) * 2 * L);
  w->cur = (double *)malloc(sizeof(double) * 12 * L);
  w->trial = (double *)malloc(sizeof(double) * 12 * L);
  nerf_range(L, s, w->cur, 0, L - 1);
  w->valid = L - 1;
}

static void ws_free(chain_ws *w) { free(w->sp); free(w->cur); free(w->trial); }

static void ws_extend(chain_ws *w, int32_t upto) {
  if (upto > w->L - 1) upto = w->L - 1;
  if (upto > w->valid) { nerf_range(w->L, w->s, w->cur, w->valid + 1, upto); w->valid = upto; }
}

/* Evaluate proposal k: s'_k = wrap(s_k + delta), G(s') for the residues it moves
 * (up to the window end for a localized proposal), and dE over the changed pairs. */
static double ws_eval(const oracle_cfg *cfg, const double *y, chain_ws *w, int32_t k,
                      double delta, int32_t global, double *S, int32_t *last_out) {
  int32_t L = w->L, lo, hi, p = pivot_of(k);
  window_of(cfg, k, global, &lo, &hi);
  int32_t last = global ? L - 1 : hi;
  ws_extend(w, last);
  memcpy(w->sp, w->s, sizeof(double) * 2 * L);
  w->sp[k] = wrap_angle(w->s[k] + delta);
  int32_t from = p < 1 ? 0 : p - 1; /* seed residue for the rebuild */
  if (from > lo) from = lo;
  if (p > from)
    memcpy(AT(w->trial, from, 0), AT(w->cur, from, 0), sizeof(double) * 12 * (size_t)(p - from));
  nerf_range(L, w->sp, w->trial, p, last);
  *last_out = last;
  return delta_e_atoms(cfg, y, w->cur, w->trial, k, global, 1, S);
}

static void ws_accept(chain_ws *w, int32_t k, int32_t last) {
  int32_t p = pivot_of(k);
  w->s[k] = w->sp[k];
  if (p <= last)
    memcpy(AT(w->cur, p, 0), AT(w->trial, p, 0), sizeof(double) * 12 * (size_t)(last - p + 1));
  w->valid = last;
}

/* One chain through sweeps [t_begin, t_begin + n_sweeps) (Algorithm 1 with the
 * alternation schedule; acceptance by the MH equation). */
static void run_chain(const oracle_cfg *cfg, const double *y, uint32_t chain, int64_t t_begin,
                      int64_t n_sweeps, int32_t mode, double *s, double *s_best, double *v,
                      int64_t *cnt, double target, double *step_log, uint8_t *acc_log,
                      double *anchor_log) {
  int32_t L = cfg->L, n = 2 * L;
  chain_ws w;
  ws_init(&w, L, s);
  int64_t step = 0, ai = 0;
  for (int64_t t = t_begin; t < t_begin + n_sweeps; ++t) {
    int32_t global = oracle_is_global(cfg, t);
    double beta = oracle_beta(cfg, t), sigma = oracle_sigma(cfg, t);
    oracle_cfg ct = *cfg;               /* this sweep's localization radius */
    ct.window_d = oracle_window_d(cfg, t);
    for (int32_t k = 0; k < n; ++k, ++step) {
      double delta, log_u2, S;
      int32_t last;
      oracle_proposal(cfg->seed, chain, t, k, sigma, &delta, &log_u2);
      double dE;
      if (mode == 0) {
        /* brute force: both energies from full rebuilds of s and s' */
        dE = oracle_delta_e(&ct, y, s, k, delta, global, 0, &S);
        memcpy(w.sp, s, sizeof(double) * n);
        w.sp[k] = wrap_angle(s[k] + delta);
        last = L - 1;
      } else {
        dE = ws_eval(&ct, y, &w, k, delta, global, &S, &last);
      }
      int acc = (dE <= 0.0) || (log_u2 < -beta * dE);
      if (step_log) { step_log[2 * step] = dE; step_log[2 * step + 1] = delta; }
      if (acc_log) acc_log[step] = (uint8_t)acc;
      if (acc) {
        if (mode == 0) { s[k] = w.sp[k]; nerf_range(L, s, w.cur, 0, L - 1); w.valid = L - 1; }
        else ws_accept(&w, k, last);
        cnt[global ? 1 : 0] += 1;
      }
    }
    if (((t + 1) % cfg->anchor_every) == 0) {
      ws_extend(&w, L - 1);
      double V = oracle_energy_full(cfg, y, w.cur);
      v[0] = V;
      if (V < v[1]) { v[1] = V; memcpy(s_best, s, sizeof(double) * n); }
      if (cnt[2] < 0 && V <= target) cnt[2] = t + 1;
      cnt[3] += 1;
      if (anchor_log) anchor_log[ai] = V;
      ++ai;
    }
  }
  ws_free(&w);
}

int32_t oracle_run(const oracle_cfg *cfg, const double *y, int32_t n_chains,
                   const uint32_t *chain_ids, int64_t t_begin, int64_t n_sweeps,
                   int32_t mode, int32_t n_threads, double *s, double *s_best, double *v,
                   int64_t *counters, double target, double *step_log, uint8_t *acc_log,
                   double *anchor_log) {
  if (!cfg_ok(cfg) || n_chains < 1 || n_sweeps < 0 || t_begin < 0 || !y || !s || !s_best ||
      !v || !counters || t_begin + n_sweeps > 0xFFFFFFFFLL)
    return -1;
  int32_t n = 2 * cfg->L;
  int64_t steps = n_sweeps * n, na = anchors_in(cfg, t_begin, n_sweeps);
#ifdef _OPENMP
  if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
  for (int32_t c = 0; c < n_chains; ++c) {
    uint32_t id = chain_ids ? chain_ids[c] : (uint32_t)c;
    run_chain(cfg, y, id, t_begin, n_sweeps, mode, s + (size_t)c * n, s_best + (size_t)c * n,
              v + 2 * c, counters + 4 * c, target, step_log ? step_log + 2 * steps * c : NULL,
              acc_log ? acc_log + steps * c : NULL, anchor_log ? anchor_log + na * c : NULL);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Replay: step the oracle's own chain, compare each proposal with the device
 * trace (increment, dE, decision) and each anchor with the device's anchored
 * energy.  A decision that differs is accepted as a near-tie fork only when the
 * device's decision is the correct one for its own dE and that dE passed the
 * tolerance; the replay then continues on the device's branch. */
int32_t oracle_replay(const oracle_cfg *cfg, const double *y, uint32_t chain_id,
                      const double *s0, int64_t t_begin, int64_t n_sweeps,
                      const double *gpu_dE, const double *gpu_delta, const uint8_t *gpu_acc,
                      const double *gpu_anchor, double rel_tol, double abs_tol,
                      double anchor_rel_tol, double *s_out, oracle_replay_report *rep) {
  memset(rep, 0, sizeof(*rep));
  rep->first_fail_step = -1;
  if (!cfg_ok(cfg)) return -1;
  int32_t L = cfg->L, n = 2 * L;
  double *s = (double *)malloc(sizeof(double) * n);
  memcpy(s, s0, sizeof(double) * n);
  chain_ws w;
  ws_init(&w, L, s);
  int64_t step = 0, ai = 0;
  for (int64_t t = t_begin; t < t_begin + n_sweeps; ++t) {
    int32_t global = oracle_is_global(cfg, t);
    double beta = oracle_beta(cfg, t), sigma = oracle_sigma(cfg, t);
    oracle_cfg ct = *cfg;
    ct.window_d = oracle_window_d(cfg, t);
    for (int32_t k = 0; k < n; ++k, ++step) {
      double delta, log_u2, S;
      int32_t last;
      oracle_proposal(cfg->seed, chain_id, t, k, sigma, &delta, &log_u2);
      double dE = ws_eval(&ct, y, &w, k, delta, global, &S, &last);
      int acc_or = (dE <= 0.0) || (log_u2 < -beta * dE);
      int acc_g = gpu_acc[step] ? 1 : 0;
      double dg = gpu_dE[step];
      int fail = 0;
      if (fabs(gpu_delta[step] - delta) > 1e-12 * (1.0 + fabs(delta))) { rep->n_delta_fail++; fail = 1; }
      double err = fabs(dg - dE);
      if (!(err <= rel_tol * S + abs_tol)) { rep->n_de_fail++; fail = 1; }
      if (err > rep->max_de_abs_err) rep->max_de_abs_err = err;
      if (S > 0.0 && err / S > rep->max_de_rel_err) rep->max_de_rel_err = err / S;
      /* the device's decision must follow from its own dE (up to FP64 rounding of the threshold) */
      int acc_own = (dg <= 0.0) || (log_u2 < -beta * dg);
      double m_own = log_u2 + beta * dg;
      if (acc_own != acc_g && !(dg > 0.0 && fabs(m_own) <= 1e-12 * (1.0 + fabs(log_u2)))) {
        rep->n_logic_fail++;
        fail = 1;
      }
      if (acc_g != acc_or) {
        rep->n_forks++;
        double m = fabs(log_u2 + beta * dE);
        if (m > rep->max_fork_margin) rep->max_fork_margin = m;
      }
      if (fail && rep->first_fail_step < 0) rep->first_fail_step = step;
      if (acc_g) ws_accept(&w, k, last);
    }
    if (((t + 1) % cfg->anchor_every) == 0) {
      ws_extend(&w, L - 1);
      double V = oracle_energy_full(cfg, y, w.cur);
      if (gpu_anchor) {
        double e = fabs(gpu_anchor[ai] - V) / (fabs(V) > 1e-300 ? fabs(V) : 1.0);
        if (e > rep->max_anchor_rel_err) rep->max_anchor_rel_err = e;
        if (!(e <= anchor_rel_tol)) {
          rep->n_anchor_fail++;
          if (rep->first_fail_step < 0) rep->first_fail_step = step;
        }
      }
      ++ai;
    }
  }
  rep->n_steps = step;
  rep->n_anchors = ai;
  if (s_out) memcpy(s_out, s, sizeof(double) * n);
  ws_free(&w);
  free(s);
  return (rep->first_fail_step < 0) ? 0 : 1;
}

/* ------------------------------------------------------------------------- */
/* Limited-memory BFGS (Liu and Nocedal 1989) with a backtracking Armijo line
 * search whose reference value is the largest of the last M accepted values
 * (the nonmonotone rule of Grippo, Lampariello and Lucidi 1986; M = 1 is the
 * monotone rule).  The paper pairs its sampler with a nonmonotone Armijo
 * L-BFGS (Sec. 3, the L-BFGS columns of Fig. 3); the exact rules used here are
 * the ones written below. */

static double dotn(int32_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Two-loop recursion: d = -H g, with H the inverse-Hessian approximation built
 * from H0 = gamma I by the BFGS update with the k stored pairs, oldest first
 * (pairs i = 0 .. k-1 in S[i*n..], Y[i*n..], oldest at 0). */
void oracle_lbfgs_direction(int32_t n, int32_t k, const double *S, const double *Y,
                            const double *g, double gamma, double *d) {
  double *a = (double *)malloc(sizeof(double) * (k > 0 ? k : 1));
  for (int32_t e = 0; e < n; ++e) d[e] = g[e];
  for (int32_t i = k - 1; i >= 0; --i) {
    const double *s = S + (size_t)i * n, *y = Y + (size_t)i * n;
    double rho = 1.0 / dotn(n, y, s);
    a[i] = rho * dotn(n, s, d);
    for (int32_t e = 0; e < n; ++e) d[e] -= a[i] * y[e];
  }
  for (int32_t e = 0; e < n; ++e) d[e] *= gamma;
  for (int32_t i = 0; i < k; ++i) {
    const double *s = S + (size_t)i * n, *y = Y + (size_t)i * n;
    double rho = 1.0 / dotn(n, y, s);
    double b = rho * dotn(n, y, d);
    for (int32_t e = 0; e < n; ++e) d[e] += (a[i] - b) * s[e];
  }
  for (int32_t e = 0; e < n; ++e) d[e] = -d[e];
  free(a);
}

static double max_abs(int32_t n, const double *v) {
  double m = 0.0;
  for (int32_t i = 0; i < n; ++i)
    if (fabs(v[i]) > m) m = fabs(v[i]);
  return m;
}

int32_t oracle_lbfgs(int32_t n, double *x, const oracle_lbfgs_opts *o, oracle_fg_fn fg, void *ctx,
                     double *f_out, int32_t *iters_out, double *f_trace, double *x_trace) {
  if (n < 1 || !o || o->m < 1 || o->nonmonotone < 1 || o->max_ls < 1 || o->n_iter < 0) return -1;
  const int32_t m = o->m, M = o->nonmonotone;
  double *g = (double *)malloc(sizeof(double) * n), *d = (double *)malloc(sizeof(double) * n);
  double *xn = (double *)malloc(sizeof(double) * n), *gn = (double *)malloc(sizeof(double) * n);
  double *S = (double *)malloc(sizeof(double) * (size_t)m * n);
  double *Y = (double *)malloc(sizeof(double) * (size_t)m * n);
  double *fh = (double *)malloc(sizeof(double) * M);
  double f;
  fg(ctx, x, &f, g);
  if (f_trace) f_trace[0] = f;
  if (x_trace) memcpy(x_trace, x, sizeof(double) * n);
  int32_t k = 0, nf = 1, it = 0, status = 1;
  fh[0] = f;
  for (it = 0; it < o->n_iter; ++it) {
    double gmax = max_abs(n, g);
    if (gmax <= o->gtol) { status = 0; break; }
    /* search direction */
    double gamma = o->step0 / gmax;
    if (k > 0) {
      const double *s = S + (size_t)(k - 1) * n, *y = Y + (size_t)(k - 1) * n;
      gamma = dotn(n, s, y) / dotn(n, y, y);
    }
    oracle_lbfgs_direction(n, k, S, Y, g, gamma, d);
    double gd = dotn(n, g, d);
    if (!(gd < 0.0)) { /* not a descent direction: drop the history, scaled steepest descent */
      k = 0;
      gamma = o->step0 / gmax;
      for (int32_t e = 0; e < n; ++e) d[e] = -gamma * g[e];
      gd = dotn(n, g, d);
    }
    /* Armijo backtracking against the largest of the last M accepted values */
    double fref = fh[0];
    for (int32_t i = 1; i < (nf < M ? nf : M); ++i)
      if (fh[i] > fref) fref = fh[i];
    double alpha = 1.0, fnew = 0.0;
    int32_t ok = 0;
    for (int32_t ls = 0; ls < o->max_ls; ++ls) {
      for (int32_t e = 0; e < n; ++e) xn[e] = x[e] + alpha * d[e];
      fg(ctx, xn, &fnew, gn);
      if (fnew <= fref + o->c1 * alpha * gd) { ok = 1; break; }
      alpha *= o->shrink;
    }
    if (!ok) { status = 2; break; }
    /* curvature pair s = xn - x, y = gn - g, kept only when s.y is clearly positive;
     * with a full history the oldest pair makes room */
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int32_t e = 0; e < n; ++e) {
      double se = xn[e] - x[e], ye = gn[e] - g[e];
      sy += se * ye; ss += se * se; yy += ye * ye;
    }
    if (sy > 1e-8 * sqrt(ss * yy)) {
      if (k == m) {
        memmove(S, S + n, sizeof(double) * (size_t)(m - 1) * n);
        memmove(Y, Y + n, sizeof(double) * (size_t)(m - 1) * n);
        --k;
      }
      for (int32_t e = 0; e < n; ++e) {
        S[(size_t)k * n + e] = xn[e] - x[e];
        Y[(size_t)k * n + e] = gn[e] - g[e];
      }
      ++k;
    }
    memcpy(x, xn, sizeof(double) * n);
    memcpy(g, gn, sizeof(double) * n);
    f = fnew;
    fh[nf % M] = f;
    ++nf;
    if (f_trace) f_trace[it + 1] = f;
    if (x_trace) memcpy(x_trace + (size_t)(it + 1) * n, x, sizeof(double) * n);
  }
  if (f_out) *f_out = f;
  if (iters_out) *iters_out = it;
  free(g); free(d); free(xn); free(gn); free(S); free(Y); free(fh);
  return status;
}

typedef struct {
  const oracle_cfg *cfg;
  const double *y;
} protein_fg_ctx;

static void protein_fg(void *ctx, const double *x, double *f, double *g) {
  const protein_fg_ctx *p = (const protein_fg_ctx *)ctx;
  oracle_grad(p->cfg, p->y, x, f, g);
}

int32_t oracle_lbfgs_protein(const oracle_cfg *cfg, const double *y, double *s,
                             const oracle_lbfgs_opts *o, double *V_out, int32_t *iters_out,
                             double *f_trace, double *x_trace) {
  if (!cfg || cfg->L < 2) return -1;
  protein_fg_ctx p = {cfg, y};
  int32_t st = oracle_lbfgs(2 * cfg->L, s, o, protein_fg, &p, V_out, iters_out, f_trace, x_trace);
  for (int32_t k = 0; k < 2 * cfg->L; ++k) s[k] = wrap_angle(s[k]);
  return st;
}

/* Step-by-step check of a device L-BFGS run: X [n_it + 1][n] are the device's
 * iterates.  For each k the oracle rebuilds its own state at X[k] (values and
 * gradients at the device's iterates, curvature pairs from consecutive iterates,
 * the same storage and reset rules), takes one iteration (direction and line
 * search) and compares its step with X[k+1] - X[k]:
 *   |dx_dev - dx_or|_inf <= step_tol |dx_or|_inf,
 * or, if the device stopped its line search at another trial, the Armijo test
 * that separates the two trials must be a near-tie (|f - threshold| <= tie_tol
 * (|f_ref| + 1)), counted as a fork.  The replay always continues from X[k+1]. */
int32_t oracle_lbfgs_replay(const oracle_cfg *cfg, const double *y, int32_t n_it, const double *X,
                            const oracle_lbfgs_opts *o, double step_tol, double tie_tol,
                            oracle_lbfgs_replay_report *rep) {
  if (!cfg || !o || !X || !rep || n_it < 0 || o->m < 1 || o->nonmonotone < 1 || o->max_ls < 1) return -1;
  const int32_t n = 2 * cfg->L, m = o->m, M = o->nonmonotone;
  memset(rep, 0, sizeof(*rep));
  rep->first_fail = -1;
  double *g = (double *)malloc(sizeof(double) * n), *gn = (double *)malloc(sizeof(double) * n);
  double *d = (double *)malloc(sizeof(double) * n), *xt = (double *)malloc(sizeof(double) * n);
  double *gt = (double *)malloc(sizeof(double) * n);
  double *S = (double *)malloc(sizeof(double) * (size_t)m * n);
  double *Y = (double *)malloc(sizeof(double) * (size_t)m * n);
  double *fh = (double *)malloc(sizeof(double) * M);
  double *fl = (double *)malloc(sizeof(double) * o->max_ls);
  double f, fn;
  oracle_grad(cfg, y, X, &f, g);
  fh[0] = f;
  int32_t k = 0, nf = 1;
  for (int32_t it = 0; it < n_it; ++it) {
    const double *x = X + (size_t)it * n, *xn = X + (size_t)(it + 1) * n;
    double gmax = max_abs(n, g);
    double gamma = o->step0 / gmax;
    if (k > 0) gamma = dotn(n, S + (size_t)(k - 1) * n, Y + (size_t)(k - 1) * n) /
                       dotn(n, Y + (size_t)(k - 1) * n, Y + (size_t)(k - 1) * n);
    oracle_lbfgs_direction(n, k, S, Y, g, gamma, d);
    double gd = dotn(n, g, d);
    if (!(gd < 0.0)) {
      k = 0;
      gamma = o->step0 / gmax;
      for (int32_t e = 0; e < n; ++e) d[e] = -gamma * g[e];
      gd = dotn(n, g, d);
    }
    double fref = fh[0];
    for (int32_t i = 1; i < (nf < M ? nf : M); ++i)
      if (fh[i] > fref) fref = fh[i];
    /* the oracle's line search, keeping every trial's Armijo margin */
    int32_t j_or = -1;
    double alpha = 1.0;
    for (int32_t j = 0; j < o->max_ls; ++j) {
      for (int32_t e = 0; e < n; ++e) xt[e] = x[e] + alpha * d[e];
      oracle_grad(cfg, y, xt, &fl[j], gt);
      fl[j] -= fref + o->c1 * alpha * gd;   /* margin: accepted iff <= 0 */
      if (fl[j] <= 0.0) { j_or = j; break; }
      alpha *= o->shrink;
    }
    /* which trial did the device take? */
    double dnorm = max_abs(n, d), best = INFINITY;
    int32_t j_dev = -1;
    double a = 1.0;
    for (int32_t j = 0; j < o->max_ls; ++j, a *= o->shrink) {
      double e_max = 0.0;
      for (int32_t e = 0; e < n; ++e) {
        double q = fabs((xn[e] - x[e]) - a * d[e]);
        if (q > e_max) e_max = q;
      }
      double rel = e_max / (a * dnorm > 0.0 ? a * dnorm : 1.0);
      if (rel < best) { best = rel; j_dev = j; }
    }
    int32_t bad = 0;
    if (j_dev == j_or) {
      if (best > rep->max_step_err) rep->max_step_err = best;
      if (!(best <= step_tol)) bad = 1;
    } else if (j_or < 0 || j_dev < 0 || best > step_tol) {
      bad = 1;
    } else {
      /* the first trial where the two searches disagree must be a near-tie */
      int32_t jm = j_dev < j_or ? j_dev : j_or;
      if (fabs(fl[jm]) <= tie_tol * (fabs(fref) + 1.0)) rep->n_forks++;
      else bad = 1;
    }
    if (bad) {
      rep->n_fail++;
      if (rep->first_fail < 0) rep->first_fail = it;
    }
    /* continue from the device's iterate */
    oracle_grad(cfg, y, xn, &fn, gn);
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int32_t e = 0; e < n; ++e) {
      double se = xn[e] - x[e], ye = gn[e] - g[e];
      sy += se * ye; ss += se * se; yy += ye * ye;
    }
    if (sy > 1e-8 * sqrt(ss * yy)) {
      if (k == m) {
        memmove(S, S + n, sizeof(double) * (size_t)(m - 1) * n);
        memmove(Y, Y + n, sizeof(double) * (size_t)(m - 1) * n);
        --k;
      }
      for (int32_t e = 0; e < n; ++e) {
        S[(size_t)k * n + e] = xn[e] - x[e];
        Y[(size_t)k * n + e] = gn[e] - g[e];
      }
      ++k;
    }
    memcpy(g, gn, sizeof(double) * n);
    f = fn;
    fh[nf % M] = f;
    ++nf;
    rep->n_steps++;
  }
  free(g); free(gn); free(d); free(xt); free(gt); free(S); free(Y); free(fh); free(fl);
  return rep->n_fail ? 1 : 0;
}
