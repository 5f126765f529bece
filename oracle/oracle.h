/*
 * oracle.h -- FP64 CPU oracle for Alternating Metropolis-Hastings (AMH).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * HIP path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product library never does.
 * It shares no code, header or constant table with the HIP path.
 *
 * Conventions (all in double precision):
 *   - state s[2L]: s[2c] = phi_c, s[2c+1] = psi_c, radians, wrapped to (-pi, pi]
 *     (Sec. 2.1, the mapping of Fig. 2);
 *   - atoms[L][4][3]: N, CA, C, CB of each residue, Angstrom;
 *   - distogram table y[P][n_bins] = -ln p, packed i<j rows,
 *     row r(i,j) = i*L - i*(i+1)/2 + (j-i-1)  (Eq. of the AlphaFold1 energy);
 *   - energies in nats; beta multiplies V.
 */
#ifndef AMH_ORACLE_H
#define AMH_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t L;            /* residues, >= 2 */
  int32_t n_bins;       /* distogram bins, >= 4; last bin is no-contact */
  double d_min;         /* left edge of bin 0 (A) */
  double bin_w;         /* bin width (A); knot b at d_min + bin_w*(b+0.5) */
  int32_t window_d;     /* localization radius d; window half-width h = d/2 residues */
  int32_t global_every; /* cycle length; sweep t is global iff global_every > 0 and
                           t % global_every >= global_every - n_global */
  int32_t anchor_every; /* anchors after sweep t iff (t+1)%anchor_every==0; >= 1 */
  int32_t n_global;     /* global sweeps per cycle (the last n_global of every
                           global_every sweeps); 0 means 1 */
  double sigma;         /* proposal standard deviation (rad) */
  double T0, T1;        /* geometric temperature schedule over total_sweeps */
  int64_t total_sweeps; /* S */
  uint64_t seed;        /* Philox key */
  double sigma_end;     /* > 0: proposal width decays geometrically to sigma_end over S */
  int32_t n_cascade;    /* extra localization radii taken in turn with window_d, 0..3 */
  int32_t cascade_d[3]; /* sweep t uses radius r = t % (1 + n_cascade): 0 window_d, else cascade_d[r-1] */
} oracle_cfg;

typedef struct {
  int64_t n_steps;          /* proposals replayed */
  int64_t n_forks;          /* decisions that differ at a certified near-tie */
  int64_t n_de_fail;        /* |dE_gpu - dE_or| above tolerance */
  int64_t n_delta_fail;     /* proposal increments that differ */
  int64_t n_logic_fail;     /* GPU decision inconsistent with its own dE */
  int64_t first_fail_step;  /* -1 if none */
  int64_t n_anchors;
  int64_t n_anchor_fail;
  double max_de_abs_err;
  double max_de_rel_err;    /* |dE_gpu - dE_or| / S_or */
  double max_anchor_rel_err;
  double max_fork_margin;   /* largest |ln u2 + beta dE_or| among forks (diagnostic) */
} oracle_replay_report;

/* Philox4x32-10 (Salmon et al., SC'11): one block. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oracle_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out);

/* Proposal increment (Box-Muller, cosine branch) and log of the acceptance uniform
 * for proposal k of sweep t of chain `chain`. */
void oracle_proposal(uint64_t seed, uint32_t chain, int64_t t, int32_t k, double sigma,
                     double *delta, double *log_u2);

double oracle_beta(const oracle_cfg *cfg, int64_t t);
int32_t oracle_is_global(const oracle_cfg *cfg, int64_t t);
double oracle_sigma(const oracle_cfg *cfg, int64_t t);
int32_t oracle_window_d(const oracle_cfg *cfg, int64_t t);
/* Noisy restart: s_k += amplitude (2u - 1), u from Philox at (k, tag, chain, 1), wrapped. */
void oracle_perturb(uint64_t seed, uint32_t chain, uint32_t tag, double amplitude, int32_t n,
                    double *s);

/* Geometry G(s): NeRF chain of ideal backbone + virtual C-beta. */
void oracle_nerf(int32_t L, const double *s, double *atoms);
void oracle_geometry_constants(double *out /* [10] */);

/* Pair energy E_ij(d): Catmull-Rom over -ln p at the bin centres. */
double oracle_pair_energy(const double *y_row, int32_t n_bins, double d_min, double bin_w, double d);
double oracle_pair_energy_deriv(const double *y_row, int32_t n_bins, double d_min, double bin_w, double d);

/* Energies of a conformation: V (all i<j, Neumaier sum) and V_local(x, k, d). */
double oracle_energy_full(const oracle_cfg *cfg, const double *y, const double *atoms);
double oracle_energy_window(const oracle_cfg *cfg, const double *y, const double *atoms, int32_t k);
/* Neumaier (compensated) sum of n doubles. */
double oracle_neumaier_sum(int64_t n, const double *x);

/* dE of setting s_k <- wrap(s_k + delta); mode 0 = brute (whole window/all pairs),
 * 1 = incremental (changed pairs only).  S_out (may be NULL) receives the sum of
 * |E_old| + |E_new| over the changed pairs. */
double oracle_delta_e(const oracle_cfg *cfg, const double *y, const double *s, int32_t k,
                      double delta, int32_t global, int32_t mode, double *S_out);

/* Gradient of V with respect to s (analytic, by the rotation argument). */
void oracle_grad(const oracle_cfg *cfg, const double *y, const double *s, double *V_out, double *g);

/* L-BFGS with a (nonmonotone) Armijo backtracking line search.
 *   n_iter       accepted iterations at most;  m  stored curvature pairs (>= 1);
 *   nonmonotone  M >= 1: trial accepted iff f(x + a d) <= max(last M accepted f) + c1 a g.d;
 *   max_ls       trials per line search (a = 1, shrink, shrink^2, ...);
 *   gtol         stop when max|g| <= gtol;
 *   step0        with no stored pair the direction is -(step0 / max|g|) g.
 * A curvature pair (s, y) is stored iff s.y > 1e-8 |s| |y|; a direction with g.d >= 0
 * drops the history.  Returns 0 (gtol reached), 1 (iteration limit), 2 (line search
 * failed; x is the last accepted point) or -1 (invalid options). */
typedef struct {
  int32_t n_iter, m, nonmonotone, max_ls;
  double c1, shrink, gtol, step0;
} oracle_lbfgs_opts;

typedef void (*oracle_fg_fn)(void *ctx, const double *x, double *f, double *g);

/* d = -H g by the two-loop recursion over k pairs (oldest first) from H0 = gamma I. */
void oracle_lbfgs_direction(int32_t n, int32_t k, const double *S, const double *Y,
                            const double *g, double gamma, double *d);
/* Minimise fg from x (in/out).  f_trace [n_iter + 1] and x_trace [n_iter + 1][n] (or
 * NULL) receive f and x at the start and after each accepted iteration. */
int32_t oracle_lbfgs(int32_t n, double *x, const oracle_lbfgs_opts *o, oracle_fg_fn fg, void *ctx,
                     double *f_out, int32_t *iters_out, double *f_trace, double *x_trace);
/* Minimise V(s) of a protein; s is wrapped into (-pi, pi] on return (x_trace is not). */
int32_t oracle_lbfgs_protein(const oracle_cfg *cfg, const double *y, double *s,
                             const oracle_lbfgs_opts *o, double *V_out, int32_t *iters_out,
                             double *f_trace, double *x_trace);

/* Step-by-step check of a device L-BFGS run from its iterates X [n_it + 1][2L]
 * (see oracle.c): returns 0 if every step matches, 1 otherwise, -1 on bad input. */
typedef struct {
  int64_t n_steps;     /* iterations checked */
  int64_t n_forks;     /* line searches that stopped at another trial at a near-tie */
  int64_t n_fail;      /* steps that differ beyond step_tol and are not forks */
  int64_t first_fail;  /* -1 if none */
  double max_step_err; /* max |dx_dev - dx_or|_inf / |dx_or|_inf over matched steps */
} oracle_lbfgs_replay_report;
int32_t oracle_lbfgs_replay(const oracle_cfg *cfg, const double *y, int32_t n_it, const double *X,
                            const oracle_lbfgs_opts *o, double step_tol, double tie_tol,
                            oracle_lbfgs_replay_report *rep);

/* Initialise chain state: v[2c] = v[2c+1] = V(s0_c), s_best = s. */
void oracle_chain_init(const oracle_cfg *cfg, const double *y, int32_t n_chains,
                       const double *s, double *s_best, double *v);

/* Run sweeps [t_begin, t_begin+n_sweeps) for n_chains chains.
 *   s, s_best   [C][2L] in/out;  v [C][2] in/out = (V at last anchor, best V);
 *   counters    [C][4]  in/out = (local accepts, global accepts, first sweep with
 *                                 anchored V <= target or -1, anchors);
 *   step_log    [C][n_sweeps*2L][2] (dE, delta) or NULL;  acc_log [C][n_sweeps*2L] or NULL;
 *   anchor_log  [C][n_anchor_in_range] or NULL.
 * Returns 0, or -1 on invalid input. */
int32_t oracle_run(const oracle_cfg *cfg, const double *y, int32_t n_chains,
                   const uint32_t *chain_ids, int64_t t_begin, int64_t n_sweeps,
                   int32_t mode, int32_t n_threads, double *s, double *s_best, double *v,
                   int64_t *counters, double target, double *step_log, uint8_t *acc_log,
                   double *anchor_log);

/* Replay one traced chain against a device trace (see oracle_replay_report). */
int32_t oracle_replay(const oracle_cfg *cfg, const double *y, uint32_t chain_id,
                      const double *s0, int64_t t_begin, int64_t n_sweeps,
                      const double *gpu_dE, const double *gpu_delta, const uint8_t *gpu_acc,
                      const double *gpu_anchor, double rel_tol, double abs_tol,
                      double anchor_rel_tol, double *s_out, oracle_replay_report *rep);

#ifdef __cplusplus
}
#endif
#endif
