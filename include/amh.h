/*
 * amh.h -- C ABI of libamh.so, the MI355X (gfx950) implementation of the
 * Alternating Metropolis-Hastings (AMH) sampler of Ghantasala, Jaiswal and Datta,
 * "An Efficient MCMC Approach to Energy Function Optimization in Protein
 * Structure Prediction" (arXiv 2211.03193).
 *
 * The calls follow the paper's problem statement: torsions in (the state vector
 * s of Sec. 2.1, s[2c] = phi_c, s[2c+1] = psi_c), distogram tables in (the
 * -log P(|x_i - x_j|) terms of the AlphaFold1 energy, Sec. 2.3), energies and
 * conformations out (minimum energies per run, Sec. 2.3 and Fig. 3).
 *
 * Conventions for every call:
 *   - pointers named *_dev are device pointers (HIP global memory) owned by the
 *     caller; the library never frees them;
 *   - work is enqueued on the stream given to amh_init (or to the call) and is
 *     ordered with it; outputs are valid once the stream has reached the call;
 *   - units: radians, Angstrom, energies in nats; beta = 1/T multiplies V;
 *   - every function returns an amh_status and never aborts; on failure
 *     amh_last_error() returns a message (thread-local);
 *   - an amh_ctx must not be used by two host threads at once.
 */
#ifndef AMH_H
#define AMH_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMH_OK = 0,
  AMH_E_INVAL = -1,       /* invalid argument or configuration (nothing was enqueued) */
  AMH_E_NOMEM = -2,       /* device allocation failed */
  AMH_E_DEVICE = -3,      /* HIP runtime error */
  AMH_E_NUMERIC = -4,     /* non-finite table entry, energy or energy change */
  AMH_E_UNSUPPORTED = -5, /* call not provided by this build */
  AMH_E_BUSY = -6         /* request cannot be admitted now (serving) */
} amh_status;

typedef struct amh_ctx amh_ctx;

/* Run configuration.  Every field is validated on the host by amh_init before any
 * device work; an invalid field returns AMH_E_INVAL. */
typedef struct {
  int32_t L;              /* residues, 2 <= L <= 1024; n = 2L torsions */
  int32_t n_chains;       /* independent chains C >= 1 (Sec. 2.4, inter-block parallelism) */
  int32_t n_bins;         /* distogram bins, 4 <= n_bins <= 64; the last is no-contact */
  int32_t window_d;       /* localization radius d >= 0: V_local sums pairs with both
                             residues in [k/2 - d/2, k/2 + d/2] (local energy, Sec. 2.3) */
  double d_min;           /* left edge of bin 0 (A); knot b sits at d_min + bin_w (b + 1/2) */
  double bin_w;           /* bin width (A) > 0 */
  int32_t global_every;   /* sweep t is a global-MH sweep iff global_every > 0 and
                             (t+1) % global_every == 0, otherwise localized (Algorithm 1) */
  int32_t anchor_every;   /* anchors (FP64 energy, best state) after sweep t iff
                             (t+1) % anchor_every == 0; >= 1 */
  double sigma;           /* proposal standard deviation (rad) >= 0 (Sec. 2.3: 10 deg) */
  double T0, T1;          /* temperature T_t = T0 (T1/T0)^(t/(S-1)), both > 0 */
  int64_t total_sweeps;   /* S >= 1, defines the schedule; amh_sweep may run it in pieces */
  uint64_t seed;          /* Philox4x32-10 key (low word, high word) */
  uint32_t chain_offset;  /* global id of chain 0: chain c draws from counter (k, t, offset+c, 0) */
  int32_t chains_per_group; /* chains that share one workgroup, 0 = choose (1, 2 or 4) */
  int32_t waves_per_group;  /* wavefronts per workgroup (<= 8), 0 = choose; >= chains_per_group */
  int32_t reserved;
} amh_config;

/* Create a sampler.
 *   y_dev  [P][n_bins] float32, P = L(L-1)/2, row r(i,j) = i*L - i(i+1)/2 + (j-i-1)
 *          for i < j, entry b = -ln p_ij(bin b).  Copied (repacked) into the context;
 *          the caller may free it once the stream has passed amh_init.
 *   s0_dev [C][2L] float64 starting torsions (rad), or NULL for the extended chain
 *          s = pi everywhere (Algorithm 1 input).
 *   stream hipStream_t to order all work of the context on (NULL = default stream).
 * Returns AMH_E_INVAL for a bad configuration (no device work), AMH_E_NUMERIC when
 * the table holds a non-finite entry (after one stream synchronisation). */
amh_status amh_init(const amh_config* cfg, const float* y_dev, const double* s0_dev,
                    void* stream, amh_ctx** out);

/* Advance every chain by n_sweeps >= 0 sweeps of 2L single-torsion proposals,
 * local or global by the schedule (Algorithm 1), asynchronously on the context
 * stream.  Fails with AMH_E_INVAL if the run would pass total_sweeps. */
amh_status amh_sweep(amh_ctx* ctx, int64_t n_sweeps);

/* Energies of conformations, accumulated in float64 (Neumaier):
 *   s_in_dev != NULL: V of B conformations s_in_dev [B][2L];
 *   s_in_dev == NULL: V of the context's chains (B must equal n_chains), which = 0
 *                     for the current state, 1 for the best state seen at anchors.
 * Outputs (any may be NULL): V_out_dev [B], s_out_dev [B][2L] (the torsions used),
 * cb_out_dev [B][L][3] float32 C-beta coordinates G(s). */
amh_status amh_energy(amh_ctx* ctx, const double* s_in_dev, int32_t B, int32_t which,
                      double* V_out_dev, double* s_out_dev, float* cb_out_dev);

/* Stateless geometry x = G(s) (Sec. 2.1): atoms_out_dev [B][L][4][3] float32 holds
 * N, CA, C, C-beta of every residue for s_dev [B][2L] float64. */
amh_status amh_conformation(const double* s_dev, int32_t B, int32_t L, float* atoms_out_dev,
                            void* stream);

/* Checkpoint / resume.  amh_get_state copies the context state out (any pointer may
 * be NULL): s [C][2L], s_best [C][2L], v [C][2] = (V at last anchor, best V),
 * counters [C][4] = (local accepts, global accepts, sweeps to target or -1,
 * anchors), atoms [C][L][4][3] float64 (N, CA, C, C-beta) and the
 * host sweep counter *t_out.  amh_set_state loads it back; with atoms_dev given,
 * continuing from a restored state reproduces the uninterrupted run bit for bit;
 * with atoms_dev NULL the coordinates are rebuilt from s (exact at anchor sweeps,
 * where the sampler rebuilds them too). */
amh_status amh_get_state(amh_ctx* ctx, double* s_dev, double* s_best_dev, double* v_dev,
                         int64_t* counters_dev, double* atoms_dev, int64_t* t_out);
amh_status amh_set_state(amh_ctx* ctx, const double* s_dev, const double* s_best_dev,
                         const double* v_dev, const int64_t* counters_dev,
                         const double* atoms_dev, int64_t t);

/* Time-to-target: the first anchor with V <= target records its sweep count in
 * counters[c][2] (default target: -infinity, never reached). */
amh_status amh_set_target(amh_ctx* ctx, double target);

/* Per-proposal trace of up to 4 chains (parity checks).  From the next amh_sweep
 * on, proposal k of sweep t of traced chain slot m is written at index
 * (t - t_first) * 2L + k of dE_dev [4][capacity], delta_dev [4][capacity]
 * (float64) and acc_dev [4][capacity] (uint8), and its anchors at
 * anchor_dev [4][anchor_capacity]; records past a capacity are dropped.
 * chain_ids[m] = -1 disables slot m.  n = 0 turns tracing off. */
amh_status amh_set_trace(amh_ctx* ctx, int32_t n, const int32_t* chain_ids, double* dE_dev,
                         double* delta_dev, uint8_t* acc_dev, int64_t capacity,
                         double* anchor_dev, int64_t anchor_capacity);

/* Philox4x32-10 blocks, the counter-based generator behind every proposal (Sec. 2.4
 * names an RNG per chain; this build draws proposal k of sweep t of chain c from
 * the counter (k, t, c, 0)): out_dev[i][0..3] = Philox(ctr_dev[i][0..3], key) for
 * n blocks of four uint32 words; key low word first. */
amh_status amh_philox(const uint32_t* ctr_dev, int64_t n, uint64_t key, uint32_t* out_dev,
                      void* stream);

/* Synchronise the context stream and report asynchronous numeric errors
 * (AMH_E_NUMERIC) raised by earlier calls. */
amh_status amh_poll(amh_ctx* ctx);

/* Launch shape chosen for the sweep kernel and the current sweep index. */
amh_status amh_info(amh_ctx* ctx, int32_t* chains_per_group, int32_t* waves_per_group,
                    int32_t* lds_bytes, int64_t* t);

/* Gradient dV/ds of B conformations (the adjoint of G and the spline energy). */
amh_status amh_grad(amh_ctx* ctx, const double* s_dev, int32_t B, double* V_out_dev,
                    double* g_out_dev);

/* Serving: admit a folding job into a running server (continuous batching). */
amh_status amh_submit(void* server, const void* job, uint64_t* job_id);

amh_status amh_destroy(amh_ctx* ctx);
const char* amh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
