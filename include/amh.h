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
  AMH_E_UNSUPPORTED = -5, /* call or option not provided by this library version */
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
  int32_t global_every;   /* cycle length: sweep t is a global-MH sweep iff global_every > 0
                             and t % global_every >= global_every - n_global, otherwise
                             localized (Algorithm 1's alternation, localized first) */
  int32_t anchor_every;   /* anchors (FP64 energy, best state) after sweep t iff
                             (t+1) % anchor_every == 0; >= 1 */
  double sigma;           /* proposal standard deviation (rad) >= 0 (Sec. 2.3: 10 deg) */
  double T0, T1;          /* temperature T_t = T0 (T1/T0)^(t/(S-1)), both > 0 */
  int64_t total_sweeps;   /* S >= 1, defines the schedule; amh_sweep may run it in pieces */
  uint64_t seed;          /* Philox4x32-10 key (low word, high word) */
  uint32_t chain_offset;  /* global id of chain 0: chain c draws from counter (k, t, offset+c, 0) */
  int32_t chains_per_group; /* chains that share one workgroup, 0 = choose (1, 2 or 4) */
  int32_t waves_per_group;  /* wavefronts per workgroup (<= 8), >= chains_per_group; 0 = choose:
                               8 when the grid has at most one workgroup per compute unit,
                               else 2 * chains_per_group (at least 4) */
  int32_t n_global;       /* global sweeps per cycle, 0..global_every (0 means 1) */
  double sigma_end;       /* > 0: the proposal width decays geometrically from sigma to
                             sigma_end over the schedule (Sec. 2.3, Sec. 3: 10 to 4 deg);
                             0 = constant sigma */
  int32_t n_cascade;      /* extra localization radii, 0..3 (Sec. 2.2: cascaded ranges): */
  int32_t cascade_d[3];   /* localized sweep t uses window_d if t % (1 + n_cascade) == 0,
                             else cascade_d[t % (1 + n_cascade) - 1] (each >= 0) */
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

/* Noisy restart (the second scheme of Sec. 3 adds a uniform draw in [-10, 10] degrees
 * to every torsion): every torsion of every chain moves by amplitude (2u - 1), u from
 * Philox at counter (k, tag, chain_offset + c, 1) with the context's key, and is
 * wrapped into (-pi, pi]; the coordinates are rebuilt, the current V re-anchored in
 * float64, and the best state replaced where V is lower.  Counters and the sweep
 * index are kept.  amplitude >= 0 (rad); use a new tag for every restart. */
amh_status amh_perturb(amh_ctx* ctx, double amplitude, uint32_t tag);

/* Bound on the wait of a pipelined localized sweep for the previous sweep's progress
 * (1 <= polls <= 2^24, the default; each poll sleeps ~128 cycles).  A wait that runs
 * out gives up instead of hanging, flags the context, and the next amh_poll returns
 * AMH_E_DEVICE; the chains' state is then undefined.  For testing the error path. */
amh_status amh_set_wait_bound(amh_ctx* ctx, int32_t polls);

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
 * names an RNG per chain; proposal k of sweep t of chain c is drawn from
 * the counter (k, t, c, 0)): out_dev[i][0..3] = Philox(ctr_dev[i][0..3], key) for
 * n blocks of four uint32 words; key low word first. */
amh_status amh_philox(const uint32_t* ctr_dev, int64_t n, uint64_t key, uint32_t* out_dev,
                      void* stream);

/* Executed work of the global sweeps (the pair sums of the full energy, Sec. 2.3,
 * evaluated as in Sec. 2.4: pair distances first, energies only where they count).
 * counters_dev: int64[3] on the device, owned by the caller, or NULL to stop
 * counting.  Every later amh_sweep adds, at the end of its launch:
 *   [0] tiles of 8 x 8 residue pairs of the changed-pair rectangle that survive the
 *       bounding-sphere test (the others hold only pairs beyond the last knot),
 *   [1] pair distances tested inside the rectangle in those tiles,
 *   [2] near pairs whose energy was evaluated (one 16-byte stencil each).
 * The rest of the work is fixed by the schedule (localized pairs, candidate tiles,
 * transitions, anchors) and needs no counting.  Stream-ordered like amh_sweep. */
amh_status amh_set_work_counters(amh_ctx* ctx, int64_t* counters_dev);

/* Synchronise the context stream and report asynchronous numeric errors
 * (AMH_E_NUMERIC) raised by earlier calls. */
amh_status amh_poll(amh_ctx* ctx);

/* Launch shape chosen for the context (chains and wavefronts per workgroup and LDS
 * bytes of a launch that runs any sweeps: the batched launches' own-shape plan) and
 * the current sweep index.  amh_sweep runs a range of sweeps as one launch per run of
 * consecutive sweeps of one kind, localized or global; amh_info_launches gives their
 * shapes. */
amh_status amh_info(amh_ctx* ctx, int32_t* chains_per_group, int32_t* waves_per_group,
                    int32_t* lds_bytes, int64_t* t);

/* Launch shapes of amh_sweep's localized-sweep launches (consecutive localized sweeps
 * of a workgroup's chains are pipelined over its wavefronts) and global-sweep
 * launches: chains and wavefronts per workgroup and LDS bytes.  Any output pointer
 * may be NULL. */
amh_status amh_info_launches(amh_ctx* ctx, int32_t* local_chains_per_group, int32_t* local_waves_per_group,
                             int32_t* local_lds_bytes, int32_t* global_chains_per_group,
                             int32_t* global_waves_per_group, int32_t* global_lds_bytes);

/* Energy and gradient dV/ds of B conformations, in float64 (the distogram energy
 * of Sec. 2.3 through the geometry G(s) of Sec. 2.1; the paper minimises the same
 * energy with L-BFGS, Sec. 3).  Turning torsion k moves the residues from its pivot
 * on rigidly about the bond axis, so dV/ds_k = u_k . sum_{j >= p} (x_j - a_k) x F_j
 * with F_j = dV/dx_j (C-beta forces); dV/ds is zero for phi_0 and psi_{L-1}.
 *   s_dev      [B][2L] torsions, or NULL for the context's current chains (B must
 *              equal n_chains);
 *   V_out_dev  [B] or NULL;  g_out_dev [B][2L] or NULL (not both NULL).
 * The results are reproducible bit for bit (the forces are summed as integer
 * multiples of 2^-44).  A conformation with a non-finite torsion, or whose pair forces
 * add up to 2^13 or more within one block of 64 x 64 residue pairs, gets V = NaN (its
 * g is then unspecified).  Non-finite energies raise AMH_E_NUMERIC at the next
 * amh_poll. */
amh_status amh_grad(amh_ctx* ctx, const double* s_dev, int32_t B, double* V_out_dev,
                    double* g_out_dev);

/* Options of amh_minimize (all validated on the host; AMH_E_INVAL otherwise). */
typedef struct {
  int32_t n_iter;       /* accepted iterations at most, >= 0 */
  int32_t m;            /* curvature pairs kept, 1 .. 64 */
  int32_t nonmonotone;  /* M, 1 .. 64: a trial step is accepted iff
                           V(s + a d) <= max(last M accepted V) + c1 a g.d (M = 1: monotone) */
  int32_t max_ls;       /* trial steps a = 1, shrink, shrink^2, ... per iteration, >= 1 */
  double c1;            /* Armijo constant in (0, 1) */
  double shrink;        /* backtracking factor in (0, 1) */
  double gtol;          /* stop once max |dV/ds| <= gtol (>= 0) */
  double step0;         /* with no curvature pair the direction is -(step0 / max|g|) g (> 0, rad) */
} amh_lbfgs_opts;

/* L-BFGS minimisation of V(s) (Liu and Nocedal 1989, two-loop recursion) with a
 * nonmonotone Armijo backtracking line search (Grippo, Lampariello and Lucidi 1986),
 * the minimiser the paper pairs with its sampler (Sec. 3, Fig. 3).  A curvature pair
 * (s, y) is kept iff s.y > 1e-8 |s| |y|; a direction with g.d >= 0 drops the history.
 * One workgroup per conformation; a float64 workspace of B (5 + 2m) 2L doubles is
 * allocated by the context on first use (and grown, after a stream synchronisation).
 *   s_dev          [B][2L] in/out, or NULL for the context's current chains (B must
 *                  equal n_chains): then the chains' current V, best V / best state and
 *                  coordinates are updated, so sampling can continue from the minimum;
 *   V_out_dev      [B] final V or NULL;  iters_out_dev [B] accepted iterations or NULL;
 *   status_out_dev [B] or NULL: 0 gradient below gtol, 1 iteration limit, 2 line
 *                  search failed (the last accepted point is returned);
 *   f_trace_dev    [B][n_iter + 1] or NULL: V at the start and after each accepted
 *                  iteration (entries past the last iteration are left untouched);
 *   x_trace_dev    [B][n_iter + 1][2L] or NULL: the iterates themselves (not wrapped),
 *                  likewise; for step-by-step checks.
 * Torsions are returned wrapped into (-pi, pi]. */
amh_status amh_minimize(amh_ctx* ctx, double* s_dev, int32_t B, const amh_lbfgs_opts* opts,
                        double* V_out_dev, int32_t* iters_out_dev, int32_t* status_out_dev,
                        double* f_trace_dev, double* x_trace_dev);

/* amh_minimize for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels
 * and results, but the float64 workspace is the library's fixed scratch array
 * (8 Mi doubles = 64 MiB per device, held from the library's load until the process
 * ends; its device address is looked up once per device by amh_init).  The call
 * allocates nothing and calls no allocating routine.
 *   Arguments, layouts and outputs are those of amh_minimize.
 *   B (5 + 2m) 2L must not exceed 8,388,608 (e.g. B <= 499 at L = 400, m = 8),
 *   else AMH_E_INVAL and nothing is launched.
 * Every call on one device shares that device's scratch array (the workspace is
 * written before it is read, so no clearing is needed): calls that overlap on one
 * GPU (two streams, two host threads, or two contexts) race and give undefined
 * results; order them on one stream or synchronise between them. */
amh_status amh_minimize_noalloc(amh_ctx* ctx, double* s_dev, int32_t B,
                                const amh_lbfgs_opts* opts, double* V_out_dev,
                                int32_t* iters_out_dev, int32_t* status_out_dev,
                                double* f_trace_dev, double* x_trace_dev);

/* ---- Serving: a continuous-batching request loop --------------------------------
 * Folding jobs (one protein each) are queued by amh_submit and admitted in arrival
 * order while a slot is free and the device memory they need fits the budget.
 * Each amh_server_step advances every admitted job by sweeps_per_round sweeps in
 * shared batched launches (jobs of different lengths side by side), reads back each
 * job's counters, retires jobs that reached their target energy or their last sweep
 * (keeping a host copy of the best state) and admits waiting jobs into the freed
 * memory.  Chain state stays on the device between steps.  A job's sweeps do not
 * depend on the other jobs in its launches: its result is the same alone and in the
 * mix.  One host thread drives a server. */
typedef struct amh_server amh_server;

typedef struct {
  int64_t hbm_budget_bytes; /* device bytes admitted jobs may hold (tables + chain state) */
  int32_t max_active;       /* admitted jobs at most (1 = one job at a time, in order) */
  int32_t sweeps_per_round; /* R >= 1: sweeps per job per amh_server_step (see below) */
  int32_t plan;             /* launch plan of the shared launches, 0..5 (see amh_batch_tune) */
  int32_t reserved;
  int64_t round_pairs;      /* 0: every job advances R sweeps per step.  > 0: a job whose R
                               sweeps cost P pair evaluations (all its chains) advances
                               R * clamp(round_pairs / P, 1, 64) sweeps, so small jobs
                               keep pace with large ones in the shared launches.  The
                               count depends only on the job and these options. */
} amh_server_opts;

/* Optional per-proposal trace of one chain of a served job: the server hands it to
 * amh_set_trace when it admits the job, so the trace covers the job's sweeps from
 * the first.  The device buffers are the caller's and must stay valid until the job
 * is done; layouts and capacities as in amh_set_trace (one chain). */
typedef struct {
  int32_t chain;          /* chain of the job to trace, 0 <= chain < n_chains */
  int32_t reserved;
  double* dE_dev;         /* [capacity] */
  double* delta_dev;      /* [capacity] */
  uint8_t* acc_dev;       /* [capacity] */
  int64_t capacity;       /* proposals, >= 1 */
  double* anchor_dev;     /* [anchor_capacity] or NULL */
  int64_t anchor_capacity;
} amh_job_trace;

typedef struct {
  amh_config cfg;        /* the job's run, with its own seed (Philox key) */
  const float* y_host;   /* [L(L-1)/2][n_bins] -ln p in host memory, copied by amh_submit */
  double target;         /* the job ends at the first anchor where a chain has V <= target */
  const amh_job_trace* trace;   /* NULL, or a trace request (copied by amh_submit) */
} amh_job;

typedef struct {
  int32_t state;            /* 0 waiting, 1 admitted, 2 done, 3 failed */
  int32_t reached;          /* 1 once a chain reached the target */
  int64_t sweeps;           /* sweeps run so far */
  int64_t sweeps_to_target; /* smallest sweep count at which a chain reached it, or -1 */
  double best_V;            /* lowest anchored energy over the chains (after a step) */
  double t_submit, t_admit, t_target, t_done; /* seconds, steady clock; -1 until they happen */
  int64_t bytes;            /* device bytes the job holds while admitted (budget accounting) */
} amh_job_status;

/* Create a server whose work is ordered on `stream` (a hipStream_t, NULL = default). */
amh_status amh_server_create(const amh_server_opts* opts, void* stream, amh_server** out);

/* Queue a job (job points to an amh_job); *job_id receives its handle.  The table is
 * copied: the caller may free y_host on return.  AMH_E_BUSY if the job alone needs
 * more than the whole budget; AMH_E_INVAL for an invalid job. */
amh_status amh_submit(void* server, const void* job, uint64_t* job_id);

/* One round: admit, advance every admitted job, retire finished ones.  Synchronises
 * the stream once per round (to read the jobs' counters back). */
amh_status amh_server_step(amh_server* server, int32_t* n_active, int32_t* n_pending);

/* Status of a job; s_best_host [C][2L] (done jobs only) and v_host [C][2] = (V at the
 * last anchor, best V) per chain may be NULL. */
amh_status amh_server_job(amh_server* server, uint64_t job_id, amh_job_status* out,
                          double* s_best_host, double* v_host);

/* Synchronise and free the server and every job it holds. */
amh_status amh_server_destroy(amh_server* server);

/* ---- Batches: many proteins (contexts of different L) in one launch ----------
 * The chains of every member context are independent (Sec. 2.4, inter-block
 * parallelism), so one launch can advance the chains of several proteins: each
 * workgroup runs one chain group of one member, with the LDS of the launch sized
 * for its longest member and the grid ordered by decreasing work per workgroup.
 * Members with different launch shapes (chains per workgroup, wavefronts) are
 * advanced by one launch per shape.  Trajectories do not depend on the launch
 * shape or on the batch: a member advanced in a batch follows exactly the sweeps
 * it would follow alone (same Philox counters, same arithmetic). */
typedef struct amh_batch amh_batch;

/* Group n >= 1 distinct contexts created on one stream.  The batch borrows them:
 * they stay owned by the caller, must outlive the batch, and remain usable alone
 * (amh_energy, amh_get_state, ...). */
amh_status amh_batch_create(amh_ctx* const* ctxs, int32_t n, amh_batch** out);

/* Advance every member by n_sweeps >= 0 sweeps (each member's own schedule from its
 * own sweep counter); AMH_E_INVAL if any member would pass its total_sweeps. */
amh_status amh_batch_sweep(amh_batch* batch, int64_t n_sweeps);

/* The same with a sweep count per member (n_sweeps [n members], host array, each >= 0):
 * member i advances n_sweeps[i] sweeps in the same launches (a member with 0 sweeps
 * only passes through).  AMH_E_INVAL, with nothing advanced, if any member would pass
 * its total_sweeps. */
amh_status amh_batch_sweep_each(amh_batch* batch, const int64_t* n_sweeps);

/* Autotuner: time each launch plan on sweeps_per_trial real sweeps of every member
 * (they count as part of the run: 6 * sweeps_per_trial sweeps in all), keep the
 * fastest.  Plans: 0 = each context's own shape; 1..5 = (chains per workgroup,
 * wavefronts) of (1,4), (2,4), (2,8), (4,4), (4,8), with fewer chains per workgroup
 * for members whose length does not fit the LDS.  ms_out [6] (or NULL) receives the
 * time of each trial, *plan_out (or NULL) the plan kept. */
amh_status amh_batch_tune(amh_batch* batch, int64_t sweeps_per_trial, float* ms_out,
                          int32_t* plan_out);

/* Select a launch plan (0..5, as above) without timing. */
amh_status amh_batch_set_plan(amh_batch* batch, int32_t plan);

/* Current plan, number of launches per sweep call and total workgroups. */
amh_status amh_batch_info(const amh_batch* batch, int32_t* plan, int32_t* n_launches,
                          int32_t* workgroups);

/* Synchronise the stream and free the batch (not its members). */
amh_status amh_batch_destroy(amh_batch* batch);

amh_status amh_destroy(amh_ctx* ctx);
const char* amh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
