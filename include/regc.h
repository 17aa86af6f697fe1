/*
 * regc.h -- C ABI of libregc_hip.so: replica-exchange grand-canonical (REGC)
 * Metropolis sampling of a Lennard-Jones gas on a frozen LJ slab, and multistate
 * reweighting of the samples, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Zhou, Scheffler, Ghiringhelli, "Determining Surface Phase Diagrams
 * Including Anharmonic Effects", arXiv:1908.11118.  The problem statement the
 * interface follows (Sec. I and Sec. IV): the inputs are the potential energy
 * function and the T and mu ranges; the outputs are per-state samples, partition
 * function estimates (free energies), phase probabilities and the phase map.
 *
 * Conventions
 *  - Reduced LJ units, k_B = 1, beta = 1/T.  Thermal wavelength
 *    Lambda(T) = lambda1 / sqrt(T) (Sec. II.A.1, Eq. (1)), so the activity of
 *    state s is ln z_s = beta_s mu_s - 3 ln Lambda(T_s).
 *  - State grid: state s = l * n_mu + m for temperature T[l] and chemical
 *    potential mu[m] (Sec. II.A.2, the L x M extended ensemble).
 *  - A walker w is one configuration slot; label[w] is the state it currently
 *    samples.  Replica exchange permutes labels, never coordinates.
 *  - Every pointer argument is a HOST pointer unless its name ends in _dev.
 *    Inputs are read during the call and copied; the caller keeps ownership.
 *    Output buffers are allocated by the caller.  The context owns all device
 *    memory it allocates and frees it in regc_destroy.
 *  - Every function returns REGC_OK (0) or a negative error code; nothing is
 *    thrown across the ABI.  regc_last_error() gives a thread-local message
 *    for the last failure on the calling thread.
 *  - Work is enqueued on the context's stream (regc_set_stream; default: the
 *    null stream).  Functions that return data to the host synchronise that
 *    stream first.  Calls on one context must not overlap.
 */
#ifndef REGC_H
#define REGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define REGC_OK 0
#define REGC_EINVAL (-1)       /* bad sizes or parameters (see each function) */
#define REGC_ENOMEM (-2)       /* device or host allocation failed */
#define REGC_EHIP (-3)         /* a HIP runtime call failed; message has hipGetErrorString */
#define REGC_ECAPACITY (-4)    /* sample or trace buffer too small; nothing was run */
#define REGC_ESTATE (-5)       /* call made in the wrong order */
#define REGC_EUNSUPPORTED (-6) /* option or combination of options not supported */
#define REGC_ENOCONV (-7)      /* reweighting did not converge; last iterate returned */

/* ---- enumerations --------------------------------------------------------- */
#define REGC_MODE_LJ 0     /* LJ gas on a frozen LJ slab */
#define REGC_MODE_IDEAL 1  /* no interactions (epsilon = 0): ideal gas */

#define REGC_FP64 0        /* all arithmetic in FP64 (trajectory-parity mode) */
#define REGC_FP32PAIR 1    /* coordinates, trial positions and pair terms in FP32; energies,
                              decisions, swaps in FP64 */

/* per-state counters returned by regc_get_stats, REGC_NSTAT per state */
#define REGC_NSTAT 10
#define REGC_ST_DISP_ATT 0
#define REGC_ST_DISP_ACC 1
#define REGC_ST_INS_ATT 2
#define REGC_ST_INS_ACC 3
#define REGC_ST_DEL_ATT 4
#define REGC_ST_DEL_ACC 5
#define REGC_ST_CAP_REJ 6    /* insertion attempted at N = n_max */
#define REGC_ST_EMPTY_REJ 7  /* displacement or removal attempted at N = 0 */
#define REGC_ST_WALL_REJ 8   /* displacement left the gas region in z */
#define REGC_ST_CORE_REJ 9   /* new pair closer than hc_frac * sigma */

/* ---- problem description -------------------------------------------------- */
/* Pair potential (Appendix): phi(r) = 4 eps [(sig/r)^12 - (sig/r)^6], truncated
 * at rcut and, when shifted != 0, shifted by -phi(rcut).  gg: gas-gas,
 * gs: gas-slab.  The frozen slab atoms do not interact with each other
 * (Sec. III.A).  A trial that creates a pair closer than hc_frac * sigma is
 * rejected without evaluating exp (exact whenever beta*phi(hc_frac*sigma)
 * exceeds ~745 plus the largest attraction, e.g. hc_frac = 0.5, eps = 1, T <= 2). */
typedef struct {
    double eps_gg, sig_gg, eps_gs, sig_gs;
    double rcut;
    double hc_frac;
    int shifted;
    int mode;            /* REGC_MODE_* */
} regc_potential;

/* Surface and gas region.  slab_xyz: n_slab x 3 doubles (x, y, z), copied at
 * create.  Gas region [0,lx) x [0,ly) x [z_lo, z_hi], periodic in x and y,
 * hard walls in z (Sec. III.A: insertion zone above the topmost surface atoms).
 * lx and ly must be at least 2*rcut (minimum image).  n_max caps N. */
typedef struct {
    int n_slab;
    const double *slab_xyz;
    double lx, ly, z_lo, z_hi;
    double lambda1;
    int n_max;
} regc_system;

/* Explicit grid values: T[n_t] > 0, mu[n_mu]. */
typedef struct {
    int n_t, n_mu;
    const double *t, *mu;
} regc_grid;

/* Schedule and implementation options.
 *  seed            Philox4x32-10 key (low word, high word).
 *  precision       REGC_FP64 or REGC_FP32PAIR.
 *  p_disp, p_ins   move mix; removal gets 1 - p_disp - p_ins.  p_ins must equal
 *                  the removal probability (detailed balance, Sec. II.A.1).
 *  max_disp        half-width of the cubic displacement (Sec. II.A.3).
 *  trials_per_sweep  K trials per sweep, independent of the state; 0 -> n_max+1.
 *  swap_every      replica-exchange step after every swap_every sweeps (0: never).
 *  sample_every    record (E, N, state) of all walkers every sample_every sweeps
 *                  (0: never), before that sweep's exchange step.
 *  swap_scheme     0: even/odd T pairs and even/odd mu pairs; 1: T, mu and the two
 *                  diagonals inside 2x2 blocks (four types, p = 1/4 each, Sec. II.A.2)
 *                  whose origin (ol, om) in {0,1}^2 is drawn per exchange step (bits
 *                  29 and 28 of the type word), so blocks of both tilings alternate.
 *  sample_capacity samples the context can hold (records x walkers); 0 -> enough
 *                  for 1024 records.
 *  trace_capacity  sweeps of accept-bit trace the context can hold (0: no trace).
 *  walkers_per_block  waves (one walker each) per workgroup, 1..8; 0 -> auto.
 *  sweeps_per_launch  upper bound of sweeps per kernel launch; 0 -> swap_every.
 *  slab_bins       -1 off, 1 on, 0 auto: slab atoms sorted into x-y columns no
 *                  narrower than rcut + max_disp; each trial scans the 3x3 block of columns.
 *  split           wavefronts per walker: 1, 2, 4, or 0 (auto: 2 when the sweep schedule
 *                  runs at most 4 walkers per compute unit and walkers_per_block is 0,
 *                  else 1); above 1, walkers_per_block is 1 and the waves share each
 *                  trial's candidates.
 *  cull            1: squared distances first, LJ terms only for pairs inside the
 *                  cutoff (compacted in LDS); 0 or -1: every candidate in full.
 *  graph_intervals 0: launch kernels one by one; R > 0: capture R exchange intervals
 *                  (sweep launches, exchange, sweep-clock advance) in a hipGraph once
 *                  and replay it; the run is split into an eager prefix up to the next
 *                  exchange boundary, whole replays, and an eager remainder.  In graph
 *                  mode regc_timing_get's sweep figures cover whole replays.
 *  schedule        0: the sweeps above.  1: the paper's REGC step (Sec. II.A; the unit
 *                  of regc_run, sample_every and the trace becomes the step): a coin
 *                  (Philox block (0, step, 0xFFFFFFFF, 6), open uniform of word 0)
 *                  below x0 gives every walker one particle-exchange attempt (trial 0:
 *                  removal when A0 < 2^31, else insertion), otherwise the step is the
 *                  replica-exchange step `step`; then every walker makes mc_cycles
 *                  cycles of N displacement attempts (trials 1 .. mc_cycles N, N after
 *                  trial 0).  p_disp, p_ins, trials_per_sweep and swap_every are not
 *                  used.  Single-class contexts, no graph replay, no learned proposal.
 *  x0              probability of the particle-exchange attempt (schedule 1).
 *  mc_cycles       MC cycles after each attempt (schedule 1).
 *  md_steps        schedule 1: > 0 replaces the MC cycles by md_steps velocity-Verlet
 *                  steps (unit mass) of every walker: forces of the truncated-shifted
 *                  LJ energy, positions wrapped in x, y and reflected at the z walls,
 *                  then the stochastic velocity-rescaling thermostat (Bussi, Donadio,
 *                  Parrinello 2007; R1 from Philox block (1 + s, step, walker, 2), the
 *                  chi-square part from blocks (1 + s, step, walker, 16 + b)).  Missing
 *                  velocities (new context, regc_set_walkers, regc_restore) are drawn
 *                  from the Maxwell-Boltzmann law at the state's T at the next step
 *                  (particle i: block (2^31 + i, step, walker, 4)); an inserted
 *                  particle's from block (0, step, walker, 3); after an exchange the
 *                  velocities are scaled by sqrt(T_new / T_old).  Normals by Box-Muller.
 *  md_dt, md_tau   time step and thermostat time constant (0: no thermostat).
 *  resync_every    sweep schedule without the learned proposal: after every
 *                  resync_every-th sweep (before its sample) each walker's running
 *                  energy is replaced by its full recomputation in the context's
 *                  precision (pair terms in FP32 or FP64, sums in FP64), so the FP32
 *                  pair mode's accumulated rounding never grows; 0: default (100 in
 *                  REGC_FP32PAIR, never in REGC_FP64, whose running sums match the
 *                  oracle's), -1: never.
 *  batch_trials    sweep schedule without the learned proposal: 2 or 4 evaluates that
 *                  many consecutive trials of a walker at once (one wavefront per walker,
 *                  64 / batch_trials lanes per trial, or with split equal to batch_trials
 *                  one wavefront per trial) on the configuration at the start
 *                  of the batch, then decides them in order, correcting each trial's
 *                  energy change by its pair terms with the moves accepted before it in
 *                  the batch and leaving to the next batch a trial whose particle index
 *                  or particle an earlier accepted move changed: the accept/reject
 *                  sequence and configurations are those of one trial at a time.  1: one
 *                  trial at a time (split and cull apply).  0: 1.
 *  slab_cell       width of the slab's x-y columns as a multiple (>= 1) of the
 *                  smallest one, rcut + max_disp (0: 1): wider columns hold more atoms
 *                  each and fewer per block, the tuner's cell-size choice.
 *  persistent      R > 0: up to R whole exchange intervals per kernel launch, the
 *                  exchange steps inside the launch between grid-wide barriers (a
 *                  cooperative launch: every workgroup resident at once, else
 *                  EUNSUPPORTED); sweep schedule only, without graph replay, cull,
 *                  batched trials, the learned proposal, observables or minima
 *                  (those runs use separate launches).  0: off.  The accept/reject
 *                  sequence is that of separate launches.
 *  balance         one-trial sweep kernel: 1: before every sweep launch a small kernel
 *                  orders each class's walkers by their current particle count and deals
 *                  them round-robin to the class's workgroups, so that every workgroup
 *                  holds walkers of all costs and the compute units finish together
 *                  (classes whose walker count is not a multiple of the walkers per
 *                  workgroup keep their order); -1: walkers in index order; 0 (default):
 *                  1 when there are more than four walkers per compute unit, else -1.
 *                  Which wave runs a walker does not change its trials or results. */
typedef struct {
    uint64_t seed;
    int precision;
    double p_disp, p_ins, max_disp;
    int trials_per_sweep;
    int swap_every, sample_every, swap_scheme;
    int64_t sample_capacity;
    int64_t trace_capacity;
    int walkers_per_block;
    int sweeps_per_launch;
    int slab_bins;
    int split;
    int cull;
    int graph_intervals;
    int schedule;
    double x0;
    int mc_cycles;
    int md_steps;
    double md_dt, md_tau;
    int resync_every;
    int batch_trials;
    double slab_cell;
    int persistent;
    int balance;
} regc_opts;

typedef struct regc_ctx regc_ctx;
typedef struct regc_mbar regc_mbar;

/* ---- sampling --------------------------------------------------------------- */
/* Fills *o with the defaults named above (seed 1, FP64, 0.5/0.25/0.2, ...). */
void regc_default_opts(regc_opts *o);

/* Creates a context for one REGC simulation on the current HIP device: all
 * walkers start empty (N = 0, E = 0) with label[w] = w (a reading; the paper
 * does not state the initial state).  EINVAL on bad sizes, T <= 0, a T or mu
 * that is not finite, lx or ly below 2 rcut, p_ins != removal probability,
 * z_hi <= z_lo.
 * EUNSUPPORTED for an unknown mode or precision. */
int regc_create(const regc_potential *pot, const regc_system *sys, const regc_grid *grid,
                const regc_opts *opts, regc_ctx **out);

/* Uneven batch: n_class independent REGC simulations (own slab, box, n_max and
 * grid each; shared potential and options) advanced by the same kernel launches.
 * Walkers of class c follow those of class c-1; exchanges stay within a class;
 * samples are stored per class.  Class c, walker w of that class is global
 * walker offset_c + w (see regc_get_layout). */
int regc_create_batch(int n_class, const regc_potential *pot, const regc_system *sys,
                      const regc_grid *grid, const regc_opts *opts, regc_ctx **out);

/* n_class, and for each class its first global walker and its walker count. */
int regc_get_layout(const regc_ctx *ctx, int *n_class, int *offsets, int *counts);

/* Work of this context goes to stream (a hipStream_t, e.g. torch's current
 * stream handle); NULL selects the null stream. */
int regc_set_stream(regc_ctx *ctx, void *stream);

/* Advances every walker by n_sweeps sweeps (Sec. II.A: GC insertion/removal and
 * displacement trials, then replica exchange every swap_every sweeps).  Returns
 * after enqueueing; ECAPACITY (and runs nothing) when the samples or trace of
 * these sweeps would not fit. */
int regc_run(regc_ctx *ctx, int64_t n_sweeps);

/* Waits for all enqueued work of the context. */
int regc_sync(regc_ctx *ctx);

/* Global sweep counter (sweeps done since create or restore). */
int regc_get_sweep(const regc_ctx *ctx, int64_t *sweep);

/* Walker state: n[W], e[W] (running FP64 total energy), label[W]; xyz may be
 * NULL, else W x n_max x 3 doubles (rows beyond n[w] are zero). */
int regc_get_walkers(regc_ctx *ctx, int32_t *n, double *e, int32_t *label, double *xyz);

/* Replaces all walker configurations: n[W], xyz W x n_max x 3.  Energies are
 * recomputed on the device in the context's precision.  label may be NULL
 * (unchanged); otherwise it must be a permutation within each class.  EINVAL,
 * before anything changes, for an N outside 0..n_max, a particle outside the
 * gas region (or not finite), or labels that are not such a permutation. */
int regc_set_walkers(regc_ctx *ctx, const int32_t *n, const double *xyz, const int32_t *label);

/* Full recomputation of every walker's energy from its coordinates in the
 * context's precision (pairs in FP32 or FP64, sums in FP64): e_out[W]. */
int regc_energies(regc_ctx *ctx, double *e_out);

/* Number of samples held (records x walkers of all classes). */
int regc_sample_count(const regc_ctx *ctx, int64_t *count);

/* Copies up to cap samples in record order (each record lists all walkers in
 * walker order): e (FP64 energy), n (particle count), state (label at record
 * time, within the class).  *n_out receives the number copied. */
int regc_get_samples(regc_ctx *ctx, double *e, int32_t *n, int32_t *state, int64_t cap,
                     int64_t *n_out);

/* Device addresses of the sample arrays (valid until destroy or clear). */
int regc_samples_device(regc_ctx *ctx, const double **e_dev, const int32_t **n_dev,
                        const int32_t **state_dev, int64_t *count);

/* Drops all stored samples and histograms (the sweep counter is kept). */
int regc_clear_samples(regc_ctx *ctx);

/* stats: S_total x REGC_NSTAT counters by state; swap_att/swap_acc: 4 x S_total
 * attempts/acceptances by swap type and lower state of the pair.  S_total is the
 * total number of states (sum over classes); any pointer may be NULL. */
int regc_get_stats(regc_ctx *ctx, int64_t *stats, int64_t *swap_att, int64_t *swap_acc);

/* Work counters of the sweep kernel since create: candidates = pair terms a trial
 * needs (the one-trial kernel: gas and slab candidates at the old and the new
 * position of a displacement; the batched kernel, which keeps each particle's slab
 * energy: gas candidates at both positions, slab candidates at the new one),
 * within_cutoff = those with r < rcut (the batched kernel counts them only while
 * regc_count_pairs is on).  Either pointer may be NULL. */
int regc_get_pair_counts(regc_ctx *ctx, int64_t *candidates, int64_t *within_cutoff);

/* on != 0: the batched-trial kernel also counts the pair terms inside the cutoff
 * (a diagnostic variant of the kernel, a little slower); 0: it does not. */
int regc_count_pairs(regc_ctx *ctx, int on);

/* Histogram of recorded N per state: S_total x (n_max_all + 1) counts, where
 * n_max_all is the largest n_max over the classes. */
int regc_get_histograms(regc_ctx *ctx, int64_t *n_hist);

/* Accept-bit trace of the sweeps run since create/clear_trace:
 * bits [sweeps][W][ceil(K/32)], n_per_sweep [sweeps][W] (N at each sweep end).
 * *n_out receives the number of sweeps copied (at most cap_sweeps). */
int regc_get_trace(regc_ctx *ctx, uint32_t *bits, int32_t *n_per_sweep, int64_t cap_sweeps,
                   int64_t *n_out);

/* Per-kernel timing with HIP events on the context stream (for benchmarks).
 * enable != 0 starts recording and resets the totals. */
int regc_timing_enable(regc_ctx *ctx, int enable);
/* ms_sweep: summed duration of the sweep-kernel launches, n_sweep: their count;
 * ms_swap / n_swap the same for exchange launches (any pointer may be NULL). */
int regc_timing_get(regc_ctx *ctx, double *ms_sweep, int64_t *n_sweep, double *ms_swap,
                    int64_t *n_swap);

/* Serialises the complete sampling state (walkers, labels, sweep counter,
 * counters) into buf.  With buf == NULL only *size is set.  Samples and traces
 * are not included.  restore requires a context created with the same inputs
 * (EINVAL otherwise) and rejects, before changing anything, a buffer whose N
 * lie outside 0..n_max or whose labels are not a permutation of the class's
 * states matching its walker-of-state table. */
int regc_checkpoint(regc_ctx *ctx, void *buf, size_t cap, size_t *size);
int regc_restore(regc_ctx *ctx, const void *buf, size_t size);

void regc_destroy(regc_ctx *ctx);

/* ---- multistate reweighting (Sec. II.B) ------------------------------------ */
/* A reweighting problem on an n_t x n_mu grid (state s = l*n_mu + m), with
 * reduced potential u_s(E, N) = beta_s E - N ln z_s (Eq. (8) with the paper's
 * sign of mu N, plus the Lambda(T) term of Eq. (1)).  n_max bounds N. */
int regc_mbar_create(const regc_grid *grid, double lambda1, int n_max, regc_mbar **out);
int regc_mbar_set_stream(regc_mbar *mb, void *stream);

/* Loads ns samples (E, N, state).  With on_device != 0 the three pointers are
 * device addresses (read during the call); otherwise host.  N outside 0..n_max
 * or a state outside the grid gives EINVAL.  The call replaces earlier samples,
 * their solution and observables; after a failed call the handle holds none
 * (regc_mbar_solve then returns ESTATE). */
int regc_mbar_set_samples(regc_mbar *mb, int64_t ns, const double *e, const int32_t *n,
                          const int32_t *state, int on_device);

/* Loads the samples of class cls of a sampling context (device to device),
 * dropping the first skip_records records (burn-in).  The reweighting grid
 * must be that class's grid.  EINVAL when nothing is left. */
int regc_mbar_load_run(regc_mbar *mb, regc_ctx *ctx, int cls, int64_t skip_records);

/* Fixed-point solver of regc_mbar_solve: method 0 plain iteration, 1 (default)
 * Anderson acceleration with `memory` past iterates (1..32, default 8). */
int regc_mbar_set_solver(regc_mbar *mb, int method, int memory);

/* Solves the self-consistent equations (Eq. (9)) for the free energies f_s =
 * -ln c_s of the sampled states, gauge f = 0 at the first sampled state, until
 * max |delta f| < tol or max_iter iterations.  f_out[S] (unsampled states get
 * their reweighted value).  iters/delta may be NULL.  ENOCONV if not converged. */
int regc_mbar_solve(regc_mbar *mb, double tol, int max_iter, double *f_out, int *iters,
                    double *delta);

/* Reweighted averages on a target grid (Eq. (9) at new states and Eq. (10)/(11)):
 * f[t] = -ln c_t, mean_n, mean_e, mean_e2 (for C = beta^2 var E), p_n [t][n_max+1]
 * = probability of each N (phase), phase[t] = most probable N (smallest on ties).
 * t = l*n_mu' + m over the target grid.  Any output may be NULL except mean_n. */
int regc_mbar_targets(regc_mbar *mb, const regc_grid *targets, double *f, double *mean_n,
                      double *mean_e, double *mean_e2, double *p_n, int32_t *phase);

/* regc_mbar_targets without p_n, for callers that cannot allocate memory (code
 * under stream capture, serving loops, hosts that forbid allocation): it calls no
 * allocator and keeps its device intermediates (target constants, per-chunk partial
 * sums, outputs before the copy) in a fixed 4 MiB array of the library that every
 * GPU holds from the first call on it (with that GPU current) until the process ends.
 * Limits: n_t <= 1024, n_t * n_mu <= 4096, and nT + 6 nK + 4 nT * chunks <= 2^19
 * doubles, where chunks is the number of 2048-sample chunks of the samples cut at
 * each N (EINVAL beyond, nothing launched).  Outputs are host arrays as in
 * regc_mbar_targets and equal to its outputs; the call synchronises the handle's
 * stream.  Calls that overlap on one GPU (from several host threads) share the
 * array and race. */
int regc_mbar_targets_static(regc_mbar *mb, const regc_grid *targets, double *f, double *mean_n,
                             double *mean_e, double *mean_e2, int32_t *phase);

/* Estimates with their errors (Sec. II.B gives the estimator, not its error; the
 * error definitions are readings of this library):
 *  - at every sampled state s, the direct mean of N over the samples holding s and
 *    its standard error by batch means: the samples of s in the order given, cut
 *    into n_batches batches (batch b: series positions floor(b n_s / B) ..
 *    floor((b+1) n_s / B) - 1), SE = sqrt(var(batch means) / B), (B - 1) variance;
 *    NaN for a state with fewer than B samples;
 *  - at every target, bootstrap standard errors of <N>, coverage and heat capacity:
 *    the samples form records of record_size consecutive samples (0: the number of
 *    grid states, i.e. one sample of every walker of a run per record); replicate
 *    b (0..n_boot-1) concatenates ceil(R / block_records) blocks of block_records
 *    records (0: R / n_batches), block j starting at record
 *    floor(w (R - block_records + 1) / 2^32), w = word 0 of Philox4x32-10 block
 *    (j, b, 0xFFFFFFFE, 7) keyed by seed, cut to R records; the self-consistent
 *    equations are re-solved with every sample weighted by its record's multiplicity
 *    (started from the full solution) and the averages re-evaluated; SE = standard
 *    deviation over the replicates, (n_boot - 1) divisor;
 *  - coverage theta = <N> / n_sites (monolayers of n_sites surface sites; n_sites > 0
 *    is required when coverage or se_coverage is requested);
 *  - heat capacity at constant mu, configurational: C = beta^2 (<E^2> - <E>^2). */
typedef struct {
    int n_batches;          /* >= 2 (default 20) */
    int n_boot;             /* 0 (no bootstrap: its outputs are NaN) or >= 2 (default 100) */
    int64_t record_size;    /* samples per record; 0 -> number of grid states */
    int64_t block_records;  /* records per bootstrap block; 0 -> records / n_batches (at least 1) */
    uint64_t seed;          /* Philox key of the block starts (default 1) */
    double n_sites;         /* surface sites for the coverage */
} regc_reweight_opts;

void regc_default_reweight_opts(regc_reweight_opts *o);

/* Solves (as regc_mbar_solve, from f = 0) and returns, on the target grid t =
 * l*n_mu' + m: mean_n, se_n (bootstrap), phase (as regc_mbar_targets), coverage and
 * se_coverage, heat_cap and se_heat_cap, p_n [t][n_max+1]; on the sampled grid:
 * f_states [S], mean_state_n and se_state_n [S] (batch means).  Any output may be
 * NULL.  EINVAL when the samples are not whole records or a block is longer than
 * the records; ENOCONV (outputs still filled) when the solve or a replicate's solve
 * did not converge.  Afterwards the handle holds the full-data solution, as after
 * regc_mbar_solve. */
int regc_reweight(regc_mbar *mb, const regc_grid *targets, double tol, int max_iter, const regc_reweight_opts *opts,
                  double *f_states, double *mean_state_n, double *se_state_n, double *mean_n, double *se_n,
                  int32_t *phase, double *coverage, double *se_coverage, double *heat_cap, double *se_heat_cap,
                  double *p_n);

/* Per-state mean of N and its batch-means standard error, the definition of
 * regc_reweight's se_state_n: the samples of each state in the order given, cut into
 * n_batches batches (batch b: series positions floor(b n_s / B) .. floor((b+1) n_s / B)
 * - 1), SE = sqrt(var(batch means) / B) with the (B - 1) variance; NaN for a state
 * with fewer than B samples.  state [ns] in 0..n_states-1 and n [ns] >= 0 are host
 * arrays, or device arrays when on_device; mean and se [n_states] are host arrays.
 * Runs on `stream` (a hipStream_t, NULL: the null stream) and returns after it.
 * EINVAL on an out-of-range state or a negative N. */
int regc_batch_means(int64_t ns, const int32_t *state, const int32_t *n, int n_states, int n_batches,
                     int on_device, double *mean, double *se, void *stream);

/* Timing of the last solve: milliseconds in the iteration kernels and their
 * iteration count. */
int regc_mbar_timing(regc_mbar *mb, double *ms_iter_total, int64_t *n_iter);

void regc_mbar_destroy(regc_mbar *mb);

/* ---- structural observables (Sec. III.A) and their reweighting (Eq. (11)) ---- */
/* Per recorded sample, counts from the walker's configuration:
 *   n_z = ceil((z_hi - z_lo)/dz) axial bins: particles with floor((z - z_lo)/dz) = k
 *   (clamped to the last bin);
 *   n_r lateral bins: unordered pairs of particles both in the layer
 *   layer_lo <= z < layer_hi whose minimum-image distance in x-y lies in
 *   [k dr, (k+1) dr);
 *   1 more: the number of particles in the layer.
 * n_obs = n_z + n_r + 1 (n_z of the largest gas height for a batch). */
typedef struct {
    double dz;
    double layer_lo, layer_hi;
    double dr;
    int n_r;
} regc_observables;

/* Records the observables with every sample from now on (spec NULL: stop).  Call
 * before the sampling to analyse; not with graph replay (EUNSUPPORTED).  Runs
 * split their launches at sample boundaries while observables are on. */
int regc_set_observables(regc_ctx *ctx, const regc_observables *spec);
/* Device view of the observable records [records][W][n_obs] (uint32), in the order
 * of the samples (regc_get_samples). */
int regc_observables_device(regc_ctx *ctx, const uint32_t **obs_dev, int *n_obs);

/* Host copy of the observable records held (as regc_get_samples: n_out records of
 * W walkers, at most cap_records). */
int regc_get_observables(regc_ctx *ctx, uint32_t *obs, int64_t cap_records, int64_t *n_out);
/* Observables of the samples given to regc_mbar_set_samples, same order, obs
 * [ns][n_obs] uint32 (host, or device when on_device).  regc_mbar_load_run loads
 * them with the samples when the run recorded observables.  After a failed call
 * the handle holds no observables. */
int regc_mbar_set_observables(regc_mbar *mb, const uint32_t *obs, int n_obs, int on_device);
/* Reweighted observables on a target grid (after regc_mbar_solve): mean
 * [nT*nMu][n_obs] = sum_n w_n(t) obs_n; cond [nT][n_max+1][n_obs] = the average
 * conditional on N (the phase of Sec. II.B), which depends on T only (0 where no
 * sample has that N).  The joint average of Eq. (11) as printed is p(N) cond,
 * p(N) from regc_mbar_targets.  Either output may be NULL. */
int regc_mbar_observables(regc_mbar *mb, const regc_grid *targets, double *mean, double *cond);

/* ---- aiAT@REGC (Sec. III.A, Eq. (12)) ---- */
/* From now on, at every sample point, keep per class and N the recorded
 * configuration of lowest energy (walkers in index order, replaced only by a
 * strictly lower energy).  Not with graph replay. */
int regc_track_minima(regc_ctx *ctx, int on);
/* e_min [n_max+1] of class cls (HUGE_VAL where N was never recorded) and, if xyz is
 * not NULL, the configurations xyz [n_max+1][n_max][3] (first N rows valid). */
int regc_get_minima(regc_ctx *ctx, int cls, double *e_min, double *xyz);
/* The aiAT@REGC phase at each mu: the recorded N of lowest
 * dG_N = E_min(N) - E_min(0) - N mu (free energies approximated by the lowest
 * energies, the frozen slab contributing nothing; smallest N on ties, -1 if no N
 * was recorded).  Host computation on the e_min array. */
int regc_aiat_phase(const double *e_min, int n_max, int n_mu, const double *mu, int32_t *phase);

/* ---- learned insertion proposal (not in the paper; keeps its statistics) ---- */
/* A multilayer perceptron maps the 16^3 occupancy grid of the gas region (voxel
 * (iz*16 + iy)*16 + ix, cells of lx/16 x ly/16 x (z_hi - z_lo)/16, indices clamped)
 * to a 4096-bin categorical over insertion voxels: occupancy -> 128 -> 128 -> 128
 * -> 4096 with GELU (erf form) after the hidden layers.  bfloat16 weights and
 * activations on MFMA, FP32 accumulation, FP32 master weights and Adam state.
 * Parameter vector (FP32, regc_mlp_param_count entries): W1 [4096][128]
 * (voxel-major), b1 [128], W2 [128][128] ([out][in]), b2, W3, b3, W4 [4096][128],
 * b4 [4096].  A training example is a configuration given as the voxel of each
 * particle (vox [nmax] per example, n particles), one particle left out (excl, or
 * -1 for none) and, for training, the left-out particle's voxel as target. */
typedef struct regc_mlp regc_mlp;

int regc_mlp_param_count(int64_t *count);
/* params may be NULL (all zero). */
int regc_mlp_create(const float *params, regc_mlp **out);
int regc_mlp_set_stream(regc_mlp *mlp, void *stream);
/* Replaces the parameters and resets the Adam state. */
int regc_mlp_set_params(regc_mlp *mlp, const float *params);
int regc_mlp_get_params(regc_mlp *mlp, float *params);
/* Logits [B][4096] of B examples (B a positive multiple of 64); host arrays
 * vox [B][nmax] (uint16 voxel indices), n [B], excl [B]. */
int regc_mlp_forward(regc_mlp *mlp, int B, int nmax, const uint16_t *vox, const int32_t *n, const int32_t *excl,
                     float *logits);
/* Mean cross-entropy of target [B] and its gradient (FP32, parameter layout;
 * grads may be NULL); no update. */
int regc_mlp_loss_grads(regc_mlp *mlp, int B, int nmax, const uint16_t *vox, const int32_t *n,
                        const int32_t *excl, const int32_t *target, double *loss, float *grads);
/* One Adam step (as regc_mlp_train's) on the given batch (host arrays as
 * regc_mlp_loss_grads); loss and grads (may be NULL) receive the batch's mean loss and
 * the gradient the step applied. */
int regc_mlp_step(regc_mlp *mlp, int B, int nmax, const uint16_t *vox, const int32_t *n, const int32_t *excl,
                  const int32_t *target, double lr, double *loss, float *grads);
/* `steps` Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8) on batches drawn from a
 * device data set of n_examples configurations (vox_dev [n_examples][nmax],
 * n_dev [n_examples]): example and left-out particle from Philox keyed by seed;
 * an empty configuration is passed over for the next non-empty one (at most 256
 * further; a batch slot left empty adds nothing to the loss or its gradient).
 * mean_loss (may be NULL) receives the last batch's loss (mean over the batch).
 * EINVAL, before any step, when an example's N lies outside 0..nmax or one of
 * its first N voxel indices is 4096 or more (the set is scanned once per call). */
int regc_mlp_train(regc_mlp *mlp, int64_t n_examples, int nmax, const uint16_t *vox_dev, const int32_t *n_dev,
                   int64_t steps, int batch, double lr, uint64_t seed, double *mean_loss);
/* Accumulated training time in ms and steps. */
int regc_mlp_timing(regc_mlp *mlp, double *ms, int64_t *steps);
void regc_mlp_destroy(regc_mlp *mlp);

/* Sampling with the learned proposal.  An insertion draws, with probability alpha
 * ((B3 + 1/2) / 2^32 < alpha, B3 the last word of the trial's second Philox
 * block), a voxel v from the network's categorical for the current occupancy --
 * FP64: by Gumbel-max, argmax_v logit_v - ln(-ln u_v), u_v the open uniform of
 * word v%4 of Philox block (trial, sweep, walker, 16 + v/4); FP32 pair mode: by
 * inverse CDF over a fixed voxel order with one 53-bit uniform from words x, y of
 * block (trial, sweep, walker, 16) over the weights expf(logit - max) summed in
 * FP64, whose probabilities (w_v / sum) the acceptance uses -- and a uniform point inside
 * it (the trial's uniforms A2, A3, B0); otherwise a uniform point of V as in the
 * plain method.  The proposal density
 *   q(r|X) = alpha P(v(r)|occ(X)) / V_vox + (1 - alpha) / V
 * replaces 1/V in the insertion acceptance (Eq. (3) divided by V q) and in the
 * removal acceptance (Eq. (2) multiplied by V q(r_i | X without i), the network
 * evaluated on the occupancy left after the removal), the Metropolis-Hastings form
 * that keeps Eq. (1) the stationary law for any network.  Displacements are
 * unchanged.  The call copies the network's current parameters (bfloat16) into the
 * context: call it again after training to refresh.  This call sets the same
 * network and alpha for every class of the context; mlp = NULL or alpha = 0
 * restores the plain method.  Alpha outside [0, 1] is EINVAL; a context of more
 * than 8 classes or one run with the paper's REGC step (schedule 1) is
 * EUNSUPPORTED.  With a proposal set on any class, every walker runs in a
 * workgroup of its own (256 threads); the walkers_per_block, split and cull
 * options then have no effect (slab binning still applies). */
int regc_set_proposal(regc_ctx *ctx, regc_mlp *mlp, double alpha);

/* The same for class cls (0-based, in the order given to regc_create_batch) of a
 * batch: one network per slab class, whose 16^3 grid spans that class's box.  A
 * class without a network (never set, mlp = NULL or alpha = 0) inserts uniformly
 * as in the plain method.  cls out of range is EINVAL. */
int regc_set_class_proposal(regc_ctx *ctx, int cls, regc_mlp *mlp, double alpha);

/* The network of class cls exactly as the sampler evaluates it (its precision build:
 * FP64 contexts the sequential FP32 sums of the parity build, FP32 contexts the MFMA
 * layers), for checking it against a reference: n_conf configurations xyz
 * [n_conf][n_max][3] (host, n_max the largest over classes) of n[c] particles, the
 * occupancy taken without particle skip[c] (-1: none).  Outputs (host): logits
 * [n_conf][4096], lse [n_conf] (the log-normaliser the sampler uses) and lnp
 * [n_conf][4096], the log-probability of each voxel as the acceptance uses it.
 * ESTATE when the class has no network. */
int regc_proposal_eval(regc_ctx *ctx, int cls, int n_conf, const int32_t *n, const double *xyz, const int32_t *skip,
                       float *logits, double *lse, double *lnp);

/* Training data for the proposal network: writes, asynchronously on the
 * context's stream, the voxel of every particle of every walker into the device
 * array vox_dev [W][n_max] (uint16, rows padded with 0 beyond N; n_max the
 * largest over classes) and N into n_dev [W].  Both are device pointers the
 * caller owns (e.g. slices of a data set appended to after each sweep). */
int regc_capture_voxels(regc_ctx *ctx, uint16_t *vox_dev, int32_t *n_dev);

/* Counters of the learned proposal accumulated by the context: [0] network
 * passes, [1] insertions served by the cached pass of the unchanged occupancy,
 * [2] insertions drawn from the network, [3] of them accepted. */
int regc_get_proposal_stats(regc_ctx *ctx, int64_t counts[4]);

/* ---- errors ---------------------------------------------------------------- */
const char *regc_strerror(int code);
const char *regc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* REGC_H */
