/*
 * nbody.h -- C ABI of the MI355X (gfx950) direct N-body hot-path library.
 *
 * The library computes the hot path of a direct-summation gravitational
 * N-body integrator with a 4th-order Hermite predictor/corrector and
 * individual block time steps, as used by Groen, Portegies Zwart, McMillan &
 * Makino, "Distributed N-body Simulation on the Grid Using Dedicated
 * Hardware" (section 2 for the scheme, section 4.1 for the step list, and
 * section 4.4 for the step list when a force accelerator does the pairwise
 * sums).  One block step is:
 *
 *   select   the next system time t = min_i(t_i + dt_i) and the block of
 *            n active particles due at t          (section 4.1, step 2)
 *   predict  positions and velocities of all N particles to t
 *                                                 (section 4.1, step 3)
 *   force    acceleration, jerk (and potential) on the n active particles
 *            from all N particles                 (section 4.1, step 4)
 *   correct  the n active particles and give each a new block step
 *                                                 (section 4.1, step 5)
 *
 * Units: G = 1.  Softening enters as s = |r|^2 + eps^2.  Block steps are
 * powers of two between 2^dt_min_log2 and 2^dt_max_log2 (the paper uses
 * 2^-22 and 2^-3).  Times are kept as integer ticks of 2^dt_min_log2.
 *
 * Memory and ownership.  Every pointer named *_dev is a device pointer.  The
 * caller owns the particle state (nbody_state), all output buffers and the
 * HIP stream; the library never frees them.  The context owns its internal
 * buffers: the predicted j-particle buffer, the active list, the work plan,
 * partial sums, counters, and the captured HIP graph.  All work is enqueued
 * asynchronously on the caller's stream unless a call returns host values.
 *
 * Errors.  Every call returns an int status (NBODY_OK = 0 or a negative
 * code) and never aborts or throws.  Host-checkable arguments are checked
 * before anything is enqueued.  Faults found on the device (non-finite
 * state, index out of range, a corrected particle that was not due) set a
 * device error word that the next synchronising call (nbody_sync,
 * nbody_step_block with outputs, nbody_run_until, nbody_get_stats) reports
 * and clears.
 *
 * Threads.  A context is not thread safe: calls on one context must not
 * overlap.  Distinct contexts are independent.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define NBODY_OK 0
#define NBODY_EINVAL (-1)       /* bad argument (checked on the host)            */
#define NBODY_ESTATE (-2)       /* call out of order, or a particle not due      */
#define NBODY_ENOMEM (-3)       /* device allocation failed                      */
#define NBODY_EDEVICE (-4)      /* HIP runtime error                             */
#define NBODY_ENONFINITE (-5)   /* the device produced a non-finite value        */
#define NBODY_EUNSUPPORTED (-6) /* valid but not supported by this library       */
#define NBODY_ERANGE (-7)       /* the device met a particle index out of range  */
#define NBODY_EIO (-8)          /* checkpoint file not writable / readable / valid */
#define NBODY_ESCRATCH (-9)     /* more particles than nbody_force_jerk_static holds */
#define NBODY_EEXTENT (-10)     /* mixed: a particle 256 or more from its cluster's origin */

/* arithmetic of the pairwise force sum */
#define NBODY_PREC_FP64 0  /* every operation in FP64                             */
#define NBODY_PREC_MIXED 1 /* FP64 coordinates and differences of positions,
                              FP32 pairwise terms, FP64 accumulation            */

/*
 * The mixed form stores each predicted position as a float on a 2^-16 grid
 * plus a float remainder, both relative to an origin of the particle's
 * cluster: the centre of the cluster's bounding box at nbody_init, rounded
 * to a multiple of 64 (so a cluster around the coordinate origin keeps it),
 * kept in checkpoints.  The grid parts are then exact, and so are their
 * differences, while every coordinate stays less than 256 length units from
 * the origin.  A prediction outside that range sets the device error word,
 * reported as NBODY_EEXTENT by the next synchronising call: rescale the
 * units, split the cluster, or use NBODY_PREC_FP64.  A cluster may lie
 * anywhere, but must stay less than 512 units wide around its centre.
 */

typedef struct nbody_ctx nbody_ctx;

/*
 * Particle state, structure of arrays, n_total entries per array, device
 * memory owned by the caller.  pos/vel/mass are inputs to nbody_init; the
 * library updates pos, vel, acc, jerk, t_tick and level in place as particles
 * are corrected.  acc/jerk hold the values at the particle's own time t_i.
 */
typedef struct {
    double *pos[3];   /* x, y, z                                            */
    double *vel[3];   /* vx, vy, vz                                         */
    double *acc[3];   /* acceleration at t_i                                */
    double *jerk[3];  /* time derivative of the acceleration at t_i        */
    double *mass;     /* read only                                          */
    int64_t *t_tick;  /* t_i = t_tick * 2^dt_min_log2                       */
    int8_t *level;    /* block step of particle i: dt_i = 2^-level[i]      */
} nbody_state;

/*
 * Run parameters.  n_clusters > 1 makes an ensemble of independent systems
 * that share nothing but the launches: cluster k holds particles
 * [cluster_offset[k], cluster_offset[k+1]) and has its own clock; one block
 * step of the ensemble advances every unfinished cluster by its own next
 * block step.  cluster_offset is a HOST array of n_clusters+1 entries, may be
 * NULL when n_clusters == 1, and is copied by nbody_create.
 */
typedef struct {
    int64_t n_total;               /* particles in all clusters, 1..2^31-1       */
    int32_t n_clusters;            /* >= 1                                        */
    const int64_t *cluster_offset; /* host, n_clusters+1, increasing, 0..n_total */
    double eps;                    /* softening length, >= 0                      */
    double eta;                    /* Aarseth step accuracy parameter, > 0        */
    double eta_init;               /* start-up step parameter (eta_init|a|/|j|)   */
    int32_t dt_min_log2;           /* smallest step 2^dt_min_log2, >= -40         */
    int32_t dt_max_log2;           /* largest step, dt_min_log2 <= it <= 0        */
    int32_t precision;             /* NBODY_PREC_FP64 or NBODY_PREC_MIXED         */
} nbody_params;

/*
 * Launch shape of the force kernel for one block-size class (chosen by
 * nbody_autotune or set by hand).  Blocks are sorted into NBODY_SIZE_CLASSES
 * classes by their mean size n over the active clusters: class 0 for
 * n >= 2048, 1 for n >= 256, 2 for n >= 32, 3 for n >= 4, 4 below.
 * i_per_lane in {1,2} (2 only with j_lanes = 1); j_lanes in {1,4,16,64,256}
 * is the number of lanes that share one i-particle and split its j loop;
 * j_tile = 256 j-particles staged in LDS per round; grid is the number of
 * persistent workgroups (0 = CUs x occupancy).
 */
#define NBODY_SIZE_CLASSES 5
typedef struct {
    int32_t size_class;
    int32_t i_per_lane;
    int32_t j_lanes;
    int32_t j_tile;
    int32_t grid;
} nbody_tuning;

/* Counters accumulated on the device since nbody_init (nbody_get_stats). */
typedef struct {
    int64_t block_steps;   /* block steps with n > 0, summed over clusters    */
    int64_t updates;       /* corrected particles (sum of block sizes)        */
    double interactions;   /* pairwise force evaluations, n*N summed          */
    int64_t dt_clamped;    /* steps that wanted less than 2^dt_min_log2       */
} nbody_stats;

/* Human readable text for a status code; never NULL. */
const char *nbody_strerror(int status);

/*
 * Create a context for the given parameters and caller-owned state.
 * `stream` is a hipStream_t (NULL = the null stream).  Allocates the
 * context's device buffers: 124 + 8 * (dt_max_log2 - dt_min_log2 + 1) B per
 * particle (j-particle records, results, active list, per-level lists), 56 B
 * per partial-sum slot (clamp(8 N, 2^20, 2^24) slots) and the per-cluster plan.
 * The state is not read until nbody_init.
 * Errors: EINVAL (bad sizes, offsets, eps, eta, step range, precision or a
 * NULL state array), ENOMEM, EDEVICE.
 */
int nbody_create(const nbody_params *params, const nbody_state *state, void *stream,
                 nbody_ctx **out);

/* Release the context's device buffers and graph; caller memory untouched. */
int nbody_destroy(nbody_ctx *ctx);

/*
 * Start-up (section 4.1, step 1): set every t_i to 0, compute acceleration
 * and jerk of every particle from all particles of its cluster (one full
 * n = N sweep), and give each particle its start-up block step: the largest
 * power of two not above eta_init |a|/|j|, clamped to the step range.
 * Resets the counters and the device error word, and (mixed form) sets each
 * cluster's origin.  Errors: EEXTENT (mixed form, a cluster 512 or more
 * units wide), ENONFINITE, EDEVICE.
 */
int nbody_init(nbody_ctx *ctx);

/*
 * Predict all particles to time t (section 4.1, step 3) into the context's
 * j-particle buffer:  d = t - t_i,  xp = x + v d + a d^2/2 + jerk d^3/6,
 * vp = v + a d + jerk d^2/2, in FP64.  t must be a multiple of
 * 2^dt_min_log2 and not before any particle's t_i (the latter is not
 * checked).  Single-cluster contexts only (EUNSUPPORTED otherwise).
 */
int nbody_predict(nbody_ctx *ctx, double t);

/*
 * Force, jerk and potential on the n listed particles from all particles
 * (section 4.1, step 4), at the positions and velocities predicted by the
 * last nbody_predict, which must have been made at the same t (ESTATE
 * otherwise):
 *   a_i    =  sum_{j != i} m_j r s^{-3/2}
 *   jerk_i =  sum_{j != i} m_j [w s^{-3/2} - 3 (r.w) r s^{-5/2}]
 *   pot_i  = -sum_{j != i} m_j s^{-1/2}
 * with r = x_j - x_i, w = v_j - v_i, s = |r|^2 + eps^2.
 * i_list_dev: int32[n] particle indices, duplicates allowed; an index
 * outside [0, n_total) makes the next synchronising call return ERANGE (the
 * slot's outputs are then unspecified).  Outputs are FP64 structure of
 * arrays: acc_dev[c*n + k] is component c of particle i_list[k];
 * jerk_dev likewise; pot_dev[k] (pot_dev may be NULL).  1 <= n <= n_total.
 * Single-cluster contexts only.
 *
 * The mixed form evaluates in FP64 the pairs whose acceleration term may
 * exceed a tenth of |a_i|, or whose jerk term may exceed twice |jerk_i|; it
 * sizes that near field from the acceleration and jerk stored in the state
 * for particle i, and from each cluster's largest and smallest mass and
 * largest speed as nbody_init (or nbody_load) found them.  So the mixed form
 * returns ESTATE before nbody_init or nbody_load, and masses must not change
 * after nbody_init (call it again after changing them).
 */
int nbody_force_jerk(nbody_ctx *ctx, const int32_t *i_list_dev, int64_t n, double t,
                     double *acc_dev, double *jerk_dev, double *pot_dev);

/*
 * Hermite corrector (section 4.1, step 5) for the n listed particles, which
 * must all be due at t (t_i + dt_i = t) and distinct; otherwise the next
 * synchronising call returns ESTATE (a particle listed twice is corrected
 * once, from the slot that claims it first).  acc_dev/jerk_dev hold the new
 * acceleration and jerk at t in the layout nbody_force_jerk writes.  Updates
 * pos, vel, acc, jerk, t_tick and level of those particles:
 *   a2 = [-6(a0-a1) - dt(4j0+2j1)]/dt^2,  a3 = [12(a0-a1) + 6dt(j0+j1)]/dt^3
 *   x1 = xp + a2 dt^4/24 + a3 dt^5/120,   v1 = vp + a2 dt^3/6 + a3 dt^4/24
 * and the next step from Aarseth's criterion with eta,
 *   dt' = sqrt(eta (|a1||a2'| + |j1|^2) / (|j1||a3| + |a2'|^2)),  a2' = a2 + dt a3,
 * quantised: halve until dt <= dt' (not below the minimum); double once if
 * dt' >= 2dt, t is a multiple of 2dt and 2dt is within the maximum.
 * A non-finite result makes the next synchronising call return ENONFINITE.
 * Single-cluster contexts only.
 */
int nbody_correct(nbody_ctx *ctx, const int32_t *i_list_dev, int64_t n, double t,
                  const double *acc_dev, const double *jerk_dev);

/*
 * One block step of every cluster, driven entirely from the device: select,
 * predict, force, correct.  The call first checks that the state is a
 * synchronised block-step state (below) and synchronises to do so; it returns
 * the new time of cluster 0 and the block size summed over clusters in
 * t_out / n_out when these are non-NULL.
 *
 * Synchronised block-step state (section 4.1): within each cluster every
 * particle's last time t_i precedes every particle's next time t_i + dt_i,
 * and t_i is a multiple of dt_i.  nbody_init and block steps keep it;
 * explicit corrections keep it when they correct whole blocks.  Otherwise
 * (for example after correcting only part of a due block) nbody_step_block
 * and nbody_run_until return ESTATE and step nothing.
 */
int nbody_step_block(nbody_ctx *ctx, double *t_out, int64_t *n_out);

/*
 * Block steps until no cluster has a next block time <= t_end (section 4.1,
 * step 6).  Steps are replayed from a captured HIP graph in batches; with
 * steps of 2^dt_max_log2 or less and t_end a multiple of 2^dt_max_log2,
 * every particle ends exactly at t_end.  t_end must be a multiple of
 * 2^dt_min_log2.  The state must be a synchronised block-step state (see
 * nbody_step_block), else ESTATE.  Synchronises; *n_steps_out (may be NULL)
 * receives the number of ensemble block steps that did work.
 */
int nbody_run_until(nbody_ctx *ctx, double t_end, int64_t *n_steps_out);

/*
 * Checkpoint and resume of a long integration (section 4.1: the run is a loop
 * of block steps over caller-owned state, so the state plus the context's
 * configuration is everything a run needs to continue).
 *
 * nbody_save synchronises, then writes to `path` (host file name): the
 * configuration (n_total, clusters and their offsets, eps, eta, eta_init, the
 * step range, precision), the statistics, the tuning table, the mixed form's
 * near-field scales of each cluster (set by nbody_init, see nbody_force_jerk),
 * and the particle state (pos, vel, acc, jerk, mass as FP64; t_tick; level).  Little-endian
 * binary with a version and a 64-bit checksum; written to "<path>.part" and
 * renamed, so an existing file is only ever replaced by a complete one.
 * ESTATE before nbody_init; a pending device error is reported instead of
 * saving; EIO if the file cannot be written.
 *
 * nbody_load reads such a file into a context created with the same
 * configuration (EINVAL otherwise; nbody_init is not needed) and copies the
 * state into the caller's state arrays, replacing their contents; statistics
 * and tuning continue from the file.  EIO if the file cannot be read, is not a
 * checkpoint of this version, is truncated or fails its checksum; nothing is
 * changed then.  A run continued from a checkpoint on the same device takes
 * the same block steps and gives bitwise the same state as one that was not
 * interrupted.  Synchronises.
 */
int nbody_save(nbody_ctx *ctx, const char *path);
int nbody_load(nbody_ctx *ctx, const char *path);

/* Wait for the context's work and report (then clear) the device error word. */
int nbody_sync(nbody_ctx *ctx);

/* Synchronise and read the counters since nbody_init (the error word too). */
int nbody_get_stats(nbody_ctx *ctx, nbody_stats *out);

/*
 * Copy the predicted positions and velocities from the last nbody_predict
 * (or block step) into caller buffers pos_dev[c*n_total + i],
 * vel_dev[c*n_total + i] in FP64 (mixed contexts keep predicted velocities
 * in FP32; they are widened).  For checking the predictor.
 */
int nbody_read_predicted(nbody_ctx *ctx, double *pos_dev, double *vel_dev);

/* Read (out->size_class selects the class) / set the launch shape of one
 * class; EINVAL for an unknown class or an unsupported shape. */
int nbody_get_tuning(const nbody_ctx *ctx, nbody_tuning *out);
int nbody_set_tuning(nbody_ctx *ctx, const nbody_tuning *tuning);

/*
 * In-kernel prediction.  Bit k of class_mask: in the block steps of a single
 * cluster (nbody_step_block, nbody_run_until), blocks of size class k whose
 * tuned shape is a lane-group shape (j_lanes 4 to 256) skip the prediction
 * pass over all N particles; their force launch predicts each j- and
 * i-particle it reads from the state instead, with the same arithmetic (the
 * prediction of section 4.1, step 3, done where the force pipeline reads the
 * particle, as GRAPE predicts the j-particles on the board: section 4.4,
 * steps 3 and 4), so results are bitwise the same either way.  Ensembles and
 * the explicit calls always use the prediction pass.  The default is 0 (every
 * block uses the prediction pass, which is faster on this hardware); the
 * option is for experiments and for workloads whose blocks are tiny.  Drops
 * the captured graph; not stored by nbody_save.  EINVAL for bits beyond the
 * classes.
 */
int nbody_set_fused_predict(nbody_ctx *ctx, int32_t class_mask);

/*
 * Autotuner: for blocks of n_probe particles per cluster (1 <= n_probe; a
 * cluster smaller than n_probe uses all its particles), time one force
 * evaluation with every supported launch shape of the class that block size
 * falls in (best of four timed calls after one warm-up), and keep for that
 * class the fastest; when the fastest is a lane-group shape, the widest lane
 * group within 3% of it.
 * Runs on the j-particle buffer of the last prediction (valid after
 * nbody_init) and writes only the context's scratch buffers: the particle
 * state is not changed.  Synchronises.  *best receives the chosen shape;
 * *best_ms (may be NULL) its time for one force evaluation in milliseconds.
 */
int nbody_autotune(nbody_ctx *ctx, int64_t n_probe, nbody_tuning *best, double *best_ms);

/*
 * Allocation-free force evaluation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It computes what nbody_force_jerk computes (the same
 * kernels and arithmetic, both precisions) without a context: on the n
 * listed particles, from all n_j particles given, at the positions and
 * velocities given (no prediction; the evaluation time is the particles').
 * The buffers its kernels need beyond the inputs and outputs (the j-particle
 * records, near-field hints, partial sums of split j ranges, the work plan
 * and counters) live in one statically sized device array of the library,
 * about 35 MB on each GPU it runs on, held until the process ends; the call
 * allocates nothing, sets no memory with hipMemset and does not synchronise.
 *
 * in: host struct of device pointers (SoA FP64, n_j entries each).  In the
 *   mixed form the near field is sized as in nbody_force_jerk, from
 *   acc_hint/jerk_hint (the particles' acceleration and jerk at or shortly
 *   before this time, e.g. from the previous evaluation; all six NULL: a first
 *   pass without the near field supplies them, doubling the work), and the
 *   masses are always tested pair by pair.  The FP64 form ignores the hints.
 *   The mixed records take as origin the centre of the particles' bounding
 *   box, rounded to a multiple of 64; particles 256 or more units from it
 *   (a system 512 or more units wide) are outside the mixed form's error
 *   bound, which this call cannot report: use the FP64 form for them.
 * i_list_dev, n, acc_dev, jerk_dev, pot_dev: as in nbody_force_jerk
 *   (pot_dev may be NULL); an index outside [0, n_j) leaves that slot's
 *   outputs unspecified (it is not reported: there is no context).
 * stream: hipStream_t (NULL = the null stream).  Asynchronous.
 *
 * Errors (host-checked, nothing enqueued): EINVAL for NULL pointers, bad eps
 * or precision, n or n_j below 1, or only some hint arrays given; ESCRATCH
 * for n_j or n above NBODY_STATIC_MAX_PARTICLES (2^18, also the j-memory
 * size of the GRAPE-6Af boards of the paper, section 5); EDEVICE on a HIP
 * error.  All calls on one GPU share the array: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 */
#define NBODY_STATIC_MAX_PARTICLES 262144
typedef struct {
    int64_t n_j;                 /* particles, 1..NBODY_STATIC_MAX_PARTICLES  */
    const double *pos[3];        /* x, y, z                                   */
    const double *vel[3];        /* vx, vy, vz                                */
    const double *mass;          /* m                                         */
    const double *acc_hint[3];   /* mixed: |a| hints by particle, or NULL     */
    const double *jerk_hint[3];  /* mixed: |jerk| hints by particle, or NULL  */
    double eps;                  /* softening length, >= 0                    */
    int32_t precision;           /* NBODY_PREC_FP64 or NBODY_PREC_MIXED       */
} nbody_direct;

int nbody_force_jerk_static(const nbody_direct *in, const int32_t *i_list_dev, int64_t n,
                            double *acc_dev, double *jerk_dev, double *pot_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
