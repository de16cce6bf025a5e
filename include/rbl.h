/*
 * rbl.h -- C-ABI of librbl: the random-batch list (RBL) short-range force
 * path of a Lennard-Jones molecular-dynamics step on an AMD Instinct MI355X
 * (gfx950), after Liang, Xu & Zhao, "Random-batch list algorithm for
 * short-range molecular dynamics simulations" (arXiv:2105.04884).
 *
 * Radius names (the paper swaps them):
 *   r_s = core radius: pairs closer than r_s are summed exactly, eq. (3);
 *   r_c = outer cut-off: pairs with r_s <= r < r_c form the shell zone, from
 *         which each particle draws a batch of P partners whose summed force
 *         is scaled by n_i/P, eq. (4).
 *
 * Conventions for every call:
 *  - Return value: RBL_OK (0), a warning (> 0) or an error (< 0).  No C++
 *    exception crosses this boundary.  rbl_last_error() returns a message
 *    for the last failing call on the calling thread.
 *  - Arguments are checked before any work is queued; a failing check
 *    queues nothing.
 *  - Work is queued on the HIP stream given to rbl_create and runs
 *    asynchronously unless the call says it synchronises.  Device-side
 *    errors (non-finite positions) surface at the next synchronising call.
 *  - Device pointers point to GPU memory owned by the caller and must stay
 *    valid until the queued work has finished.  Host pointers are read or
 *    written before the call returns.
 *  - Particle arrays are in the caller's order ("ID" = index in the
 *    caller's arrays) and laid out as structure of arrays: pos[0..n) holds
 *    x, pos[n..2n) y, pos[2n..3n) z (same for velocities and forces).
 *    For an ensemble the replicas are concatenated in replica order.
 *  - A context is not thread-safe; use one per host thread.
 *  - Units are reduced LJ units: epsilon = sigma = mass = 1 (with particle
 *    types, lengths are in units of the sigma that pair_coeffs scales).
 */
#ifndef RBL_H
#define RBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbl_ctx rbl_ctx;

typedef enum rbl_status {
    RBL_OK = 0,
    RBL_W_SKIN = 1,        /* warning: some particle moved more than skin/2 between list builds */
    RBL_E_ARG = -1,        /* invalid argument (NULL pointer, non-positive size, bad radius, P out of range) */
    RBL_E_BOX = -2,        /* a box edge is not larger than 2 (r_c + skin) (largest pair cut-off with
                              particle types), or a type's stencil spans more than 15 cells */
    RBL_E_STATE = -3,      /* call needs a list build first, or the build lacks the list asked for */
    RBL_E_CAPACITY = -4,   /* neighbour rows exceeded their capacity and could not be regrown */
    RBL_E_NONFINITE = -5,  /* a position was NaN or infinite at a list build */
    RBL_E_HIP = -6,        /* HIP runtime error */
    RBL_E_NOMEM = -7       /* device allocation failed */
} rbl_status;

enum { RBL_PREC_FP64 = 0, RBL_PREC_MIXED = 1 };
enum { RBL_PAIR_LJ = 0, RBL_PAIR_LJ_ERFC = 1 };
enum { RBL_LIST_CORE = 1, RBL_LIST_SHELL = 2, RBL_LIST_FULL = 4 };
enum { RBL_SHELL_LIST = 0, RBL_SHELL_STENCIL = 1, RBL_SHELL_PAPER = 2 };

/* Largest batch size P accepted by rbl_forces, rbl_step and
 * rbl_export_batches. */
#define RBL_MAX_P 128

typedef struct rbl_config {
    int64_t n;                 /* particles over all replicas, >= 1 */
    int32_t n_replicas;        /* independent systems sharing the launches, >= 1 */
    int32_t precision;         /* RBL_PREC_FP64: all pair arithmetic in FP64.
                                  RBL_PREC_MIXED: distances, r^2 and the core/shell/cut-off
                                  classification in FP64; r^-2, r^-6 and the force
                                  magnitude in FP32; per-particle force, energy and
                                  virial accumulated in FP64. */
    int32_t pair;              /* RBL_PAIR_LJ, or RBL_PAIR_LJ_ERFC (adds q_i q_j erfc(alpha r)/r) */
    int32_t lists;             /* RBL_LIST_* mask built by rbl_build (default core|shell) */
    double skin;               /* Verlet skin (default 0.3): lists hold candidates within
                                  r_s + skin (core), [max(r_s - skin, 0), r_c + skin) (shell)
                                  and r_c + skin (full) */
    double alpha;              /* erfc screening parameter for RBL_PAIR_LJ_ERFC */
    int32_t shift;             /* 1: pair energy shifted to zero at r_c (default 1) */
    int32_t momentum_fix;      /* 1: subtract the average net force per replica from the
                                  RBL force (default 1; Sec. II, Appendix A) */
    int32_t predraw;           /* 1: rbl_step draws the batches of a whole list lifetime at
                                  each rebuild (bit-identical to drawing inline; default 1) */
    int32_t graphs;            /* 1: rbl_step replays each list lifetime as a captured HIP
                                  graph on an internal stream (default 1; not while
                                  per-kernel profiling is on) */
    int32_t lanes;             /* lanes per particle of the pre-drawn RBL and full-list force
                                  kernels: 1, 2 or 4; 0 (default) lets the first rbl_step of
                                  the context time the three and keep the fastest (see
                                  rbl_tuning).  The choice changes the order of the per-
                                  particle sums, so bit-identical runs need the same value. */
    int32_t persistent;        /* force-kernel launch: 1 one block per work tile, 2 a
                                  persistent grid of the blocks the device keeps resident,
                                  each walking tiles in turn; 0 (default) lets the first
                                  rbl_step of the context time both and keep the faster
                                  (see rbl_launch_modes).  Results are the same. */
    double capacity_factor;    /* rows are first sized to capacity_factor x the longest row
                                  seen + 8 (default 1.25; the fused build's LDS shell-list
                                  room takes at most 1.1); rows that overflow later are
                                  regrown (rbl_build) or the run is repeated with longer rows
                                  (rbl_step), so results never depend on it */
    const int64_t* replica_offsets; /* host, n_replicas + 1 prefix offsets into the particle
                                       arrays; NULL when n_replicas == 1 */
    const double* charges;     /* device, n charges in caller order, or NULL (all zero) */
    int32_t shell_source;      /* population each batch is drawn from, eq. (4):
                                  RBL_SHELL_LIST (default): the particle's shell row,
                                  n_i = its length;
                                  RBL_SHELL_STENCIL: every particle of the 5x5x5 stencil
                                  cells around the particle's cell, itself included (the
                                  form of Sec. II), n_i = N_I of that cell; partners
                                  outside [r_s, r_c) add zero.  Batches are then always
                                  drawn at the list build (predraw is implied) and no
                                  shell row is needed by rbl_forces or rbl_step.
                                  RBL_SHELL_PAPER: the same form on the grid Sec. II and
                                  Fig. 1 describe: cells of edge w = (r_s + skin)(1 + 1e-6),
                                  the (2h+1)^3 cells around the particle's cell with
                                  h = floor((r_c + skin)/w) + 1 (an axis of at most 2h+1
                                  cells taken whole), members listed by ascending z, y, x
                                  cell index, then ID; 2 (2h+1)^2 <= 256 is required
                                  (rbl_build fails with RBL_E_ARG otherwise). */
    int32_t rebuild_check;     /* 0 (default): rbl_step rebuilds the lists before every force
                                  evaluation s with s % rebuild_every == 0.  1: rebuilds
                                  before evaluation s when some particle has moved more than
                                  skin/2 since the last build (|x_i(s) - x_i(b)|^2 >
                                  (skin/2)^2, in FP64) or s - b == rebuild_every, b being the
                                  step of the last build: lists then hold every pair within
                                  the radii at every step (the standard Verlet-list
                                  criterion), and the rebuild is decided on the device
                                  inside the captured lifetimes. */
    int32_t core_filter;       /* Core rows filtered to the partners within r_s + skin/2
                                  (with types r_s sigma_ab + skin/2), in runs with
                                  rebuild_check with one lane per particle in the RBL force
                                  kernel and core rows of at most 64 entries: filtered again
                                  at every rebuild and
                                  whenever some particle has moved skin/4 (less a rounding
                                  margin) since, so that every partner that can reach r < r_s
                                  is kept and the forces are those of the built rows bit for
                                  bit, with fewer partners read per step.  0: off; 1: on;
                                  2 (default): off in the context's first such run (often a
                                  lattice start) and decided once at its end, by timing the
                                  force kernel on its final state and lists (kept if a
                                  filtered step saves enough to repay a filtering within
                                  0.4 rebuild_every steps; with lanes = 0 a pre-drawn RBL
                                  kernel of 2 or 4 lanes is weighed against one lane with
                                  the filter and moved to it if that is faster; off for
                                  RBL_SHELL_PAPER, whose lifetimes are short), see
                                  rbl_core_filter.  While in use the context holds one
                                  more core-row array (the core rows' room in ints per
                                  particle), its lengths and FP32 positions, 16 bytes per
                                  particle beside the rows.  Other values: RBL_E_ARG. */
    int32_t n_types;           /* 0 (default): one particle type, eq. (1) with epsilon = sigma = 1.
                                  1..4: particle types whose interaction lengths differ (Sec. II):
                                  pair (a, b) interacts by eq. (1) with its own epsilon_ab and
                                  sigma_ab, has the core radius r_s sigma_ab and the cut-off
                                  r_c sigma_ab (r_s, r_c of rbl_build in units of sigma; with
                                  `shift` its energy is zero at its own cut-off), and its
                                  lists use those radii with the skin.  The cells are sized by
                                  the smallest pair cut-off (edge >= (r_c sigma_min + skin)/2),
                                  and a particle of type a searches the cells within
                                  h_a = ceil((r_c max_b sigma_ab + skin)(1 + 1e-6) / w) of its
                                  own along each axis, w the narrowest cell edge of any
                                  replica: one stencil per type, as Sec. II describes.
                                  Box edges must exceed 2 (r_c sigma_max + skin), and h_a <= 15
                                  (else rbl_build fails with RBL_E_BOX).  Not with charges, and
                                  with shell_source RBL_SHELL_LIST only.  The lists are built
                                  as explicit rows (no fused build), so rbl_step draws its
                                  batches in the force kernel and takes P <= 32; rbl_rdf takes
                                  r_max <= r_c sigma_min. */
    const int32_t* types;      /* host, n types in caller order (values 0 .. n_types - 1), or
                                  NULL when n_types == 0; copied by rbl_create */
    const double* pair_coeffs; /* host, n_types x n_types x 2 doubles: (epsilon_ab, sigma_ab) of
                                  pair (a, b) at [(a n_types + b) 2], symmetric, epsilon >= 0,
                                  sigma > 0; NULL when n_types == 0; copied by rbl_create */
} rbl_config;

/* Fills *cfg with the defaults above for n particles in one replica. */
void rbl_config_init(rbl_config* cfg, int64_t n);

/* Creates a context.  hip_stream: a hipStream_t (NULL = the null stream).
 * Errors: RBL_E_ARG (bad config), RBL_E_NOMEM, RBL_E_HIP. */
rbl_status rbl_create(const rbl_config* cfg, void* hip_stream, rbl_ctx** out);

/* Frees everything the context owns.  NULL is accepted. Synchronises. */
rbl_status rbl_destroy(rbl_ctx* ctx);

/*
 * Builds the cell list and the neighbour lists at positions `pos` (device,
 * SoA [3][n] FP64), Sec. II: particles are binned into cells of edge
 * >= (r_c + skin)/2 and each particle's candidates are searched in the 5x5x5
 * block of cells around its own.  Positions are wrapped into the box for the
 * build (the caller's array is not modified).  `box` (host) holds 3 edges
 * per replica.  Rows list their partners in the order of the cell traversal
 * (cells by z-major index, particles within a cell by ID), and a batch
 * position k in [0, n_i) refers to the k-th shell partner in that order.
 * Synchronises (once, to size list capacities).
 * Errors: RBL_E_ARG (NULL, r_s <= 0, r_c <= r_s), RBL_E_BOX, RBL_E_NONFINITE,
 * RBL_E_NOMEM, RBL_E_HIP.
 */
rbl_status rbl_build(rbl_ctx* ctx, const double* pos, const double* box,
                     double r_s, double r_c);

/*
 * RBL force at positions `pos` (device, SoA FP64, usually close to the
 * positions of the last build), eq. (3) + eq. (4):
 *   F_i = sum_{j in core, r < r_s} f_ij
 *       + (n_i/P) sum_{j in B_i, r_s <= r < r_c} f_ij
 * where B_i is P members of the draw population (cfg.shell_source: the
 * shell row, or all particles of the stencil cells) drawn without
 * replacement (Floyd's algorithm on Philox4x32-10, key = seed, counter =
 * (replica-local particle ID, step mod 2^32, replica, block)); when
 * n_i <= P the whole population is used unscaled.  With momentum_fix the average net force of each replica is
 * subtracted afterwards.  force: device SoA [3][n] (written).  ev: device,
 * 2 doubles per replica (potential energy U, virial W = sum over pairs of
 * r.f, both with the same estimator), or NULL.  1 <= P <= RBL_MAX_P.
 * Errors: RBL_E_ARG, RBL_E_STATE (no build, or the build has no core list,
 * or, with RBL_SHELL_LIST, no shell list).
 */
rbl_status rbl_forces(rbl_ctx* ctx, int P, uint64_t seed, uint64_t step,
                      const double* pos, double* force, double* ev);

/*
 * rbl_forces for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as rbl_forces (bit-identical forces and
 * [U, W]); it calls no hipMalloc, hipFree or other allocating routine.  Its
 * scratch (per-wavefront force partials, reduction partials, per-replica
 * sums, and for the stencil population or P > 32 the drawn batches and
 * population sizes) lives in one static device array of 64 MiB per device
 * (kept until the process ends), whose address rbl_create takes on its
 * device.  Nothing in it needs clearing between calls: every call writes
 * what it reads.  Limit: 160 n_slots/64 + 40 (red_blocks + 1) n_replicas
 * bytes, plus 4 P n_slots (+ 4 n_slots for the stencil population) when
 * batches are drawn, must fit in 64 MiB (n_slots: see rbl_info); otherwise
 * RBL_E_CAPACITY and nothing is queued.  All calls on one device share the
 * array, so calls that overlap on one device (other streams, other host
 * threads) race: order them on one stream.  The context's own stored
 * batches are left as they were.
 */
rbl_status rbl_forces_noalloc(rbl_ctx* ctx, int P, uint64_t seed, uint64_t step,
                              const double* pos, double* force, double* ev);

/* Direct-truncation force at `pos` from the full list (needs
 * RBL_LIST_FULL in cfg.lists): F_i = sum_{j, r < r_c} f_ij.  No mean-force
 * subtraction.  Same pointer conventions as rbl_forces. */
rbl_status rbl_full_forces(rbl_ctx* ctx, const double* pos, double* force, double* ev);

/*
 * Velocity-Verlet molecular dynamics (Algorithm 1, NVE), in place on the
 * device arrays pos and vel (SoA FP64).  The lists are built at the first
 * force evaluation and again before every force evaluation whose index s
 * (counted from step0) satisfies s % rebuild_every == 0; positions are
 * wrapped into the box at each build.  Force evaluation s draws batches with
 * Philox step counter s.  Per step:
 *   v += (dt/2) F;  x += dt v;  [rebuild];  F = force(s + 1);  v += (dt/2) F
 * use_full = 1 runs the direct-truncation force instead (needs no shell list).
 * force (device, may be NULL) receives the final force, ev (device, may be
 * NULL) the final [U, W] per replica.  Box and radii are those of the last
 * rbl_build.  Returns RBL_W_SKIN if any particle moved more than skin/2
 * within one list lifetime.  P is at most RBL_MAX_P when the batches are
 * drawn at the list builds (cfg.predraw, one particle type), and at most 32
 * when the force kernel draws them from explicit shell rows (predraw off,
 * particle types, or a stencil too wide for the fused build).
 * Errors: RBL_E_ARG, RBL_E_STATE, RBL_E_NONFINITE, RBL_E_NOMEM, RBL_E_HIP.
 */
rbl_status rbl_step(rbl_ctx* ctx, double* pos, double* vel, double* force,
                    int64_t nsteps, double dt, int P, uint64_t seed, int64_t step0,
                    int rebuild_every, int use_full, double* ev);

/*
 * Continues the last completed rbl_step (or rbl_continue) of this context
 * for nsteps >= 1 more steps of the same schedule (Algorithm 1), from the
 * state that run left in the context's device memory: its positions and
 * velocities, the force of its last evaluation, and the lists and batches
 * in use then.  dt, P, seed, rebuild_every and use_full are that run's;
 * the steps are numbered on from its end (force evaluations end+1 ..
 * end+nsteps), so that rbl_step over a + b steps and rbl_step over a steps
 * followed by rbl_continue over b steps give bit-identical results.  The
 * thermostat is the one set now.  pos, vel, force (device SoA [3][n], each
 * may be NULL) receive the final state in the caller's order; ev (device,
 * may be NULL) the final [U, W] per replica.  With all of them NULL the
 * state stays in the context: a caller that advances a system in pieces
 * pays no list build from its arrays and no copy per piece.  Lists whose
 * rows outgrow their room are regrown and the call repeated from its
 * starting state with a list build at its first step (the results are
 * then those of an rbl_step started there).
 * Errors: RBL_E_ARG (nsteps < 1), RBL_E_STATE (no completed run, or a call
 * since then that loaded positions or drew batches: rbl_build, rbl_forces,
 * rbl_full_forces, rbl_export_batches, rbl_rdf), RBL_E_NONFINITE,
 * RBL_E_CAPACITY, RBL_E_NOMEM, RBL_E_HIP.  Returns RBL_W_SKIN as rbl_step.
 */
rbl_status rbl_continue(rbl_ctx* ctx, double* pos, double* vel, double* force,
                        int64_t nsteps, double* ev);

/* The last rbl_step / rbl_continue: attempts = passes it took (1, or more
 * when a list outgrew its room and the call was repeated), end_step = index
 * of its last force evaluation, resumable = 1 if rbl_continue may follow,
 * builds = list builds of its last pass (the entry build of an rbl_step
 * included), build_step = force evaluation of the last build.  Any pointer
 * may be NULL. */
rbl_status rbl_last_run(rbl_ctx* ctx, int32_t* attempts, int64_t* end_step, int32_t* resumable,
                        int64_t* builds, int64_t* build_step);

/* ---- parity exports (host buffers, caller-allocated; synchronising) ---- */

/* Row lengths of the last build for the particles rows[0..nrows) (IDs; NULL
 * = all n): counts[k] core, counts[nrows+k] shell, counts[2 nrows+k] full
 * (0 for a list that was not built).  With a stencil draw population
 * (RBL_SHELL_STENCIL, RBL_SHELL_PAPER) and no shell rows built, the shell
 * column holds N_I once a batch has been drawn from the last build (a force
 * call, a batch export or a run), else 0. */
rbl_status rbl_row_counts(rbl_ctx* ctx, int64_t nrows, const int64_t* rows, int64_t* counts);

/* Rows of the last build as CSR over the requested rows; partners are
 * particle IDs in row order.  *_off are prefix offsets of rbl_row_counts
 * (nrows + 1 entries); an index pointer may be NULL to skip that list. */
rbl_status rbl_export_lists(rbl_ctx* ctx, int64_t nrows, const int64_t* rows,
                            const int64_t* core_off, int32_t* core_idx,
                            const int64_t* shell_off, int32_t* shell_idx,
                            const int64_t* full_off, int32_t* full_idx);

/* The batches rbl_forces would draw: batch[k*P + m] = ID of the m-th drawn
 * partner of particle rows[k] (in increasing batch position), -1 past
 * count[k] = min(n_i, P).  With RBL_SHELL_STENCIL, n_i is N_I and the
 * partners are stencil particles (the particle itself among them). */
rbl_status rbl_export_batches(rbl_ctx* ctx, int P, uint64_t seed, uint64_t step,
                              int64_t nrows, const int64_t* rows,
                              int32_t* batch, int32_t* count);

/* The batches stored on the device now, as the force kernels read them
 * (eq. (4); Algorithm 1, the random choice of p partners): after an
 * rbl_step or rbl_continue whose loop draws at each list build (cfg.predraw,
 * or the stencil population), those the last build drew for every force
 * evaluation of its list lifetime; after rbl_forces or rbl_export_batches
 * that drew one step, that step.  *nsteps, *P_out and *step0 (each may be
 * NULL) receive how many steps are stored, the batch size and the first
 * step; with batch and count both NULL nothing else is done.  Otherwise
 * batch (host, [nsteps][nrows][P]) receives, for step step0 + r and particle
 * rows[k], the IDs of its drawn partners in increasing batch position, -1
 * past count[k] = min(n_i, P) (host, [nrows]).  Synchronises.
 * Errors: RBL_E_ARG (row out of range, only one of batch and count given),
 * RBL_E_STATE (nothing stored: no build, or the last run drew inline). */
rbl_status rbl_export_drawn_batches(rbl_ctx* ctx, int64_t nrows, const int64_t* rows,
                                    int32_t* batch, int32_t* count, int32_t* nsteps,
                                    int32_t* P_out, int64_t* step0);

/* Cell binning of the last build: ncell[3r..3r+2] cells per axis of replica
 * r; slot_of_id[i] = position of particle i in the cell-sorted order of its
 * replica (0-based within the replica); cell_count (may be NULL) per cell,
 * replicas concatenated (size: sum of ncell products). */
rbl_status rbl_export_binning(rbl_ctx* ctx, int32_t* ncell, int64_t* slot_of_id,
                              int32_t* cell_count);

/* ---- control ---- */

/* Waits for the context's queued work and returns pending device errors
 * (RBL_E_NONFINITE) or warnings (RBL_W_SKIN), clearing them. */
rbl_status rbl_sync(rbl_ctx* ctx);

/* Per-kernel timing with HIP events on the context's stream while enabled:
 * the force kernels and the fused list build carry a start and a stop event
 * in their dispatch (the kernel's own duration), other kernels have events
 * recorded around the launch.  rbl_kernel_stats fills, for kernel class
 * `kind` (0 force RBL, 1 force full, 2 list build, 3 binning, 4 integrate,
 * 5 reduce, 6 predraw), the number of launches and their summed duration in
 * milliseconds since profiling was enabled; it synchronises. */
rbl_status rbl_set_profiling(rbl_ctx* ctx, int on);
rbl_status rbl_kernel_stats(rbl_ctx* ctx, int kind, int64_t* launches, double* total_ms);

/* Lanes per particle chosen for the RBL (pre-drawn batches) and the
 * full-list force kernels, and the times measured by the autotuner:
 * force_us[3k + q] = microseconds per launch at 1, 2, 4 lanes (q = 0, 1, 2)
 * for k = 0 (RBL) and k = 1 (full list); zeros before tuning.  Any pointer
 * may be NULL. */
rbl_status rbl_tuning(rbl_ctx* ctx, int32_t* lpp_rbl, int32_t* lpp_full, double* force_us);

/* Launch mode chosen for the RBL and the full-list force kernels (1:
 * persistent grid, 0: one block per tile) and the autotuner's times:
 * force_us[2k + q] = microseconds per launch for k = 0 (RBL), 1 (full list)
 * with q = 0 one block per tile, q = 1 persistent; zeros before tuning.
 * Any pointer may be NULL.  Used by callers that size launches (the
 * persistent grid of the large single-system workload). */
rbl_status rbl_launch_modes(rbl_ctx* ctx, int32_t* persistent_rbl, int32_t* persistent_full,
                            double* force_us);

/* Core-row filter (rbl_config.core_filter): *used = 1 if the last rbl_step /
 * rbl_continue read filtered core rows; the times of the core_filter = 2
 * decision: force_us[0] an unfiltered force launch, [1] a launch on the
 * filtered rows, [2] the filtering launch, in microseconds (zeros before
 * the decision); *mean_kept the mean length of the filtered rows at the
 * last filtering (0 if none).  Any pointer may be NULL; with mean_kept the
 * call copies the row lengths to the host and synchronises. */
rbl_status rbl_core_filter(rbl_ctx* ctx, int32_t* used, double* force_us, double* mean_kept);

/* Size information: n_slots (particles plus per-replica padding to 64) and
 * current list capacities (entries per row). */
rbl_status rbl_info(rbl_ctx* ctx, int64_t* n_slots, int32_t* cap_core,
                    int32_t* cap_shell, int32_t* cap_full);

/* ---- thermostat and observables ---- */

/*
 * Langevin thermostat for rbl_step (Sec. II: m dv = (F - gamma v) dt +
 * sqrt(2 gamma kT) dW; Sec. III: velocity Verlet with underdamped Langevin
 * dynamics).  gamma = 0 (the default) is plain velocity Verlet (NVE).  With
 * gamma > 0 each step is the BAOAB splitting (Leimkuhler & Matthews 2013):
 *   v += (dt/2) F;  x += (dt/2) v;  v = c v + sqrt(kT (1 - c^2)) xi;
 *   x += (dt/2) v;  [rebuild];  F = force(s);  v += (dt/2) F
 * with c = exp(-gamma dt) and xi three standard normal numbers per particle:
 * Box-Muller on the Philox4x32-10 block (key = seed of rbl_step, counter =
 * (replica-local ID, s mod 2^32, replica, 2^31)), s being the force
 * evaluation the step leads to.  Unit mass.  kT: host, one bath temperature
 * per replica (may be NULL when gamma = 0).  Applies to later rbl_step calls.
 * Errors: RBL_E_ARG (gamma < 0 or not finite, kT missing, negative or not
 * finite).
 */
rbl_status rbl_set_thermostat(rbl_ctx* ctx, double gamma, const double* kT);

/*
 * Continuous trajectory for the mean-squared displacement eta(t) of
 * Sec. III: out = pos + k L per component, where k counts the box lengths
 * that the list builds of rbl_step took off each particle when wrapping it
 * into the box (counted since the context was created; a run that is
 * repeated after a capacity overflow counts once).  pos: positions written
 * by the last rbl_step; pos, out: device SoA [3][n] (may alias).
 * Errors: RBL_E_ARG, RBL_E_STATE (no box yet).
 */
rbl_status rbl_unwrap(rbl_ctx* ctx, const double* pos, double* out);

/* out[r] = (1/n_r) sum_{i in replica r} |a_i - b_i|^2 (device, one double per
 * replica): with unwrapped positions at two times, the mean-squared
 * displacement of Sec. III.  a, b: device SoA [3][n].  Deterministic
 * (fixed-order sums).  Errors: RBL_E_ARG, RBL_E_STATE (no replica table). */
rbl_status rbl_msd(rbl_ctx* ctx, const double* a, const double* b, double* out);

/*
 * Pair-distance histogram behind the radial distribution function of
 * Sec. III, g(r) = (1/(N rho)) sum_i sum_{j != i} <delta(r_ij - r)>/(4 pi r^2):
 * counts[r*nbins + k] += the number of ordered pairs (i, j), i != j, of
 * replica r at positions `pos` whose minimum-image distance lies in
 * [k dr, (k+1) dr), dr = r_max/nbins (bins decided on r^2 against the squared
 * edges).  counts: device uint64 [n_replicas][nbins], accumulated (the caller
 * zeroes it), so frames can be summed; g(r) of bin k is then
 * counts / (frames N rho 4/3 pi ((k+1)^3 - k^3) dr^3).  Pairs are found
 * through the cells of the last build, so pos must be within skin/2 of the
 * positions of that build (as after rbl_step).  pos: device SoA [3][n].
 * Errors: RBL_E_ARG (NULL, r_max not in (0, r_c], nbins not in 1..2^20),
 * RBL_E_STATE (no build).
 */
rbl_status rbl_rdf(rbl_ctx* ctx, const double* pos, double r_max, int nbins, uint64_t* counts);

/*
 * Potential energy per particle and pressure with the mean-field tail
 * corrections of Sec. III (sigma = epsilon = 1, tails beyond r_c):
 *   u = U/N + (8/3) pi rho (1/(3 r_c^9) - 1/r_c^3),
 *   P = rho T + W/(3V) + (16/3) pi rho^2 (2/(3 r_c^9) - 1/r_c^3),
 * with U, W the [U, W] pair of a force call (`ev`, device, 2 doubles per
 * replica; W/(3V) is the (8/V) sum (2 r^-12 - r^-6) of Sec. III).  out
 * (host, 4 doubles per replica): u; P with T = the thermostat's kT (NaN
 * without a thermostat); the kinetic temperature sum v^2/(3 n_r - 3) from
 * vel (device SoA, or NULL: NaN); P with that kinetic temperature.
 * Synchronises.  Errors: RBL_E_ARG, RBL_E_STATE (no box, or a pair that is
 * not the unshifted LJ: cfg.shift must be 0 and cfg.pair RBL_PAIR_LJ).
 */
rbl_status rbl_thermo(rbl_ctx* ctx, const double* vel, const double* ev, double* out);

const char* rbl_last_error(void);
const char* rbl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RBL_H */
