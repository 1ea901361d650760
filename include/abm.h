/*
 * abm.h -- C ABI of the MI355X spherical-agent mechanics library (libabm.so).
 *
 * One iteration of the thesis's agent-based mechanics (arXiv 2503.10796):
 *   - uniform-grid neighbour search: box length = largest agent diameter or a
 *     user value, agent box from its centre, 27 surrounding boxes (Sec 4.4.3,
 *     Sec 5.3.1), open boundary: the grid spans the agents' bounding box
 *     (Sec 4.4.11);
 *   - pairwise sphere-sphere force F_N = k*delta - gamma*sqrt(r*delta),
 *     r = r1*r2/(r1+r2), along the centre line (Sec 4.5.1, Eq 4.1-4.2);
 *   - displacement F*dt/m when |F| exceeds the adherence threshold, capped in
 *     norm at the maximum displacement (Sec 5.5; Tutorial E.15);
 *   - static-agent skip of the force calculation (Sec 5.5);
 *   - grow-or-divide cell rule with appended daughters (Algorithm 2,
 *     Sec 5.3.2);
 *   - periodic Morton-order re-sort of agent storage (Sec 5.4.2, Fig 5.4);
 *   - copy semantics: every agent reads the start-of-iteration state and new
 *     agents appear in the next iteration (Sec 5.2.1).
 *   - Brownian step and apoptosis with parallel removal (Algorithm 2,
 *     Sec 5.3.2, Table 4.2).
 * Plus batched independent simulations (parameter sweeps, Sec 4.3 execution
 * modes C-E), a surrogate MLP trained with BF16 matrix-core kernels, the SIR
 * epidemiology model with toroidal or closed space (Algorithms 3-5,
 * Sec 4.4.11) and extracellular diffusion with soma clustering (Eq 4.3,
 * Algorithms 6-7).
 *
 * Conventions for every entry point:
 *   - Return value: ABM_OK (0) or a negative ABM_ERR_* code; the message of
 *     the last failure on the calling thread is abm_last_error().
 *   - Pointers flagged "on_device" are HIP device pointers, otherwise host
 *     pointers.  The caller owns every buffer it passes; the library reads or
 *     writes it only during the call, in stream order on the handle's stream,
 *     and has finished with it when the call returns.
 *   - All device state of a handle lives inside the caller's workspace
 *     (size from the *_workspace_bytes call, 256-byte aligned); the library
 *     allocates no device memory in create/step/query.  The workspace must
 *     outlive the handle.
 *   - Handles are not thread-safe; one handle per thread at a time.
 *   - Nothing falls back to the CPU: every step runs in HIP kernels.
 */
#ifndef ABM_H
#define ABM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABM_OK 0
#define ABM_ERR_ARG (-1)       /* bad parameters or sizes */
#define ABM_ERR_CAPACITY (-2)  /* agents or grid boxes would exceed the capacity */
#define ABM_ERR_NONFINITE (-3) /* a non-finite position, diameter or force */
#define ABM_ERR_HIP (-4)       /* HIP runtime failure */

/* flags of abm_params.flags */
#define ABM_DIAG 1u /* diagnostic sweep: every pair within the box length is visited and
                      neighbours are counted; writes the fields of ABM_RECORD plus NBR_COUNT */
#define ABM_RECORD 2u /* the production sweep (half shell, reach culling, unit skipping,
                        box-wise path unchanged) also writes each agent's force, displacement,
                        contact count and box of the iteration (NBR_COUNT is -1) */

/* Model parameters of one simulation.
 * dt, k, gamma: time step and the constants of Eq 4.1 (k = 2, gamma = 1 in the thesis).
 * adherence: force threshold that |F| must exceed to move the agent (Sec 5.5; Table 4.2: 1.8).
 * mass: agent mass in F*dt/m (Tutorial E.15 uses 0.1).
 * max_disp: cap on the Euclidean norm of one step's displacement.
 * box_len: grid box length; 0 = largest agent diameter (Sec 4.4.3).
 * div_vol: > 0 enables Algorithm 2: cells grow by their growth rate per step
 *          below this volume and divide at or above it; 0 = no growth.
 * shift_frac: on division mother and daughter move shift_frac * r_mother in
 *          opposite directions along a uniformly random unit vector.
 * detect_static: 1 = skip the force of agents meeting the four conditions of Sec 5.5
 *          (not with brownian_rate > 0: every agent then moves every iteration).
 * resort_every: Morton re-sort of agent storage every so many iterations (0 = never;
 *          < 0 = let abm_batch_tune pick it, never until then).
 * seed, sim_id: key and counter words of the Philox4x32-10 draws (division
 *          directions and the cell behaviour below).
 * Cell behaviour of Algorithm 2 (Table 4.2), per iteration:
 * brownian_rate: length of a random step along the normalised vector of three
 *          uniforms in (-1, 1), added before the mechanical displacement (0 = off).
 * death_prob, min_age: a cell of at least min_age iterations is removed with
 *          probability death_prob (0 = off); removals take effect for the next
 *          iteration and are no change for the static rule (Sec 5.5, condition iv).
 * division_prob: a cell at or above div_vol divides with this probability and
 *          otherwise neither grows nor divides; must be in (0, 1] when div_vol > 0
 *          (1 = the deterministic grow-or-divide rule).
 * Daughters start at age 0; the mother keeps her age. */
typedef struct abm_params {
    double dt, k, gamma, adherence, mass, max_disp;
    double box_len;
    double div_vol;
    double shift_frac;
    int32_t detect_static;
    int32_t resort_every;
    uint64_t seed;
    uint32_t sim_id;
    uint32_t flags;
    double brownian_rate, death_prob, division_prob;
    int32_t min_age;
    int32_t reserved; /* 0 */
} abm_params;

/* Fields for abm_*_query.  Arrays are in the library's current storage order
 * (it changes on a Morton re-sort); match agents across calls by ABM_UID.
 * Element types: POS, FORCE, DISP: 3 doubles per agent (x,y,z interleaved);
 * DIAM, VOL, GROWTH: double; UID: uint64; STATIC: uint8; NZ, NBR_COUNT,
 * CONTACT_COUNT, AGE (iterations since creation): int32; BOX: int64 linear box id (x fastest) in the grid of
 * the last iteration.  FORCE, DISP, NBR_COUNT, CONTACT_COUNT and BOX are the
 * values of the last iteration run with ABM_DIAG or ABM_RECORD set (NBR_COUNT
 * and CONTACT_COUNT are -1 and FORCE is 0 for agents skipped as static;
 * NBR_COUNT is -1 under ABM_RECORD alone).  Under ABM_RECORD without
 * ABM_DIAG the sweep does not visit aligned 4x4x4 box blocks whose agents
 * are all static, and the fields of those agents keep older values (their
 * STATIC flag of the start of the iteration tells them apart).  They are indexed like the state
 * at the start of that iteration: read them after an iteration without a
 * Morton re-sort (a re-sort permutes the state, not these fields). */
enum abm_field {
    ABM_POS = 0, ABM_DIAM = 1, ABM_VOL = 2, ABM_GROWTH = 3, ABM_UID = 4, ABM_STATIC = 5,
    ABM_NZ = 6, ABM_NBR_COUNT = 7, ABM_CONTACT_COUNT = 8, ABM_FORCE = 9, ABM_DISP = 10,
    ABM_BOX = 11, ABM_AGE = 12
};

typedef struct abm_batch abm_batch;
typedef struct abm_batch abm_pop; /* a population is a batch of one simulation */

/* ------------------------------------------------------------------------- */
/* Batched simulations: n_sims independent populations advanced together,     */
/* one captured HIP graph launch per iteration.                                */
/* ------------------------------------------------------------------------- */

/* Workspace bytes for n_sims simulations with these agent and grid-box
 * capacities (arrays of n_sims).  The grid of a simulation needs 64 box
 * slots per aligned 4x4x4 block of boxes that it touches, i.e.
 * 64 * ceil(dx/4) * ceil(dy/4) * ceil(dz/4) for dx x dy x dz boxes; a larger
 * grid fails the step with ABM_ERR_CAPACITY.  Returns 0 for invalid sizes. */
size_t abm_batch_workspace_bytes(int n_sims, const int64_t *capacity, const int64_t *box_capacity);

/* Create a batch.  per_sim: n_sims parameter sets.  n0: initial agents per
 * simulation.  xyz (sum(n0) x 3, simulation-major), diam, vol, growth and uid
 * (sum(n0) each) are host or device arrays per inputs_on_device; vol = NULL
 * derives pi d^3/6, growth = NULL means 0, uid = NULL numbers each
 * simulation's agents 0..n0-1.  Capacities as in abm_batch_workspace_bytes.
 * hip_stream: stream for all work of this handle (NULL = default stream).
 * Errors: ABM_ERR_ARG (n0 > capacity, bad parameters, workspace too small),
 * ABM_ERR_NONFINITE (non-finite input), ABM_ERR_HIP. */
int abm_batch_create(int n_sims, const abm_params *per_sim, const int64_t *n0, const double *xyz,
                     const double *diam, const double *vol, const double *growth, const uint64_t *uid,
                     int inputs_on_device, const int64_t *capacity, const int64_t *box_capacity,
                     void *workspace, size_t ws_bytes, void *hip_stream, abm_batch **out);

/* Restore per-agent static flags, non-zero-force counts and ages, the next
 * uid and the iteration counter of every simulation (checkpoint resume:
 * query a running batch, create a new one from the queried arrays, restore;
 * also the way to give a new population its initial ages).  is_static
 * (uint8), nz (int32) and age (int32, >= 0) are sum(n) arrays in the
 * creation order; next_uid has n_sims entries; any of the four may be NULL
 * (ages then start at 0).  Only valid right after abm_batch_create, before
 * any step, tune or other restore (ABM_ERR_ARG otherwise: the state is no
 * longer in creation order). */
int abm_batch_restore(abm_batch *b, const uint8_t *is_static, const int32_t *nz, const int32_t *age,
                      const uint64_t *next_uid, int64_t iteration, int on_device);

/* Advance every simulation by n_iter iterations (stream-ordered, graph
 * launched; the call waits for the stream once at the end to read the status).
 * ABM_ERR_CAPACITY: a division or the grid would exceed a capacity; the
 * batch is left at the last completed iteration.  ABM_ERR_NONFINITE: a
 * non-finite position or force appeared. */
int abm_batch_step(abm_batch *b, int n_iter);

/* Current agent counts (n_sims entries, host). */
int abm_batch_num_agents(abm_batch *b, int64_t *n_out);

/* Number of agents (whole batch) whose force, contact and move decisions the
 * last iteration took on the FP64 path because the FP32 sweep could not
 * certify them (guard bands around the decision thresholds, Eq 4.1-4.2 and
 * the adherence rule of Sec 5.5).  A statistic; *n_out is host memory. */
int abm_batch_fp64_agents(abm_batch *b, int64_t *n_out);

/* Copy one field of simulation `sim` into dst (capacity `cap` elements of the
 * field's type); *n_out receives the number of agents. */
int abm_batch_query(abm_batch *b, int sim, int field, void *dst, int dst_on_device, int64_t cap, int64_t *n_out);

/* Grid of the last iteration of simulation `sim`: lo[3], L, dims[3]. */
int abm_batch_grid(abm_batch *b, int sim, double lo[3], double *L, int64_t dims[3]);

/* Spheroid statistics of every simulation: centroid (n_sims x 3), radius of
 * gyration and largest distance from the centroid (n_sims each), and the
 * 32-bin radial density histogram on [0, hist_rmax) in agents per 1000 um^3
 * (agents beyond hist_rmax go to the last bin) (n_sims x 32).  Host arrays;
 * any may be NULL.  FP64 reductions in a fixed order (deterministic). */
int abm_batch_stats(abm_batch *b, double hist_rmax, double *centroid, double *r_gyr, double *r_max, float *hist);

/* Histograms only, to host or device memory (n_sims x 32 floats). */
int abm_batch_hist(abm_batch *b, double hist_rmax, float *out, int out_on_device);

/* Autotune the launch schedule of the batch by timing candidates from a
 * snapshot of the state, one stage after the other: the persistent work
 * groups of the unit sweep (512..4096), the work groups and waves per work
 * group of the box-wise sweep (512..4096 x 2 or 4 waves), and, when some
 * simulation sets resort_every < 0, the Morton re-sort period (5, 10 or 20
 * iterations, each timed over 20 iterations so that its re-sorts count;
 * Sec 5.4.2, Fig 5.14).  Stages 1-2 time n_trial_iters iterations per
 * candidate.  The batch is restored afterwards, so results are unchanged.
 * This call allocates (and frees) one snapshot of the workspace.  Writes the
 * chosen sweep work-group count to *grid_out (may be NULL); the whole
 * schedule is read with abm_batch_schedule.  (The sweep's work unit, an
 * aligned 4x4x4 block of boxes, is fixed: the box-slot layout is built on it.) */
int abm_batch_tune(abm_batch *b, int n_trial_iters, int *grid_out);

/* The launch schedule in use: unit-sweep work groups, box-wise work groups
 * and waves per work group, Morton re-sort period (0 = never).  Any pointer
 * may be NULL. */
int abm_batch_schedule(abm_batch *b, int *sweep_grid, int *dense_grid, int *dense_waves, int *resort_every);

/* Set the number of persistent workgroups of the force sweep (a multiple of
 * 8, one share per XCD; default 2048). */
int abm_batch_set_sweep_grid(abm_batch *b, int workgroups);

/* Measurement: with timing on, abm_batch_step replays each iteration as two
 * graph launches (the force sweep, then the rest) with HIP events recorded on
 * the handle's stream around the sweep.  abm_batch_sweep_time returns the
 * summed sweep milliseconds and the number of sweeps since its last call
 * (and resets both).  Results are identical with timing on or off. */
int abm_batch_set_timing(abm_batch *b, int on);
int abm_batch_sweep_time(abm_batch *b, double *ms_total, int64_t *n_sweeps);

/* Release the handle (the workspace stays the caller's). */
int abm_batch_destroy(abm_batch *b);

/* ------------------------------------------------------------------------- */
/* Single population: thin wrappers of the batch calls with n_sims = 1.       */
/* ------------------------------------------------------------------------- */
size_t abm_pop_workspace_bytes(const abm_params *p, int64_t capacity, int64_t box_capacity);
int abm_pop_create(const abm_params *p, int64_t n, const double *xyz, const double *diam, const double *vol,
                   const double *growth, const uint64_t *uid, int inputs_on_device, void *workspace,
                   size_t ws_bytes, int64_t capacity, int64_t box_capacity, void *hip_stream, abm_pop **out);
int abm_pop_step(abm_pop *p, int n_iter);
int abm_pop_num_agents(abm_pop *p, int64_t *n);
int abm_pop_query(abm_pop *p, int field, void *dst, int dst_on_device, int64_t cap, int64_t *n_out);
int abm_pop_stats(abm_pop *p, double hist_rmax, double centroid[3], double *r_gyr, double *r_max, float hist[32]);
int abm_pop_destroy(abm_pop *p);

/* ------------------------------------------------------------------------- */
/* Surrogate MLP (35 -> 256 -> 256 -> 256 -> 32, exact-erf GELU on the hidden */
/* layers), BF16 matrix-core GEMMs with FP32 accumulation, FP32 master        */
/* weights, mean-squared-error loss, Adam.  Parameter layout of get/set: per  */
/* layer W as [out, in] row-major then b as [out].                            */
/* ------------------------------------------------------------------------- */
typedef struct abm_mlp abm_mlp;

/* Workspace bytes for an MLP with these layer widths and maximum batch. */
size_t abm_mlp_workspace_bytes(const int *dims, int n_dims, int max_batch);

/* Create with He-normal weights (std sqrt(2/fan_in)) and zero biases drawn
 * from Philox4x32-10 keyed by seed.  dims must be 35,256,256,256,32 or any
 * widths that are multiples of 16 except the input width. */
int abm_mlp_create(const int *dims, int n_dims, int max_batch, uint64_t seed, void *workspace, size_t ws_bytes,
                   void *hip_stream, abm_mlp **out);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the MSE of a batch
 * (x: batch x dims[0], y: batch x dims[last], device FP32).  The loss is
 * written to *loss_out (host) when loss_out is not NULL. */
int abm_mlp_train_step(abm_mlp *m, const float *x, const float *y, int batch, float lr, float *loss_out);

/* Loss and gradient (FP32, parameter layout above, device pointer) of a batch
 * without updating the weights. */
int abm_mlp_grads(abm_mlp *m, const float *x, const float *y, int batch, float *grads_out, float *loss_out);

/* Forward pass: y = MLP(x) for a batch (device FP32). */
int abm_mlp_infer(abm_mlp *m, const float *x, float *y, int batch);

/* The forward pass of abm_mlp_infer (the same kernels and arithmetic, so the
 * same y bit for bit) for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  It calls no
 * allocating routine: its activations go to a fixed device array of 12 MiB
 * inside the library, which every GPU the library runs on holds until the
 * process ends.  Limits: batch 1..4096 and input and hidden widths up to 512
 * (ABM_ERR_ARG beyond them; max_batch of the handle does not apply).  The
 * first call on a device looks up that device's copy of the array with the
 * device current, so call it with the handle's device current.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * x: batch x dims[0], y: batch x dims[last], device FP32, on the handle's stream. */
int abm_mlp_infer_noalloc(abm_mlp *m, const float *x, float *y, int batch);

/* Copy the FP32 master parameters out of / into the handle (device FP32). */
int abm_mlp_get_params(abm_mlp *m, float *dst, size_t n);
int abm_mlp_set_params(abm_mlp *m, const float *src, size_t n);
size_t abm_mlp_num_params(abm_mlp *m);
int abm_mlp_destroy(abm_mlp *m);

/* ------------------------------------------------------------------------- */
/* SIR epidemiology (Sec 4.6.3): persons in a cubic space [0, S]^3 with a      */
/* state each (susceptible, infected, recovered).  Per iteration, from the    */
/* start-of-iteration state (copy semantics, Sec 5.2.1), every person runs    */
/* its behaviours in the order:                                               */
/*   infection  a susceptible person that draws U < infection_prob becomes    */
/*              infected if an infected person is strictly within the         */
/*              infection radius (Algorithm 3)                                */
/*   recovery   an infected person (also one infected just now) recovers if   */
/*              it draws U < recovery_prob (Algorithm 4)                      */
/*   movement   a step of length `speed` along three uniforms in (-1, 1)      */
/*              normalised to unit length, then the boundary (Algorithm 5,    */
/*              Sec 4.4.11): toroidal wraps every coordinate into [0, S) with */
/*              fmod, closed clamps it to [0, S].                             */
/* On the torus, distances are minimum-image.  Draws: Philox4x32-10 with      */
/* counter (uid, iteration, sim_id) and key (seed low XOR tag, seed high),    */
/* tags 'INFE', 'RECO', 'MOVE'; a word w gives (w + 1/2) 2^-32.  Positions    */
/* are FP64 and every operation is IEEE-rounded as written, so results are    */
/* deterministic and independent of the storage order.                       */
/* ------------------------------------------------------------------------- */
#define ABM_SIR_SUSCEPTIBLE 0
#define ABM_SIR_INFECTED 1
#define ABM_SIR_RECOVERED 2
#define ABM_BOUNDARY_TOROIDAL 0
#define ABM_BOUNDARY_CLOSED 1

/* Fields of abm_sir_query: positions (double, n x 3 interleaved), states
 * (uint8), uids (uint32).  Rows are in the handle's storage order (persons
 * are re-sorted by grid box every few iterations), the same order for every
 * field between two steps. */
#define ABM_SIR_POS 0
#define ABM_SIR_STATE 1
#define ABM_SIR_UID 2

typedef struct abm_sir_params {
    double space;          /* side S of the cubic space (> 0) */
    double radius;         /* infection radius (> 0) */
    double infection_prob; /* in [0, 1] */
    double recovery_prob;  /* in [0, 1] */
    double speed;          /* step length per iteration (>= 0) */
    int32_t boundary;      /* ABM_BOUNDARY_TOROIDAL or ABM_BOUNDARY_CLOSED */
    uint32_t sim_id;       /* counter word of the draws */
    uint64_t seed;
} abm_sir_params;

typedef struct abm_sir abm_sir;

/* Workspace bytes for n persons (n < 2^31) and a history of hist_cap
 * iterations of counts; 0 for invalid arguments. */
size_t abm_sir_workspace_bytes(const abm_sir_params *p, int64_t n, int hist_cap);

/* Create from host arrays: pos (n x 3 interleaved, every coordinate in
 * [0, S]), state (n bytes, 0..2); person k gets uid k.  The workspace
 * (device memory of at least abm_sir_workspace_bytes) is owned by the caller
 * and must outlive the handle; every kernel runs on hip_stream (NULL: the
 * default stream).  Errors: ABM_ERR_ARG (bad parameters or inputs, workspace
 * too small), ABM_ERR_NONFINITE (a non-finite coordinate), ABM_ERR_HIP. */
int abm_sir_create(const abm_sir_params *p, int64_t n, const double *pos, const uint8_t *state, int hist_cap,
                   void *workspace, size_t ws_bytes, void *hip_stream, abm_sir **out);

/* Advance n_iter iterations.  counts (host, n_iter x 3 int64, or NULL)
 * receives the numbers of susceptible, infected and recovered persons after
 * each iteration.  Synchronises the stream when counts is not NULL. */
int abm_sir_step(abm_sir *s, int n_iter, int64_t *counts);

/* Copy one field (ABM_SIR_*) to dst (host, or device when dst_on_device);
 * cap: rows dst holds (ABM_ERR_ARG if fewer than the persons). */
int abm_sir_query(abm_sir *s, int field, void *dst, int dst_on_device, int64_t cap);

/* Iterations done and persons per state now (host). */
int abm_sir_counts(abm_sir *s, int64_t *iteration, int64_t counts[3]);

/* Grid of the neighbour search (an index of the infected persons, rebuilt
 * every iteration): boxes per axis and box length (>= 2 radius). */
int abm_sir_grid(abm_sir *s, int64_t *dims, double *box_len);

/* Timing of the person kernel (infection, recovery, movement, binning of the
 * persons infected after it):
 * with timing on, every iteration brackets it with HIP events on the
 * handle's stream; abm_sir_kernel_time returns the total and the count of the
 * iterations timed since the last call, and resets them. */
int abm_sir_set_timing(abm_sir *s, int on);
int abm_sir_kernel_time(abm_sir *s, double *ms_total, int64_t *n_launches);

int abm_sir_destroy(abm_sir *s);

/* ------------------------------------------------------------------------- */
/* Extracellular diffusion with secreting, chemotactic cells (Sec 4.5.2,      */
/* Eq 4.3; soma clustering, Sec 4.7.1, Algorithms 6-7).  n_substances         */
/* concentration grids of R^3 points at the voxel centres of the cubic space  */
/* [lo, lo + S]^3 (dx = S / R); a position belongs to voxel                   */
/* floor((x - lo) / dx), clamped to [0, R - 1].  Per iteration, from the      */
/* start-of-iteration state:                                                  */
/*   chemotaxis  every cell moves by gradient_weight along the normalised     */
/*               central-difference gradient (u[+1] - u[-1]) / (2 dx) of its  */
/*               substance at its voxel (no move where it vanishes); the      */
/*               new coordinates are clamped to the space (Algorithm 7)       */
/*   secretion   every voxel gains secretion times the number of cells of     */
/*               that substance's type in it at the start (Algorithm 6)       */
/*   diffusion   Eq 4.3, evaluated left to right as                           */
/*               u (1 - mu dt) + c ((u[x+1] - 2u) + u[x-1]) + c (... y) +     */
/*               c (... z), c = (nu dt) / (dx dx), zero beyond the grid (the  */
/*               substances diffuse out of the space).                        */
/* All arithmetic is FP64 and IEEE-rounded as written (no contraction), so    */
/* results do not depend on the order in which cells or voxels are visited.   */
/* ------------------------------------------------------------------------- */
#define ABM_SOMA_POS 0  /* double, n_cells x 3 interleaved */
#define ABM_SOMA_TYPE 1 /* int32, n_cells */
#define ABM_SOMA_CONC 2 /* double, n_substances x R^3 (x fastest, then y, z) */

typedef struct abm_soma_params {
    double lo;              /* lower corner of the space on every axis */
    double space;           /* side S (> 0) */
    int32_t resolution;     /* grid points per axis R (1 .. 2048) */
    int32_t n_substances;   /* 1 .. 16; cells of type t follow substance t */
    double diffusion;       /* nu (>= 0) */
    double decay;           /* mu (>= 0) */
    double dt;              /* time step (> 0) */
    double secretion;       /* quantity per cell and iteration */
    double gradient_weight; /* length of a chemotaxis step */
} abm_soma_params;

typedef struct abm_soma abm_soma;

/* Workspace bytes for n_cells cells (0 allowed: diffusion alone); 0 for
 * invalid arguments. */
size_t abm_soma_workspace_bytes(const abm_soma_params *p, int64_t n_cells);

/* Create from host arrays: pos (n_cells x 3 interleaved, inside the space),
 * type (n_cells int32 in [0, n_substances)), conc (n_substances x R^3
 * initial concentrations, or NULL for zero).  The workspace (device memory of
 * at least abm_soma_workspace_bytes) is owned by the caller and must outlive
 * the handle; kernels run on hip_stream.  Errors: ABM_ERR_ARG (bad
 * parameters or inputs, workspace too small), ABM_ERR_NONFINITE (a
 * non-finite position or concentration), ABM_ERR_HIP. */
int abm_soma_create(const abm_soma_params *p, int64_t n_cells, const double *pos, const int32_t *type,
                    const double *conc, void *workspace, size_t ws_bytes, void *hip_stream, abm_soma **out);

/* Advance n_iter iterations (asynchronous on the handle's stream). */
int abm_soma_step(abm_soma *s, int n_iter);

/* Copy one field (ABM_SOMA_*) to dst (host, or device when dst_on_device);
 * cap: elements dst holds (rows for POS and TYPE, values for CONC);
 * ABM_ERR_ARG if it is too small.  Cells keep their creation order. */
int abm_soma_query(abm_soma *s, int field, void *dst, int dst_on_device, int64_t cap);

/* Timing of the diffusion kernel (Eq 4.3 over every substance): with timing
 * on, every iteration brackets it with HIP events on the handle's stream;
 * abm_soma_kernel_time returns the total and the count of the iterations
 * timed since the last call, and resets them. */
int abm_soma_set_timing(abm_soma *s, int on);
int abm_soma_kernel_time(abm_soma *s, double *ms_total, int64_t *n_launches);

int abm_soma_destroy(abm_soma *s);

/* Message of the last failed call on this thread ("" if none). */
const char *abm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ABM_H */
