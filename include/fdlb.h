/*
 * fdlb.h -- C ABI of libfdlb, an MI355X (gfx950) implementation of the
 * finite-difference lattice Boltzmann method of Ghiroldi & Gibelli,
 * "A finite-difference lattice Boltzmann approach for gas microflows"
 * (arXiv 1308.0692).
 *
 * The method: discrete velocities xi_alpha and weights w_alpha from a
 * half-range (or full-range) Gauss-Hermite rule (Table I, tensor product in
 * two dimensions); weighted populations f_alpha (Eq. 2) obey the linearised
 * BGKW model of Eq. (1) with the isothermal equilibrium of Eq. (5); density
 * and momentum are the sums of Eqs. (6)-(7); solid walls re-emit the
 * populations that leave them with the diffuse Maxwell condition of Eq. (8),
 * whose wall density comes from the impermeability sum of Eq. (9).  One time
 * step relaxes with an explicit Euler step and then transports with a
 * first-order upwind difference (the paragraph that introduces the fully
 * discrete scheme, before the Couette problem).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Geometry: the unit square, N_x x N_y cell-centred cells (dx = 1/N_x,
 *    dy = 1/N_y); walls lie on the outer cell faces.  An axis is either
 *    bounded by two walls or periodic; a periodic axis must have exactly one
 *    cell (the paper's planar Couette flow), so transport along it vanishes.
 *  - Walls: index 0 bottom (y = 0), 1 top (y = 1), 2 left (x = 0), 3 right
 *    (x = 1).  wall_u[i] is the wall's tangential speed: along +x for the
 *    bottom/top walls, along +y for the left/right walls.  A periodic axis has
 *    no walls: the speeds given for them are ignored.  Either kind of rule
 *    may serve either kind of axis: a half-range rule on a bounded axis is the
 *    paper's method, a full-range one its standard lattice.
 *  - Wall density (Eq. 9): the flux arriving at a wall face divided by the
 *    flux the emission of Eq. (8) carries away per unit density,
 *    rho_w = sum_{xi.n<0} |xi.n| f / sum_{xi.n>0} (xi.n) w, which keeps every
 *    wall impermeable.  For a half-range rule the denominator is
 *    (2 pi)^(-1/2) and this is Eq. (9) as printed.  A population moving along
 *    a wall (xi.n = 0, odd full-range rules) neither arrives nor leaves.
 *  - Velocity order: alpha = j * Q_x + i, i indexing the x rule and j the y
 *    rule, both rules with nodes ascending.
 *  - Host arrays of cell fields are row-major [y][x] (N_x fastest), doubles.
 *    Population arrays are [alpha][y][x], doubles, raw f_alpha (not deviations).
 *  - Device memory is owned by the caller: the library never allocates or
 *    frees device memory, and keeps none beyond what fdlb_bind hands it except
 *    one static array of FDLB_STATIC_SCRATCH_BYTES per GPU that its code
 *    object carries (the workspace of fdlb_step_static).  Host buffers passed
 *    in are owned by the caller and not retained after return.
 *  - Streams: `stream` arguments are hipStream_t values passed as void*;
 *    NULL means the default stream.  Every call that launches work enqueues
 *    it on the bound stream.  Calls documented as synchronous wait for that
 *    stream; all others return without waiting.
 *  - Errors: every int-returning function returns FDLB_OK (0), a negative
 *    error code, or a positive warning.  fdlb_last_error() gives a message
 *    for the calling thread.  No C++ exception crosses this interface.  A
 *    handle must not be used from two threads at once; distinct handles are
 *    independent.
 */
#ifndef FDLB_H
#define FDLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FDLB_OK 0
#define FDLB_ENOTCONVERGED 1 /* warning: max_steps reached above the tolerance */
#define FDLB_EINVAL (-1)     /* invalid argument */
#define FDLB_EUNSTABLE (-2)  /* CFL > 1 or dt/Kn > 1 without allow_unstable */
#define FDLB_EHIP (-3)       /* a HIP runtime call failed (message has the HIP error) */
#define FDLB_EDIVERGED (-4)  /* non-finite residual or |u| > 0.5 during a solve */
#define FDLB_ESTATE (-5)     /* call out of order (e.g. not bound) */
#define FDLB_ENOMEM (-6)     /* host allocation failed */

/* ---- enumerations -------------------------------------------------------- */
#define FDLB_HALF 0 /* half-range Gauss-Hermite rule, n nodes per half-line */
#define FDLB_FULL 1 /* full-range Gauss-Hermite rule, n nodes */
#define FDLB_FP64 0 /* populations stored and updated in double */
#define FDLB_FP32 1 /* deviations f_alpha - w_alpha stored and updated in float;
                       wall densities and the residual in double */
#define FDLB_MIXED 2 /* FDLB_FP32 kernels until a steady solve nears its tolerance,
                        then the state is widened in place and FDLB_FP64 kernels
                        finish; the state buffers are sized for double */

/* FDLB_MIXED leaves float, during fdlb_solve_steady / fdlb_batch_solve with
 * tol < FDLB_MIXED_SWITCH_R, at the first host check whose residual is below
 * FDLB_MIXED_SWITCH_R, or once the lowest residual seen has not fallen by 10 %
 * for FDLB_MIXED_STALL_STEPS steps.  Float deviations carry about 7 digits,
 * which puts the float residual floor near 1e-8 (rounding makes the float
 * iteration cycle instead of settling; 1.1-2.3e-8 on the cavities measured),
 * so the switch level sits just above it. */
#define FDLB_MIXED_SWITCH_R 3e-8
#define FDLB_MIXED_STALL_STEPS 4000
#define FDLB_WALL_BOTTOM 0
#define FDLB_WALL_TOP 1
#define FDLB_WALL_LEFT 2
#define FDLB_WALL_RIGHT 3

/* ---- quadrature (Eq. 4, Table I, tensor product after Table I) ----------- */

/*
 * Half-range rule for the weight (2 pi)^(-1/2) exp(-xi^2/2) on [0, inf),
 * mirrored onto (-inf, 0]: the n-point Gauss rule of each half-line.  Writes
 * 2n nodes in ascending order and their weights (summing to 1) into
 * caller-owned arrays of 2n doubles.  n in 1..16, else FDLB_EINVAL.
 * Host only; needs no GPU.
 */
int fdlb_quad_half_range(int n_per_half, double *nodes, double *weights);

/*
 * Full-range Gauss-Hermite rule for the same weight on the whole line
 * (probabilists' Hermite roots): n nodes ascending and weights summing to 1.
 * n in 1..32, else FDLB_EINVAL.  Host only.
 */
int fdlb_quad_full_range(int n, double *nodes, double *weights);

/* ---- problem description --------------------------------------------------- */

typedef struct fdlb_problem_desc {
    int32_t nx, ny;                 /* cells; >= 1 */
    double lx, ly;                  /* domain lengths in units of the length l of Kn (0 means 1) */
    int32_t periodic_x, periodic_y; /* 1: periodic axis (then that N must be 1) */
    double wall_u[4];               /* tangential wall speeds (see conventions) */
    double kn;                      /* Knudsen number of Eq. (1); INFINITY allowed */
    double cfl;                     /* Courant number in (0, 1]; 0.9 is customary */
    int32_t qx_kind, qx_n;          /* FDLB_HALF (n per half) or FDLB_FULL (n total) */
    int32_t qy_kind, qy_n;
    int32_t precision;              /* FDLB_FP64, FDLB_FP32 or FDLB_MIXED */
    int32_t allow_unstable;         /* 1: accept CFL > 1 or dt/Kn > 1 (tests only) */
} fdlb_problem_desc;

typedef struct fdlb_problem fdlb_problem; /* opaque host handle */

/*
 * Validate a description and build the velocity set, the time step
 * dt = cfl / max_alpha(|xi_x| N_x / l_x [x bounded] + |xi_y| N_y / l_y [y bounded])
 * and omega = dt / Kn (0 for Kn = INFINITY).  Cells are l_x / N_x by l_y / N_y.  Host only (no GPU call); the
 * handle owns only host memory.  FDLB_EINVAL for bad sizes or rules.
 * Every rule needs at least 2 nodes (per half-line
 * for half-range) so that it integrates xi^2 exactly and the relaxation of
 * Eqs. (1), (5) conserves momentum; FDLB_EINVAL otherwise.  FDLB_EUNSTABLE if
 * cfl > 1 or omega > 1 and allow_unstable is 0.
 */
int fdlb_problem_create(const fdlb_problem_desc *desc, fdlb_problem **out);
void fdlb_problem_destroy(fdlb_problem *p); /* NULL is a no-op; no GPU call */

int fdlb_problem_q(const fdlb_problem *p);         /* number of velocities, or < 0 */
double fdlb_problem_dt(const fdlb_problem *p);     /* time step (NaN for NULL) */
double fdlb_problem_omega(const fdlb_problem *p);  /* dt / Kn */
/* Copy the velocity set (Q entries each, velocity order above) into caller arrays. */
int fdlb_problem_velocities(const fdlb_problem *p, double *xi_x, double *xi_y, double *w);

/*
 * Device memory the caller must provide: the state (two population buffers
 * of Q N_x N_y values each, in the problem's precision) and a workspace
 * (moments, wall fluxes, residual partials, tables, outputs).  Both sizes
 * are in bytes; base addresses must be 256-byte aligned.
 */
size_t fdlb_state_bytes(const fdlb_problem *p);
size_t fdlb_workspace_bytes(const fdlb_problem *p);

/*
 * Hand the library device buffers of at least the sizes above and the stream
 * to use.  Uploads the velocity tables (asynchronously, on the stream).  The
 * buffers stay owned by the caller and must outlive the binding; binding
 * again replaces the previous binding.  The state is undefined until one of
 * the init/upload calls below.
 */
int fdlb_bind(fdlb_problem *p, void *d_state, void *d_workspace, void *stream);

/* ---- initial state --------------------------------------------------------- */

/*
 * Seed every cell at equilibrium, f_alpha = w_alpha rho (1 + xi_alpha . u)
 * (Eqs. 3, 5), from host arrays of N_x N_y doubles ([y][x]).  NULL rho means
 * rho = 1, NULL ux/uy mean zero.  With renormalize_mass, rho is first scaled
 * so that its sum over cells is N_x N_y (the steady state scales with the
 * total mass, which the scheme conserves).  Resets the step counter.
 */
int fdlb_init_equilibrium(fdlb_problem *p, const double *rho, const double *ux, const double *uy,
                          int renormalize_mass);

/*
 * Same from device arrays of N_x N_y floats each (e.g. a network's output),
 * laid out [y][x]; none may be NULL.  Renormalisation as above, on device
 * (asynchronous): a density field whose sum is not positive leaves a NaN
 * state, which the next fdlb_solve_steady reports as FDLB_EDIVERGED (the host
 * variant returns FDLB_EINVAL instead).
 */
int fdlb_init_equilibrium_dev(fdlb_problem *p, const float *d_rho, const float *d_ux, const float *d_uy,
                              int renormalize_mass);

/*
 * Replace the state by raw populations from a host array of Q N_x N_y doubles
 * ([alpha][y][x]); the FP32 path stores f - w rounded to float.  With
 * fdlb_state_download this is checkpoint/resume.  Synchronous.
 */
int fdlb_state_upload(fdlb_problem *p, const double *f_host);
int fdlb_state_download(fdlb_problem *p, double *f_host); /* synchronous */

/*
 * Exact checkpoint of the carried state (current populations in the stored
 * precision, their moment and wall-flux buffers, the step counter) as an
 * opaque host byte buffer of fdlb_checkpoint_bytes() bytes, owned by the
 * caller.  Loading it into a problem built from the same description and
 * marching on gives bit-identical results to never having stopped.  The
 * buffer opens with a header naming the problem (grid, both velocity rules,
 * precision), checked first: a checkpoint of another problem gives
 * FDLB_EINVAL and leaves the state untouched.  A checkpoint saved after a
 * steady solve restores as a state that marches on (the solve's request to
 * stop at its converged step is not restored).  Synchronous.
 */
size_t fdlb_checkpoint_bytes(const fdlb_problem *p);
int fdlb_checkpoint_save(fdlb_problem *p, void *host_buf);
int fdlb_checkpoint_load(fdlb_problem *p, const void *host_buf);

/* ---- time marching ------------------------------------------------------------ */

/*
 * Advance nsteps time steps, asynchronously on the bound stream.  Each step
 * relaxes every population by an explicit Euler step of Eq. (1) toward the
 * equilibrium of Eq. (5), re-emits the populations leaving each wall with
 * Eq. (8) and the wall density of Eq. (9), transports with the first-order
 * upwind difference of the fully discrete scheme, and forms the moments of
 * Eqs. (6)-(7) and the step's residual (fdlb_last_residual).
 * A launch of at most 1024 tiles (blocks) reduces each step's residual inside
 * the next step's launch (one extra block) and once more at the end of the
 * call; larger grids launch a reduction kernel after every step.  Either way
 * the control block holds every step's residual when the call's work ends.
 */
int fdlb_step(fdlb_problem *p, int64_t nsteps);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fdlb_step
 * on a state buffer the caller passes, with no workspace from the caller and
 * no allocation by the library.  The moments, wall fluxes, residual partial
 * sums, control block and velocity table live in one static device array of
 * FDLB_STATIC_SCRATCH_BYTES per GPU, which the library holds from its first
 * use on that GPU until the process ends.
 *   p        a problem from fdlb_problem_create with precision FDLB_FP32 or
 *            FDLB_FP64 (FDLB_MIXED gives FDLB_EINVAL).  It need not be bound;
 *            if it is, its binding, state and step counter are not touched.
 *            Its tile choice (fdlb_problem_set_tile) is used.
 *   d_state  device buffer of fdlb_state_bytes(p) bytes, 256-byte aligned,
 *            owned by the caller: two halves of fdlb_state_bytes(p)/2 bytes.
 *            On entry the first half holds the populations as deviations
 *            h_alpha = f_alpha - w_alpha in the storage type (float for
 *            FDLB_FP32, double for FDLB_FP64), planes [alpha][y][x] in the
 *            velocity order above (the layout of a bound state buffer after an
 *            init).  On return of the work, the state after nsteps steps is
 *            in half (nsteps mod 2); the other half is overwritten.  The steps
 *            are those fdlb_step takes from the same state (bit-identical on
 *            the same tile).
 *   nsteps   >= 0.
 *   stream   hipStream_t (as void*) of the current device; the work is
 *            enqueued on it and the call returns without waiting for it.
 * Errors: FDLB_EINVAL for a NULL or misaligned buffer, nsteps < 0, a
 * FDLB_MIXED problem, or a problem whose workspace (without the host staging
 * area) exceeds FDLB_STATIC_SCRATCH_BYTES (every grid of at most 512 x 512
 * cells fits, at any Q); nothing is enqueued then.  FDLB_EHIP for HIP errors.
 * Calls on one GPU share its array: calls whose work overlaps on one GPU
 * (two streams, or two threads) race and give undefined results; calls in
 * stream order do not interfere, each rewriting what it reads before it
 * reads it.  The state buffer must hold finite values.
 */
#define FDLB_STATIC_SCRATCH_BYTES ((size_t)16 << 20)
int fdlb_step_static(fdlb_problem *p, void *d_state, int64_t nsteps, void *stream);

/*
 * Advance nsteps steps as fdlb_step does (same states), but with a reduction
 * kernel after every step and HIP events recorded on the bound stream around
 * every kernel launch; returns the summed device time of the fused step
 * kernels and of the residual-reduction kernels, in milliseconds (either
 * pointer may be NULL).  Synchronous.
 */
int fdlb_step_timed(fdlb_problem *p, int64_t nsteps, double *ms_step_kernels, double *ms_reduce_kernels);

/*
 * Residual of the most recent step, R = ||u^{n+1} - u^n||_2 / ||u^{n+1}||_2
 * over all cells (both velocity components), and the number of steps since
 * the last init.  The paper states no stopping rule; this relative change of
 * the velocity field (Eq. 7) per step is the one every solve here uses.
 * Synchronous.
 */
int fdlb_last_residual(fdlb_problem *p, double *residual, int64_t *steps);

typedef struct fdlb_report {
    int64_t steps;          /* steps taken by the call */
    int64_t first_below;    /* step count at which R first fell below tol, or -1 */
    double residual;        /* residual of the last step */
    double wall_s;          /* wall time of the call (host clock, after sync) */
    double updates_per_s;   /* N_x N_y Q steps / wall_s */
    double bytes_per_s;     /* algorithmic bytes (2 x population size per update) / wall_s */
    int32_t status;         /* same as the return value */
    int32_t history_len;    /* entries written to history */
    int32_t history_cap;    /* capacity of history (set by the caller) */
    int32_t pad_;
    double *history;        /* caller-owned, may be NULL: residual at every check */
    int64_t steps_fp32;     /* steps of the call taken in float (FDLB_MIXED: before the switch) */
} fdlb_report;

/*
 * March until the residual of a step falls below tol or max_steps steps have
 * been taken.  The device stops updating the state at the first step whose
 * residual is below tol (or that diverges), so the state returned is that
 * step's; the host reads the control block every check_every steps (the only
 * device-to-host synchronisation in the loop).  use_graph = 1 replays
 * check_every steps as one captured HIP graph.  A later fdlb_step resumes
 * unconditional stepping.  Synchronous.  Returns FDLB_OK, FDLB_ENOTCONVERGED
 * or FDLB_EDIVERGED.
 */
int fdlb_solve_steady(fdlb_problem *p, double tol, int64_t max_steps, int32_t check_every,
                      int32_t use_graph, fdlb_report *report);

/*
 * A faster steady iteration of the same discrete model (the paper calls for better
 * solvers than plain time marching): with on != 0, every later step of the problem
 * moves each population by its own multiple of the step's change,
 *   h <- h + s_alpha (S h - h),
 * S the step of the scheme, instead of h <- S h.  A fixed point of one is a fixed point
 * of the other, so a steady solve reaches the same steady state (to the tolerance of
 * its residual); the iterates are then pseudo-time levels, not the time evolution.
 * The stretch s_alpha >= 1 is as large as a Fourier analysis of one velocity's update
 * (equilibrium held fixed) allows with the problem's own margin:
 *   s_alpha = max(1, min(cfl / (nu_alpha (1 - omega) + omega / 2), 1 / omega, 64)),
 *   nu_alpha = dt (|xi_x| N_x / l_x + |xi_y| N_y / l_y)  (bounded axes only),
 * so that s (omega + 2 nu (1 - omega)) <= 2 cfl and the stretched relaxation rate s omega <= 1
 * (the slow velocities no longer wait for the fastest one's step).  The coupling of the
 * velocities through the equilibrium is not covered by that analysis; the iteration was
 * stable on every problem tried.  Typical gains: 2-5x fewer iterations for Kn >= 0.05,
 * less at smaller Kn where 1 / omega bounds the stretch.  fdlb_problem_pseudo_weights
 * copies s_alpha as the kernels use it (rounded to float; Q doubles, velocity order of the
 * ABI).  Off by default; host only.
 */
int fdlb_set_pseudo_time(fdlb_problem *p, int on);
int fdlb_problem_pseudo_weights(const fdlb_problem *p, double *stretch);

/* ---- outputs ---------------------------------------------------------------------- */

/*
 * Cell fields of the current state into host arrays of N_x N_y doubles
 * ([y][x]; any pointer may be NULL): density (Eq. 6), velocity (Eq. 7) and
 * the xy stress sum_alpha xi_x xi_y g_alpha of the post-relaxation state.
 * Synchronous.
 */
int fdlb_moments(fdlb_problem *p, double *rho, double *ux, double *uy, double *pxy);

/*
 * Face state along one wall after relaxation: arriving and grazing
 * populations carry the wall cell's value, leaving ones the emission of
 * Eq. (8) with rho_w of Eq. (9).  Per face (N_x faces for bottom/top, N_y
 * for left/right; pointers may be NULL): density, tangential velocity and
 * xy stress.  FDLB_EINVAL for a wall of a periodic axis.  Synchronous.
 */
int fdlb_wall_profile(fdlb_problem *p, int wall, double *rho, double *u_t, double *pxy);

/* ---- tuning --------------------------------------------------------------------- */

/*
 * Tile shapes of the step kernel.  fdlb_tile_count() gives the number of
 * compiled shapes; fdlb_tile_describe writes text such as
 * "vx4 lx32 k2 w4 nt (128x16)": cells per lane along x, lanes along x, rows
 * per lane, waves stacked along y, then "aN" (velocities split over N waves),
 * "xN" (N waves side by side), "nt" (non-temporal population stores) and
 * "pN" (N velocity planes prefetched) when present, and the tile's size in
 * cells; a buffer too short gets a truncated,
 * NUL-terminated text.
 * fdlb_problem_set_tile selects one (-1: the built-in heuristic); shapes that
 * do not fit the problem give FDLB_EINVAL.  fdlb_autotune times every
 * fitting shape for `steps` steps on the bound buffers (the state is
 * re-seeded at rest afterwards) and keeps the fastest; synchronous.
 */
int fdlb_tile_count(int precision);
int fdlb_tile_describe(int precision, int tile, char *buf, size_t len);
int fdlb_problem_set_tile(fdlb_problem *p, int tile);
int fdlb_problem_get_tile(const fdlb_problem *p);
int fdlb_autotune(fdlb_problem *p, int steps, double *best_ms_per_step);

/*
 * On-disk cache of the tile choices of fdlb_autotune and fdlb_batch_autotune: with a
 * non-empty path (a text file, created if absent), a tuning first looks up its key -- the
 * device (architecture and name), a hash of the compiled tile shapes, the precision and the
 * problem's sizes (every member's for a batch) -- and, on a hit whose tile still fits, sets
 * that tile (and re-seeds as a tuning does) without timing anything, returning the cached
 * time per step; otherwise it times the shapes and appends the result.  Lines that do not
 * parse, and files that cannot be read or written, are ignored.  NULL or "" disables the
 * cache (the default).  Process-wide; safe to call from any thread.
 */
int fdlb_set_tune_cache(const char *path);

/* ---- mixed precision (FDLB_MIXED) ------------------------------------------------- */

/*
 * Precision the kernels of a problem run in now: FDLB_FP32 or FDLB_FP64.  A
 * FDLB_MIXED problem starts every new state (init, upload) in FDLB_FP32, and
 * its tile calls above act on the table of this precision (fdlb_autotune
 * restarts the float phase and tunes it).
 */
int fdlb_problem_active_precision(const fdlb_problem *p);

/*
 * Widen the float state of a FDLB_MIXED problem to double in place (exact)
 * and recompute its moments and wall fluxes in double; marching then goes on
 * with the FDLB_FP64 kernels, from the same step count.  A no-op if already
 * in double; FDLB_EINVAL for other precisions.  Steady solves call it
 * themselves (see FDLB_MIXED_SWITCH_R).  Synchronous.
 */
int fdlb_promote(fdlb_problem *p);

/* ---- batches ---------------------------------------------------------------------- */

typedef struct fdlb_batch fdlb_batch; /* opaque: many independent problems, one launch per step */

/*
 * Build a batch of n problems (each validated as by fdlb_problem_create; all
 * must share the precision).  Every instance's state and workspace live in
 * one caller-provided arena each.  Host only.
 */
int fdlb_batch_create(const fdlb_problem_desc *descs, int n, fdlb_batch **out);
void fdlb_batch_destroy(fdlb_batch *b);
size_t fdlb_batch_state_bytes(const fdlb_batch *b);
size_t fdlb_batch_workspace_bytes(const fdlb_batch *b);
int fdlb_batch_bind(fdlb_batch *b, void *d_state, void *d_workspace, void *stream);
/* Seed instance i as fdlb_init_equilibrium / fdlb_init_equilibrium_dev do. */
int fdlb_batch_init_equilibrium(fdlb_batch *b, int i, const double *rho, const double *ux,
                                const double *uy, int renormalize_mass);
int fdlb_batch_init_equilibrium_dev(fdlb_batch *b, int i, const float *d_rho, const float *d_ux,
                                    const float *d_uy, int renormalize_mass);
/*
 * March every instance until its own residual falls below tol or max_steps.
 * Instances retire individually: an instance stops being updated at the first
 * step below tol (or at divergence), on the device, and leaves the launch at
 * the next host check.  All active instances advance together: one step-kernel
 * launch per time step for the whole batch (two while FDLB_MIXED instances run
 * in both precisions), with each instance's residual reduced as for a single
 * problem (inline for small instances, a shared reduction launch per step for
 * large ones); the host polls every check_every steps; use_graph replays
 * check_every steps as one captured graph.  All instances must have been initialised (and have taken
 * step counts of equal parity).  reports: caller array of n entries (may be
 * NULL; each entry's history/history_cap are honoured).
 * Returns FDLB_OK when every instance converged, FDLB_ENOTCONVERGED if some
 * did not, FDLB_EDIVERGED if some diverged (each report says which).
 * Synchronous.
 */
int fdlb_batch_solve(fdlb_batch *b, double tol, int64_t max_steps, int32_t check_every,
                     int32_t use_graph, fdlb_report *reports);
int fdlb_batch_moments(fdlb_batch *b, int i, double *rho, double *ux, double *uy, double *pxy);
/* Face state along one wall of instance i, as fdlb_wall_profile gives it for a problem. */
int fdlb_batch_wall_profile(fdlb_batch *b, int i, int wall, double *rho, double *u_t, double *pxy);
int fdlb_batch_state_download(fdlb_batch *b, int i, double *f_host);
/* Number of velocities of instance i (the Q of its state layout), or FDLB_EINVAL for an index
 * out of range. */
int fdlb_batch_problem_q(const fdlb_batch *b, int i);
/*
 * Instance i's raw populations from a host array in the layout of fdlb_state_upload
 * ([Q][ny][nx] float64, Eq. (2) velocities); like fdlb_batch_init_equilibrium it restarts
 * that instance (step parity 0, a mixed-precision instance back in its float phase).
 * FDLB_EINVAL for an index out of range or a NULL array.  Synchronous.
 */
int fdlb_batch_state_upload(fdlb_batch *b, int i, const double *f_host);
/*
 * One tile shape serves the whole batch (it must fit every problem).  fdlb_batch_autotune
 * times every fitting shape on the whole batch for `steps` steps (every problem is re-seeded
 * at rest afterwards) and keeps, among the shapes within 5 % of the fastest, the one that
 * splits a tile's velocities over the most waves (a batch shrinks as its members converge, and
 * its smaller launches pack the shorter blocks of such shapes better); best_ms_per_step is that
 * shape's time.  Synchronous.
 */
int fdlb_batch_set_tile(fdlb_batch *b, int tile);
int fdlb_batch_get_tile(const fdlb_batch *b);
int fdlb_batch_autotune(fdlb_batch *b, int steps, double *best_ms_per_step);
/*
 * FDLB_MIXED batches: each instance leaves float on its own (see FDLB_MIXED_SWITCH_R); while
 * some instances run in float and others in double, every step launches the two groups one
 * after the other.  The tile calls above act on the float group; the double group starts with
 * the built-in choice, and fdlb_batch_autotune also times its shapes with every instance
 * promoted to double (best_ms_per_step reports the float group's figure).
 * fdlb_batch_active_precision gives instance i's current precision.
 */
int fdlb_batch_active_precision(const fdlb_batch *b, int i);
/*
 * Tail of a batch solve: once at most max_members instances remain active (and the solve began
 * with more), each precision group switches to the built-in tile choice for its largest remaining
 * instance, if that shape fits every instance; the batch's own tiles are restored when the solve
 * returns.  A shape chosen for many concurrent instances trades latency for throughput, which
 * the last instances no longer need.  Default 8; 0 disables (every step then uses the batch's
 * tile, so an instance's results are bit-identical to a single solve with that tile).
 */
int fdlb_batch_set_retile(fdlb_batch *b, int max_members);
/* Velocity-local pseudo-time steps for every instance (see fdlb_set_pseudo_time). */
int fdlb_batch_set_pseudo_time(fdlb_batch *b, int on);

/* ---- learned warm start ----------------------------------------------------------------- */

/*
 * A small network maps (Kn, x, y) to the steady fields (rho, u_x, u_y) of a problem; its
 * prediction seeds the state at equilibrium (Eqs. 3, 5, via fdlb_init_equilibrium_dev with
 * mass renormalisation) and the solver then iterates to the tolerance as usual, so the
 * network only changes where the iteration starts.
 *
 * Network: inputs a = ((log10 Kn + 0.5) / 1.5, 2x - 1, 2y - 1) (cell centres on the unit
 * square; Kn in [0.01, 10] maps to [-1, 1]); hidden layers of width 128 with tanh; outputs
 * y = ((rho - 1) / u_w, u_x / u_w, u_y / u_w), u_w the fastest wall speed (the linearised
 * problem is linear in u_w).  Parameters: one float vector, layer by layer, W_l row-major
 * by output then b_l (W_0: 128 x 3, hidden W_l: 128 x 128, W_L: 3 x 128); 50,435 of them
 * for four hidden layers.  The 128 x 128 products use bf16 operands with fp32
 * accumulation on the matrix cores; everything else is fp32.  Loss: mean squared error
 * over samples and outputs.  Optimiser: Adam with bias correction.
 */
typedef struct fdlb_mlp fdlb_mlp; /* opaque host handle */

/* hidden_layers 1..8; max_batch (samples per training step) 1..2^22.  Host only. */
int fdlb_mlp_create(int hidden_layers, int64_t max_batch, fdlb_mlp **out);
void fdlb_mlp_destroy(fdlb_mlp *m);
int64_t fdlb_mlp_param_count(const fdlb_mlp *m);
size_t fdlb_mlp_workspace_bytes(const fdlb_mlp *m); /* bf16 weights, bf16 activation and gradient transposes, partial gradients */

/* Glorot-uniform weights (bound sqrt(6 / (fan_in + fan_out)), splitmix64 stream from
 * `seed`) and zero biases into a caller host array of fdlb_mlp_param_count floats. */
int fdlb_mlp_init_params(const fdlb_mlp *m, uint64_t seed, float *host_params);

/*
 * Caller-owned device buffers: parameters, gradient, Adam first and second moments
 * (param_count floats each; the moments must be zero before Adam step 1) and the workspace
 * (256-byte aligned).  Every call below is asynchronous on `stream` unless it says otherwise.
 */
int fdlb_mlp_bind(fdlb_mlp *m, float *d_params, float *d_grad, float *d_adam_m, float *d_adam_v,
                  void *d_workspace, void *stream);

/* Inference: d_out[n][3] = network(d_in[n][3]) for any n >= 0. */
int fdlb_mlp_forward(fdlb_mlp *m, const float *d_in, int64_t n, float *d_out);

/*
 * One training evaluation: forward pass, loss and gradient (written to the bound gradient
 * buffer) of the mean squared error over n samples (1 <= n <= max_batch).  Sample g is row
 * d_rows[g] of d_in[.][3] and d_target[.][3] (d_rows may be NULL: row g).
 */
int fdlb_mlp_backward(fdlb_mlp *m, const float *d_in, const float *d_target, const int32_t *d_rows, int64_t n);
/* Loss of the last fdlb_mlp_backward (synchronous). */
int fdlb_mlp_last_loss(fdlb_mlp *m, double *loss);

/* Adam update of the parameters from the bound gradient; step counts from 1. */
int fdlb_mlp_adam_step(fdlb_mlp *m, double lr, double beta1, double beta2, double eps, int64_t step);

/*
 * `steps` minibatch steps, each fdlb_mlp_backward then fdlb_mlp_adam_step, enqueued back to back
 * (the same arithmetic in the same order as the two calls, the update applied inside the
 * gradient reduction, hence the same parameters to the bit).
 * Step s uses the samples d_rows[s batch .. min((s + 1) batch, n_rows)) (device int32 row indices,
 * e.g. a permutation of 0..n_rows-1), learning rate lr[s] (host array of `steps` values) and Adam
 * step count first_step + s.  FDLB_EINVAL if batch is not in 1..max_batch, if a step would start
 * past n_rows, or for NULL arrays.  Asynchronous on the bound stream.
 */
int fdlb_mlp_train(fdlb_mlp *m, const float *d_in, const float *d_target, const int32_t *d_rows, int64_t n_rows,
                   int64_t batch, int64_t steps, const double *lr, double beta1, double beta2, double eps,
                   int64_t first_step);

/*
 * Predicted fields of an nx x ny problem with Knudsen number kn and fastest wall speed
 * u_w, into device arrays of nx ny floats ([y][x]): rho = 1 + u_w y_0, u = u_w (y_1, y_2).
 */
int fdlb_mlp_predict_fields(fdlb_mlp *m, double kn, int nx, int ny, double u_w, float *d_rho, float *d_ux,
                            float *d_uy);

/*
 * Training samples from the current state of a problem (or instance i of a batch): for every
 * cell ([y][x] order) the network input and the target fields as defined above, into device
 * arrays of nx ny x 3 floats each.  FDLB_EINVAL for Kn = INFINITY or no moving wall.
 * Asynchronous on the problem's stream.
 */
int fdlb_field_samples(fdlb_problem *p, float *d_in, float *d_target);
int fdlb_batch_field_samples(fdlb_batch *b, int i, float *d_in, float *d_target);

/* ---- hybrid half-range / full-range channel ------------------------------------------
 *
 * The coupling the paper proposes in its closing remarks: away from walls a half-range
 * model with N velocities behaves like a full-range one with N/2^d, so half-range nodes are
 * kept only in the Knudsen layers next to the walls and the bulk runs on the cheaper
 * full-range set.  Built here for the planar Couette channel (plates at y = 0 and y = 1,
 * x periodic with one cell, the geometry of Eqs. 10-11), one channel per workgroup with the
 * whole state resident in LDS for the duration of a launch.
 *
 * Scheme: ny cells across the channel; the first and the last `layer` cells carry the x rule
 * times a half-range y rule of n_half nodes per half-line (the layer set, Q_l = Q_x 2 n_half
 * velocities), the others the x rule times an n_full-node full-range y rule (the bulk set,
 * Q_b = Q_x n_full).  Each cell relaxes with its own set (Eqs. 1, 5-7), the plates act on
 * the layer cells as the walls of the plain scheme (Eqs. 8-9), and every population then
 * moves by the donor cell in y.  A donor cell in the other zone is seen through that zone's
 * post-relaxation distribution carried to this zone's y nodes, for each x node, by a
 * truncated Hermite expansion: c_m = (1/m!) sum_a g_a He_m(xi_a) over the source nodes,
 * g'_k = w'_k sum_{m <= K} c_m He_m(xi'_k), with K = n_full - 1 from bulk to layer (the
 * polynomial through the bulk values) and K = min(n_half, n_full) - 1 from layer to bulk
 * (the degree whose coefficients the half-range rule integrates exactly).  Both maps carry
 * every w * polynomial of degree <= K exactly, the equilibrium among them; the interface is
 * conservative only to that extent (the defect vanishes with the Knudsen layer's remnant at
 * the interface).  dt = cfl / (ny max |xi_y|) over the y rules present, omega = dt / Kn.
 * With 2 layer == ny there is no bulk and the channel is the plain half-range scheme.
 *
 * State layout (doubles, raw f): the 2 layer cells' populations plane by plane,
 * [alpha][c] with alpha = y node * Q_x + x node and c over the layer cells in ascending y
 * (bottom layer, then top layer), followed by the bulk cells' populations [k][b] the same
 * way.  One channel holds 2 layer Q_l + (ny - 2 layer) Q_b doubles.
 */
typedef struct fdlb_hybrid_desc {
    int32_t ny;              /* cells across the channel, 2..4096 */
    int32_t layer;           /* half-range cells next to each plate, 1..ny/2 */
    double kn;               /* Knudsen number of Eq. (1), > 0; INFINITY allowed */
    double u_bottom, u_top;  /* tangential plate speeds along +x */
    double cfl;              /* Courant number in (0, 1] */
    int32_t qx_kind, qx_n;   /* x rule (FDLB_HALF or FDLB_FULL, at least 2 nodes per rule / half) */
    int32_t n_half;          /* half-range y nodes per half-line in the layers, 2..8 */
    int32_t n_full;          /* full-range y nodes in the bulk, 2..16 */
} fdlb_hybrid_desc;

typedef struct fdlb_hybrid fdlb_hybrid; /* opaque: a batch of channels */

/* Validate n descriptions (1..65536) and build the velocity sets, time steps and interface
 * maps.  Host only.  FDLB_EINVAL for a bad description, FDLB_EUNSTABLE for omega > 1 or
 * cfl > 1; Q_x 2 n_half <= 512. */
int fdlb_hybrid_create(const fdlb_hybrid_desc *descs, int n, fdlb_hybrid **out);
void fdlb_hybrid_destroy(fdlb_hybrid *h); /* NULL is a no-op; no GPU call */

/* Sizes, in bytes, of the caller-provided device state arena (every channel's populations,
 * 256-byte aligned each) and workspace (tables, control blocks, staging). */
size_t fdlb_hybrid_state_bytes(const fdlb_hybrid *h);
size_t fdlb_hybrid_workspace_bytes(const fdlb_hybrid *h);
/* Layout of channel i: velocities of the layer and bulk sets, doubles of its state, dt and
 * omega.  Any pointer may be NULL. */
int fdlb_hybrid_info(const fdlb_hybrid *h, int i, int32_t *q_layer, int32_t *q_bulk,
                     int64_t *state_doubles, double *dt, double *omega);

/* Bind the arenas (256-byte aligned) and a stream; uploads the tables (synchronous).
 * FDLB_EINVAL if a channel's LDS footprint (16 bytes per population, 64-232 bytes per cell
 * for its moments and their partial sums, and its tables) exceeds what one workgroup may
 * hold on the current device. */
int fdlb_hybrid_bind(fdlb_hybrid *h, void *d_state, void *d_workspace, void *stream);

/* Seed channel i at f = w (rho + xi . rho u) on each cell's own set from host arrays of ny
 * doubles (NULL: rho = 1, u = 0).  Synchronous. */
int fdlb_hybrid_init_equilibrium(fdlb_hybrid *h, int i, const double *rho, const double *ux,
                                 const double *uy);
/* Copy channel i's state (layout above) from / to a host array.  Synchronous. */
int fdlb_hybrid_set_state(fdlb_hybrid *h, int i, const double *host_state);
int fdlb_hybrid_get_state(fdlb_hybrid *h, int i, double *host_state);

/* Advance every channel by exactly nsteps steps.  Asynchronous. */
int fdlb_hybrid_step(fdlb_hybrid *h, int64_t nsteps);

/*
 * March every channel until the residual of a step, R = ||u^{n+1} - u^n||_2 / ||u^{n+1}||_2
 * over the channel's cells, falls below tol (the state is that step's) or max_steps steps
 * have been taken.  The residual is evaluated every step inside the launch; a launch runs
 * at most `chunk` steps (<= 0: 100000) and converged channels leave the next launch.
 * reps (may be NULL) receives n reports: steps, first_below, residual, wall_s, updates/s
 * (cells x own velocities x steps / wall_s), status; history (if given) the residual of
 * every step up to its capacity.  Synchronous.  FDLB_OK if every channel converged,
 * FDLB_ENOTCONVERGED or FDLB_EDIVERGED (a non-finite residual) otherwise.
 */
int fdlb_hybrid_solve(fdlb_hybrid *h, double tol, int64_t max_steps, int64_t chunk,
                      fdlb_report *reps);

/* Cell fields of channel i (host arrays of ny doubles, any may be NULL): rho, u_x, u_y
 * (Eqs. 6-7 over the cell's own set) and the xy stress of the post-relaxation state.
 * Synchronous. */
int fdlb_hybrid_moments(fdlb_hybrid *h, int i, double *rho, double *ux, double *uy, double *pxy);

/*
 * Face values of channel i into out[8]: u_x and p_xy of the face state at the bottom plate
 * (arriving populations of the wall cell after relaxation, emission of Eq. 8), the same at
 * the top plate, then the y-flux of x-momentum through the lower interface as the layer
 * cell's and as the bulk cell's update transport it, and through the upper interface as the
 * bulk cell's and the layer cell's update do (NaN without a bulk).  At a steady state the
 * flux is uniform inside each zone; the two values at an interface differ by the coupling's
 * conservation defect.  Synchronous.
 */
int fdlb_hybrid_faces(fdlb_hybrid *h, int i, double *out);

/* ---- measurement helpers ------------------------------------------------------------ */

/* Copy `bytes` bytes device-to-device with the library's streaming copy kernel
 * (for the achievable-bandwidth ceiling); asynchronous on the stream. */
int fdlb_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *stream);

/*
 * Streaming probes of the achievable HBM bandwidth, one kernel per mode, each
 * thread keeping four 16-byte accesses in flight:
 *   FDLB_COPY_PLAIN     copy, plain loads and stores
 *   FDLB_COPY_NT_LOAD   copy, non-temporal loads, plain stores
 *   FDLB_COPY_NT_STORE  copy, plain loads, non-temporal stores (the step kernels' mix)
 *   FDLB_COPY_NT        copy, non-temporal loads and stores (fdlb_stream_copy)
 *   FDLB_COPY_READ      read d_src only; d_dst receives one 16-byte sum per block
 *                       (it must hold 512 KiB)
 *   FDLB_COPY_WRITE     write d_dst only (d_src unused)
 * FDLB_EINVAL for another mode.  Asynchronous on the stream.
 */
#define FDLB_COPY_PLAIN 0
#define FDLB_COPY_NT_LOAD 1
#define FDLB_COPY_NT_STORE 2
#define FDLB_COPY_NT 3
#define FDLB_COPY_READ 4
#define FDLB_COPY_WRITE 5
int fdlb_stream_probe(void *d_dst, const void *d_src, size_t bytes, int mode, void *stream);

/* Message for the last error on the calling thread ("" if none). */
const char *fdlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDLB_H */
