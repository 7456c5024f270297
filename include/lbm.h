/*
 * liblbm -- MI355X (gfx950) implementation of the thermal lattice Boltzmann
 * scheme with arbitrary specific-heat ratio of Hu, Zhang & Geng
 * (arXiv:1608.06345): two reduced distributions per cell, g (mass and
 * momentum) and h (internal energy), on the D2Q37 and D3Q107 velocity sets,
 * advanced by a fused BGK collide-and-stream step (lbm_create, lbm_create_ex)
 * or by the paper's finite-difference form (lbm_create_fd), one solve per
 * handle or many per pool (lbm_pool_*).
 *
 * The method, section by section:
 *   Sec. II   the reduced distributions g and h; the moments
 *             rho = sum g_i, rho u = sum g_i xi_i,
 *             rho E = sum xi_i^2 g_i / 2 + sum h_i;
 *             the specific-heat ratio gamma = (delta + D + 2) / (delta + D)
 *             through delta internal degrees of freedom; the dimensionless
 *             energy E = u^2/2 + (D + delta) T / 2; the BGK targets
 *             F_i (for g) and (delta/2) T F_i (for h).
 *   Sec. III  explicit first-order time stepping of both BGK equations.
 *   Sec. IV   the fourth-order Hermite equilibrium F_i and the velocity sets
 *             (Table I: D2Q37, Table II: D3Q107, xi_i = r e_i, r ~ 1.19698).
 *   Sec. V    the shock-tube set-up: periodic transverse axes, open ends
 *             along x, and the lattice time conversion t = step / (X r),
 *             i.e. every population moves e_i cells per step.
 *
 * Conventions shared by every call
 *   - Every call returns an lbm_status code; nothing aborts or throws.
 *   - Cell index = x + nx * (y + ny * z); 2D grids have nz = 1.
 *   - Host arrays are owned and allocated by the caller; the library copies
 *     them synchronously.  "_dev" variants take device pointers and run
 *     asynchronously on the handle's stream.
 *   - Vector fields are component-major: u[k * ncells + cell].
 *   - All device memory of a solve is owned by the library; it is released
 *     by lbm_destroy.
 *   - A handle is not thread-safe; separate handles are independent.
 *   - State convention: S_0 is the equilibrium of the initial fields and one
 *     step is S_{n+1} = Stream(Collide(S_n)) (lattice streaming) or one
 *     explicit finite-difference step (lbm_create_fd).  lbm_moments and
 *     lbm_totals report S_n, the pre-collision state after n steps.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_solver *lbm_handle;

enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument (see each call) */
    LBM_ENOMEM = -2,     /* device allocation failed */
    LBM_EDEVICE = -3,    /* a HIP runtime call failed */
    LBM_ESTATE = -4,     /* call out of order (e.g. step before init) */
    LBM_ENONFINITE = -5, /* a conservation total is NaN or infinite */
    LBM_EBUSY = -6,      /* pool: no free slot or arena space right now */
    LBM_ESCRATCH = -7    /* grid too large for lbm_moments_noalloc's scratch */
};

enum lbm_velocity_set { LBM_D2Q37 = 37, LBM_D3Q107 = 107 };

/* Boundary condition per axis, 2 bits each: bc = bx | by << 2 | bz << 4.
 * PERIODIC wraps.  ZERO_GRADIENT is the reading of the paper's "open"
 * boundary (Sec. V): populations streaming in from beyond the end are the
 * post-collision populations of the end cell (pull source clamped). */
enum lbm_bc { LBM_BC_PERIODIC = 0, LBM_BC_ZERO_GRADIENT = 1 };
#define LBM_BC(bx, by, bz) \
    ((uint32_t)(bx) | ((uint32_t)(by) << 2) | ((uint32_t)(bz) << 4))

/* Storage and arithmetic precision of the populations.
 * FP64: populations and collision in double.
 * FP32_DEV: populations stored in float as deviations from the rest
 *   equilibrium, g_i - w_i and h_i - w_i delta/2 (reference rho0 = T0 = 1),
 *   collision in float computed directly on the deviations; readouts and
 *   conservation totals in double.
 * FP16_SCALED: as FP32_DEV, but each deviation is stored in IEEE half
 *   precision divided by its weight w_i (the per-population scale that puts
 *   all populations in one range); half the bytes of FP32_DEV, with the
 *   accuracy of an 11-bit significand per stored value.  That rounding is
 *   not conservative: totals drift at its level (a random walk of about
 *   w_i |d_i| 2^-12 per stored value and step). */
enum lbm_precision { LBM_FP64 = 0, LBM_FP32_DEV = 1, LBM_FP16_SCALED = 2 };

/* Create a solve (Secs. II-IV).
 *   dim           2 or 3
 *   velocity_set  LBM_D2Q37 with dim 2, LBM_D3Q107 with dim 3
 *   gamma         specific-heat ratio; delta = 2/(gamma-1) - dim, values
 *                 within 1e-9 of 0 taken as 0; delta < 0 is rejected
 *   tau_f, tau_g  relaxation times of g and h in lattice units (> 1/2).
 *                 The paper uses one tau for both (Sec. II); two different
 *                 values conserve mass and momentum but not total energy.
 *   nx, ny, nz    grid size (>= 1; nz must be 1 when dim is 2)
 *   bc            LBM_BC(bx, by, bz)
 *   out           receives the handle
 * Errors: EINVAL for any argument outside the above, or a grid whose one
 * population array exceeds 2^31 - 1 bytes; ENOMEM if device memory cannot be
 * allocated; EDEVICE for other HIP failures.  lbm_create uses LBM_FP64. */
int lbm_create(int dim, int velocity_set, double gamma, double tau_f,
               double tau_g, int64_t nx, int64_t ny, int64_t nz, uint32_t bc,
               lbm_handle *out);
int lbm_create_ex(int dim, int velocity_set, double gamma, double tau_f,
                  double tau_g, int64_t nx, int64_t ny, int64_t nz,
                  uint32_t bc, int precision, lbm_handle *out);

/* Collision of a solve.
 * PAPER: the BGK collision of Secs. II-III, g toward F with tau_f and h
 *   toward (delta/2) T F with tau_g.  With tau_f != tau_g it does not
 *   conserve total energy: a cell's energy changes by (a_f - a_g)
 *   (E_tr^eq - E_tr) per step (a = 1/tau per lattice step, dt/tau per
 *   finite-difference step; E_tr = sum xi^2 g / 2, E_tr^eq = rho (u^2 +
 *   D T) / 2).
 * ENERGY_CONSERVING: not in the paper.  h relaxes toward ((delta/2) T +
 *   kappa) F with kappa rho = (1 - a_f / a_g)(E_tr^eq - E_tr), which
 *   conserves total energy exactly for any tau_f, tau_g and is the paper's
 *   collision when tau_f = tau_g.  Mass, momentum and g's relaxation are
 *   unchanged. */
enum lbm_collision { LBM_COLLISION_PAPER = 0, LBM_COLLISION_ENERGY_CONSERVING = 1 };

/* Select the collision (default PAPER).  Must precede lbm_init_fields:
 * ESTATE once the handle holds a state; EINVAL for other modes. */
int lbm_set_collision(lbm_handle h, int mode);

/* Create a solve that advances by the finite-difference form of Sec. III
 * instead of lattice streaming: explicit Euler in time with step dt,
 *   g_i(t+dt) = g_i - dt xi_i . grad g_i - (dt/tau_f) (g_i - F_i),
 *   h_i(t+dt) = h_i - dt xi_i . grad h_i - (dt/tau_g) (h_i - (delta/2) T F_i),
 * every term at time t, the convection per axis by the third-order
 * upwind-biased difference of Sec. III (stencil x-2s .. x+s against the
 * sign s of xi_a).  Units: grid step 1, particle speeds xi_i = r e_i, so one
 * lattice step of lbm_create corresponds to dt = 1/r; tau_f and tau_g are
 * relaxation times in the units of dt (no half-step shift).  Open ends take
 * a neighbour beyond the end as the end cell's value (zero gradient).
 *   dt      time step, 0 < dt <= 1/(3r) (the fastest speed, 3r, then moves
 *           at most one cell per step)
 *   tau_f, tau_g   > 0 with dt/tau <= 1 (the explicit relaxation must not
 *           overshoot the equilibrium)
 * Stability: forward Euler with the upwind-biased difference alone
 * amplifies every mode; the relaxation damps the departures from
 * equilibrium, and the scheme is stable for per-axis Courant numbers
 * |xi_a| dt up to ~0.6-0.7 at dt/tau in 0.2-1 (less with weaker damping):
 * for the fastest D2Q37 population (3r, 3r) that is 3 r dt <= ~0.3, for
 * D3Q107's (3r, r, r) 3 r dt <= ~0.36.  Larger steps are accepted up to the
 * bound below but grow without limit.
 * precision: LBM_FP64 or LBM_FP32_DEV; LBM_FP16_SCALED is rejected (EINVAL):
 * re-rounding every value to half at each of the many short steps costs
 * percents of the velocity.
 * Other arguments and errors as lbm_create_ex.  lbm_step(n) takes
 * n such steps; lbm_moments and lbm_totals report the state at step n;
 * init_fields sets the state to the equilibrium of the fields. */
int lbm_create_fd(int dim, int velocity_set, double gamma, double tau_f,
                  double tau_g, double dt, int64_t nx, int64_t ny, int64_t nz,
                  uint32_t bc, int precision, lbm_handle *out);

/* Release every device resource of the handle (NULL is accepted). */
int lbm_destroy(lbm_handle h);

/* Run the handle's work on `stream` (a hipStream_t; NULL is the device's
 * null stream).  Until this is called a handle uses a non-blocking stream of
 * its own.  The stream is borrowed, not owned: it must outlive its use. */
int lbm_set_stream(lbm_handle h, void *stream);
/* Kernel layout of the step (a tuning choice; results agree to round-off).
 *   LANE      fused kernel, one lane holds all 2Q populations of a cell
 *             (half storage: as 2Q halves in Q g/h words);
 *   SPLIT     fused kernel, a lane pair holds them, g in lane l and h in
 *             lane l + 32 of the wave;
 *   TWO_PASS  (lbm_create_fd solves only) the finite-difference step as a
 *             moments pass plus updates of chunks of populations, which
 *             keeps each chunk's neighbour rows in cache; where nx is a
 *             multiple of 256 the updates stage each population's stencil
 *             rows in LDS (same results to rounding);
 *   SPLIT_LDS (D3Q107 lattice streaming, nx a multiple of 128) SPLIT with
 *             the pulled rows staged in LDS: a workgroup loads each
 *             population's shifted row once, four cells a lane, and each
 *             lane reads its pulled value from LDS (same results to
 *             rounding);
 *   AUTO      (the default) lattice streaming: LANE for D2Q37 and for half
 *             storage, SPLIT for D3Q107 in FP64 and FP32, whose 214
 *             populations do not fit one lane's registers; finite
 *             differences: TWO_PASS, except LANE for
 *             D2Q37 in FP64 when nx is not a multiple of 256, where the
 *             fused kernel is faster than the two-pass step without LDS.
 * EINVAL for other values, for TWO_PASS on a lattice-streaming solve, and for
 * SPLIT_LDS on any other solve. */
enum lbm_variant {
    LBM_VARIANT_AUTO = 0,
    LBM_VARIANT_LANE = 1,
    LBM_VARIANT_SPLIT = 2,
    LBM_VARIANT_TWO_PASS = 3,
    LBM_VARIANT_SPLIT_LDS = 4
};
int lbm_set_variant(lbm_handle h, int variant);

/* Block until the handle's stream is idle. */
int lbm_synchronize(lbm_handle h);

/* Initial state S_0: g_i = F_i(rho, u, T), h_i = (delta/2) T F_i (Sec. II,
 * Sec. IV), and step count 0.  rho, T: [ncells]; u: [dim][ncells]; FP64 host
 * arrays.  EINVAL on a NULL pointer. */
int lbm_init_fields(lbm_handle h, const double *rho, const double *u,
                    const double *T);
/* Same from device arrays, asynchronous on the handle's stream; the arrays
 * must stay valid until the stream reaches this point. */
int lbm_init_fields_dev(lbm_handle h, const double *rho, const double *u,
                        const double *T);

/* Advance n >= 0 steps, asynchronously on the handle's stream.  One step of
 * lattice streaming is S_{n+1} = Stream(Collide(S_n)): the BGK collision of
 * both reduced distributions toward their Sec. IV equilibria (the relaxation
 * of the Sec. II BGK equations, discretised explicitly in time as in
 * Sec. III), then every population moves e_i cells, the lattice time step
 * implied by Sec. V's time conversion t = step / (X r).  With lbm_create_fd
 * a step is instead one explicit finite-difference step of size dt
 * (Sec. III).  ESTATE before init; EINVAL for n < 0. */
int lbm_step(lbm_handle h, int64_t n);

/* Moments of S_n (Sec. II): rho [ncells], u [dim][ncells] and the specific
 * total energy E = (sum xi^2 g / 2 + sum h) / rho [ncells], in FP64 host
 * arrays; synchronous.  ESTATE before init. */
int lbm_moments(lbm_handle h, double *rho, double *u, double *E);
/* Same into device arrays, asynchronous on the handle's stream. */
int lbm_moments_dev(lbm_handle h, double *rho, double *u, double *E);

/* Temperature of S_n (Sec. II: E = |u|^2/2 + (D + delta) T / 2, so
 * T = (2E - |u|^2) / (D + delta)), formed per cell in FP64 on the device from
 * the same moment sums lbm_moments reports.  T [ncells] FP64 host array;
 * synchronous.  ESTATE before init; EINVAL on a NULL pointer. */
int lbm_temperature(lbm_handle h, double *T);
/* Same into a device array, asynchronous on the handle's stream. */
int lbm_temperature_dev(lbm_handle h, double *T);

/* lbm_moments without any device allocation, for callers that cannot
 * allocate device memory (tight serving loops retiring results, harnesses
 * that forbid allocation).  Same arguments, results (bit for bit) and errors
 * as lbm_moments; the fields are staged in a fixed 64 MiB device array that
 * the library holds on each device it runs on until the process ends,
 * instead of a buffer allocated per call.  Limit: (2 + dim) * ncells * 8
 * bytes <= 64 MiB, i.e. ncells <= 2097152 in 2D and 1677721 in 3D; larger
 * grids return LBM_ESCRATCH.  Every call on one device shares that device's
 * array: calls that overlap on one device (from two threads, or on two
 * streams) race.  Synchronous, so not for use under graph capture. */
int lbm_moments_noalloc(lbm_handle h, double *rho, double *u, double *E);

/* Domain totals of S_n in FP64, from the Sec. II moments summed over every
 * cell: mass = sum rho, mom[k] = sum rho u_k
 * (mom has dim entries), energy = sum rho E; deterministic summation order.
 * Synchronous.  ESTATE before init; ENONFINITE (totals still written) if any
 * total is NaN or infinite. */
int lbm_totals(lbm_handle h, double *mass, double *mom, double *energy);

/* Read-only facts about a solve. */
typedef struct {
    int dim, q, precision;
    int64_t nx, ny, nz;
    uint32_t bc;
    double gamma, delta, tau_f, tau_g, r;
    int64_t steps;          /* steps taken since the last init */
    size_t device_bytes;    /* device memory held by the handle */
    int scheme;             /* 0: lattice streaming, 1: finite differences */
    double dt;              /* finite-difference time step (0 for lattice) */
    int collision;          /* enum lbm_collision */
} lbm_info;
int lbm_get_info(lbm_handle h, lbm_info *info);

/* Device bytes a lattice-streaming solve of this shape holds (two
 * distributions, two ping-pong copies, plus reduction scratch); 0 for
 * invalid arguments.  A finite-difference solve holds a per-cell record on
 * top (lbm_info.device_bytes has the total). */
size_t lbm_footprint_bytes(int dim, int velocity_set, int precision,
                           int64_t nx, int64_t ny, int64_t nz);

/* The library's lattice (Sec. IV, Tables I-II): e [q][3] (z = 0 in 2D), w [q]
 * and the scale r, derived by the library from the Gauss-Hermite moment
 * conditions.  Any output pointer may be NULL.  Returns q, or EINVAL. */
int lbm_lattice(int velocity_set, int8_t *e, double *w, double *r);

/* ------------------------------------------------------------------------
 * Batched multi-solve pool (serving form).
 *
 * Many independent solves -- D2Q37 and D3Q107 grids of any size, each with
 * its own gamma, tau_f, tau_g, boundary conditions and number of steps --
 * stay resident in one device arena and are advanced together: every step is
 * one launch per velocity set over all resident solves (plus one tiny
 * counter launch), and lbm_pool_run replays K such steps from a captured
 * hipGraph.  Membership lives in device tables, so solves can be admitted and
 * released between replays without re-capturing (continuous batching).  Each
 * solve follows exactly the single-solve scheme and state convention above
 * (lattice streaming, the paper's collision: the finite-difference form and
 * the energy-conserving collision are single-solve options); its arithmetic
 * does not depend on which other solves are resident.
 * All pool memory is owned by the pool.  A pool is not thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct lbm_pool *lbm_pool_handle;

/* One solve request.  dim 2 uses D2Q37, dim 3 uses D3Q107; gamma, tau_f,
 * tau_g, grid and bc as in lbm_create; steps >= 0 is the number of steps the
 * pool runs it for. */
typedef struct {
    int dim;
    double gamma, tau_f, tau_g;
    int64_t nx, ny, nz;
    uint32_t bc;
    int64_t steps;
} lbm_request;

typedef struct {
    size_t budget_bytes;       /* arena size */
    size_t used_bytes;         /* held by resident solves */
    size_t largest_free_bytes; /* biggest request that fits now */
    int max_slots, resident, graphs;
} lbm_pool_info;

/* Create a pool: an arena of budget_bytes of device memory, up to max_slots
 * (1..65536) resident solves, all stored in `precision`.  EINVAL for bad
 * arguments; ENOMEM if the arena cannot be allocated. */
int lbm_pool_create(size_t budget_bytes, int max_slots, int precision,
                    lbm_pool_handle *out);
int lbm_pool_destroy(lbm_pool_handle p);
/* Run the pool's work on `stream` (as lbm_set_stream). */
int lbm_pool_set_stream(lbm_pool_handle p, void *stream);

/* Arena bytes a request occupies (both distributions, both ping-pong
 * sides); 0 if the request is invalid in any respect lbm_pool_admit rejects
 * with EINVAL (shape, gamma giving delta < 0, rates, steps, bc).  This is the
 * admission footprint. */
size_t lbm_pool_request_bytes(const lbm_request *r, int precision);

/* Admit a request with its initial fields (as lbm_init_fields: host
 * arrays rho [N], u [dim][N], T [N]; the _dev form takes device arrays on the
 * pool's stream).  On success *slot receives the slot id and the solve is at
 * step 0.  EINVAL for an invalid request; ENOMEM if it can never fit the
 * arena; EBUSY if no slot or no contiguous arena space is free now (retry
 * after releasing finished solves). */
int lbm_pool_admit(lbm_pool_handle p, const lbm_request *r, const double *rho,
                   const double *u, const double *T, int *slot);
int lbm_pool_admit_dev(lbm_pool_handle p, const lbm_request *r,
                       const double *rho, const double *u, const double *T,
                       int *slot);

/* Advance every resident solve that has steps left by up to `ticks` steps
 * (0..4096), asynchronously, as one replay of a captured graph (captured on
 * first use for each ticks value).  lbm_pool_run_eager enqueues the same
 * launches without a graph. */
int lbm_pool_run(lbm_pool_handle p, int ticks);
int lbm_pool_run_eager(lbm_pool_handle p, int ticks);

/* Synchronise, then list (up to max_finished) slots that have run all their
 * steps and were not listed before.  Their state stays resident until
 * lbm_pool_release. */
int lbm_pool_poll(lbm_pool_handle p, int *finished, int max_finished,
                  int *n_finished);
/* Steps a slot has taken so far (synchronous). */
int lbm_pool_slot_steps(lbm_pool_handle p, int slot, int64_t *steps_done);

/* Moments / totals of a slot's S_n (n = its steps done), as lbm_moments,
 * lbm_moments_dev and lbm_totals.  EINVAL for a slot that is not resident. */
int lbm_pool_moments(lbm_pool_handle p, int slot, double *rho, double *u,
                     double *E);
int lbm_pool_moments_dev(lbm_pool_handle p, int slot, double *rho, double *u,
                         double *E);
int lbm_pool_totals(lbm_pool_handle p, int slot, double *mass, double *mom,
                    double *energy);
/* Temperature of a slot's S_n, as lbm_temperature (Sec. II). */
int lbm_pool_temperature(lbm_pool_handle p, int slot, double *T);

/* Free a slot and its arena space (synchronises the pool's stream first). */
int lbm_pool_release(lbm_pool_handle p, int slot);
int lbm_pool_get_info(lbm_pool_handle p, lbm_pool_info *info);

/* Static description of a status code. */
const char *lbm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
