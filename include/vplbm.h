/*
 * vplbm.h — C ABI of the MI355X (gfx950) volume-penalization lattice Boltzmann library.
 *
 * The operation: Benamour, Liberge & Beghein, "A volume penalization lattice Boltzmann method for
 * simulating flows in the presence of obstacles" (arXiv:1812.05401), Section 2.  A D2Q9 lattice
 * is advanced on every node, fluid and solid alike; obstacles enter only through the penalization
 * body force f = -rho (chi/eta)(u - u_s) (Eq. 17), with the velocity solved implicitly (Eq. 18) and
 * the force injected by the Guo term (SRT, Eqs. 2 and 7) or the Lu term (MRT, Eqs. 10-16).
 *
 * Conventions shared by every call:
 *   - Lattice units, dx = dt = 1.  Node (x, y) sits at integer coordinates 0 <= x < nx, 0 <= y < ny.
 *   - Directions alpha = 0..8 follow Eq. 3: 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
 *   - Host arrays are row-major, x fastest: field[y*nx + x]; populations pop[(a*ny + y)*nx + x].
 *   - Every host pointer is owned by the caller and only read or written during the call (or,
 *     for asynchronous calls, copied before the call returns).  The library owns all device memory.
 *   - Every call returns 0 (VPLBM_OK) or a negative error code; vplbm_last_error() then holds a
 *     message for the calling thread.  No C++ exception crosses the ABI.
 *   - A handle is not thread-safe: use one handle per thread or lock around calls.
 *   - The stored state is the post-collision population.  Step n (n = 0, 1, ...) streams it,
 *     applies the edge rules, computes the moments and the penalized velocity, collides and stores;
 *     bodies are placed at time t = n during step n.
 */
#ifndef VPLBM_H
#define VPLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VPLBM_ABI_VERSION 1
#define VPLBM_MAX_BODIES 8
/* doubles per step in the observable ring: mass, then (fx, fy) for each of the 8 bodies */
#define VPLBM_RING_WIDTH (1 + 2 * VPLBM_MAX_BODIES)

enum vplbm_error {
    VPLBM_OK = 0,
    VPLBM_EINVAL = -1,     /* bad argument, bad configuration, NULL or destroyed handle */
    VPLBM_ENOMEM = -2,     /* device or host allocation failed */
    VPLBM_EHIP = -3,       /* a HIP runtime call failed (message has the HIP error string) */
    VPLBM_EUNSTABLE = -4,  /* the simulation produced a non-finite or non-positive density */
    VPLBM_EBUDGET = -5,    /* a pool request can never fit the pool's memory budget */
    VPLBM_ESTATE = -6      /* the call is not valid in the object's current state */
};

/* Collision (Section 2.1).  VPLBM_MRT uses the rates of Eq. 14 with s_n = 1/tau and s_q from
   Lambda (Eq. 15); VPLBM_SRT is the single rate 1/tau with the Guo term (Eqs. 2, 7). */
enum vplbm_collision { VPLBM_SRT = 0, VPLBM_MRT = 1 };

/* Storage of the populations.  F64 stores f.  F32, F32D, F16S and BF16S store f - w_alpha (the
   lattice weights of Eq. 5, i.e. the deviation from the rest state at rho = 1) rounded to nearest
   even in binary32 / binary32 / binary16 / bfloat16.  Every format computes on f - w_alpha: F64
   and F32D in FP64, F32, F16S and BF16S in FP32.  F32D moves F32's bytes; only its storage is
   rounded to binary32, so long runs keep the mass and forces of an FP64 run, at some FP64
   arithmetic cost.  F16SR and BF16SR are F16S and BF16S with stochastic rounding: each stored h
   is rounded up or down at random with probabilities that make the rounding error zero-mean,
   which keeps the mass of long 16-bit runs from drifting; the random bits come from a
   counter-based hash of (node, step), so runs are reproducible.  get/set_populations convert to
   and from f in FP64; a get followed by a set
   restores the stored bits, except that in F32 and F32D a stored |f - w_alpha| below about 2^-33
   (where FP64's rounding of f reaches half its binary32 ulp) may come back changed by < 2^-56. */
enum vplbm_storage {
    VPLBM_F64 = 0, VPLBM_F32 = 1, VPLBM_F16S = 2, VPLBM_BF16S = 3, VPLBM_F32D = 4,
    VPLBM_F16SR = 5, VPLBM_BF16SR = 6
};

/* Edge rules.  x edges: both PERIODIC, or VELOCITY (Zou-He inlet at x = 0 imposing (u_in_x,
   u_in_y)) with OUTFLOW (zero-gradient outlet at x = nx-1) or CONVECTIVE (the populations
   entering from x = nx obey df/dt + U df/dx = 0 with U = u_in_x, implicitly upwind: the outlet
   condition of the paper's cylinder case, Section 3.3).  y edges: both PERIODIC or both FREESLIP
   (specular reflection, wall half a link outside the first and last rows). */
enum vplbm_bc { VPLBM_PERIODIC = 0, VPLBM_VELOCITY = 1, VPLBM_OUTFLOW = 2, VPLBM_FREESLIP = 3,
                VPLBM_CONVECTIVE = 4 };

/* Obstacle shapes; a node belongs to a body when its centre lies inside (boundary included).
   DISK_OUTSIDE is the complement of a disk (|x - c| >= r), e.g. a fixed outer cylinder. */
enum vplbm_shape { VPLBM_DISK = 0, VPLBM_RECT = 1, VPLBM_DISK_OUTSIDE = 2 };

typedef struct {
    uint32_t abi_version;        /* must be VPLBM_ABI_VERSION */
    int32_t nx, ny;              /* lattice size, 3 <= nx, ny and nx * ny < 2^31 */
    int32_t collision;           /* enum vplbm_collision */
    int32_t storage;             /* enum vplbm_storage */
    double tau;                  /* relaxation time, > 1/2; viscosity nu = (tau - 1/2)/3 (Eq. 6) */
    double lambda;               /* MRT: Lambda of Eq. 15 (> 0); ignored for SRT */
    double eta;                  /* penalization parameter of Eq. 17, > 0 (the paper uses 1e-7) */
    double rho0, ux0, uy0;       /* uniform initial state: f = f^eq(rho0, u0) (u_s inside bodies) */
    int32_t bc_xlo, bc_xhi, bc_ylo, bc_yhi;   /* enum vplbm_bc */
    double u_in_x, u_in_y;       /* inlet velocity for bc_xlo = VPLBM_VELOCITY, |u_in_x| < 1 */
    int32_t reduce;              /* 1: per-step FP64 mass and body-force reductions; 0: none */
    int32_t ring;                /* steps kept in the observable ring (0: 4096) */
    void *stream;                /* hipStream_t the work is ordered on (e.g. torch's current
                                    stream); NULL: a stream owned by the handle */
} vplbm_config;

typedef struct {
    int32_t kind;                /* enum vplbm_shape */
    double cx, cy;               /* centre at t = 0 */
    double r;                    /* radius (DISK, DISK_OUTSIDE) */
    double hx, hy;               /* half-sides (RECT) */
    double ux, uy, omega;        /* rigid velocity: u_s(x) = U + omega e_z x (x - c(t)) */
    double ax, ay, freq;         /* prescribed motion c(t) = c0 + a sin(2 pi freq t); adds
                                    a 2 pi freq cos(2 pi freq t) to U.  Needs device masks. */
} vplbm_body;

typedef struct {
    int64_t step;                /* index of the last executed step, -1 before the first */
    double mass;                 /* sum of rho over all nodes in that step (reduce = 1) */
    double fx[VPLBM_MAX_BODIES]; /* force of the fluid on body k: minus the sum of the     */
    double fy[VPLBM_MAX_BODIES]; /* penalization force over the body's nodes in that step  */
    int32_t nbodies;
    int32_t status;              /* 0 ok, 1 unstable (non-finite or non-positive density seen);
                                    pool requests: 2 = device memory refused (VPLBM_FAILED) */
} vplbm_obs;

typedef struct vplbm_sim_s *vplbm_sim;

/* Create a simulation: validates cfg, allocates the two population buffers, the mask and the
   observable ring on the device, and sets f = f^eq(rho0, u0) everywhere (no bodies yet).
   Work is ordered on cfg->stream.  On error *out is NULL. */
int vplbm_create(const vplbm_config *cfg, vplbm_sim *out);

/* Set the obstacles (Section 2.2: chi and u_s).  bodies[0..nbodies) (nbodies <= 8) give the
   solid velocity of body k; body_id, if not NULL, is a host nx*ny plane with 0 = fluid and
   k = bodies[k-1], copied in; if NULL the mask is rasterized on the device from the shapes (the
   lowest-index body owns a node) and, for moving bodies, rebuilt before every step.  A moving
   body requires body_id == NULL.  Before the first step this also resets the populations to the
   uniform initial state with u_s inside the bodies.  Stream-ordered. */
int vplbm_set_mask(vplbm_sim s, const uint8_t *body_id, const vplbm_body *bodies, int32_t nbodies);

/* Advance nsteps >= 0 steps (asynchronous on the stream).  Pairs of steps share one kernel launch
   (the first kept on chip; see vplbm_steps_per_launch), an odd last step takes its own, and chunks
   of 128 steps are replayed from a captured HIP graph (the environment variable
   VPLBM_GRAPH_STEPS at create sets another even chunk; 0 launches every step directly).  Returns
   VPLBM_EUNSTABLE if an earlier vplbm_observables saw status 1. */
int vplbm_step(vplbm_sim s, int64_t nsteps);

/* Observables of the last executed step; if rho/ux/uy are not NULL they receive (host, nx*ny,
   FP64) the density and penalized velocity (Eqs. 8, 9, 18) of the current state, i.e. the
   moments the next step computes.  Synchronizes the stream. */
int vplbm_observables(vplbm_sim s, vplbm_obs *out, double *rho, double *ux, double *uy);

/* Destroy the handle and free its device memory.  NULL-safe.  Synchronizes the stream. */
int vplbm_destroy(vplbm_sim s);

/* Message for the last error on the calling thread ("" if none).  Valid until the next call. */
const char *vplbm_last_error(void);

/* ---- extensions ------------------------------------------------------------------------- */

/* Set f = f^eq(rho, u) per node from host FP64 fields (nx*ny each).  Stream-ordered. */
int vplbm_init_fields(vplbm_sim s, const double *rho, const double *ux, const double *uy);

/* Copy the populations to / from a host FP64 array [9][ny][nx] (decoded from / encoded to the
   storage format).  set also sets the step counter to `step` (checkpoint/resume).  Both
   synchronize the stream. */
int vplbm_get_populations(vplbm_sim s, double *pop);
int vplbm_set_populations(vplbm_sim s, const double *pop, int64_t step);

/* Convergence residual (the relative L2 norm of Eq. 20 applied to the change of the velocity
   field): residual = sqrt(sum |u - u_prev|^2 / sum |u|^2) over the fluid nodes of the current
   state, where u_prev is the velocity at the previous call.  The first call stores the field and
   returns +inf; a zero field returns 0.  u is the velocity field vplbm_observables returns (the
   penalized velocity the next step would take).  The sums run in FP64 in a fixed order, so the
   value does not depend on scheduling.  The first call allocates 16 bytes per node for the
   snapshot.  Synchronizes. */
int vplbm_residual(vplbm_sim s, double *residual);

/* Copy the current body-id plane (host nx*ny).  Synchronizes. */
int vplbm_get_mask(vplbm_sim s, uint8_t *body_id);

/* Copy the per-step observables of steps [first, first+count) from the device ring into
   out[count][VPLBM_RING_WIDTH] (mass, fx0, fy0, ..., fx7, fy7).  The steps must still be in the
   ring (the last `ring` steps).  Synchronizes. */
int vplbm_force_series(vplbm_sim s, int64_t first, int64_t count, double *out);

/* Momentum exchange (the force evaluation of the paper's Section 3.3, after Ladd) on each body
   for the current state: over every link between a fluid node x_f and a solid node x_s = x_f +
   xi_a of body k, the momentum xi_a (g_a(x_f) + g_abar(x_s)) that the next streaming carries
   into the body.  Links through periodic edges wrap, through other edges they do not exist.
   fx, fy: host arrays of VPLBM_MAX_BODIES.  Its time mean equals that of the penalization force
   in vplbm_obs (the body's own momentum changes average out).  Synchronizes. */
int vplbm_momentum_exchange(vplbm_sim s, double *fx, double *fy);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): vplbm_momentum_exchange without any allocation and
   without synchronizing.  out: device memory of 2 * VPLBM_MAX_BODIES doubles, receiving (fx0, fy0,
   fx1, fy1, ...) of the current state, written asynchronously on the simulation's stream (the
   caller synchronizes before reading).  The sums run in a fixed order, so repeated calls give the
   same value.  Partial sums go through a static device array of the library, one per GPU (65,536
   rows of 17 doubles, 8.5 MiB, held until the process ends) and shared by every call on that
   GPU: calls that overlap on one GPU (on different streams) race.  EINVAL: bad handle, out NULL
   or not device memory, or a lattice of more than 16,777,216 nodes (the rows the array holds). */
int vplbm_momentum_exchange_noalloc(vplbm_sim s, double *out);

/* Number of steps done and the handle's stream (hipStream_t). */
int vplbm_steps_done(vplbm_sim s, int64_t *steps);
int vplbm_stream(vplbm_sim s, void **stream);

/* Lattice updates per kernel launch for this simulation: 3 for binary32 storage (the two
   intermediate steps kept on chip, 64 x 14 tiles; the convective outlet included), 2 for the
   other formats (pairs of steps, the intermediate one kept on chip), 1 when the environment variable
   VPLBM_TWO_STEP=0 was set at create; VPLBM_THREE_STEP=0 at create caps it at 2.  Moving bodies
   get a mask of their own for each intermediate step.  What remains of a call after its full
   launches takes launches of one or two steps.  Every launch shape gives bitwise the same
   populations (the update of Section 2 per node and step).  EINVAL: bad handle or NULL out. */
int vplbm_steps_per_launch(vplbm_sim s, int32_t *steps);

/* Algorithmic HBM bytes of one lattice update for a storage format: 9 population loads,
   9 population stores and the 1-byte mask. */
int vplbm_bytes_per_update(int32_t storage, int64_t *bytes);

/* ---- serving pool -----------------------------------------------------------------------
 * Many independent simulations resident on one GPU at once, advanced together: every call to
 * vplbm_pool_advance replays one captured HIP graph of `steps_per_launch` steps of a batched
 * step kernel (three steps per launch for binary32 storage and two for the other formats, the
 * intermediate steps kept on chip, what remains of a replay last) with one
 * workgroup per tile of a device table spanning all resident simulations (each simulation's
 * per-node arithmetic is the single-simulation step's), then
 * retires the finished ones and admits queued requests, first come first served, while the
 * memory budget and the slots allow.  A simulation's results do not depend on what else is
 * resident: fields are bitwise identical alone and in a mix, and the final mass and body forces
 * are summed per tile in a fixed order.  Bodies must be static (no prescribed motion) and are
 * rasterized on the device.  Every edge condition of a single simulation is accepted, the
 * convective outlet included (its requests take the launches of their storage format).
 */
typedef struct vplbm_pool_s *vplbm_pool;

enum vplbm_request_state {
    VPLBM_QUEUED = 0,    /* submitted, waiting for memory or a slot */
    VPLBM_RUNNING = 1,   /* resident, advancing */
    VPLBM_DONE = 2,      /* finished; results held until vplbm_pool_result */
    VPLBM_FAILED = 3,    /* became unstable (status 1; results hold the last observables), or
                            the device refused its memory while nothing else was resident
                            (status 2; no step done, no fields) */
    VPLBM_CANCELLED = 4  /* cancelled; results hold the steps done (and the fields if kept) */
};

typedef struct {
    uint32_t abi_version;       /* must be VPLBM_ABI_VERSION */
    uint64_t budget_bytes;      /* device memory the resident simulations may use together */
    int32_t max_slots;          /* resident simulations at most, 1..1024 */
    int32_t steps_per_launch;   /* steps per vplbm_pool_advance (graph length), 1..4096 */
    void *stream;               /* hipStream_t for all pool work; NULL: a stream of the pool's */
} vplbm_pool_config;

int vplbm_pool_create(const vplbm_pool_config *cfg, vplbm_pool *out);

/* Queue a simulation for `nsteps` >= 1 steps from its uniform initial state (cfg->stream is
   ignored; cfg->reduce is ignored: the final step's mass and forces are always reduced).
   keep_fields = 1 also keeps the final density and velocity fields for vplbm_pool_result.
   Returns VPLBM_EBUDGET if the simulation alone exceeds the budget, VPLBM_EINVAL for a bad
   config or moving bodies.  *id receives the request id (>= 0). */
int vplbm_pool_submit(vplbm_pool p, const vplbm_config *cfg, const vplbm_body *bodies,
                      int32_t nbodies, int64_t nsteps, int32_t keep_fields, int64_t *id);

/* Admission cap on the lattice nodes of the resident simulations (0, the default: none).  A
   queued request is admitted only while the resident nodes plus its own stay within the cap, or
   when nothing is resident.  Resident simulations advance in lock step, every launch taking each
   of them the same steps, so every resident node slows every other simulation down: a cap near what fills the GPU keeps
   small requests batched while long ones do not crowd each other, which shortens the tail of
   time-to-result at high load.  Takes effect at the next vplbm_pool_advance. */
int vplbm_pool_set_admission(vplbm_pool p, uint64_t max_resident_nodes);

/* Early stop for a steady run (a QUEUED request): every `every` >= 1 steps (checked at the end of
   each graph replay, so at multiples of steps_per_launch at the earliest) the pool computes the
   request's convergence residual on the device, as vplbm_residual defines it with u_prev the
   field of the previous check, and once it is below `tol` > 0 the request runs one more step
   (whose mass and forces are reduced) and finishes.  It costs 16 bytes per node more, charged
   against the budget (VPLBM_EBUDGET if the request no longer fits it). */
int vplbm_pool_set_stop(vplbm_pool p, int64_t id, double tol, int64_t every);

/* The last residual the pool computed for a request with an early stop (+inf before the second
   check); valid until vplbm_pool_result releases the request. */
int vplbm_pool_residual(vplbm_pool p, int64_t id, double *residual);

/* Wait for the previous graph replay, retire finished simulations, admit queued ones, and replay
   the graph for the next steps_per_launch steps (asynchronous).  Any output pointer may be
   NULL. */
int vplbm_pool_advance(vplbm_pool p, int32_t *running, int32_t *queued, int32_t *finished_total);

/* Cancel a request.  A QUEUED one leaves the queue at once; a RUNNING one is retired at the next
   vplbm_pool_advance, which releases its memory (if it finished in the launch that was in
   flight, it is DONE instead).  Its result then has the steps done, zero mass and forces, and,
   if it kept them and was running, the fields of its state at that point.  VPLBM_ESTATE if it
   already finished. */
int vplbm_pool_cancel(vplbm_pool p, int64_t id);

/* State and steps done of a request. */
int vplbm_pool_status(vplbm_pool p, int64_t id, int32_t *state, int64_t *steps_done);

/* Results of a DONE, FAILED or CANCELLED request: final observables and, if the request kept them, the
   host FP64 fields (nx*ny each; pass NULL to skip).  Releases the request. */
int vplbm_pool_result(vplbm_pool p, int64_t id, vplbm_obs *out, double *rho, double *ux, double *uy);

/* Device bytes the pool charges a simulation against its budget. */
int vplbm_pool_bytes_needed(const vplbm_config *cfg, uint64_t *bytes);

/* Wait for outstanding work, free everything.  NULL-safe. */
int vplbm_pool_destroy(vplbm_pool p);

#ifdef __cplusplus
}
#endif
#endif /* VPLBM_H */
