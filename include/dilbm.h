/*
 * dilbm.h -- C ABI of libdilbm.so, an MI355X (gfx950) implementation of the time step of
 * the diffuse-interface lattice Boltzmann method (DI-LBM) for fluid-particle flows of
 * Liu, Huang, Chai & Shi.
 *
 * One step (Section 2.3 of the paper) does, on the GPU:
 *   1. rebuild the diffuse solid field phi of Eq. (14) from the body positions;
 *   2. collide every node with Eq. (13): BGK relaxation towards f^eq(rho, u) with the
 *      corrected velocity u of Eq. (17), plus phi times the force term F_i of Eq. (15)
 *      built from the uncorrected velocity u* of Eq. (16);
 *   3. stream (pull form) and take the moments of Eq. (5) at every node;
 *   4. reduce the hydrodynamic force and torque of Eqs. (18)-(19) per body (FP64), and
 *      move the bodies with Eqs. (22)-(24) plus the repulsion of Eqs. (28)-(29) (FP64).
 *
 * Conventions for every call:
 *   - Lattice units: dx = dt = 1.  Node (i, j) sits at (i + 0.5, j + 0.5).
 *   - D2Q9 directions in the order of Eq. (3): c_0 = (0,0); c_1..c_4 = (1,0), (0,1),
 *     (-1,0), (0,-1); c_5..c_8 = (1,1), (-1,1), (-1,-1), (1,-1).
 *   - Field arrays are row-major [ny][nx]; population arrays are [9][ny][nx] and hold the
 *     deviation from the rest state, f_i - w_i * rho0, as FP64.
 *   - All pointers are HOST pointers unless stated otherwise.  The caller owns every
 *     array; the library copies in and out and keeps no pointer after a call returns.
 *     A handle is owned by the library until its destroy call.
 *   - Every call returns a dilbm_status.  On DILBM_EINVAL / DILBM_ENOMEM the handle is
 *     left as it was.  DILBM_EUNSTABLE (rho <= 0, |u| > 0.5 or a non-finite value at some
 *     node) and DILBM_ECAPACITY (more bodies near one tile than list_capacity) poison
 *     the handle: afterwards only the get_* calls, dilbm_last_error and destroy work;
 *     other calls return DILBM_ESTATE.
 *   - A handle is used by one host thread at a time; distinct handles are independent.
 *
 * Readings of the paper that this library follows (the paper is silent or ambiguous):
 *   c_s^2 = 1/3; l > 0 inside the solid in Eq. (14) and phi := 0 below l = -cutoff*eps;
 *   several bodies covering one node are weighted by w_b = phi_b * min(1, 1/sum phi) and
 *   their Eq. (15) terms are summed; the solid velocity at a node is U + omega x r;
 *   distances use the periodic minimum image; a uniform fluid body force G enters by the
 *   forcing of Guo, Zheng & Shi (Phys. Rev. E 65, 046308, 2002) with u* carrying G/2;
 *   walls are static diffuse slabs across the periodic seams (streaming is periodic on
 *   both axes); the body update is forward Euler in velocity and trapezoidal in position
 *   with dt = 1; a body's mass is rho_s * pi * R^2 and its inertia m R^2 / 2.
 */
#ifndef DILBM_H
#define DILBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DILBM_ABI_VERSION 2u

typedef enum dilbm_status {
  DILBM_OK = 0,
  DILBM_EINVAL = -1,     /* a bad argument; nothing changed */
  DILBM_ENOMEM = -2,     /* device or host memory exhausted; nothing changed */
  DILBM_EDEVICE = -3,    /* a HIP runtime error */
  DILBM_EUNSTABLE = -4,  /* the flow blew up; handle poisoned */
  DILBM_ESTATE = -5,     /* call not allowed in the handle's state */
  DILBM_EABI = -6,       /* abi_version mismatch */
  DILBM_ECAPACITY = -7,  /* a per-tile body list overflowed; handle poisoned */
  DILBM_EAGAIN = -8      /* pool: not enough free memory right now; retry later */
} dilbm_status;

enum { DILBM_STORE_FP32 = 0, DILBM_STORE_FP16 = 1 };
/* fp16_scale_log2 = DILBM_FP16_SCALE_AUTO: the library takes the largest k at which every
 * equilibrium state with 0 < rho <= 2 rho0 and |u| <= 0.5 (the speeds a step accepts) is
 * stored at no more than half of FP16's largest finite value (65504), the rest being
 * headroom for the non-equilibrium part: k = 10 on D2Q9, 11 on D3Q19, 8 on D3Q27 for
 * rho0 = 1.  A power-of-two scale changes no relative precision in FP16's normal range;
 * a larger k keeps smaller deviations out of the subnormals but lets a state inside that
 * range overflow (a non-finite population: DILBM_EUNSTABLE at the next step). */
enum { DILBM_FP16_SCALE_AUTO = -1 };
/* Scale of Eqs. (18)-(19).  MOMENTUM_EXCHANGE: F_b = -sum_n w_b rho (u_s - u*), the
 * momentum the fluid gains from the body in the collision (the appendix's macroscopic
 * force), which balances the fluid momentum exactly.  PAPER_LITERAL: -sum_n w_b sum_i c_i
 * F_i as printed, which is (1 - 1/(2 tau)) times the former. */
enum { DILBM_FORCE_MOMENTUM_EXCHANGE = 0, DILBM_FORCE_PAPER_LITERAL = 1 };
enum { DILBM_WALL_Y = 1u, DILBM_WALL_X = 2u };
/* Open ends in x: the boundary treatment the paper applies to its physical boundaries
 * (Section 3), non-equilibrium extrapolation (Guo, Zheng & Shi 2002).  The inlet column
 * x = 0 and the outlet column x = nx - 1 take, after each collision, f^eq of their
 * boundary state plus (1 - 1/tau) times the non-equilibrium part of the neighbouring
 * column (x = 1, x = nx - 2) at the same step; the neighbour's velocity includes half the
 * body force, as in its own collision.  Boundary columns exert no force on bodies: keep
 * bodies' supports off the two outermost columns on each side. */
enum { DILBM_XBC_PERIODIC = 0, DILBM_XBC_INLET_OUTLET = 1 };
enum { DILBM_INLET_VELOCITY = 0, DILBM_INLET_PRESSURE = 1 };
enum { DILBM_OUTLET_PRESSURE = 0, DILBM_OUTLET_ZERO_GRADIENT = 1 };

typedef struct dilbm_params {
  uint32_t abi_version;        /* must be DILBM_ABI_VERSION, else DILBM_EABI */
  int32_t nx, ny;              /* lattice size, 1 <= n <= 65536 each, nx*ny < 2^31 */
  double tau;                  /* BGK relaxation time of Eq. (13), > 0.5 */
  double rho0;                 /* rest density (also rho_f of Eq. (22)), > 0 */
  double interface_width;      /* epsilon of Eq. (14), > 0 */
  double phi_cutoff;           /* phi := 0 where l < -phi_cutoff * epsilon; > 0 */
  double body_force[2];        /* G: uniform force density on the fluid at every node */
  double gravity[2];           /* g of Eq. (22): the body feels (rho0/rho_s - 1) m g */
  uint32_t wall_mask;          /* DILBM_WALL_* bits; 0 = fully periodic */
  double wall_half_thickness;  /* h: a wall slab is |distance to the seam| < h */
  int32_t force_mode;          /* DILBM_FORCE_* */
  double coll_eps_p;           /* eps_P  of Eq. (28) */
  double coll_eps_p_overlap;   /* eps_P' of Eq. (28) */
  double coll_eps_w;           /* eps_W  of Eq. (29) */
  double coll_eps_w_overlap;   /* eps_W' of Eq. (29) */
  double coll_xi;              /* xi of Eqs. (28)-(29) */
  int32_t storage;             /* DILBM_STORE_*: population storage; arithmetic is FP32 */
  int32_t fp16_scale_log2;     /* FP16 storage keeps 36 (f - w rho0) * 2^k; k in [0, 24],
                                  or DILBM_FP16_SCALE_AUTO (default) */
  int32_t list_capacity;       /* bodies per tile list; 0 = min(n_bodies, 128) */
  int32_t tile;                /* tile shape id (dilbm_tile_shape); -1 = default: 256 x 1
                                  for FP32 storage with nx >= 1024, else 64 x 4.  Shape 5
                                  (512 x 1, two nodes per lane) needs FP16 storage and an
                                  even nx */
  int32_t x_boundary;          /* DILBM_XBC_*; INLET_OUTLET needs nx >= 3, no DILBM_WALL_X */
  int32_t inlet_kind;          /* DILBM_INLET_*: VELOCITY prescribes inlet_velocity and
                                  takes rho from the neighbour; PRESSURE prescribes
                                  inlet_density and takes u from the neighbour */
  int32_t inlet_profile;       /* velocity inlet: 0 uniform; 1 parabolic 4 s (1 - s) across
                                  the channel (between the y wall slabs, else the full
                                  height), peak inlet_velocity */
  int32_t outlet_kind;         /* DILBM_OUTLET_*: PRESSURE prescribes outlet_density and
                                  takes u from the neighbour; ZERO_GRADIENT takes both */
  double inlet_velocity[2];
  double inlet_density;        /* > 0 when used */
  double outlet_density;       /* > 0 when used */
  int32_t device;              /* HIP device ordinal */
  void *stream;                /* hipStream_t to run on, or NULL for a library stream */
} dilbm_params;

typedef struct dilbm_solver dilbm_solver;

/* Fill *p with defaults: tau 0.8, rho0 1, interface width 2, cutoff 4, no forces, no
 * walls, h = 2 * interface width, momentum-exchange force scale, eps_P = eps_P' = 1e4,
 * eps_W = eps_W' = 5e3, xi = 1, FP32 storage, FP16 scale DILBM_FP16_SCALE_AUTO, device 0,
 * no stream.  nx and ny are set to 0 and must be filled in. */
void dilbm_params_init(dilbm_params *p);

/* Number of tile shapes and the node extent (tx, ty) of shape `id`: shapes 0-4 hold 256
 * nodes (one per lane of a 256-thread block), shape 5 holds 512 (two per lane). */
int32_t dilbm_num_tile_shapes(void);
dilbm_status dilbm_tile_shape(int32_t id, int32_t *tx, int32_t *ty);

/* Device bytes a solve with these parameters and n bodies occupies. */
dilbm_status dilbm_footprint(const dilbm_params *p, int32_t n_bodies, uint64_t *bytes);

/* Create a solve with the fluid at rest (f = w rho0) and no bodies (Section 2.3, step 1).
 * Allocates its device memory on p->device. */
dilbm_status dilbm_create(const dilbm_params *p, dilbm_solver **out);

/* Replace the whole body set at the current step boundary; populations are untouched.
 * The state per body is what Eqs. (22)-(24) evolve: centre X_s, velocity u_s, spin
 * omega_s, with mass rho_s pi R^2 and inertia m R^2 / 2 (Section 3.2 gives the particle
 * by its diameter and density ratio); the solid field of Eq. (14) is rebuilt from it.
 * pos/vel are [n][2], omega/radius/density [n]; vel, omega and fixed may be NULL (zero).
 * radius and density must be > 0.  fixed[b] != 0 makes body b move with its given
 * velocity and spin (its hydrodynamic force is still computed).  Positions are wrapped
 * into [0, nx) x [0, ny).  0 <= n <= 2^27 - 1 (DILBM_EINVAL beyond). */
dilbm_status dilbm_set_particles(dilbm_solver *s, int32_t n, const double *pos,
                                 const double *vel, const double *omega, const double *radius,
                                 const double *density, const uint8_t *fixed);

/* Set / read the populations of the current state: f_dev[9][ny][nx] = f_i - w_i rho0. */
dilbm_status dilbm_set_populations(dilbm_solver *s, const double *f_dev);
dilbm_status dilbm_get_populations(dilbm_solver *s, double *f_dev);

/* Advance nsteps >= 0 steps of the procedure of Section 2.3: per step, the solid field
 * of Eq. (14) from the body state, the collision of Eq. (13) with Eqs. (15)-(17) and the
 * streaming, the force and torque of Eqs. (18)-(19), and the body update of
 * Eqs. (22)-(24) with the repulsion of Eqs. (28)-(29).  Synchronous: returns when the
 * steps are done.  The device's error flags are read back after every chunk of steps
 * (32 by default) while the next chunk runs, so a blow-up or a list overflow ends the
 * call at most two chunks after the step where it happened (DILBM_EUNSTABLE /
 * DILBM_ECAPACITY, handle poisoned; the step count then includes those chunks). */
dilbm_status dilbm_step(dilbm_solver *s, int64_t nsteps);

/* rho and the corrected velocity u of Eq. (17) of the current state, each [ny][nx];
 * any pointer may be NULL. */
dilbm_status dilbm_get_fields(dilbm_solver *s, double *rho, double *ux, double *uy);

/* The same for the rectangle [x0, x0 + w) x [y0, y0 + h) only; each array is [h][w].
 * For lattices too large to copy whole. */
dilbm_status dilbm_get_fields_region(dilbm_solver *s, int32_t x0, int32_t y0, int32_t w,
                                     int32_t h, double *rho, double *ux, double *uy);

/* The same as dilbm_get_fields_region for callers that cannot allocate memory (code
 * under HIP graph capture elsewhere in the process, tight serving loops, harnesses that
 * forbid hipMalloc): it allocates nothing.  The values go through a fixed device staging
 * array of 3 x 2^20 FP64 (24 MiB, held on each GPU the library runs on until the process
 * ends) instead of a buffer of the handle's.  w * h must be at most 2^20 (1048576) nodes,
 * else DILBM_EINVAL and nothing is read.  All calls on one GPU share the array: calls
 * that overlap on one GPU (other threads, other handles) race and must be serialised by
 * the caller. */
dilbm_status dilbm_get_fields_region_noalloc(dilbm_solver *s, int32_t x0, int32_t y0, int32_t w,
                                             int32_t h, double *rho, double *ux, double *uy);

/* Force [n][2] and torque [n] on each body by the fluid in the last completed step
 * (zeros before the first step), Eqs. (18)-(19) with the sign printed there. */
dilbm_status dilbm_get_particle_forces(dilbm_solver *s, double *force, double *torque);

/* Body state at the current step: pos/vel [n][2], omega [n]; any may be NULL. */
dilbm_status dilbm_get_particles(dilbm_solver *s, double *pos, double *vel, double *omega);

/* Force [2] on all wall slabs together by the fluid in the last completed step. */
dilbm_status dilbm_get_wall_force(dilbm_solver *s, double *force);

/* Steps completed so far. */
dilbm_status dilbm_get_step_count(dilbm_solver *s, int64_t *steps);

/* Number of bodies the handle holds (size the get_* arrays with it).  After a
 * set_particles that failed with DILBM_ECAPACITY the new body set is in place. */
dilbm_status dilbm_get_body_count(dilbm_solver *s, int32_t *n);

/* Kernel timing: while enabled, dilbm_step launches kernels directly (no graph) and
 * brackets every collide-stream launch with HIP events on the solve's stream; the get
 * call returns the summed milliseconds and the number of launches since enabling. */
dilbm_status dilbm_set_kernel_timing(dilbm_solver *s, int32_t enable);
dilbm_status dilbm_get_kernel_timing(dilbm_solver *s, double *collide_ms, int64_t *launches);
/* The duration of each timed collide-stream launch since timing was enabled, in launch
 * order: copies min(cap, count) values (milliseconds) into ms[] and sets *count to the
 * number recorded.  ms may be NULL when cap is 0. */
dilbm_status dilbm_get_kernel_launch_times(dilbm_solver *s, double *ms, int64_t cap,
                                           int64_t *count);

void dilbm_destroy(dilbm_solver *s);  /* NULL-safe */

/* Message of the last failed call on s (or of this thread's last failed create when s is
 * NULL); never NULL. */
const char *dilbm_last_error(const dilbm_solver *s);

/* ---------------------------------------------------------------------------------
 * Pool: many independent solves advanced together.  Every step of the pool is one
 * collide-stream launch and one body launch for all member solves; K-step sequences
 * are captured in a HIP graph.  Solves may join and leave between runs (continuous
 * batching).  Each member follows exactly the per-solve semantics above.
 * The pool's solve memory comes from one device arena: either the caller's (`arena`,
 * `arena_bytes`, device memory that must outlive the pool) or, when arena is NULL, one
 * the pool allocates with arena_bytes.
 * ------------------------------------------------------------------------------- */
typedef struct dilbm_pool dilbm_pool;

dilbm_status dilbm_pool_create(int32_t device, void *stream, void *arena, uint64_t arena_bytes,
                               dilbm_pool **out);

/* Admit a solve that will run `nsteps` steps, with bodies as in dilbm_set_particles
 * (p->device and p->stream are ignored).  Returns DILBM_EAGAIN if its footprint does
 * not fit in the arena's free space now, DILBM_ENOMEM if it can never fit. */
dilbm_status dilbm_pool_submit(dilbm_pool *pool, const dilbm_params *p, int32_t n,
                               const double *pos, const double *vel, const double *omega,
                               const double *radius, const double *density,
                               const uint8_t *fixed, int64_t nsteps, int64_t *ticket);

/* Enqueue up to `steps` steps for every member that has steps left (fewer for members
 * that finish earlier).  After each K-step chunk the members' sticky error words are
 * copied to the host asynchronously; the call waits for the previous chunk's copy (the
 * device keeps the current chunk queued) and stops every member whose solve has become
 * unstable or overflowed a list: it leaves the pool at most one chunk after the failure,
 * dilbm_pool_query reports it done, and its results calls return the error.  The call
 * returns with the last chunk still running; dilbm_pool_sync waits for it and applies
 * the same check. */
dilbm_status dilbm_pool_run(dilbm_pool *pool, int32_t steps);

/* Wait for everything enqueued so far. */
dilbm_status dilbm_pool_sync(dilbm_pool *pool);

/* Steps enqueued for a ticket, and whether all its steps have completed on the GPU
 * (non-blocking). */
dilbm_status dilbm_pool_query(dilbm_pool *pool, int64_t ticket, int64_t *steps_enqueued,
                              int32_t *done);

/* Results of a ticket; wait for the ticket's enqueued steps first. */
dilbm_status dilbm_pool_get_fields(dilbm_pool *pool, int64_t ticket, double *rho, double *ux,
                                   double *uy);
dilbm_status dilbm_pool_get_particles(dilbm_pool *pool, int64_t ticket, double *pos,
                                      double *vel, double *omega);
dilbm_status dilbm_pool_get_particle_forces(dilbm_pool *pool, int64_t ticket, double *force,
                                            double *torque);

/* Leave the pool and give the memory back (after the ticket's work has completed). */
dilbm_status dilbm_pool_release(dilbm_pool *pool, int64_t ticket);

/* Pool tuning: steps per captured graph (1..256) and tile shape for solves admitted
 * later.  dilbm_pool_autotune times every tile shape with 16-step graphs, then 128-step
 * graphs with the best shape, on the current members, and keeps the fastest per node
 * update.  Each candidate's first graph launch captures the graph and is not timed; then
 * whole graph launches covering at least steps_per_trial steps are timed with events.
 * Every trial step is a real step of the members (about 5 x 32 + 256 steps at
 * steps_per_trial <= 16). */
dilbm_status dilbm_pool_set_launch(dilbm_pool *pool, int32_t graph_steps, int32_t tile);
dilbm_status dilbm_pool_autotune(dilbm_pool *pool, int32_t steps_per_trial,
                                 int32_t *best_graph_steps, int32_t *best_tile);

/* Free arena bytes, member count, and the last error message of the pool. */
dilbm_status dilbm_pool_stats(dilbm_pool *pool, uint64_t *free_bytes, int32_t *members);
const char *dilbm_pool_last_error(const dilbm_pool *pool);

void dilbm_pool_destroy(dilbm_pool *pool);  /* NULL-safe; waits for enqueued work */

#ifdef __cplusplus
}
#endif
#endif
