/*
 * dilbm3d.h -- C ABI of the three-dimensional DI-LBM step in libdilbm.so (D3Q19 or D3Q27
 * lattice, spherical particles), on MI355X (gfx950).
 *
 * The paper (Liu, Huang, Chai & Shi) states DI-LBM in two dimensions and motivates it by
 * the cost of solid volume fractions in three.  These calls take the same step as
 * dilbm.h, Section 2.3, with every equation carried over to three dimensions:
 *   1. the diffuse solid field phi of Eq. (14) with l = R - |x - X| for a sphere;
 *   2. the collision of Eq. (13) with the corrected velocity of Eq. (17), phi times the
 *      force term of Eq. (15) and the uncorrected velocity of Eq. (16);
 *   3. pull streaming over the D3Q19 or D3Q27 velocities and the moments of Eq. (5);
 *   4. the hydrodynamic force and torque of Eqs. (18)-(19) per sphere (torque r x F, a
 *      vector; FP64 accumulation) and the motion of Eqs. (22)-(24) with the repulsion
 *      of Eqs. (28)-(29) (FP64).
 *
 * Conventions (as dilbm.h unless stated):
 *   - Lattice units.  Node (i, j, k) sits at (i + 0.5, j + 0.5, k + 0.5).
 *   - D3Q19 directions: 0 rest; 1..6 = +x, -x, +y, -y, +z, -z; 7..18 the edge
 *     directions in opposite pairs: (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1),
 *     (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).  Weights
 *     1/3, 1/18, 1/36; c_s^2 = 1/3.  D3Q27 (lattice = 27) keeps these 19 and adds the
 *     corner directions 19..26 in opposite pairs: (1,1,1), (-1,-1,-1), (1,1,-1),
 *     (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1); weights 8/27, 2/27, 1/54,
 *     1/216, c_s^2 = 1/3 (both are the standard three-dimensional counterparts of the
 *     D2Q9 velocities and weights of Eqs. (3)-(4)).
 *   - Field arrays are [nz][ny][nx]; population arrays are [q][nz][ny][nx] (q = 19 or
 *     27) and hold f_i - w_i * rho0 as FP64.  Per-sphere vectors are [n][3] (x, y, z).
 *   - Host pointers; the caller owns every array; status codes and handle poisoning
 *     as in dilbm.h (DILBM_EUNSTABLE and DILBM_ECAPACITY poison the handle).
 *   - Populations are stored on the device in FP32 as f_i - w_i rho0, or in FP16 as
 *     S (f_i - w_i rho0) 2^k with stochastic rounding in the step (storage =
 *     DILBM_STORE_FP16, as in dilbm.h; structure of arrays, one plane per direction);
 *     all arithmetic of the node update is FP32, the sphere forces, torques and motion
 *     are FP64.
 *   - A sphere's mass is rho_s * 4/3 pi R^3 and its moment of inertia 2/5 m R^2; the
 *     spin update has no gyroscopic term (the inertia is isotropic).
 *   - Streaming is periodic on all three axes; walls are static diffuse slabs across
 *     the periodic seams, as in two dimensions.
 *   - Open ends in x (x_boundary = DILBM_XBC_INLET_OUTLET, the constants of dilbm.h):
 *     non-equilibrium extrapolation (Guo, Zheng & Shi 2002), the treatment the paper
 *     gives its physical boundaries (Section 3), as in two dimensions.  After each
 *     collision the inlet plane x = 0 and the outlet plane x = nx - 1 take f^eq of their
 *     boundary state plus (1 - 1/tau) times the non-equilibrium part of the neighbouring
 *     plane (x = 1, x = nx - 2) at the same step; the neighbour's velocity includes half
 *     the body force.  The boundary planes exert no force on spheres or walls: keep the
 *     spheres' supports off the two outermost planes on each side.
 */
#ifndef DILBM3D_H
#define DILBM3D_H

#include <stdint.h>

#include "dilbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DILBM3D_ABI_VERSION 4u

enum { DILBM3D_WALL_Y = 1u, DILBM3D_WALL_X = 2u, DILBM3D_WALL_Z = 4u };

typedef struct dilbm3d_solver dilbm3d_solver;

typedef struct dilbm3d_params {
  uint32_t abi_version;        /* DILBM3D_ABI_VERSION, else DILBM_EABI */
  int32_t nx, ny, nz;          /* >= 1 each; one population buffer (q planes of nz * ny
                                  rows; a row nx values rounded up to 128 bytes) < 4 GB */
  double tau;                  /* BGK relaxation time, > 0.5 */
  double rho0;                 /* rest density, > 0 */
  double interface_width;      /* epsilon of Eq. (14), > 0 */
  double phi_cutoff;           /* phi := 0 where l < -phi_cutoff * epsilon; > 0 */
  double body_force[3];        /* uniform fluid body force density G */
  double gravity[3];           /* g of Eq. (22): acts on the spheres only */
  uint32_t wall_mask;          /* DILBM3D_WALL_* */
  double wall_half_thickness;  /* h: slab surfaces at h and N - h on each walled axis */
  int32_t force_mode;          /* DILBM_FORCE_MOMENTUM_EXCHANGE or DILBM_FORCE_PAPER_LITERAL */
  double coll_eps_p, coll_eps_p_overlap, coll_eps_w, coll_eps_w_overlap, coll_xi; /* (28)-(29) */
  int32_t list_capacity;       /* spheres listed per tile; 0 = min(n, 128); <= 1024 */
  int32_t lattice;             /* 19 (D3Q19; 0 also means 19) or 27 (D3Q27) */
  int32_t storage;             /* DILBM_STORE_FP32 or DILBM_STORE_FP16, as in dilbm.h */
  int32_t fp16_scale_log2;     /* FP16 storage keeps S (f - w rho0) * 2^k; k in [0, 24],
                                  or DILBM_FP16_SCALE_AUTO (dilbm.h; the default) */
  int32_t x_boundary;          /* DILBM_XBC_*; INLET_OUTLET needs nx >= 3, no DILBM3D_WALL_X */
  int32_t inlet_kind;          /* DILBM_INLET_VELOCITY (inlet_velocity prescribed, rho from
                                  the neighbour) or DILBM_INLET_PRESSURE (inlet_density
                                  prescribed, u from the neighbour) */
  int32_t inlet_profile;       /* velocity inlet: 0 uniform; 1 parabolic 4 s (1 - s) across
                                  y (between the y wall slabs, else the full height), uniform
                                  in z; 2 the product of that and the same across z (a duct);
                                  peak inlet_velocity */
  int32_t outlet_kind;         /* DILBM_OUTLET_PRESSURE (outlet_density prescribed, u from
                                  the neighbour) or DILBM_OUTLET_ZERO_GRADIENT (both) */
  double inlet_velocity[3];
  double inlet_density;        /* > 0 when used */
  double outlet_density;       /* > 0 when used */
  int32_t device;              /* HIP device ordinal */
  void *stream;                /* hipStream_t to run on, or NULL for a library-owned one */
} dilbm3d_params;

/* Fill *p with defaults: abi_version, rho0 = 1, interface_width = 2, phi_cutoff = 4,
 * wall_half_thickness = 4, collision constants 1e4 / 1e4 / 5e3 / 5e3 and xi = 1, FP32
 * storage, fp16_scale_log2 = DILBM_FP16_SCALE_AUTO, periodic in x (inlet and outlet densities 1); the
 * caller sets nx, ny, nz and tau.  Returns DILBM_EINVAL for p == NULL. */
dilbm_status dilbm3d_params_init(dilbm3d_params *p);

/* Create a solver with the fluid at rest (f = w rho0) and no spheres.  *out receives the
 * handle (NULL on failure).  DILBM_EINVAL for bad parameters, DILBM_EABI for a version
 * mismatch, DILBM_ENOMEM when the device buffers do not fit. */
dilbm_status dilbm3d_create(const dilbm3d_params *p, dilbm3d_solver **out);

/* Replace the spheres: 0 <= n <= 2^27 - 1 (DILBM_EINVAL beyond); pos [n][3] (wrapped into the domain), radius [n] > 0 and
 * density [n] > 0 are required, vel [n][3], omega [n][3] and fixed [n] (nonzero: the
 * sphere keeps its velocity and spin and is not integrated) may be NULL (zero). */
dilbm_status dilbm3d_set_particles(dilbm3d_solver *s, int32_t n, const double *pos,
                                   const double *vel, const double *omega,
                                   const double *radius, const double *density,
                                   const uint8_t *fixed);

/* Populations in and out, [q][nz][ny][nx] deviations f_i - w_i rho0 at the current step,
 * q = 19 or 27 (the lattice; stored as FP32 or FP16: values are rounded to nearest on the
 * way in). */
dilbm_status dilbm3d_set_populations(dilbm3d_solver *s, const double *f_dev);
dilbm_status dilbm3d_get_populations(dilbm3d_solver *s, double *f_dev);

/* Advance nsteps >= 0 steps (the procedure of Section 2.3 per step: Eqs. (13)-(19) on the
 * fluid, the open ends if any, Eqs. (22)-(24) and (28)-(29) on the spheres); synchronous.  The sticky error
 * flags are checked every 32 steps while later steps run: a solve that becomes unstable
 * (rho <= 0, |u| > 0.5 or a non-finite value) or overflows a tile sphere list stops
 * within 64 steps of the failure, the call returns the error, and the solver refuses
 * further steps (DILBM_ESTATE). */
dilbm_status dilbm3d_step(dilbm3d_solver *s, int64_t nsteps);

/* Steps taken so far (including those a failed call ran before it stopped). */
dilbm_status dilbm3d_get_step_count(dilbm3d_solver *s, int64_t *steps);

/* rho and the corrected velocity of Eq. (17) at every node (the boundary state on the
 * inlet and outlet planes), [nz][ny][nx] each; any pointer may be NULL. */
dilbm_status dilbm3d_get_fields(dilbm3d_solver *s, double *rho, double *ux, double *uy,
                                double *uz);

/* Hydrodynamic force [n][3] and torque [n][3] on each sphere from the last step
 * (Eqs. (18)-(19)); either may be NULL. */
dilbm_status dilbm3d_get_particle_forces(dilbm3d_solver *s, double *force, double *torque);

/* Sphere state at the current step: pos, vel, omega, [n][3] each; any may be NULL. */
dilbm_status dilbm3d_get_particles(dilbm3d_solver *s, double *pos, double *vel,
                                   double *omega);

/* Force of the fluid on the wall slabs in the last step, [3]. */
dilbm_status dilbm3d_get_wall_force(dilbm3d_solver *s, double *force);

/* Time every collide launch with HIP events on the solver's stream (enable != 0), and
 * read the total milliseconds and launch count since timing was enabled. */
dilbm_status dilbm3d_set_kernel_timing(dilbm3d_solver *s, int32_t enable);
dilbm_status dilbm3d_get_kernel_timing(dilbm3d_solver *s, double *collide_ms,
                                       int64_t *launches);
/* Each timed collide launch since timing was enabled, in launch order: min(cap, count)
 * durations in milliseconds into ms[], *count = the number recorded. */
dilbm_status dilbm3d_get_kernel_launch_times(dilbm3d_solver *s, double *ms, int64_t cap,
                                             int64_t *count);

/* Release the handle and its device memory; NULL is a no-op. */
void dilbm3d_destroy(dilbm3d_solver *s);

/* Batches: several solves advanced together, one collide launch over all members' tiles
 * and one sphere launch over all their spheres per step (the Section 2.3 step of each
 * member, with the arithmetic of dilbm3d_step).  Members must share the device, the
 * lattice, the population storage and the tile width (all with rows of 256 nodes or
 * more, or all shorter); they run on the first member's stream.  The batch refers to its
 * members and owns none of them: once a member is destroyed the batch may only be
 * destroyed (dilbm3d_batch_step would read the destroyed member).  Members may still
 * be stepped, read or given new spheres on their own between batch calls; each call
 * takes their current state.  *out receives the handle (NULL on failure); DILBM_EINVAL
 * for n < 1, a NULL or repeated member or members that differ as above, DILBM_ESTATE
 * for a poisoned member. */
typedef struct dilbm3d_batch dilbm3d_batch;
dilbm_status dilbm3d_batch_create(dilbm3d_solver *const *members, int32_t n,
                                  dilbm3d_batch **out);

/* Advance every member nsteps >= 0 steps (< 2^31); synchronous.  The members' error
 * words are read every 32 steps while later steps run: when a member fails, the call
 * stops within 64 steps, every member has advanced the same number of steps
 * (dilbm3d_get_step_count), every failing member is poisoned as by dilbm3d_step and the
 * call returns the error of the first (the message names its index). */
dilbm_status dilbm3d_batch_step(dilbm3d_batch *b, int64_t nsteps);

/* Release the batch (not its members); NULL is a no-op. */
void dilbm3d_batch_destroy(dilbm3d_batch *b);

/* Message of the batch's last failure ("" if none); for b == NULL, the calling thread's
 * last failure of a dilbm3d_* call. */
const char *dilbm3d_batch_last_error(const dilbm3d_batch *b);

/* Message of the handle's last failure ("" if none); for s == NULL, the calling
 * thread's last failure of a dilbm3d_* call. */
const char *dilbm3d_last_error(const dilbm3d_solver *s);

#ifdef __cplusplus
}
#endif
#endif
