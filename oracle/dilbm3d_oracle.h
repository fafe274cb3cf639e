/*
 * dilbm3d_oracle.h -- interface of the FP64 CPU reference of the three-dimensional DI-LBM
 * time step (D3Q19 or D3Q27 lattice, spherical particles).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU library's 3-D path
 * is checked against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Method: the DI-LBM step of Section 2.3 (Eqs. (13)-(19)) and the particle dynamics of
 * Eqs. (22)-(24) and (28)-(29), written for three dimensions: the diffuse solid field of
 * Eq. (14) with l = R - |x - X| for a sphere, the rigid-body solid velocity U + omega x r,
 * torque r x F as a vector, and a sphere's mass 4/3 pi R^3 rho_s and moment of inertia
 * 2/5 m R^2.  The D3Q19 velocity set and weights (1/3, 1/18, 1/36) are the standard
 * three-dimensional counterpart of Eqs. (3)-(4), with the same c_s^2 = 1/3.
 *
 * Units are lattice units (dx = dt = 1).  Node (i, j, k) sits at (i + 0.5, j + 0.5, k + 0.5).
 * Population arrays are [19][nz][ny][nx], row-major, FP64, and hold DEVIATIONS from the
 * rest state: f_i - w_i * rho0.  Velocity order: 0 rest; 1-6 (+x, -x, +y, -y, +z, -z);
 * 7-18 the twelve edge directions in opposite pairs (+x+y, -x-y), (+x-y, -x+y),
 * (+x+z, -x-z), (+x-z, -x+z), (+y+z, -y-z), (+y-z, -y+z).
 */
#ifndef DILBM3D_ORACLE_H
#define DILBM3D_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora3_params {
  int32_t nx, ny, nz;
  double tau;              /* BGK relaxation time, > 0.5 */
  double rho0;             /* rest density */
  double eps;              /* interface width of Eq. (14) */
  double cutoff;           /* phi := 0 where l < -cutoff * eps */
  double G[3];             /* uniform fluid body force density */
  double g[3];             /* g of Eq. (22) */
  uint32_t wall_mask;      /* diffuse slabs across the seams: bit 0 y, bit 1 x, bit 2 z */
  double wall_h;           /* half thickness of a wall slab */
  int32_t force_mode;      /* 0: momentum-exchange scale; 1: Eq. (18) taken literally */
  double eps_p, eps_p1, eps_w, eps_w1, xi;   /* Eqs. (28)-(29) */
  int32_t lattice;         /* 19 (D3Q19, also 0) or 27 (D3Q27) */
  /* open ends in x: non-equilibrium extrapolation (Guo, Zheng & Shi 2002) replaces the
   * post-collision state of the columns x = 0 (inlet) and x = nx - 1 (outlet) */
  int32_t x_boundary;      /* 0: periodic in x; 1: inlet and outlet columns */
  int32_t inlet_kind;      /* 0: velocity u_in (rho from the neighbour); 1: density rho_in */
  int32_t inlet_profile;   /* velocity inlet: 0 uniform; 1 parabolic 4 s (1 - s) across y
                              (between the y wall slabs, else the full height); 2 the
                              product of that and the same across z */
  int32_t outlet_kind;     /* 0: density rho_out (u from the neighbour); 1: zero gradient */
  double u_in[3];
  double rho_in, rho_out;
} ora3_params;

typedef struct ora3_solver ora3_solver;

/* lattice and pointwise operators: the ora3q_ forms take the velocity set (19 or 27),
 * the ora3_ forms are D3Q19 */
void   ora3q_lattice(int32_t q, int32_t *cx, int32_t *cy, int32_t *cz, double *w, double *cs2);
void   ora3q_feq(int32_t q, double rho, const double *u, double *feq);
void   ora3q_force_term(int32_t q, double tau, double rho, const double *us, const double *ustar,
                        double *F);
void   ora3q_guo_term(int32_t q, double tau, const double *u, const double *G, double *Gi);
int32_t ora3q_collide_node(int32_t q, double tau, double rho0, const double *f_dev, int32_t nb,
                           const double *phi_b, const double *us, const double *G,
                           int32_t force_mode, double *fpost_dev, double *rho_out,
                           double *u_out, double *ustar_out, double *force_b);
void   ora3_lattice(int32_t *cx, int32_t *cy, int32_t *cz, double *w, double *cs2);
void   ora3_feq(double rho, const double *u, double *feq);
void   ora3_force_term(double tau, double rho, const double *us, const double *ustar,
                       double *F);
void   ora3_guo_term(double tau, const double *u, const double *G, double *Gi);
/* One node of one step before streaming: nb bodies cover it with raw phi_b and solid
 * velocity us[3 b ..]; outputs f* - w rho0, rho, corrected u, u* and the force on each
 * body ([3 b ..]).  Returns -4 if rho <= 0, |u| > 0.5 or anything is not finite. */
int32_t ora3_collide_node(double tau, double rho0, const double *f_dev, int32_t nb,
                          const double *phi_b, const double *us, const double *G,
                          int32_t force_mode, double *fpost_dev, double *rho_out,
                          double *u_out, double *ustar_out, double *force_b);
/* Non-equilibrium extrapolation at one boundary node from its neighbour's populations
 * f_nb_dev (deviations): f*_b = f^eq(rho_b, u_b) + (1 - 1/tau) (f_nb - f^eq(rho_nb, u_nb)),
 * u_nb = (j_nb + G/2) / rho_nb.  rho_b = rho_nb if rho_from_nb, else rho_set; u_b = u_nb
 * if u_from_nb, else u_set.  Outputs f*_b - w rho0 and the boundary state. */
void   ora3q_nee_node(int32_t q, double tau, double rho0, const double *f_nb_dev,
                      const double *G, int32_t rho_from_nb, double rho_set, int32_t u_from_nb,
                      const double *u_set, double *fpost_dev, double *rho_b, double *u_b);
/* the inlet profile factor of node (j, k) (1 for a uniform inlet) */
double ora3_inlet_shape(const ora3_params *p, int32_t j, int32_t k);
void   ora3_pp_force(const double *d, double ri, double rj, double xi, double eps_p,
                     double eps_p1, double *F);
void   ora3_pw_force(const double *d, double r, double xi, double eps_w, double eps_w1,
                     double *F);
void   ora3_body_update(double m, double I, const double *F, const double *T, double *x,
                        double *u, double *om);

/* solver */
int32_t ora3_create(const ora3_params *p, ora3_solver **out);
void    ora3_destroy(ora3_solver *s);
int32_t ora3_set_particles(ora3_solver *s, int32_t n, const double *pos, const double *vel,
                           const double *omega, const double *radius, const double *density,
                           const uint8_t *fixed);
int32_t ora3_set_populations(ora3_solver *s, const double *f_dev);
int32_t ora3_get_populations(const ora3_solver *s, double *f_dev);
int32_t ora3_step(ora3_solver *s, int64_t nsteps);
int32_t ora3_get_fields(ora3_solver *s, double *rho, double *ux, double *uy, double *uz);
int32_t ora3_get_particle_forces(const ora3_solver *s, double *force, double *torque);
int32_t ora3_get_particles(const ora3_solver *s, double *pos, double *vel, double *omega);
int32_t ora3_get_wall_force(const ora3_solver *s, double *force);

#ifdef __cplusplus
}
#endif
#endif
