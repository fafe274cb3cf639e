/*
 * dilbm_oracle.h -- interface of the FP64 CPU reference of the DI-LBM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Method: Liu, Huang, Chai & Shi, "A diffuse-interface lattice Boltzmann method for
 * fluid-particle interaction problems" (DI-LBM), Section 2.3, Eqs. (13)-(19), with the
 * particle dynamics of Eqs. (22)-(24) and the collision model of Eqs. (28)-(29).
 *
 * Units are lattice units (dx = dt = 1).  Node (i, j) sits at (i + 0.5, j + 0.5).
 * Population arrays are [9][ny][nx], row-major, FP64, and hold DEVIATIONS from the
 * rest state: f_i - w_i * rho0.
 */
#ifndef DILBM_ORACLE_H
#define DILBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_params {
  int32_t nx, ny;
  double tau;              /* BGK relaxation time, > 0.5 */
  double rho0;             /* rest density */
  double eps;              /* interface width of Eq. (14) */
  double cutoff;           /* phi := 0 where l < -cutoff * eps */
  double G[2];             /* uniform fluid body force density */
  double g[2];             /* g of Eq. (22) */
  uint32_t wall_mask;      /* bit 0: diffuse slab across the y seam; bit 1: across the x seam */
  double wall_h;           /* half thickness of a wall slab */
  int32_t force_mode;      /* 0: momentum-exchange scale; 1: Eq. (18) taken literally */
  double eps_p, eps_p1, eps_w, eps_w1, xi;   /* Eqs. (28)-(29): eps_P, eps_P', eps_W, eps_W', xi */
  int32_t bb_walls_y;      /* test-only: halfway bounce-back walls at y = 0 and y = ny */
  /* open ends in x: non-equilibrium extrapolation (Guo, Zheng & Shi 2002) replaces the
   * post-collision populations of the inlet column x = 0 and the outlet column x = nx-1 */
  int32_t x_boundary;      /* 0: periodic in x; 1: inlet and outlet columns */
  int32_t inlet_kind;      /* 0: velocity (u_in prescribed, rho from the neighbour);
                              1: pressure (rho_in prescribed, u from the neighbour) */
  int32_t inlet_profile;   /* velocity inlet: 0 uniform u_in; 1 parabolic across the
                              channel between the y walls, peak u_in */
  int32_t outlet_kind;     /* 0: pressure (rho_out prescribed, u from the neighbour);
                              1: zero gradient (rho and u from the neighbour) */
  double u_in[2];
  double rho_in, rho_out;
} ora_params;

typedef struct ora_solver ora_solver;

/* lattice and pointwise operators */
void   ora_lattice(int32_t *cx, int32_t *cy, double *w, double *cs2);
void   ora_feq(double rho, double ux, double uy, double *feq);
double ora_phi(double l, double eps, double cutoff);
void   ora_force_term(double tau, double rho, double usx, double usy,
                      double ux_star, double uy_star, double *F);
void   ora_guo_term(double tau, double ux, double uy, double Gx, double Gy, double *Gi);
int32_t ora_collide_node(double tau, double rho0, const double *f_dev, int32_t nb,
                         const double *phi_b, const double *usx, const double *usy,
                         double Gx, double Gy, int32_t force_mode, double *fpost_dev,
                         double *rho_out, double *u_out, double *ustar_out, double *force_b);
/* Non-equilibrium extrapolation at one boundary node: f*_b = f^eq(rho_b, u_b) +
 * (1 - 1/tau) (f_nb - f^eq(rho_nb, u_nb)), where f_nb are the neighbour's populations
 * (deviations) and rho_nb, u_nb its moments (u with half the body force).  rho_b is
 * rho_set (rho_from_nb = 0) or rho_nb; u_b is u_set (u_from_nb = 0) or u_nb. */
void   ora_nee_node(double tau, double rho0, const double *f_nb_dev, double Gx, double Gy,
                    int32_t rho_from_nb, double rho_set, int32_t u_from_nb, double ux_set,
                    double uy_set, double *fpost_dev, double *rho_b, double *u_b);
/* prescribed inlet velocity (x component scale) at row j: 1 for a uniform inlet,
 * 4 s (1 - s) across the channel for a parabolic one */
double ora_inlet_shape(const ora_params *p, int32_t j);
void   ora_pp_force(double dx, double dy, double ri, double rj,
                    double xi, double eps_p, double eps_p1, double *F);
void   ora_pw_force(double dx, double dy, double r,
                    double xi, double eps_w, double eps_w1, double *F);
void   ora_body_update(double m, double I, double Fx, double Fy, double T,
                       double *x, double *y, double *ux, double *uy, double *om);

/* solver */
int32_t ora_create(const ora_params *p, ora_solver **out);
void    ora_destroy(ora_solver *s);
int32_t ora_set_particles(ora_solver *s, int32_t n, const double *pos, const double *vel,
                          const double *omega, const double *radius, const double *density,
                          const uint8_t *fixed);
int32_t ora_set_populations(ora_solver *s, const double *f_dev);
int32_t ora_get_populations(const ora_solver *s, double *f_dev);
int32_t ora_step(ora_solver *s, int64_t nsteps);
int32_t ora_get_fields(ora_solver *s, double *rho, double *ux, double *uy);
int32_t ora_get_particle_forces(const ora_solver *s, double *force, double *torque);
int32_t ora_get_particles(const ora_solver *s, double *pos, double *vel, double *omega);
int32_t ora_get_wall_force(const ora_solver *s, double *force);
int32_t ora_num_threads(void);
void ora_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
