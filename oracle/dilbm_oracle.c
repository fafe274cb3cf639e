/*
 * dilbm_oracle.c -- plain FP64 CPU reference of the DI-LBM time step.
 *
 * TEST INFRASTRUCTURE ONLY: the oracle that the GPU library is checked against.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it.  It shares
 * no code with the GPU library.  It is written to be read against the paper, not to be
 * fast: every node is handled by one call of ora_collide_node(), which takes the
 * paper's steps in the paper's order.
 *
 * Paper: Liu, Huang, Chai & Shi, "A diffuse-interface lattice Boltzmann method for
 * fluid-particle interaction problems".
 *   Eq. (2)  equilibrium;  Eqs. (3)-(4) D2Q9 velocities and weights;  Eq. (5) moments;
 *   Eq. (13) DI-LBM evolution;  Eq. (14) diffuse solid field phi;  Eq. (15) modified
 *   force term;  Eq. (16) uncorrected velocity;  Eq. (17) corrected velocity;
 *   Eqs. (18)-(19) hydrodynamic force and torque;  Section 2.3 step procedure;
 *   Eqs. (22)-(24) particle motion;  Eqs. (28)-(29) particle-particle and
 *   particle-wall repulsion.
 *
 * Readings where the paper is silent or ambiguous (each is stated where it is used):
 *   c_s^2 = 1/3 (the relation after Eq. (2) is cut off; 1/3 is the value for which the
 *   second moment of the equilibrium in the appendix holds with the Eq. (4) weights);
 *   l > 0 inside the solid; cell-centred nodes; minimum-image distances on periodic
 *   axes; phi := 0 below l = -cutoff*eps; several bodies at one node are weighted by
 *   w_b = phi_b * min(1, 1/sum phi); rigid-body solid velocity U + omega x r; a uniform
 *   fluid body force enters through Guo-Zheng-Shi forcing (Phys. Rev. E 65, 046308,
 *   2002) with u* carrying half of it; walls are static diffuse slabs across the
 *   periodic seams; forward-Euler velocity and trapezoidal position updates with dt=1.
 *
 * Compiled with -O2 -ffp-contract=off; results do not depend on the thread count
 * because every node is computed independently and every reduction over nodes runs
 * serially in row-major order.
 */
#include "dilbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

/* Eq. (3): c_0 = 0; c_1..c_4 = (cos, sin)((i-1) pi/2); c_5..c_8 = sqrt2 (cos, sin)((2i-1) pi/4). */
static const int32_t CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int32_t CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Eq. (4). */
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* Lattice sound speed squared (see header comment). */
static const double CS2 = 1.0 / 3.0;

/* status codes (same numbers as the public library's, defined independently here) */
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_EUNSTABLE = -4 };

void ora_lattice(int32_t *cx, int32_t *cy, double *w, double *cs2) {
  for (int i = 0; i < Q; ++i) {
    if (cx) cx[i] = CX[i];
    if (cy) cy[i] = CY[i];
    if (w) w[i] = WT[i];
  }
  if (cs2) *cs2 = CS2;
}

/* Eq. (2): f_i^eq = w_i rho [1 + c_i.u/cs2 + (c_i.u)^2/(2 cs2^2) - u^2/(2 cs2)]. */
void ora_feq(double rho, double ux, double uy, double *feq) {
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < Q; ++i) {
    const double cu = CX[i] * ux + CY[i] * uy;
    feq[i] = WT[i] * rho * (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Eq. (14): phi = (1 + tanh(2 l / eps)) / 2, l = signed distance, positive inside the
 * solid.  tanh never reaches -1, so phi is set to 0 where l < -cutoff*eps. */
double ora_phi(double l, double eps, double cutoff) {
  if (l < -cutoff * eps) return 0.0;
  return 0.5 * (1.0 + tanh(2.0 * l / eps));
}

/* Eq. (15): F_i = (1 - 1/(2 tau)) w_i rho [ c_i.(u_s - u*)/cs2
 *                 + (u_s u_s - u* u*) : (c_i c_i - cs2 I) / (2 cs2^2) ]. */
void ora_force_term(double tau, double rho, double usx, double usy, double ux_star,
                    double uy_star, double *F) {
  const double us[2] = {usx, usy};
  const double ut[2] = {ux_star, uy_star};
  for (int i = 0; i < Q; ++i) {
    const double c[2] = {(double)CX[i], (double)CY[i]};
    const double lin = (c[0] * (us[0] - ut[0]) + c[1] * (us[1] - ut[1])) / CS2;
    double quad = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        quad += (us[a] * us[b] - ut[a] * ut[b]) * (c[a] * c[b] - (a == b ? CS2 : 0.0));
    F[i] = (1.0 - 1.0 / (2.0 * tau)) * WT[i] * rho * (lin + quad / (2.0 * CS2 * CS2));
  }
}

/* Forcing term for a uniform fluid body force G (Guo, Zheng & Shi 2002):
 * G_i = (1 - 1/(2 tau)) w_i [ (c_i - u)/cs2 + (c_i.u) c_i / cs2^2 ] . G. */
void ora_guo_term(double tau, double ux, double uy, double Gx, double Gy, double *Gi) {
  for (int i = 0; i < Q; ++i) {
    const double cu = CX[i] * ux + CY[i] * uy;
    const double ax = (CX[i] - ux) / CS2 + cu * CX[i] / (CS2 * CS2);
    const double ay = (CY[i] - uy) / CS2 + cu * CY[i] / (CS2 * CS2);
    Gi[i] = (1.0 - 1.0 / (2.0 * tau)) * WT[i] * (ax * Gx + ay * Gy);
  }
}

/*
 * One node of one DI-LBM step, before streaming (Section 2.3, steps 2-4).
 *   f_dev[i]  : f_i - w_i rho0 at this node (post-stream state of time t_n)
 *   nb bodies cover the node with raw phi_b (Eq. (14)) and solid velocity u_{s,b}.
 * Outputs f*_i - w_i rho0, rho, corrected u (Eq. (17)), u* and, per body, the force
 * this node exerts on it (Eq. (18) sign: force ON the body BY the fluid).
 * Returns ORA_EUNSTABLE if rho <= 0, |u| > 0.5 or anything is not finite.
 */
int32_t ora_collide_node(double tau, double rho0, const double *f_dev, int32_t nb,
                         const double *phi_b, const double *usx, const double *usy,
                         double Gx, double Gy, int32_t force_mode, double *fpost_dev,
                         double *rho_out, double *u_out, double *ustar_out, double *force_b) {
  double f[Q];
  for (int i = 0; i < Q; ++i) f[i] = f_dev[i] + WT[i] * rho0;

  /* Eq. (5) and Eq. (16); u* carries half of the fluid body force (Guo forcing). */
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    jx += CX[i] * f[i];
    jy += CY[i] * f[i];
  }
  const double usx_star = (jx + 0.5 * Gx) / rho;
  const double usy_star = (jy + 0.5 * Gy) / rho;

  /* several bodies: w_b = phi_b * min(1, 1/sum phi), so the combined phi stays <= 1 */
  double S = 0.0;
  for (int b = 0; b < nb; ++b) S += phi_b[b];
  const double scale = S > 1.0 ? 1.0 / S : 1.0;

  /* Eq. (17): u = u* + phi (u_s - u*) / 2, summed over bodies. */
  double ux = usx_star, uy = usy_star;
  for (int b = 0; b < nb; ++b) {
    const double wb = scale * phi_b[b];
    ux += 0.5 * wb * (usx[b] - usx_star);
    uy += 0.5 * wb * (usy[b] - usy_star);
  }

  /* Eq. (13): f* = f - (f - f^eq(rho, u))/tau + phi F_i (+ body-force term). */
  double feq[Q], Gi[Q], Fb[Q], acc[Q];
  ora_feq(rho, ux, uy, feq);
  ora_guo_term(tau, ux, uy, Gx, Gy, Gi);
  for (int i = 0; i < Q; ++i) acc[i] = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double wb = scale * phi_b[b];
    ora_force_term(tau, rho, usx[b], usy[b], usx_star, usy_star, Fb);
    for (int i = 0; i < Q; ++i) acc[i] += wb * Fb[i];
    if (force_b) {
      double fx, fy;
      if (force_mode == 1) {
        /* Eq. (18) literally: -phi sum_i F_i c_i */
        fx = 0.0;
        fy = 0.0;
        for (int i = 0; i < Q; ++i) {
          fx += Fb[i] * CX[i];
          fy += Fb[i] * CY[i];
        }
        fx = -wb * fx;
        fy = -wb * fy;
      } else {
        /* the momentum the node gains from the body in this collision,
         * phi rho (u_s - u*) (the appendix's macroscopic force), with the sign of Eq. (18) */
        fx = -wb * rho * (usx[b] - usx_star);
        fy = -wb * rho * (usy[b] - usy_star);
      }
      force_b[2 * b + 0] = fx;
      force_b[2 * b + 1] = fy;
    }
  }
  int bad = !(rho > 0.0) || !(ux * ux + uy * uy <= 0.25);
  for (int i = 0; i < Q; ++i) {
    const double fp = f[i] - (f[i] - feq[i]) / tau + acc[i] + Gi[i];
    fpost_dev[i] = fp - WT[i] * rho0;
    if (!isfinite(fpost_dev[i])) bad = 1;
  }
  if (rho_out) *rho_out = rho;
  if (u_out) {
    u_out[0] = ux;
    u_out[1] = uy;
  }
  if (ustar_out) {
    ustar_out[0] = usx_star;
    ustar_out[1] = usy_star;
  }
  return bad ? ORA_EUNSTABLE : ORA_OK;
}

/* Non-equilibrium extrapolation (Guo, Zheng & Shi 2002), the boundary treatment the paper
 * applies to its physical boundaries (Section 3): the boundary node takes the equilibrium
 * of its boundary state plus the neighbour's non-equilibrium part, relaxed as in Eq. (13). */
void ora_nee_node(double tau, double rho0, const double *f_nb_dev, double Gx, double Gy,
                  int32_t rho_from_nb, double rho_set, int32_t u_from_nb, double ux_set,
                  double uy_set, double *fpost_dev, double *rho_b, double *u_b) {
  double f[Q];
  for (int i = 0; i < Q; ++i) f[i] = f_nb_dev[i] + WT[i] * rho0;
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    jx += CX[i] * f[i];
    jy += CY[i] * f[i];
  }
  const double ux = (jx + 0.5 * Gx) / rho, uy = (jy + 0.5 * Gy) / rho;
  const double rb = rho_from_nb ? rho : rho_set;
  const double uxb = u_from_nb ? ux : ux_set, uyb = u_from_nb ? uy : uy_set;
  double feq_nb[Q], feq_b[Q];
  ora_feq(rho, ux, uy, feq_nb);
  ora_feq(rb, uxb, uyb, feq_b);
  for (int i = 0; i < Q; ++i)
    fpost_dev[i] = feq_b[i] + (1.0 - 1.0 / tau) * (f[i] - feq_nb[i]) - WT[i] * rho0;
  if (rho_b) *rho_b = rb;
  if (u_b) {
    u_b[0] = uxb;
    u_b[1] = uyb;
  }
}

double ora_inlet_shape(const ora_params *p, int32_t j) {
  if (!p->inlet_profile) return 1.0;
  double y0 = 0.0, y1 = (double)p->ny;
  if ((p->wall_mask & 1u) && !p->bb_walls_y) {  /* slab across the y seam: |y - seam| < h */
    y0 = p->wall_h;
    y1 = (double)p->ny - p->wall_h;
  }
  const double sv = ((double)j + 0.5 - y0) / (y1 - y0);
  return (sv > 0.0 && sv < 1.0) ? 4.0 * sv * (1.0 - sv) : 0.0;
}

/* Eq. (28): repulsion on body i from body j; (dx, dy) = X_i - X_j, d = |X_i - X_j|. */
void ora_pp_force(double dx, double dy, double ri, double rj, double xi, double eps_p,
                  double eps_p1, double *F) {
  const double d = sqrt(dx * dx + dy * dy);
  double k = 0.0;
  if (d > ri + rj + xi) {
    k = 0.0;
  } else if (d <= ri + rj) {
    k = (ri + rj - d) / eps_p1;
  } else {
    k = (ri + rj + xi - d) * (ri + rj + xi - d) / eps_p;
  }
  F[0] = k * dx;
  F[1] = k * dy;
}

/* Eq. (29): repulsion on a body from the wall; (dx, dy) = X_i - X_i', where X_i' is the
 * mirror image of the centre across the nearest wall surface, d' = |X_i - X_i'|. */
void ora_pw_force(double dx, double dy, double r, double xi, double eps_w, double eps_w1,
                  double *F) {
  const double d = sqrt(dx * dx + dy * dy);
  double k = 0.0;
  if (d > 2.0 * r + xi) {
    k = 0.0;
  } else if (d <= 2.0 * r) {
    k = (2.0 * r - d) / eps_w1;
  } else {
    k = (2.0 * r + xi - d) * (2.0 * r + xi - d) / eps_w;
  }
  F[0] = k * dx;
  F[1] = k * dy;
}

/* Eqs. (22)-(24) with dt = 1: forward-Euler velocity and spin, trapezoidal position.
 * (Fx, Fy) is the total force and T the torque. */
void ora_body_update(double m, double I, double Fx, double Fy, double T, double *x, double *y,
                     double *ux, double *uy, double *om) {
  const double ux_new = *ux + Fx / m;
  const double uy_new = *uy + Fy / m;
  const double om_new = *om + T / I;
  *x += 0.5 * (*ux + ux_new);
  *y += 0.5 * (*uy + uy_new);
  *ux = ux_new;
  *uy = uy_new;
  *om = om_new;
}

/* ------------------------------------------------------------------------------ */
/* solver                                                                            */

struct ora_solver {
  ora_params p;
  int64_t n;     /* nx*ny */
  double *f;     /* [9][ny][nx] deviations at t_n */
  double *ftmp;
  int32_t nb;
  double *bx, *by, *bu, *bv, *bw, *br, *brho;
  uint8_t *bfix;
  double *bF, *bT; /* hydrodynamic force/torque of the last step */
  double wallF[2];
  /* per-node lists of covering bodies (CSR) */
  int64_t *off;
  int64_t e_cap;
  int32_t *e_b;
  double *e_phi, *e_usx, *e_usy, *e_rx, *e_ry, *e_F;
};

/* periodic minimum image, mapped to [-N/2, N/2) */
static double min_image(double d, double N) {
  while (d >= 0.5 * N) d -= N;
  while (d < -0.5 * N) d += N;
  return d;
}

static double wrap_coord(double x, double N) {
  x = fmod(x, N);
  if (x < 0.0) x += N;
  if (x >= N) x -= N;
  return x;
}

/* Node index range [lo, hi] (before wrapping) whose centres k+0.5 lie within H of X;
 * the whole axis when the window is as wide as the domain. */
static void axis_window(double X, double H, int32_t N, int64_t *lo, int64_t *hi) {
  if (2.0 * H + 1.0 >= (double)N) {
    *lo = 0;
    *hi = N - 1;
  } else {
    *lo = (int64_t)ceil(X - H - 0.5);
    *hi = (int64_t)floor(X + H - 0.5);
  }
}

static int64_t wrap_index(int64_t k, int32_t N) {
  k %= N;
  if (k < 0) k += N;
  return k;
}

/* Visit every (body, node) pair with phi_b > 0 in a fixed order: bodies 0..nb-1, then the
 * y-seam wall slab, then the x-seam wall slab; nodes row-major within each.  mode 0
 * counts entries per node; mode 1 fills the CSR arrays. */
static void visit_pairs(ora_solver *s, int mode, int64_t *fill) {
  const ora_params *p = &s->p;
  const int32_t nx = p->nx, ny = p->ny;
  const double lcut = -p->cutoff * p->eps;
  for (int32_t b = 0; b < s->nb; ++b) {
    const double X = s->bx[b], Y = s->by[b], R = s->br[b];
    const double H = R + p->cutoff * p->eps;
    int64_t xlo, xhi, ylo, yhi;
    axis_window(X, H, nx, &xlo, &xhi);
    axis_window(Y, H, ny, &ylo, &yhi);
    for (int64_t ky = ylo; ky <= yhi; ++ky) {
      const int64_t j = wrap_index(ky, ny);
      const double ry = min_image((double)j + 0.5 - Y, (double)ny);
      for (int64_t kx = xlo; kx <= xhi; ++kx) {
        const int64_t i = wrap_index(kx, nx);
        const double rx = min_image((double)i + 0.5 - X, (double)nx);
        /* Eq. (14) with l = R - |r| (positive inside the disc) */
        const double l = R - sqrt(rx * rx + ry * ry);
        if (l < lcut) continue;
        const int64_t node = j * nx + i;
        if (mode == 0) {
          s->off[node + 1] += 1;
        } else {
          const int64_t e = s->off[node] + fill[node]++;
          s->e_b[e] = b;
          s->e_phi[e] = ora_phi(l, p->eps, p->cutoff);
          /* rigid-body velocity of the solid at the node: U + omega x r */
          s->e_usx[e] = s->bu[b] - s->bw[b] * ry;
          s->e_usy[e] = s->bv[b] + s->bw[b] * rx;
          s->e_rx[e] = rx;
          s->e_ry[e] = ry;
        }
      }
    }
  }
  /* wall slabs: l = h - |distance to the seam|, solid velocity 0 */
  for (int wall = 0; wall < 2; ++wall) {
    if (!(p->wall_mask & (1u << wall))) continue;
    for (int64_t j = 0; j < ny; ++j) {
      for (int64_t i = 0; i < nx; ++i) {
        const double d = wall == 0 ? min_image((double)j + 0.5, (double)ny)
                                   : min_image((double)i + 0.5, (double)nx);
        const double l = p->wall_h - fabs(d);
        if (l < lcut) continue;
        const int64_t node = j * nx + i;
        if (mode == 0) {
          s->off[node + 1] += 1;
        } else {
          const int64_t e = s->off[node] + fill[node]++;
          s->e_b[e] = s->nb + wall;
          s->e_phi[e] = ora_phi(l, p->eps, p->cutoff);
          s->e_usx[e] = 0.0;
          s->e_usy[e] = 0.0;
          s->e_rx[e] = 0.0;
          s->e_ry[e] = 0.0;
        }
      }
    }
  }
}

static int build_lists(ora_solver *s) {
  const int64_t n = s->n;
  memset(s->off, 0, (size_t)(n + 1) * sizeof(int64_t));
  visit_pairs(s, 0, NULL);
  for (int64_t k = 0; k < n; ++k) s->off[k + 1] += s->off[k];
  const int64_t ne = s->off[n];
  if (ne > s->e_cap) {
    int64_t cap = ne + ne / 2 + 16;
    free(s->e_b);
    free(s->e_phi);
    free(s->e_usx);
    free(s->e_usy);
    free(s->e_rx);
    free(s->e_ry);
    free(s->e_F);
    s->e_b = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    s->e_phi = (double *)malloc((size_t)cap * sizeof(double));
    s->e_usx = (double *)malloc((size_t)cap * sizeof(double));
    s->e_usy = (double *)malloc((size_t)cap * sizeof(double));
    s->e_rx = (double *)malloc((size_t)cap * sizeof(double));
    s->e_ry = (double *)malloc((size_t)cap * sizeof(double));
    s->e_F = (double *)malloc((size_t)cap * 2 * sizeof(double));
    if (!s->e_b || !s->e_phi || !s->e_usx || !s->e_usy || !s->e_rx || !s->e_ry || !s->e_F) {
      s->e_cap = 0;
      return ORA_ENOMEM;
    }
    s->e_cap = cap;
  }
  int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  if (!fill) return ORA_ENOMEM;
  visit_pairs(s, 1, fill);
  free(fill);
  return ORA_OK;
}

int32_t ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the node loops from now on (n >= 1); results do not depend on it. */
void ora_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static int valid_params(const ora_params *p) {
  if (!p) return 0;
  if (p->nx < 1 || p->ny < 1) return 0;
  if (!(p->tau > 0.5) || !(p->rho0 > 0.0) || !(p->eps > 0.0) || !(p->cutoff > 0.0)) return 0;
  if (p->wall_mask & ~3u) return 0;
  if (p->wall_mask && !(p->wall_h > 0.0)) return 0;
  if (p->force_mode != 0 && p->force_mode != 1) return 0;
  if (p->x_boundary != 0 && p->x_boundary != 1) return 0;
  if (p->x_boundary) {
    if (p->nx < 3 || (p->wall_mask & 2u)) return 0;
    if ((p->inlet_kind != 0 && p->inlet_kind != 1) || (p->outlet_kind != 0 && p->outlet_kind != 1))
      return 0;
    if (p->inlet_profile != 0 && p->inlet_profile != 1) return 0;
    if (p->inlet_kind == 1 && !(p->rho_in > 0.0)) return 0;
    if (p->outlet_kind == 0 && !(p->rho_out > 0.0)) return 0;
  }
  return 1;
}

int32_t ora_create(const ora_params *p, ora_solver **out) {
  if (!out) return ORA_EINVAL;
  *out = NULL;
  if (!valid_params(p)) return ORA_EINVAL;
  ora_solver *s = (ora_solver *)calloc(1, sizeof(ora_solver));
  if (!s) return ORA_ENOMEM;
  s->p = *p;
  s->n = (int64_t)p->nx * p->ny;
  s->f = (double *)calloc((size_t)(Q * s->n), sizeof(double));
  s->ftmp = (double *)calloc((size_t)(Q * s->n), sizeof(double));
  s->off = (int64_t *)calloc((size_t)(s->n + 1), sizeof(int64_t));
  if (!s->f || !s->ftmp || !s->off) {
    ora_destroy(s);
    return ORA_ENOMEM;
  }
  /* Section 2.3 step 1, initialised at rest: f = f^eq(rho0, 0), i.e. zero deviation. */
  *out = s;
  return ORA_OK;
}

static void free_bodies(ora_solver *s) {
  free(s->bx);
  free(s->by);
  free(s->bu);
  free(s->bv);
  free(s->bw);
  free(s->br);
  free(s->brho);
  free(s->bfix);
  free(s->bF);
  free(s->bT);
  s->bx = s->by = s->bu = s->bv = s->bw = s->br = s->brho = s->bF = s->bT = NULL;
  s->bfix = NULL;
  s->nb = 0;
}

void ora_destroy(ora_solver *s) {
  if (!s) return;
  free(s->f);
  free(s->ftmp);
  free(s->off);
  free(s->e_b);
  free(s->e_phi);
  free(s->e_usx);
  free(s->e_usy);
  free(s->e_rx);
  free(s->e_ry);
  free(s->e_F);
  free_bodies(s);
  free(s);
}

int32_t ora_set_particles(ora_solver *s, int32_t n, const double *pos, const double *vel,
                          const double *omega, const double *radius, const double *density,
                          const uint8_t *fixed) {
  if (!s || n < 0) return ORA_EINVAL;
  if (n > 0 && (!pos || !radius || !density)) return ORA_EINVAL;
  for (int32_t b = 0; b < n; ++b)
    if (!(radius[b] > 0.0) || !(density[b] > 0.0) || !isfinite(pos[2 * b]) ||
        !isfinite(pos[2 * b + 1]))
      return ORA_EINVAL;
  free_bodies(s);
  s->nb = n;
  s->wallF[0] = s->wallF[1] = 0.0;
  size_t nn = (size_t)(n > 0 ? n : 1);
  s->bx = (double *)calloc(nn, sizeof(double));
  s->by = (double *)calloc(nn, sizeof(double));
  s->bu = (double *)calloc(nn, sizeof(double));
  s->bv = (double *)calloc(nn, sizeof(double));
  s->bw = (double *)calloc(nn, sizeof(double));
  s->br = (double *)calloc(nn, sizeof(double));
  s->brho = (double *)calloc(nn, sizeof(double));
  s->bfix = (uint8_t *)calloc(nn, 1);
  s->bF = (double *)calloc(2 * nn, sizeof(double));
  s->bT = (double *)calloc(nn, sizeof(double));
  if (!s->bx || !s->by || !s->bu || !s->bv || !s->bw || !s->br || !s->brho || !s->bfix ||
      !s->bF || !s->bT) {
    free_bodies(s);
    return ORA_ENOMEM;
  }
  for (int32_t b = 0; b < n; ++b) {
    s->bx[b] = wrap_coord(pos[2 * b], s->p.nx);
    s->by[b] = wrap_coord(pos[2 * b + 1], s->p.ny);
    s->bu[b] = vel ? vel[2 * b] : 0.0;
    s->bv[b] = vel ? vel[2 * b + 1] : 0.0;
    s->bw[b] = omega ? omega[b] : 0.0;
    s->br[b] = radius[b];
    s->brho[b] = density[b];
    s->bfix[b] = fixed ? fixed[b] : 0;
  }
  return ORA_OK;
}

int32_t ora_set_populations(ora_solver *s, const double *f_dev) {
  if (!s || !f_dev) return ORA_EINVAL;
  memcpy(s->f, f_dev, (size_t)(Q * s->n) * sizeof(double));
  return ORA_OK;
}

int32_t ora_get_populations(const ora_solver *s, double *f_dev) {
  if (!s || !f_dev) return ORA_EINVAL;
  memcpy(f_dev, s->f, (size_t)(Q * s->n) * sizeof(double));
  return ORA_OK;
}

/* Per-node pass: every node runs ora_collide_node on its own populations and its list of
 * covering bodies.  With `fout` the post-collision populations are streamed (push) into
 * fout; with rho/ux/uy the moments are stored instead. */
static int node_pass(ora_solver *s, double *fout, double *rho_o, double *ux_o, double *uy_o) {
  const ora_params *p = &s->p;
  const int32_t nx = p->nx, ny = p->ny;
  const int64_t n = s->n;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int32_t j = 0; j < ny; ++j) {
    for (int32_t i = 0; i < nx; ++i) {
      const int64_t node = (int64_t)j * nx + i;
      double fd[Q], fp[Q], rho, u[2];
      for (int q = 0; q < Q; ++q) fd[q] = s->f[q * n + node];
      const int64_t e0 = s->off[node];
      const int32_t nb = (int32_t)(s->off[node + 1] - e0);
      double *eF = nb > 0 ? s->e_F + 2 * e0 : NULL;
      int st = ora_collide_node(p->tau, p->rho0, fd, nb, nb ? s->e_phi + e0 : NULL,
                                nb ? s->e_usx + e0 : NULL, nb ? s->e_usy + e0 : NULL, p->G[0],
                                p->G[1], p->force_mode, fp, &rho, u, NULL, eF);
      if (p->x_boundary && (i == 0 || i == nx - 1)) {
        /* inlet / outlet column: its post-collision state comes from the neighbour */
        const int32_t in = (i == 0);
        const int64_t nbn = (int64_t)j * nx + (in ? 1 : nx - 2);
        double fnb[Q];
        for (int q = 0; q < Q; ++q) fnb[q] = s->f[q * n + nbn];
        int32_t rho_nb, u_nb;
        double rset, uxs = 0.0, uys = 0.0;
        if (in) {
          rho_nb = p->inlet_kind == 0;
          u_nb = p->inlet_kind == 1;
          rset = p->rho_in;
          const double sh = ora_inlet_shape(p, j);
          uxs = sh * p->u_in[0];
          uys = sh * p->u_in[1];
        } else {
          rho_nb = p->outlet_kind == 1;
          u_nb = 1;
          rset = p->rho_out;
        }
        ora_nee_node(p->tau, p->rho0, fnb, p->G[0], p->G[1], rho_nb, rset, u_nb, uxs, uys, fp,
                     &rho, u);
        for (int64_t e = 0; e < 2 * (int64_t)nb; ++e) eF[e] = 0.0;  /* no body force here */
        st = (rho > 0.0 && u[0] * u[0] + u[1] * u[1] <= 0.25) ? ORA_OK : ORA_EUNSTABLE;
        for (int q = 0; q < Q; ++q)
          if (!isfinite(fp[q])) st = ORA_EUNSTABLE;
      }
      if (st != ORA_OK) bad = 1;
      if (rho_o) rho_o[node] = rho;
      if (ux_o) ux_o[node] = u[0];
      if (uy_o) uy_o[node] = u[1];
      if (fout) {
        for (int q = 0; q < Q; ++q) {
          int64_t jj = j + CY[q];
          const int64_t ii = wrap_index(i + CX[q], nx);
          if (p->bb_walls_y && (jj < 0 || jj >= ny)) {
            /* halfway bounce-back: the population returns to its node reversed */
            static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
            fout[OPP[q] * n + node] = fp[q];
            continue;
          }
          jj = wrap_index(jj, ny);
          fout[q * n + jj * nx + ii] = fp[q];
        }
      }
    }
  }
  return bad ? ORA_EUNSTABLE : ORA_OK;
}

/* Eqs. (18)-(19): sum the per-node contributions, in row-major node order, into each
 * body (force and torque about its centre) and into the wall force. */
static void reduce_forces(ora_solver *s) {
  for (int32_t b = 0; b < s->nb; ++b) {
    s->bF[2 * b] = 0.0;
    s->bF[2 * b + 1] = 0.0;
    s->bT[b] = 0.0;
  }
  s->wallF[0] = s->wallF[1] = 0.0;
  const int64_t n = s->n;
  for (int64_t node = 0; node < n; ++node) {
    for (int64_t e = s->off[node]; e < s->off[node + 1]; ++e) {
      const int32_t b = s->e_b[e];
      const double fx = s->e_F[2 * e], fy = s->e_F[2 * e + 1];
      if (b < s->nb) {
        s->bF[2 * b] += fx;
        s->bF[2 * b + 1] += fy;
        s->bT[b] += s->e_rx[e] * fy - s->e_ry[e] * fx;
      } else {
        s->wallF[0] += fx;
        s->wallF[1] += fy;
      }
    }
  }
}

/* Section 2.3 step 5: move the bodies with Eqs. (22)-(24), adding the repulsion of
 * Eqs. (28)-(29).  Every force uses the positions at t_n. */
static void move_bodies(ora_solver *s) {
  const ora_params *p = &s->p;
  const int32_t nb = s->nb;
  if (nb == 0) return;
  double *Ft = (double *)malloc((size_t)nb * 2 * sizeof(double));
  if (!Ft) return;
  for (int32_t b = 0; b < nb; ++b) {
    const double R = s->br[b];
    const double m = s->brho[b] * M_PI * R * R;
    /* Eq. (22): F_f + (rho_f/rho_s - 1) m_s g, with rho_f = rho0 */
    double fx = s->bF[2 * b] + (p->rho0 / s->brho[b] - 1.0) * m * p->g[0];
    double fy = s->bF[2 * b + 1] + (p->rho0 / s->brho[b] - 1.0) * m * p->g[1];
    for (int32_t c = 0; c < nb; ++c) {
      if (c == b) continue;
      double Fc[2];
      ora_pp_force(min_image(s->bx[b] - s->bx[c], p->nx), min_image(s->by[b] - s->by[c], p->ny),
                   R, s->br[c], p->xi, p->eps_p, p->eps_p1, Fc);
      fx += Fc[0];
      fy += Fc[1];
    }
    /* walls: image across the nearer surface of each slab (surfaces at h and N - h) */
    if (p->wall_mask & 1u) {
      const double Y = s->by[b], h = p->wall_h, N = p->ny;
      const double dy = (Y - h <= (N - h) - Y) ? 2.0 * (Y - h) : -2.0 * ((N - h) - Y);
      double Fw[2];
      ora_pw_force(0.0, dy, R, p->xi, p->eps_w, p->eps_w1, Fw);
      fx += Fw[0];
      fy += Fw[1];
    }
    if (p->wall_mask & 2u) {
      const double X = s->bx[b], h = p->wall_h, N = p->nx;
      const double dx = (X - h <= (N - h) - X) ? 2.0 * (X - h) : -2.0 * ((N - h) - X);
      double Fw[2];
      ora_pw_force(dx, 0.0, R, p->xi, p->eps_w, p->eps_w1, Fw);
      fx += Fw[0];
      fy += Fw[1];
    }
    Ft[2 * b] = fx;
    Ft[2 * b + 1] = fy;
  }
  for (int32_t b = 0; b < nb; ++b) {
    if (s->bfix[b]) {
      /* prescribed motion: velocity and spin stay as given, Eq. (24) moves the centre */
      s->bx[b] += s->bu[b];
      s->by[b] += s->bv[b];
    } else {
      const double R = s->br[b];
      const double m = s->brho[b] * M_PI * R * R; /* disc of unit depth */
      const double I = 0.5 * m * R * R;
      ora_body_update(m, I, Ft[2 * b], Ft[2 * b + 1], s->bT[b], &s->bx[b], &s->by[b], &s->bu[b],
                      &s->bv[b], &s->bw[b]);
    }
    s->bx[b] = wrap_coord(s->bx[b], p->nx);
    s->by[b] = wrap_coord(s->by[b], p->ny);
  }
  free(Ft);
}

int32_t ora_step(ora_solver *s, int64_t nsteps) {
  if (!s || nsteps < 0) return ORA_EINVAL;
  for (int64_t t = 0; t < nsteps; ++t) {
    int st = build_lists(s); /* step 5 of the previous step: phi from the body positions */
    if (st != ORA_OK) return st;
    st = node_pass(s, s->ftmp, NULL, NULL, NULL); /* steps 2-3: Eqs. (13), (17) + stream */
    reduce_forces(s);                             /* step 4: Eqs. (18)-(19) */
    double *tmp = s->f;
    s->f = s->ftmp;
    s->ftmp = tmp;
    move_bodies(s); /* step 5: Eqs. (22)-(24) */
    if (st != ORA_OK) return st;
  }
  return ORA_OK;
}

int32_t ora_get_fields(ora_solver *s, double *rho, double *ux, double *uy) {
  if (!s) return ORA_EINVAL;
  int st = build_lists(s);
  if (st != ORA_OK) return st;
  const int64_t n = s->n;
  double *r = rho ? rho : (double *)malloc((size_t)n * sizeof(double));
  double *a = ux ? ux : (double *)malloc((size_t)n * sizeof(double));
  double *c = uy ? uy : (double *)malloc((size_t)n * sizeof(double));
  node_pass(s, NULL, r, a, c);
  if (!rho) free(r);
  if (!ux) free(a);
  if (!uy) free(c);
  return ORA_OK;
}

int32_t ora_get_particle_forces(const ora_solver *s, double *force, double *torque) {
  if (!s) return ORA_EINVAL;
  for (int32_t b = 0; b < s->nb; ++b) {
    if (force) {
      force[2 * b] = s->bF[2 * b];
      force[2 * b + 1] = s->bF[2 * b + 1];
    }
    if (torque) torque[b] = s->bT[b];
  }
  return ORA_OK;
}

int32_t ora_get_particles(const ora_solver *s, double *pos, double *vel, double *omega) {
  if (!s) return ORA_EINVAL;
  for (int32_t b = 0; b < s->nb; ++b) {
    if (pos) {
      pos[2 * b] = s->bx[b];
      pos[2 * b + 1] = s->by[b];
    }
    if (vel) {
      vel[2 * b] = s->bu[b];
      vel[2 * b + 1] = s->bv[b];
    }
    if (omega) omega[b] = s->bw[b];
  }
  return ORA_OK;
}

int32_t ora_get_wall_force(const ora_solver *s, double *force) {
  if (!s || !force) return ORA_EINVAL;
  force[0] = s->wallF[0];
  force[1] = s->wallF[1];
  return ORA_OK;
}
