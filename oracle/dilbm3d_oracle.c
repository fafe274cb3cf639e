/*
 * dilbm3d_oracle.c -- plain FP64 CPU reference of the three-dimensional DI-LBM time step
 * (D3Q19 or D3Q27, spheres).
 *
 * TEST INFRASTRUCTURE ONLY: the oracle that the GPU library's 3-D path is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code with the GPU library.  Written to be read against the paper: every
 * node is handled by one call of ora3_collide_node(), which takes the Section 2.3 steps
 * in the paper's order.
 *
 * Paper: Liu, Huang, Chai & Shi, "A diffuse-interface lattice Boltzmann method for
 * fluid-particle interaction problems".  The paper states the method in two dimensions
 * and motivates it by the cost of solid fractions in three; this file carries each
 * equation over unchanged in form:
 *   Eq. (2)  equilibrium (c_s^2 = 1/3, as for the D2Q9 lattice);  Eq. (5) moments;
 *   Eq. (13) evolution;  Eq. (14) phi with l = R - |x - X| (sphere);  Eq. (15) force
 *   term;  Eqs. (16)-(17) velocities;  Eqs. (18)-(19) force and torque (r x F, a
 *   vector);  Eqs. (22)-(24) particle motion (sphere: m = 4/3 pi R^3 rho_s,
 *   I = 2/5 m R^2, isotropic, so the spin update has no gyroscopic term);
 *   Eqs. (28)-(29) repulsion (the same scalar laws along the 3-D centre line); optional
 *   open ends in x by non-equilibrium extrapolation (Guo, Zheng & Shi 2002), the
 *   treatment the paper gives its physical boundaries (Section 3).
 * The readings of the two-dimensional oracle carry over: minimum images, the phi cutoff
 * at l = -cutoff*eps, w_b = phi_b min(1, 1/sum phi), solid velocity U + omega x r,
 * Guo-Zheng-Shi forcing for the uniform body force with u* carrying half of it, static
 * diffuse wall slabs across the periodic seams, forward-Euler velocities and
 * trapezoidal positions with dt = 1.
 *
 * Compiled with -O2 -ffp-contract=off; results do not depend on the thread count.
 */
#include "dilbm3d_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The two velocity sets, standard three-dimensional counterparts of Eqs. (3)-(4):
 * D3Q19 is the rest direction, the six axis directions and the twelve edge directions;
 * D3Q27 adds the eight corner directions.  Opposite directions are neighbours (i, i + 1)
 * for odd i, and D3Q27's first 19 directions are those of D3Q19. */
#define QMAX 27
static const int32_t CX[QMAX] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                 1, -1, 1, -1, 1, -1, -1, 1};
static const int32_t CY[QMAX] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                 1, -1, 1, -1, -1, 1, 1, -1};
static const int32_t CZ[QMAX] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                 1, -1, -1, 1, 1, -1, 1, -1};
static const double CS2 = 1.0 / 3.0;

enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_EUNSTABLE = -4 };

static int valid_q(int32_t q) { return q == 19 || q == 27; }

/* weights by |c|^2 = 0, 1, 2, 3: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216 */
static double weight(int32_t q, int i) {
  const int n = abs(CX[i]) + abs(CY[i]) + abs(CZ[i]);
  if (q == 27) return n == 0 ? 8.0 / 27.0 : (n == 1 ? 2.0 / 27.0 : (n == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
  return n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

void ora3q_lattice(int32_t q, int32_t *cx, int32_t *cy, int32_t *cz, double *w, double *cs2) {
  for (int i = 0; i < q; ++i) {
    if (cx) cx[i] = CX[i];
    if (cy) cy[i] = CY[i];
    if (cz) cz[i] = CZ[i];
    if (w) w[i] = weight(q, i);
  }
  if (cs2) *cs2 = CS2;
}

/* Eq. (2): f_i^eq = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)] */
void ora3q_feq(int32_t q, double rho, const double *u, double *feq) {
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < q; ++i) {
    const double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    feq[i] = weight(q, i) * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Eq. (15): F_i = (1 - 1/(2 tau)) [f_i^eq(rho, u_s) - f_i^eq(rho, u*)] */
void ora3q_force_term(int32_t q, double tau, double rho, const double *us, const double *ustar,
                      double *F) {
  double a[QMAX], b[QMAX];
  ora3q_feq(q, rho, us, a);
  ora3q_feq(q, rho, ustar, b);
  for (int i = 0; i < q; ++i) F[i] = (1.0 - 1.0 / (2.0 * tau)) * (a[i] - b[i]);
}

/* Guo-Zheng-Shi forcing of a uniform body force density G */
void ora3q_guo_term(int32_t q, double tau, const double *u, const double *G, double *Gi) {
  for (int i = 0; i < q; ++i) {
    const double c[3] = {CX[i], CY[i], CZ[i]};
    const double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += ((c[a] - u[a]) / CS2 + cu * c[a] / (CS2 * CS2)) * G[a];
    Gi[i] = (1.0 - 1.0 / (2.0 * tau)) * weight(q, i) * s;
  }
}

/* the D3Q19 forms of the pointwise operators */
void ora3_lattice(int32_t *cx, int32_t *cy, int32_t *cz, double *w, double *cs2) {
  ora3q_lattice(19, cx, cy, cz, w, cs2);
}
void ora3_feq(double rho, const double *u, double *feq) { ora3q_feq(19, rho, u, feq); }
void ora3_force_term(double tau, double rho, const double *us, const double *ustar, double *F) {
  ora3q_force_term(19, tau, rho, us, ustar, F);
}
void ora3_guo_term(double tau, const double *u, const double *G, double *Gi) {
  ora3q_guo_term(19, tau, u, G, Gi);
}

int32_t ora3q_collide_node(int32_t q, double tau, double rho0, const double *f_dev, int32_t nb,
                           const double *phi_b, const double *us, const double *G,
                           int32_t force_mode, double *fpost_dev, double *rho_out,
                           double *u_out, double *ustar_out, double *force_b) {
  if (!valid_q(q)) return ORA_EINVAL;
  const int Q = q;
  double f[QMAX];
  for (int i = 0; i < Q; ++i) f[i] = f_dev[i] + weight(q, i) * rho0;

  /* Eq. (5) and Eq. (16); u* carries half of the fluid body force */
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    j[0] += CX[i] * f[i];
    j[1] += CY[i] * f[i];
    j[2] += CZ[i] * f[i];
  }
  double ust[3];
  for (int a = 0; a < 3; ++a) ust[a] = (j[a] + 0.5 * G[a]) / rho;

  /* several bodies: w_b = phi_b * min(1, 1/sum phi) */
  double S = 0.0;
  for (int b = 0; b < nb; ++b) S += phi_b[b];
  const double scale = S > 1.0 ? 1.0 / S : 1.0;

  /* Eq. (17): u = u* + phi (u_s - u*) / 2, summed over bodies */
  double u[3] = {ust[0], ust[1], ust[2]};
  for (int b = 0; b < nb; ++b) {
    const double wb = scale * phi_b[b];
    for (int a = 0; a < 3; ++a) u[a] += 0.5 * wb * (us[3 * b + a] - ust[a]);
  }

  /* Eq. (13): f* = f - (f - f^eq(rho, u))/tau + phi F_i + G_i */
  double feq[QMAX], Gi[QMAX], Fb[QMAX], acc[QMAX];
  ora3q_feq(q, rho, u, feq);
  ora3q_guo_term(q, tau, u, G, Gi);
  for (int i = 0; i < Q; ++i) acc[i] = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double wb = scale * phi_b[b];
    ora3q_force_term(q, tau, rho, us + 3 * b, ust, Fb);
    for (int i = 0; i < Q; ++i) acc[i] += wb * Fb[i];
    if (force_b) {
      double fb[3];
      if (force_mode == 1) {
        /* Eq. (18) literally: -phi sum_i F_i c_i */
        fb[0] = fb[1] = fb[2] = 0.0;
        for (int i = 0; i < Q; ++i) {
          fb[0] += Fb[i] * CX[i];
          fb[1] += Fb[i] * CY[i];
          fb[2] += Fb[i] * CZ[i];
        }
        for (int a = 0; a < 3; ++a) fb[a] = -wb * fb[a];
      } else {
        /* the momentum the node gains from the body, with the sign of Eq. (18) */
        for (int a = 0; a < 3; ++a) fb[a] = -wb * rho * (us[3 * b + a] - ust[a]);
      }
      for (int a = 0; a < 3; ++a) force_b[3 * b + a] = fb[a];
    }
  }
  int bad = !(rho > 0.0) || !(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= 0.25);
  for (int i = 0; i < Q; ++i) {
    const double fp = f[i] - (f[i] - feq[i]) / tau + acc[i] + Gi[i];
    fpost_dev[i] = fp - weight(q, i) * rho0;
    if (!isfinite(fpost_dev[i])) bad = 1;
  }
  if (rho_out) *rho_out = rho;
  for (int a = 0; a < 3; ++a) {
    if (u_out) u_out[a] = u[a];
    if (ustar_out) ustar_out[a] = ust[a];
  }
  return bad ? ORA_EUNSTABLE : ORA_OK;
}

int32_t ora3_collide_node(double tau, double rho0, const double *f_dev, int32_t nb,
                          const double *phi_b, const double *us, const double *G,
                          int32_t force_mode, double *fpost_dev, double *rho_out,
                          double *u_out, double *ustar_out, double *force_b) {
  return ora3q_collide_node(19, tau, rho0, f_dev, nb, phi_b, us, G, force_mode, fpost_dev,
                            rho_out, u_out, ustar_out, force_b);
}

/* Eq. (28) along the centre line d = X_i - X_j (not normalised, as written) */
void ora3_pp_force(const double *d, double ri, double rj, double xi, double eps_p,
                   double eps_p1, double *F) {
  const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double k = 0.0;
  if (dist > ri + rj + xi) {
    k = 0.0;
  } else if (dist <= ri + rj) {
    k = (ri + rj - dist) / eps_p1;
  } else {
    k = (ri + rj + xi - dist) * (ri + rj + xi - dist) / eps_p;
  }
  for (int a = 0; a < 3; ++a) F[a] = k * d[a];
}

/* Eq. (29): d = X_i - X_i', X_i' the mirror image across the nearest wall surface */
void ora3_pw_force(const double *d, double r, double xi, double eps_w, double eps_w1,
                   double *F) {
  const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double k = 0.0;
  if (dist > 2.0 * r + xi) {
    k = 0.0;
  } else if (dist <= 2.0 * r) {
    k = (2.0 * r - dist) / eps_w1;
  } else {
    k = (2.0 * r + xi - dist) * (2.0 * r + xi - dist) / eps_w;
  }
  for (int a = 0; a < 3; ++a) F[a] = k * d[a];
}

/* Eqs. (22)-(24), dt = 1: forward-Euler velocity and spin, trapezoidal position */
void ora3_body_update(double m, double I, const double *F, const double *T, double *x,
                      double *u, double *om) {
  for (int a = 0; a < 3; ++a) {
    const double un = u[a] + F[a] / m;
    x[a] += 0.5 * (u[a] + un);
    u[a] = un;
    om[a] += T[a] / I;
  }
}

/* ------------------------------------------------------------------------------ */
/* solver                                                                            */

struct ora3_solver {
  ora3_params p;
  int32_t q;      /* 19 or 27 directions */
  int64_t n;      /* nx*ny*nz */
  double *f;      /* [q][nz][ny][nx] deviations at t_n */
  double *ftmp;
  int32_t nb;
  double *bx, *bu, *bw; /* [nb][3]: centre, velocity, spin */
  double *br, *brho;
  uint8_t *bfix;
  double *bF, *bT;      /* [nb][3] hydrodynamic force and torque of the last step */
  double wallF[3];
  /* per-node lists of covering bodies (CSR) */
  int64_t *off;
  int64_t e_cap;
  int32_t *e_b;
  double *e_phi, *e_us, *e_r, *e_F; /* phi; [3] solid velocity, arm, force */
};

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

static double phi_of(double l, const ora3_params *p) {
  if (l < -p->cutoff * p->eps) return 0.0;
  return 0.5 * (1.0 + tanh(2.0 * l / p->eps));
}

static void add_entry(ora3_solver *s, int mode, int64_t *fill, int64_t node, int32_t b,
                      double l, const double *us, const double *r) {
  if (mode == 0) {
    s->off[node + 1] += 1;
    return;
  }
  const int64_t e = s->off[node] + fill[node]++;
  s->e_b[e] = b;
  s->e_phi[e] = phi_of(l, &s->p);
  for (int a = 0; a < 3; ++a) {
    s->e_us[3 * e + a] = us[a];
    s->e_r[3 * e + a] = r[a];
  }
}

/* Every (body, node) pair with phi_b > 0, in a fixed order: bodies 0..nb-1, then the wall
 * slabs (y, x, z); nodes in memory order within each.  mode 0 counts, mode 1 fills. */
static void visit_pairs(ora3_solver *s, int mode, int64_t *fill) {
  const ora3_params *p = &s->p;
  const int32_t nx = p->nx, ny = p->ny, nz = p->nz;
  const double lcut = -p->cutoff * p->eps;
  for (int32_t b = 0; b < s->nb; ++b) {
    const double *X = s->bx + 3 * b, *U = s->bu + 3 * b, *W = s->bw + 3 * b;
    const double R = s->br[b];
    const double H = R + p->cutoff * p->eps;
    int64_t lo[3], hi[3];
    axis_window(X[0], H, nx, &lo[0], &hi[0]);
    axis_window(X[1], H, ny, &lo[1], &hi[1]);
    axis_window(X[2], H, nz, &lo[2], &hi[2]);
    for (int64_t kz = lo[2]; kz <= hi[2]; ++kz) {
      const int64_t k = wrap_index(kz, nz);
      for (int64_t ky = lo[1]; ky <= hi[1]; ++ky) {
        const int64_t j = wrap_index(ky, ny);
        for (int64_t kx = lo[0]; kx <= hi[0]; ++kx) {
          const int64_t i = wrap_index(kx, nx);
          const double r[3] = {min_image((double)i + 0.5 - X[0], nx),
                               min_image((double)j + 0.5 - X[1], ny),
                               min_image((double)k + 0.5 - X[2], nz)};
          /* Eq. (14) with l = R - |r| (positive inside the sphere) */
          const double l = R - sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
          if (l < lcut) continue;
          /* rigid-body velocity of the solid at the node: U + omega x r */
          const double us[3] = {U[0] + W[1] * r[2] - W[2] * r[1],
                                U[1] + W[2] * r[0] - W[0] * r[2],
                                U[2] + W[0] * r[1] - W[1] * r[0]};
          add_entry(s, mode, fill, (k * ny + j) * nx + i, b, l, us, r);
        }
      }
    }
  }
  /* wall slabs: l = h - |distance to the seam|, solid velocity 0 */
  static const double zero[3] = {0.0, 0.0, 0.0};
  for (int wall = 0; wall < 3; ++wall) {
    if (!(p->wall_mask & (1u << wall))) continue;
    for (int64_t k = 0; k < nz; ++k)
      for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
          const double d = wall == 0   ? min_image((double)j + 0.5, ny)
                           : wall == 1 ? min_image((double)i + 0.5, nx)
                                       : min_image((double)k + 0.5, nz);
          const double l = p->wall_h - fabs(d);
          if (l < lcut) continue;
          add_entry(s, mode, fill, (k * ny + j) * nx + i, s->nb + wall, l, zero, zero);
        }
  }
}

static int build_lists(ora3_solver *s) {
  const int64_t n = s->n;
  memset(s->off, 0, (size_t)(n + 1) * sizeof(int64_t));
  visit_pairs(s, 0, NULL);
  for (int64_t k = 0; k < n; ++k) s->off[k + 1] += s->off[k];
  const int64_t ne = s->off[n];
  if (ne > s->e_cap) {
    const int64_t cap = ne + ne / 2 + 16;
    free(s->e_b);
    free(s->e_phi);
    free(s->e_us);
    free(s->e_r);
    free(s->e_F);
    s->e_b = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    s->e_phi = (double *)malloc((size_t)cap * sizeof(double));
    s->e_us = (double *)malloc((size_t)cap * 3 * sizeof(double));
    s->e_r = (double *)malloc((size_t)cap * 3 * sizeof(double));
    s->e_F = (double *)malloc((size_t)cap * 3 * sizeof(double));
    if (!s->e_b || !s->e_phi || !s->e_us || !s->e_r || !s->e_F) {
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

static int valid_params(const ora3_params *p) {
  if (!p) return 0;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
  if (!(p->tau > 0.5) || !(p->rho0 > 0.0) || !(p->eps > 0.0) || !(p->cutoff > 0.0)) return 0;
  if (p->wall_mask & ~7u) return 0;
  if (p->wall_mask && !(p->wall_h > 0.0)) return 0;
  if (p->force_mode != 0 && p->force_mode != 1) return 0;
  if (p->lattice != 0 && !valid_q(p->lattice)) return 0;
  if (p->x_boundary != 0 && p->x_boundary != 1) return 0;
  if (p->x_boundary) {
    if (p->nx < 3 || (p->wall_mask & 2u)) return 0;
    if ((p->inlet_kind != 0 && p->inlet_kind != 1) || (p->outlet_kind != 0 && p->outlet_kind != 1))
      return 0;
    if (p->inlet_profile < 0 || p->inlet_profile > 2) return 0;
    if (p->inlet_kind == 1 && !(p->rho_in > 0.0)) return 0;
    if (p->outlet_kind == 0 && !(p->rho_out > 0.0)) return 0;
  }
  return 1;
}

/* Non-equilibrium extrapolation (Guo, Zheng & Shi 2002), the treatment the paper gives its
 * physical boundaries (Section 3): the boundary node takes the equilibrium of its boundary
 * state plus its neighbour's non-equilibrium part relaxed as in Eq. (13); the neighbour's
 * velocity carries half the body force, as in its own collision (Eq. (16)). */
void ora3q_nee_node(int32_t q, double tau, double rho0, const double *f_nb_dev,
                    const double *G, int32_t rho_from_nb, double rho_set, int32_t u_from_nb,
                    const double *u_set, double *fpost_dev, double *rho_b, double *u_b) {
  const int Q = q;
  double f[QMAX];
  for (int i = 0; i < Q; ++i) f[i] = f_nb_dev[i] + weight(q, i) * rho0;
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    j[0] += CX[i] * f[i];
    j[1] += CY[i] * f[i];
    j[2] += CZ[i] * f[i];
  }
  double u_nb[3], ub[3];
  for (int a = 0; a < 3; ++a) u_nb[a] = (j[a] + 0.5 * G[a]) / rho;
  const double rb = rho_from_nb ? rho : rho_set;
  for (int a = 0; a < 3; ++a) ub[a] = u_from_nb ? u_nb[a] : u_set[a];
  double feq_nb[QMAX], feq_b[QMAX];
  ora3q_feq(q, rho, u_nb, feq_nb);
  ora3q_feq(q, rb, ub, feq_b);
  for (int i = 0; i < Q; ++i)
    fpost_dev[i] = feq_b[i] + (1.0 - 1.0 / tau) * (f[i] - feq_nb[i]) - weight(q, i) * rho0;
  if (rho_b) *rho_b = rb;
  if (u_b)
    for (int a = 0; a < 3; ++a) u_b[a] = ub[a];
}

/* parabola 4 s (1 - s) over [a, b) at cell centre c + 1/2, zero outside */
static double parabola(int32_t c, double a, double b) {
  const double sv = ((double)c + 0.5 - a) / (b - a);
  return (sv > 0.0 && sv < 1.0) ? 4.0 * sv * (1.0 - sv) : 0.0;
}

double ora3_inlet_shape(const ora3_params *p, int32_t j, int32_t k) {
  if (!p->inlet_profile) return 1.0;
  const int wy = (p->wall_mask & 1u) != 0, wz = (p->wall_mask & 4u) != 0;
  double sh = parabola(j, wy ? p->wall_h : 0.0, wy ? p->ny - p->wall_h : (double)p->ny);
  if (p->inlet_profile == 2)
    sh *= parabola(k, wz ? p->wall_h : 0.0, wz ? p->nz - p->wall_h : (double)p->nz);
  return sh;
}

int32_t ora3_create(const ora3_params *p, ora3_solver **out) {
  if (!out) return ORA_EINVAL;
  *out = NULL;
  if (!valid_params(p)) return ORA_EINVAL;
  ora3_solver *s = (ora3_solver *)calloc(1, sizeof(ora3_solver));
  if (!s) return ORA_ENOMEM;
  s->p = *p;
  s->q = p->lattice ? p->lattice : 19;
  s->n = (int64_t)p->nx * p->ny * p->nz;
  s->f = (double *)calloc((size_t)(s->q * s->n), sizeof(double));
  s->ftmp = (double *)calloc((size_t)(s->q * s->n), sizeof(double));
  s->off = (int64_t *)calloc((size_t)(s->n + 1), sizeof(int64_t));
  if (!s->f || !s->ftmp || !s->off) {
    ora3_destroy(s);
    return ORA_ENOMEM;
  }
  /* initialised at rest: f = f^eq(rho0, 0), i.e. zero deviation */
  *out = s;
  return ORA_OK;
}

static void free_bodies(ora3_solver *s) {
  free(s->bx);
  free(s->bu);
  free(s->bw);
  free(s->br);
  free(s->brho);
  free(s->bfix);
  free(s->bF);
  free(s->bT);
  s->bx = s->bu = s->bw = s->br = s->brho = s->bF = s->bT = NULL;
  s->bfix = NULL;
  s->nb = 0;
}

void ora3_destroy(ora3_solver *s) {
  if (!s) return;
  free(s->f);
  free(s->ftmp);
  free(s->off);
  free(s->e_b);
  free(s->e_phi);
  free(s->e_us);
  free(s->e_r);
  free(s->e_F);
  free_bodies(s);
  free(s);
}

int32_t ora3_set_particles(ora3_solver *s, int32_t n, const double *pos, const double *vel,
                           const double *omega, const double *radius, const double *density,
                           const uint8_t *fixed) {
  if (!s || n < 0) return ORA_EINVAL;
  if (n > 0 && (!pos || !radius || !density)) return ORA_EINVAL;
  for (int32_t b = 0; b < n; ++b)
    if (!(radius[b] > 0.0) || !(density[b] > 0.0) || !isfinite(pos[3 * b]) ||
        !isfinite(pos[3 * b + 1]) || !isfinite(pos[3 * b + 2]))
      return ORA_EINVAL;
  free_bodies(s);
  s->nb = n;
  s->wallF[0] = s->wallF[1] = s->wallF[2] = 0.0;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  s->bx = (double *)calloc(3 * nn, sizeof(double));
  s->bu = (double *)calloc(3 * nn, sizeof(double));
  s->bw = (double *)calloc(3 * nn, sizeof(double));
  s->br = (double *)calloc(nn, sizeof(double));
  s->brho = (double *)calloc(nn, sizeof(double));
  s->bfix = (uint8_t *)calloc(nn, 1);
  s->bF = (double *)calloc(3 * nn, sizeof(double));
  s->bT = (double *)calloc(3 * nn, sizeof(double));
  if (!s->bx || !s->bu || !s->bw || !s->br || !s->brho || !s->bfix || !s->bF || !s->bT) {
    free_bodies(s);
    return ORA_ENOMEM;
  }
  const double N[3] = {s->p.nx, s->p.ny, s->p.nz};
  for (int32_t b = 0; b < n; ++b) {
    for (int a = 0; a < 3; ++a) {
      s->bx[3 * b + a] = wrap_coord(pos[3 * b + a], N[a]);
      s->bu[3 * b + a] = vel ? vel[3 * b + a] : 0.0;
      s->bw[3 * b + a] = omega ? omega[3 * b + a] : 0.0;
    }
    s->br[b] = radius[b];
    s->brho[b] = density[b];
    s->bfix[b] = fixed ? fixed[b] : 0;
  }
  return ORA_OK;
}

int32_t ora3_set_populations(ora3_solver *s, const double *f_dev) {
  if (!s || !f_dev) return ORA_EINVAL;
  memcpy(s->f, f_dev, (size_t)(s->q * s->n) * sizeof(double));
  return ORA_OK;
}

int32_t ora3_get_populations(const ora3_solver *s, double *f_dev) {
  if (!s || !f_dev) return ORA_EINVAL;
  memcpy(f_dev, s->f, (size_t)(s->q * s->n) * sizeof(double));
  return ORA_OK;
}

/* Per-node pass: ora3_collide_node on every node; with `fout` the post-collision
 * populations are streamed (push, periodic) into fout, otherwise the moments are stored. */
static int node_pass(ora3_solver *s, double *fout, double *rho_o, double *ux_o, double *uy_o,
                     double *uz_o) {
  const ora3_params *p = &s->p;
  const int32_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t n = s->n;
  int bad = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : bad)
  for (int32_t k = 0; k < nz; ++k) {
    for (int32_t j = 0; j < ny; ++j) {
      for (int32_t i = 0; i < nx; ++i) {
        const int64_t node = ((int64_t)k * ny + j) * nx + i;
        const int Q = s->q;
        double fd[QMAX], fp[QMAX], rho, u[3];
        for (int q = 0; q < Q; ++q) fd[q] = s->f[q * n + node];
        const int64_t e0 = s->off[node];
        const int32_t nb = (int32_t)(s->off[node + 1] - e0);
        int st =
            ora3q_collide_node(Q, p->tau, p->rho0, fd, nb, nb ? s->e_phi + e0 : NULL,
                               nb ? s->e_us + 3 * e0 : NULL, p->G, p->force_mode, fp, &rho, u,
                               NULL, nb ? s->e_F + 3 * e0 : NULL);
        if (p->x_boundary && (i == 0 || i == nx - 1)) {
          /* inlet / outlet column: its post-collision state comes from the neighbour */
          const int32_t in = (i == 0);
          const int64_t nbn = ((int64_t)k * ny + j) * nx + (in ? 1 : nx - 2);
          double fnb[QMAX], uset[3] = {0.0, 0.0, 0.0};
          for (int q = 0; q < Q; ++q) fnb[q] = s->f[q * n + nbn];
          int32_t rho_nb, u_nb;
          double rset;
          if (in) {
            rho_nb = p->inlet_kind == 0;
            u_nb = p->inlet_kind == 1;
            rset = p->rho_in;
            const double sh = ora3_inlet_shape(p, j, k);
            for (int a = 0; a < 3; ++a) uset[a] = sh * p->u_in[a];
          } else {
            rho_nb = p->outlet_kind == 1;
            u_nb = 1;
            rset = p->rho_out;
          }
          ora3q_nee_node(Q, p->tau, p->rho0, fnb, p->G, rho_nb, rset, u_nb, uset, fp, &rho, u);
          for (int64_t e = 0; e < 3 * (int64_t)nb; ++e) s->e_F[3 * e0 + e] = 0.0;  /* no force */
          st = (rho > 0.0 && u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= 0.25) ? ORA_OK
                                                                                : ORA_EUNSTABLE;
          for (int q = 0; q < Q; ++q)
            if (!isfinite(fp[q])) st = ORA_EUNSTABLE;
        }
        if (st != ORA_OK) bad = 1;
        if (rho_o) rho_o[node] = rho;
        if (ux_o) ux_o[node] = u[0];
        if (uy_o) uy_o[node] = u[1];
        if (uz_o) uz_o[node] = u[2];
        if (fout) {
          for (int q = 0; q < Q; ++q) {
            const int64_t ii = wrap_index(i + CX[q], nx);
            const int64_t jj = wrap_index(j + CY[q], ny);
            const int64_t kk = wrap_index(k + CZ[q], nz);
            fout[q * n + (kk * ny + jj) * nx + ii] = fp[q];
          }
        }
      }
    }
  }
  return bad ? ORA_EUNSTABLE : ORA_OK;
}

/* Eqs. (18)-(19): node contributions summed in memory order into each body (force and
 * torque r x F about its centre) and into the wall force */
static void reduce_forces(ora3_solver *s) {
  for (int64_t e = 0; e < 3 * (int64_t)s->nb; ++e) {
    s->bF[e] = 0.0;
    s->bT[e] = 0.0;
  }
  s->wallF[0] = s->wallF[1] = s->wallF[2] = 0.0;
  for (int64_t node = 0; node < s->n; ++node) {
    for (int64_t e = s->off[node]; e < s->off[node + 1]; ++e) {
      const int32_t b = s->e_b[e];
      const double *F = s->e_F + 3 * e, *r = s->e_r + 3 * e;
      if (b < s->nb) {
        for (int a = 0; a < 3; ++a) s->bF[3 * b + a] += F[a];
        s->bT[3 * b + 0] += r[1] * F[2] - r[2] * F[1];
        s->bT[3 * b + 1] += r[2] * F[0] - r[0] * F[2];
        s->bT[3 * b + 2] += r[0] * F[1] - r[1] * F[0];
      } else {
        for (int a = 0; a < 3; ++a) s->wallF[a] += F[a];
      }
    }
  }
}

/* sphere of radius R and density rho_s */
static double sphere_mass(double R, double rho_s) { return rho_s * 4.0 / 3.0 * M_PI * R * R * R; }

/* Section 2.3 step 5: Eqs. (22)-(24) with the repulsion of Eqs. (28)-(29); every force
 * uses the positions at t_n */
static void move_bodies(ora3_solver *s) {
  const ora3_params *p = &s->p;
  const int32_t nb = s->nb;
  if (nb == 0) return;
  const double N[3] = {p->nx, p->ny, p->nz};
  double *Ft = (double *)malloc((size_t)nb * 3 * sizeof(double));
  if (!Ft) return;
  for (int32_t b = 0; b < nb; ++b) {
    const double R = s->br[b];
    const double m = sphere_mass(R, s->brho[b]);
    double F[3];
    /* Eq. (22): F_f + (rho_f/rho_s - 1) m_s g, rho_f = rho0 */
    for (int a = 0; a < 3; ++a) F[a] = s->bF[3 * b + a] + (p->rho0 / s->brho[b] - 1.0) * m * p->g[a];
    for (int32_t c = 0; c < nb; ++c) {
      if (c == b) continue;
      double d[3], Fc[3];
      for (int a = 0; a < 3; ++a) d[a] = min_image(s->bx[3 * b + a] - s->bx[3 * c + a], N[a]);
      ora3_pp_force(d, R, s->br[c], p->xi, p->eps_p, p->eps_p1, Fc);
      for (int a = 0; a < 3; ++a) F[a] += Fc[a];
    }
    /* walls: image across the nearer surface of each slab (surfaces at h and N - h) */
    static const int axis_of_wall[3] = {1, 0, 2};
    for (int wall = 0; wall < 3; ++wall) {
      if (!(p->wall_mask & (1u << wall))) continue;
      const int a = axis_of_wall[wall];
      const double c = s->bx[3 * b + a], h = p->wall_h, L = N[a];
      double d[3] = {0.0, 0.0, 0.0}, Fw[3];
      d[a] = (c - h <= (L - h) - c) ? 2.0 * (c - h) : -2.0 * ((L - h) - c);
      ora3_pw_force(d, R, p->xi, p->eps_w, p->eps_w1, Fw);
      for (int e = 0; e < 3; ++e) F[e] += Fw[e];
    }
    for (int a = 0; a < 3; ++a) Ft[3 * b + a] = F[a];
  }
  for (int32_t b = 0; b < nb; ++b) {
    if (s->bfix[b]) {
      /* prescribed motion: velocity and spin stay as given, Eq. (24) moves the centre */
      for (int a = 0; a < 3; ++a) s->bx[3 * b + a] += s->bu[3 * b + a];
    } else {
      const double R = s->br[b];
      const double m = sphere_mass(R, s->brho[b]);
      const double I = 0.4 * m * R * R;
      ora3_body_update(m, I, Ft + 3 * b, s->bT + 3 * b, s->bx + 3 * b, s->bu + 3 * b,
                       s->bw + 3 * b);
    }
    for (int a = 0; a < 3; ++a) s->bx[3 * b + a] = wrap_coord(s->bx[3 * b + a], N[a]);
  }
  free(Ft);
}

int32_t ora3_step(ora3_solver *s, int64_t nsteps) {
  if (!s || nsteps < 0) return ORA_EINVAL;
  for (int64_t t = 0; t < nsteps; ++t) {
    int st = build_lists(s); /* phi from the body positions of t_n */
    if (st != ORA_OK) return st;
    st = node_pass(s, s->ftmp, NULL, NULL, NULL, NULL); /* Eqs. (13), (17), stream */
    reduce_forces(s);                                   /* Eqs. (18)-(19) */
    double *tmp = s->f;
    s->f = s->ftmp;
    s->ftmp = tmp;
    move_bodies(s); /* Eqs. (22)-(24) */
    if (st != ORA_OK) return st;
  }
  return ORA_OK;
}

int32_t ora3_get_fields(ora3_solver *s, double *rho, double *ux, double *uy, double *uz) {
  if (!s) return ORA_EINVAL;
  int st = build_lists(s);
  if (st != ORA_OK) return st;
  const size_t bytes = (size_t)s->n * sizeof(double);
  double *r = rho ? rho : (double *)malloc(bytes);
  double *a = ux ? ux : (double *)malloc(bytes);
  double *b = uy ? uy : (double *)malloc(bytes);
  double *c = uz ? uz : (double *)malloc(bytes);
  if (r && a && b && c) node_pass(s, NULL, r, a, b, c);
  if (!rho) free(r);
  if (!ux) free(a);
  if (!uy) free(b);
  if (!uz) free(c);
  return (r && a && b && c) ? ORA_OK : ORA_ENOMEM;
}

int32_t ora3_get_particle_forces(const ora3_solver *s, double *force, double *torque) {
  if (!s) return ORA_EINVAL;
  for (int64_t e = 0; e < 3 * (int64_t)s->nb; ++e) {
    if (force) force[e] = s->bF[e];
    if (torque) torque[e] = s->bT[e];
  }
  return ORA_OK;
}

int32_t ora3_get_particles(const ora3_solver *s, double *pos, double *vel, double *omega) {
  if (!s) return ORA_EINVAL;
  for (int64_t e = 0; e < 3 * (int64_t)s->nb; ++e) {
    if (pos) pos[e] = s->bx[e];
    if (vel) vel[e] = s->bu[e];
    if (omega) omega[e] = s->bw[e];
  }
  return ORA_OK;
}

int32_t ora3_get_wall_force(const ora3_solver *s, double *force) {
  if (!s || !force) return ORA_EINVAL;
  for (int a = 0; a < 3; ++a) force[a] = s->wallF[a];
  return ORA_OK;
}
