/*
 * bgk_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Laidin & Rey, arXiv 2502.02704.  Every routine is a direct, unblocked,
 * unfused transcription of the definitions it cites, written for a reader who
 * checks it against the paper by eye.  OpenMP only splits independent x cells
 * (the paper's own implementation is OpenMP, Section 4); it never changes the
 * order of any sum.  The HIP library shares nothing with this file.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - BGK rate: tau = 1, so the scheme relaxes at rate 1/eps (Section 3.1).
 *  - The fully discrete kinetic scheme and the Euler update are read with
 *    the factor dt/dx in front of the flux differences (Section 3.1, 3.2).
 *  - Upwind flux F_{i+1/2} = max(v_x,0) f_i + min(v_x,0) f_{i+1}; the printed
 *    a^- = -min(a,0) would give the wrong sign for v_x < 0.
 *  - Rusanov flux H = (h_L + h_R)/2 - S/2 (V_R - V_L) on conserved V; the
 *    printed central term is a difference and its dissipation acts on U.
 *  - Sound speed c = sqrt(gamma * theta), gamma a parameter (1 reproduces the
 *    printed c = sqrt(theta); 5/3 is the monatomic value).
 *  - Velocity points are cell centres of a uniform truncated box.
 *  - Parareal corrections act on conserved moments; error is the max over
 *    slices, x cells and components of absolute differences.
 */
#include "bgk_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0;

void bgk_oracle_set_threads(int n) { g_threads = n; }

int bgk_oracle_get_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

#define NT bgk_oracle_get_threads()

/* ---------------------------------------------------------------- grid -- */
/* Section 3: uniform finite-volume cells X_i (x) and cubes V_j (v). */

static double dx_of(const bgk_oracle_problem* p) {
  return (p->x_hi - p->x_lo) / p->nx;
}
static double dv_of(const bgk_oracle_problem* p, int a) {
  return (p->v_hi[a] - p->v_lo[a]) / p->nv[a];
}
static double vc(const bgk_oracle_problem* p, int a, int j) {
  return p->v_lo[a] + (j + 0.5) * dv_of(p, a);
}
static long nv3_of(const bgk_oracle_problem* p) {
  return (long)p->nv[0] * p->nv[1] * p->nv[2];
}
static double dv3_of(const bgk_oracle_problem* p) {
  return dv_of(p, 0) * dv_of(p, 1) * dv_of(p, 2);
}

static int check_problem(const bgk_oracle_problem* p) {
  if (!p) return ORACLE_E_INVALID;
  if (p->nx < 2) return ORACLE_E_INVALID;
  for (int a = 0; a < 3; ++a) {
    if (p->nv[a] < 1) return ORACLE_E_INVALID;
    if (!(p->v_hi[a] > p->v_lo[a])) return ORACLE_E_INVALID;
  }
  if (!(p->x_hi > p->x_lo)) return ORACLE_E_INVALID;
  if (p->bc != 0 && p->bc != 1) return ORACLE_E_INVALID;
  if (!(p->eps > 0.0)) return ORACLE_E_INVALID; /* also rejects NaN */
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return ORACLE_E_INVALID;
  if (!(p->sound_gamma > 0.0)) return ORACLE_E_INVALID;
  return ORACLE_OK;
}

/* Ghost-cell index map for the x stencil: Neumann copies the boundary cell,
 * periodic wraps around. */
static int ghost(const bgk_oracle_problem* p, int i) {
  if (i >= 0 && i < p->nx) return i;
  if (p->bc == 1) return (i + p->nx) % p->nx;
  return i < 0 ? 0 : p->nx - 1;
}

/* ---------------------------------------------------------- time steps -- */
/* Section 2.2: the fine propagator runs at the stability-limited step and
 * the span is cut into the smallest number of uniform steps not exceeding
 * it.  Without force dt_stab = cfl * dx / max_j |v_x,j|; with an exterior
 * force both explicit fluxes share the step,
 * dt_stab = cfl / (max_j |v_x,j| / dx + E_max / dv_x). */
static double emax_of(const bgk_oracle_problem* p, const double* E) {
  double m = 0.0;
  if (E)
    for (int i = 0; i < p->nx; ++i)
      if (fabs(E[i]) > m) m = fabs(E[i]);
  return m;
}

static int n_steps_impl(const bgk_oracle_problem* p, double emax, double t_span,
                        int32_t* n_steps, double* dt) {
  if (check_problem(p) || !(t_span > 0.0) || !(emax >= 0.0)) return ORACLE_E_INVALID;
  double vmax = 0.0;
  for (int j = 0; j < p->nv[0]; ++j) {
    double a = fabs(vc(p, 0, j));
    if (a > vmax) vmax = a;
  }
  double dt_stab = emax > 0.0 ? p->cfl / (vmax / dx_of(p) + emax / dv_of(p, 0))
                              : p->cfl * dx_of(p) / vmax;
  double r = t_span / dt_stab;
  int32_t n = (int32_t)ceil(r - 1e-9);
  if (n < 1) n = 1;
  if (n_steps) *n_steps = n;
  if (dt) *dt = t_span / n;
  return ORACLE_OK;
}

int bgk_oracle_n_steps(const bgk_oracle_problem* p, double t_span,
                       int32_t* n_steps, double* dt) {
  return n_steps_impl(p, 0.0, t_span, n_steps, dt);
}

int bgk_oracle_n_steps_force(const bgk_oracle_problem* p, const double* E,
                             double t_span, int32_t* n_steps, double* dt) {
  if (!E) return ORACLE_E_INVALID;
  return n_steps_impl(p, emax_of(p, E), t_span, n_steps, dt);
}

/* ------------------------------------------------------------ Maxwellian -- */
/* Equilibria of the collision operator (Section 1):
 * M(v) = rho (2 pi theta)^{-3/2} exp(-|v-u|^2 / (2 theta)). */
static double maxwellian(double rho, const double u[3], double theta,
                         const double v[3]) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) d2 += (v[a] - u[a]) * (v[a] - u[a]);
  return rho / pow(2.0 * M_PI * theta, 1.5) * exp(-d2 / (2.0 * theta));
}

static int physical(double rho, double theta) {
  return rho > 0.0 && theta > 0.0 && isfinite(rho) && isfinite(theta);
}

/* ---------------------------------------------------------------- lift -- */
/* Discrete lifting operator (Section 3.3, Definition 2). */
int bgk_oracle_lift(const bgk_oracle_problem* p, const double* W, double* f) {
  if (check_problem(p) || !W || !f) return ORACLE_E_INVALID;
  const long nv3 = nv3_of(p);
  int bad = 0;
#pragma omp parallel for num_threads(NT) reduction(| : bad)
  for (int i = 0; i < p->nx; ++i) {
    const double* w = W + 5 * (long)i;
    double u[3] = {w[1], w[2], w[3]};
    if (!physical(w[0], w[4]) || !isfinite(u[0]) || !isfinite(u[1]) ||
        !isfinite(u[2])) {
      bad = 1;
      continue;
    }
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx)
      for (int jy = 0; jy < p->nv[1]; ++jy)
        for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
          double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
          f[(long)i * nv3 + j] = maxwellian(w[0], u, w[4], v);
        }
  }
  return bad ? ORACLE_E_NONPHYSICAL : ORACLE_OK;
}

/* Lifting of order one (Definition 3 with L = 1) for the BGK operator with
 * tau = 1: the first Chapman-Enskog correction (the perturbation whose stress
 * and heat flux are the Navier-Stokes ones, mu = rho theta, kappa = 5/2 rho
 * theta),
 *   f = M[rho,u,theta] (1 - eps P),  c = v - u,
 *   P = (u_x'/theta)(c_x^2 - |c|^2/3) + (u_y'/theta) c_x c_y
 *       + (u_z'/theta) c_x c_z + (theta'/theta) c_x (|c|^2/(2 theta) - 5/2),
 * ' the x-derivative by central differences of the primitive moments, with
 * the boundary condition's ghost cells.  Needs a finite eps. */
int bgk_oracle_lift_ce(const bgk_oracle_problem* p, const double* W, double* f) {
  if (check_problem(p) || !W || !f || !isfinite(p->eps)) return ORACLE_E_INVALID;
  const long nv3 = nv3_of(p);
  const double dx = dx_of(p);
  int bad = 0;
  for (int i = 0; i < p->nx; ++i) {
    const double* w = W + 5 * (long)i;
    if (!physical(w[0], w[4]) || !isfinite(w[1]) || !isfinite(w[2]) || !isfinite(w[3]))
      bad = 1;
  }
  if (bad) return ORACLE_E_NONPHYSICAL;
#pragma omp parallel for num_threads(NT)
  for (int i = 0; i < p->nx; ++i) {
    const double* w = W + 5 * (long)i;
    const double* wl = W + 5 * (long)ghost(p, i - 1);
    const double* wr = W + 5 * (long)ghost(p, i + 1);
    double u[3] = {w[1], w[2], w[3]};
    const double th = w[4];
    double d[4];  /* u_x', u_y', u_z', theta' */
    for (int c = 0; c < 4; ++c) d[c] = (wr[1 + c] - wl[1 + c]) / (2.0 * dx);
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx)
      for (int jy = 0; jy < p->nv[1]; ++jy)
        for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
          double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
          double c[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
          double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
          double P = d[0] / th * (c[0] * c[0] - c2 / 3.0) + d[1] / th * c[0] * c[1] +
                     d[2] / th * c[0] * c[2] + d[3] / th * c[0] * (c2 / (2.0 * th) - 2.5);
          f[(long)i * nv3 + j] = maxwellian(w[0], u, th, v) * (1.0 - p->eps * P);
        }
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------- moments -- */
/* Discrete projection operator (Section 3.3, Definition 1), first-order
 * quadrature, literal two-pass form:
 *   rho = sum f dv,  rho u = sum v f dv,  3 rho theta = sum |v-u|^2 f dv.
 * Conserved energy from the Section 1 relation E = (rho|u|^2 + 3 rho theta)/2. */
/* Compensated (Neumaier) running sum: the moments below are sums over up to
 * 10^5 velocities, where a plain running sum loses up to ~1e-13 relative;
 * the compensation keeps each sum within a few ulps of the exact one, in the
 * same left-to-right order. */
typedef struct {
  double s, c;
} csum;

static void csum_add(csum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double csum_value(const csum* a) { return a->s + a->c; }

static int moments_cell(const bgk_oracle_problem* p, const double* fi,
                        double* V5, double* W5) {
  const double dv3 = dv3_of(p);
  csum rho_s = {0.0, 0.0}, mom_s[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  long j = 0;
  for (int jx = 0; jx < p->nv[0]; ++jx)
    for (int jy = 0; jy < p->nv[1]; ++jy)
      for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
        double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
        csum_add(&rho_s, fi[j] * dv3);
        for (int a = 0; a < 3; ++a) csum_add(&mom_s[a], v[a] * fi[j] * dv3);
      }
  double rho = csum_value(&rho_s);
  double u[3] = {csum_value(&mom_s[0]) / rho, csum_value(&mom_s[1]) / rho,
                 csum_value(&mom_s[2]) / rho};
  csum s2_s = {0.0, 0.0};
  j = 0;
  for (int jx = 0; jx < p->nv[0]; ++jx)
    for (int jy = 0; jy < p->nv[1]; ++jy)
      for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
        double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) d2 += (v[a] - u[a]) * (v[a] - u[a]);
        csum_add(&s2_s, d2 * fi[j] * dv3);
      }
  double s2 = csum_value(&s2_s);
  double theta = s2 / (3.0 * rho);
  if (W5) {
    W5[0] = rho;
    W5[1] = u[0];
    W5[2] = u[1];
    W5[3] = u[2];
    W5[4] = theta;
  }
  if (V5) {
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    V5[0] = rho;
    V5[1] = rho * u[0];
    V5[2] = rho * u[1];
    V5[3] = rho * u[2];
    V5[4] = 0.5 * rho * usq + 1.5 * rho * theta;
  }
  return physical(rho, theta) ? ORACLE_OK : ORACLE_E_NONPHYSICAL;
}

int bgk_oracle_moments(const bgk_oracle_problem* p, const double* f,
                       double* V, double* W) {
  if (check_problem(p) || !f) return ORACLE_E_INVALID;
  const long nv3 = nv3_of(p);
  int bad = 0;
#pragma omp parallel for num_threads(NT) reduction(| : bad)
  for (int i = 0; i < p->nx; ++i) {
    if (moments_cell(p, f + (long)i * nv3, V ? V + 5 * (long)i : NULL,
                     W ? W + 5 * (long)i : NULL))
      bad = 1;
  }
  return bad ? ORACLE_E_NONPHYSICAL : ORACLE_OK;
}

/* ------------------------------------------------------------ transport -- */
/* Section 3.1: explicit upwind finite volumes in x,
 *   f*_ij = f_ij - dt/dx (F_{i+1/2,j} - F_{i-1/2,j}),
 *   F_{i+1/2,j} = max(v_x,0) f_ij + min(v_x,0) f_{i+1,j},
 * and, with an exterior force E_i along x, Rusanov fluxes in v_x,
 *   f*_ij -= dt/dv_x (G_{i,j+1/2} - G_{i,j-1/2}),
 *   G_{i,j+1/2} = E_i/2 (f_ij + f_{i,j+1}) - E_max/2 (f_{i,j+1} - f_ij),
 * j+1 the next v_x point at the same (v_y, v_z), E_max = max_i |E_i|.  The
 * printed dissipation term differences a value with itself; it is read as
 * the Rusanov one above.  No flux crosses the ends of the truncated v_x
 * range, so the scheme conserves mass. */
/* Second order in x (order = 2): the upwind flux gains the Lax-Wendroff
 * correction limited by van Leer's limiter (the flux limiters the paper names
 * as the natural improvement, Section 3.1), written with the limited
 * difference L(a, b) = 2ab/(a+b) when ab > 0, else 0:
 *   v_x > 0: F_{i+1/2} = v_x [f_i + (1-nu)/2 L(f_i - f_{i-1}, f_{i+1} - f_i)]
 *   v_x < 0: F_{i+1/2} = v_x [f_{i+1} - (1-|nu|)/2 L(f_{i+2} - f_{i+1}, f_{i+1} - f_i)]
 * nu = v_x dt/dx; ghost cells two deep from the boundary condition.  It is
 * TVD for |nu| <= 1 and second order where the data are smooth. */
static double vl_limited(double a, double b) {
  return a * b > 0.0 ? 2.0 * a * b / (a + b) : 0.0;
}

static double flux2(double vx, double nu, double fm, double f0, double fp, double fp2) {
  /* flux through the face between f0 (cell i) and fp (cell i+1) */
  if (vx > 0.0) return vx * (f0 + 0.5 * (1.0 - nu) * vl_limited(f0 - fm, fp - f0));
  if (vx < 0.0) return vx * (fp - 0.5 * (1.0 + nu) * vl_limited(fp2 - fp, fp - f0));
  return 0.0;
}

static int transport_impl(const bgk_oracle_problem* p, const double* E, int order,
                          const double* f, double dt, double* f_star) {
  if (check_problem(p) || !f || !f_star || f == f_star) return ORACLE_E_INVALID;
  const long nv3 = nv3_of(p);
  const int nyz = p->nv[1] * p->nv[2];
  const double r = dt / dx_of(p);
  const double rv = dt / dv_of(p, 0);
  const double emax = emax_of(p, E);
#pragma omp parallel for num_threads(NT)
  for (int i = 0; i < p->nx; ++i) {
    const double* fm2 = f + (long)ghost(p, i - 2) * nv3;
    const double* fm = f + (long)ghost(p, i - 1) * nv3;
    const double* f0 = f + (long)i * nv3;
    const double* fp = f + (long)ghost(p, i + 1) * nv3;
    const double* fp2 = f + (long)ghost(p, i + 2) * nv3;
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx) {
      double vx = vc(p, 0, jx);
      double vp = vx > 0.0 ? vx : 0.0;
      double vm = vx < 0.0 ? vx : 0.0;
      double nu = vx * r;
      for (int jyz = 0; jyz < nyz; ++jyz, ++j) {
        double F_right, F_left;
        if (order == 2) {
          F_right = flux2(vx, nu, fm[j], f0[j], fp[j], fp2[j]);
          F_left = flux2(vx, nu, fm2[j], fm[j], f0[j], fp[j]);
        } else {
          F_right = vp * f0[j] + vm * fp[j];
          F_left = vp * fm[j] + vm * f0[j];
        }
        double out = f0[j] - r * (F_right - F_left);
        if (E) {
          double G_up = 0.0, G_down = 0.0;
          if (jx + 1 < p->nv[0]) {
            double a = f0[j], b = f0[j + nyz];
            G_up = 0.5 * E[i] * (a + b) - 0.5 * emax * (b - a);
          }
          if (jx > 0) {
            double a = f0[j - nyz], b = f0[j];
            G_down = 0.5 * E[i] * (a + b) - 0.5 * emax * (b - a);
          }
          out -= rv * (G_up - G_down);
        }
        f_star[(long)i * nv3 + j] = out;
      }
    }
  }
  return ORACLE_OK;
}

int bgk_oracle_transport(const bgk_oracle_problem* p, const double* f,
                         double dt, double* f_star) {
  return transport_impl(p, NULL, 1, f, dt, f_star);
}

int bgk_oracle_transport_force(const bgk_oracle_problem* p, const double* E,
                               const double* f, double dt, double* f_star) {
  if (!E) return ORACLE_E_INVALID;
  return transport_impl(p, E, 1, f, dt, f_star);
}

/* ---------------------------------------------------------- relaxation -- */
/* Section 3.1: implicit BGK term with the n+1 moments taken from f* (the
 * collision operator conserves them), so
 *   f^{n+1} = (f* + lambda M[P f*]) / (1 + lambda),  lambda = dt / eps. */
int bgk_oracle_relax(const bgk_oracle_problem* p, const double* f_star,
                     double dt, double* f_out) {
  if (check_problem(p) || !f_star || !f_out) return ORACLE_E_INVALID;
  const long nv3 = nv3_of(p);
  const double lambda = dt / p->eps;
  int bad = 0;
#pragma omp parallel for num_threads(NT) reduction(| : bad)
  for (int i = 0; i < p->nx; ++i) {
    double W5[5];
    if (moments_cell(p, f_star + (long)i * nv3, NULL, W5)) {
      bad = 1;
      continue;
    }
    double u[3] = {W5[1], W5[2], W5[3]};
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx)
      for (int jy = 0; jy < p->nv[1]; ++jy)
        for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
          double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
          double M = maxwellian(W5[0], u, W5[4], v);
          long k = (long)i * nv3 + j;
          f_out[k] = (f_star[k] + lambda * M) / (1.0 + lambda);
        }
  }
  return bad ? ORACLE_E_NONPHYSICAL : ORACLE_OK;
}

/* ---------------------------------------------------- fine propagator -- */
static int fine_steps_impl(const bgk_oracle_problem* p, const double* E, int order,
                           const double* f_in, double* f_out, double dt,
                           int32_t n_steps) {
  if (check_problem(p) || !f_in || !f_out || n_steps < 0 || !(dt > 0.0))
    return ORACLE_E_INVALID;
  const size_t n = (size_t)p->nx * nv3_of(p);
  double* cur = (double*)malloc(n * sizeof(double));
  double* star = (double*)malloc(n * sizeof(double));
  if (!cur || !star) {
    free(cur);
    free(star);
    return ORACLE_E_INVALID;
  }
  memcpy(cur, f_in, n * sizeof(double));
  int rc = ORACLE_OK;
  for (int32_t s = 0; s < n_steps && rc == ORACLE_OK; ++s) {
    rc = transport_impl(p, E, order, cur, dt, star);
    if (rc == ORACLE_OK) rc = bgk_oracle_relax(p, star, dt, cur);
  }
  if (rc == ORACLE_OK) memcpy(f_out, cur, n * sizeof(double));
  free(cur);
  free(star);
  return rc;
}

int bgk_oracle_fine_steps(const bgk_oracle_problem* p, const double* f_in,
                          double* f_out, double dt, int32_t n_steps) {
  return fine_steps_impl(p, NULL, 1, f_in, f_out, dt, n_steps);
}

int bgk_oracle_fine_steps_force(const bgk_oracle_problem* p, const double* E,
                                const double* f_in, double* f_out, double dt,
                                int32_t n_steps) {
  if (!E) return ORACLE_E_INVALID;
  return fine_steps_impl(p, E, 1, f_in, f_out, dt, n_steps);
}

static int fine_step_impl(const bgk_oracle_problem* p, const double* E, int order,
                          const double* f_in, double* f_out, double t_span,
                          int32_t* n_steps_out) {
  int32_t n;
  double dt;
  int rc = n_steps_impl(p, emax_of(p, E), t_span, &n, &dt);
  if (rc) return rc;
  if (n_steps_out) *n_steps_out = n;
  return fine_steps_impl(p, E, order, f_in, f_out, dt, n);
}

int bgk_oracle_fine_step(const bgk_oracle_problem* p, const double* f_in,
                         double* f_out, double t_span, int32_t* n_steps_out) {
  return fine_step_impl(p, NULL, 1, f_in, f_out, t_span, n_steps_out);
}

int bgk_oracle_fine_step_force(const bgk_oracle_problem* p, const double* E,
                               const double* f_in, double* f_out, double t_span,
                               int32_t* n_steps_out) {
  if (!E) return ORACLE_E_INVALID;
  return fine_step_impl(p, E, 1, f_in, f_out, t_span, n_steps_out);
}

static void conserved_to_primitive(const double* V5, double* W5) {
  double rho = V5[0];
  double u[3] = {V5[1] / rho, V5[2] / rho, V5[3] / rho};
  double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  W5[0] = rho;
  W5[1] = u[0];
  W5[2] = u[1];
  W5[3] = u[2];
  W5[4] = (2.0 * V5[4] / rho - usq) / 3.0;
}

/* Steps 5-7 of Algorithm 2: lifting, kinetic propagation, projection. */
static int propagate_impl(const bgk_oracle_problem* p, const double* E, int order,
                          int lift_order,
                          const double* V_in, double* V_out, double t_span) {
  if (check_problem(p) || !V_in || !V_out) return ORACLE_E_INVALID;
  const size_t n = (size_t)p->nx * nv3_of(p);
  double* W = (double*)malloc(5 * (size_t)p->nx * sizeof(double));
  double* f = (double*)malloc(n * sizeof(double));
  if (!W || !f) {
    free(W);
    free(f);
    return ORACLE_E_INVALID;
  }
  for (int i = 0; i < p->nx; ++i) conserved_to_primitive(V_in + 5 * i, W + 5 * i);
  int rc = lift_order == 1 ? bgk_oracle_lift_ce(p, W, f) : bgk_oracle_lift(p, W, f);
  if (rc == ORACLE_OK) rc = fine_step_impl(p, E, order, f, f, t_span, NULL);
  if (rc == ORACLE_OK) rc = bgk_oracle_moments(p, f, V_out, NULL);
  free(W);
  free(f);
  return rc;
}

int bgk_oracle_fine_propagate_moments(const bgk_oracle_problem* p,
                                      const double* V_in, double* V_out,
                                      double t_span) {
  return propagate_impl(p, NULL, 1, 0, V_in, V_out, t_span);
}

int bgk_oracle_fine_propagate_moments_force(const bgk_oracle_problem* p,
                                            const double* E, const double* V_in,
                                            double* V_out, double t_span) {
  if (!E) return ORACLE_E_INVALID;
  return propagate_impl(p, E, 1, 0, V_in, V_out, t_span);
}

/* ------------------------------------------------------------ coarse G -- */
/* Section 3.2: Euler equations in conserved variables
 *   V = (rho, rho u_x, rho u_y, rho u_z, E),
 *   h(V) = (rho u_x, rho u_x^2 + rho theta, rho u_x u_y, rho u_x u_z,
 *           u_x (E + rho theta)),
 * Rusanov flux H_{i+1/2} = (h(V_i) + h(V_{i+1}))/2 - S/2 (V_{i+1} - V_i),
 * S = max(|u_x| + c) over the two cells, update V -= dt/dx (H+ - H-). */
static int euler_prim(const double* V5, double gamma, double* ux, double* uy,
                      double* uz, double* theta, double* c) {
  double rho = V5[0];
  *ux = V5[1] / rho;
  *uy = V5[2] / rho;
  *uz = V5[3] / rho;
  double usq = (*ux) * (*ux) + (*uy) * (*uy) + (*uz) * (*uz);
  *theta = (2.0 * V5[4] / rho - usq) / 3.0;
  if (!physical(rho, *theta)) return ORACLE_E_NONPHYSICAL;
  *c = sqrt(gamma * (*theta));
  return ORACLE_OK;
}

static void euler_flux(const double* V5, double ux, double uy, double uz,
                       double theta, double* h) {
  double rho = V5[0];
  double pr = rho * theta;
  h[0] = rho * ux;
  h[1] = rho * ux * ux + pr;
  h[2] = rho * ux * uy;
  h[3] = rho * ux * uz;
  h[4] = ux * (V5[4] + pr);
}

/* With an exterior force E_i the Euler system carries the source
 * S = (0, rho E, 0, 0, rho u_x E) (Section 3.2 allows a source term), added
 * explicitly in each substep from the substep's initial state.
 *
 * viscous = 1: the compressible Navier-Stokes system of Section 1 (the
 * first-order Chapman-Enskog correction of Euler's equations), with the BGK
 * transport coefficients of tau = 1: viscosity mu = rho theta and heat
 * conductivity kappa = (5/2) rho theta (Prandtl number 1).  In 1D-3V the
 * strain terms are sigma_xx = (4/3) du_x/dx, sigma_xy = du_y/dx,
 * sigma_xz = du_z/dx.  Face viscous flux (central differences, face values
 * the mean of the two cells):
 *   D = eps/dx (0, 4/3 mu (ux_R-ux_L), mu (uy_R-uy_L), mu (uz_R-uz_L),
 *               mu (4/3 ux (ux_R-ux_L) + uy (uy_R-uy_L) + uz (uz_R-uz_L))
 *               + kappa (theta_R-theta_L)),
 * added as V += dt/dx (D_{i+1/2} - D_{i-1/2}); the substep also obeys the
 * explicit diffusion limit dt <= cfl dx^2 / (2 eps (5/3) max theta), 5/3
 * theta being the larger of the two diffusivities 4/3 mu/rho and
 * kappa/(rho c_v). */
static int coarse_impl(const bgk_oracle_problem* p, const double* E, int viscous,
                       const double* V_in, double* V_out, double t_span,
                       int32_t* n_sub_out) {
  if (check_problem(p) || !V_in || !V_out || !(t_span > 0.0))
    return ORACLE_E_INVALID;
  if (viscous && !isfinite(p->eps)) return ORACLE_E_INVALID;
  const int nx = p->nx;
  const double dx = dx_of(p);
  double* V = (double*)malloc(5 * (size_t)nx * sizeof(double));
  double* Vn = (double*)malloc(5 * (size_t)nx * sizeof(double));
  double* H = (double*)malloc(5 * (size_t)(nx + 1) * sizeof(double));
  double* spd = (double*)malloc((size_t)nx * sizeof(double));
  double* hh = (double*)malloc(5 * (size_t)nx * sizeof(double));
  double* pr = (double*)malloc(4 * (size_t)nx * sizeof(double)); /* ux uy uz theta */
  if (!V || !Vn || !H || !spd || !hh || !pr) {
    free(V); free(Vn); free(H); free(spd); free(hh); free(pr);
    return ORACLE_E_INVALID;
  }
  memcpy(V, V_in, 5 * (size_t)nx * sizeof(double));
  double t = 0.0;
  int32_t nsub = 0;
  int rc = ORACLE_OK;
  while (t_span - t > 1e-14 * t_span) {
    /* cell-wise primitive variables, wave speed and physical flux */
    double smax = 0.0, thmax = 0.0;
    for (int i = 0; i < nx && rc == ORACLE_OK; ++i) {
      double ux, uy, uz, th, c;
      rc = euler_prim(V + 5 * i, p->sound_gamma, &ux, &uy, &uz, &th, &c);
      if (rc) break;
      spd[i] = fabs(ux) + c;
      euler_flux(V + 5 * i, ux, uy, uz, th, hh + 5 * i);
      if (spd[i] > smax) smax = spd[i];
      if (th > thmax) thmax = th;
      pr[4 * i + 0] = ux;
      pr[4 * i + 1] = uy;
      pr[4 * i + 2] = uz;
      pr[4 * i + 3] = th;
    }
    if (rc) break;
    double dt = p->cfl * dx / smax;
    if (viscous) {
      double dt_visc = p->cfl * dx * dx / (2.0 * p->eps * (5.0 / 3.0) * thmax);
      if (dt_visc < dt) dt = dt_visc;
    }
    if (dt > t_span - t) dt = t_span - t;
    /* interface fluxes H_{f-1/2} for f = 0..nx, ghosts from the BC */
    for (int fc = 0; fc <= nx; ++fc) {
      int L = ghost(p, fc - 1), R = ghost(p, fc);
      double S = spd[L] > spd[R] ? spd[L] : spd[R];
      for (int c = 0; c < 5; ++c)
        H[5 * fc + c] = 0.5 * (hh[5 * L + c] + hh[5 * R + c]) -
                        0.5 * S * (V[5 * R + c] - V[5 * L + c]);
    }
    for (int i = 0; i < nx; ++i)
      for (int c = 0; c < 5; ++c)
        Vn[5 * i + c] = V[5 * i + c] - dt / dx * (H[5 * (i + 1) + c] - H[5 * i + c]);
    if (viscous) {
      /* face viscous fluxes D_{f-1/2}, f = 0..nx, into H (reused) */
      for (int fc = 0; fc <= nx; ++fc) {
        int L = ghost(p, fc - 1), R = ghost(p, fc);
        const double* a = pr + 4 * L;
        const double* b = pr + 4 * R;
        double mu = 0.5 * (V[5 * L] * a[3] + V[5 * R] * b[3]);
        double kappa = 2.5 * mu;
        double dux = b[0] - a[0], duy = b[1] - a[1], duz = b[2] - a[2];
        double uxf = 0.5 * (a[0] + b[0]), uyf = 0.5 * (a[1] + b[1]), uzf = 0.5 * (a[2] + b[2]);
        double k = p->eps / dx;
        H[5 * fc + 0] = 0.0;
        H[5 * fc + 1] = k * (4.0 / 3.0) * mu * dux;
        H[5 * fc + 2] = k * mu * duy;
        H[5 * fc + 3] = k * mu * duz;
        H[5 * fc + 4] = k * (mu * ((4.0 / 3.0) * uxf * dux + uyf * duy + uzf * duz) +
                             kappa * (b[3] - a[3]));
      }
      for (int i = 0; i < nx; ++i)
        for (int c = 1; c < 5; ++c)
          Vn[5 * i + c] += dt / dx * (H[5 * (i + 1) + c] - H[5 * i + c]);
    }
    if (E)
      for (int i = 0; i < nx; ++i) {
        Vn[5 * i + 1] += dt * V[5 * i + 0] * E[i];
        Vn[5 * i + 4] += dt * V[5 * i + 1] * E[i];
      }
    memcpy(V, Vn, 5 * (size_t)nx * sizeof(double));
    t += dt;
    ++nsub;
  }
  if (rc == ORACLE_OK) {
    /* the final state must be physical as well */
    for (int i = 0; i < nx && rc == ORACLE_OK; ++i) {
      double ux, uy, uz, th, c;
      rc = euler_prim(V + 5 * i, p->sound_gamma, &ux, &uy, &uz, &th, &c);
    }
  }
  if (rc == ORACLE_OK) memcpy(V_out, V, 5 * (size_t)nx * sizeof(double));
  if (n_sub_out) *n_sub_out = nsub;
  free(V); free(Vn); free(H); free(spd); free(hh); free(pr);
  return rc;
}

static int euler_impl(const bgk_oracle_problem* p, const double* E,
                      const double* V_in, double* V_out, double t_span,
                      int32_t* n_sub_out) {
  return coarse_impl(p, E, 0, V_in, V_out, t_span, n_sub_out);
}

int bgk_oracle_euler_coarse_step(const bgk_oracle_problem* p,
                                 const double* V_in, double* V_out,
                                 double t_span, int32_t* n_sub_out) {
  return euler_impl(p, NULL, V_in, V_out, t_span, n_sub_out);
}

int bgk_oracle_cns_coarse_step(const bgk_oracle_problem* p, const double* E,
                               const double* V_in, double* V_out, double t_span,
                               int32_t* n_sub_out) {
  return coarse_impl(p, E, 1, V_in, V_out, t_span, n_sub_out);
}

int bgk_oracle_euler_coarse_step_force(const bgk_oracle_problem* p,
                                       const double* E, const double* V_in,
                                       double* V_out, double t_span,
                                       int32_t* n_sub_out) {
  if (!E) return ORACLE_E_INVALID;
  return euler_impl(p, E, V_in, V_out, t_span, n_sub_out);
}

/* ------------------------------------------------------------ parareal -- */
static void primitive_to_conserved(const double* W5, double* V5) {
  double rho = W5[0];
  double usq = W5[1] * W5[1] + W5[2] * W5[2] + W5[3] * W5[3];
  V5[0] = rho;
  V5[1] = rho * W5[1];
  V5[2] = rho * W5[2];
  V5[3] = rho * W5[3];
  V5[4] = 0.5 * rho * usq + 1.5 * rho * W5[4];
}

/* Algorithm 2 with 0-based iteration index k:
 *   U^{n,0} = G(U^{n-1,0});
 *   for k = 0..K-1:
 *     Delta^n = P F L(U^{n-1,k}) - G(U^{n-1,k})       for n = k+1..N
 *     U^{n,k+1} = U^{n,k}                              for n <= k
 *     U^{n,k+1} = G(U^{n-1,k+1}) + Delta^n             for n = k+1..N (in order)
 *     err_k = max_{n,i,c} |U^{n,k+1} - U^{n,k}|;  stop at K or err < tol.
 * The jump loop is the parallel one (Section 2.2 and Section 4). */
/* The coarse model G of the parareal iteration: 0 the Euler system, 1 the
 * Navier-Stokes system, 2 the fine propagator itself (a check of the
 * correction: with G = F the first iteration reproduces the serial chain). */
static int coarse_of(const bgk_oracle_problem* p, const double* E, int coarse, int order,
                     int lift_order, const double* in, double* out, double dT) {
  if (coarse == 2) return propagate_impl(p, E, order, lift_order, in, out, dT);
  return coarse_impl(p, E, coarse, in, out, dT, NULL);
}

static int parareal_impl(const bgk_oracle_problem* p, const double* E, int viscous,
                         int lift_order, int order, const double* W0, int32_t n_slices, double T,
                         int32_t k_max, double tol, double* V_out,
                         double* err_hist, int32_t* k_done) {
  if (check_problem(p) || !W0 || !V_out || n_slices < 1 || k_max < 0 ||
      !(T > 0.0))
    return ORACLE_E_INVALID;
  const int nx = p->nx;
  const size_t sl = 5 * (size_t)nx;
  const double dT = T / n_slices;
  double* U = (double*)malloc(sl * (n_slices + 1) * sizeof(double));
  double* Un = (double*)malloc(sl * (n_slices + 1) * sizeof(double));
  double* D = (double*)malloc(sl * (n_slices + 1) * sizeof(double));
  if (!U || !Un || !D) {
    free(U); free(Un); free(D);
    return ORACLE_E_INVALID;
  }
  for (int i = 0; i < nx; ++i) primitive_to_conserved(W0 + 5 * i, U + 5 * i);
  int rc = ORACLE_OK;
  for (int n = 1; n <= n_slices && rc == ORACLE_OK; ++n)
    rc = coarse_of(p, E, viscous, order, lift_order, U + sl * (n - 1), U + sl * n, dT);
  int32_t kd = 0;
  for (int k = 0; k < k_max && rc == ORACLE_OK; ++k) {
    /* jumps, independent over n */
    int bad = 0;
    for (int n = k + 1; n <= n_slices; ++n) {
      double* Fv = (double*)malloc(sl * sizeof(double));
      double* Gv = (double*)malloc(sl * sizeof(double));
      int r1 = propagate_impl(p, E, order, lift_order, U + sl * (n - 1), Fv, dT);
      int r2 = r1 ? r1 : coarse_of(p, E, viscous, order, lift_order, U + sl * (n - 1), Gv, dT);
      if (r1 || r2) bad = r1 ? r1 : r2;
      else
        for (size_t q = 0; q < sl; ++q) D[sl * n + q] = Fv[q] - Gv[q];
      free(Fv);
      free(Gv);
      if (bad) break;
    }
    if (bad) {
      rc = bad;
      break;
    }
    /* frozen prefix, then the sequential correction */
    memcpy(Un, U, sl * (k + 1) * sizeof(double));
    for (int n = k + 1; n <= n_slices && rc == ORACLE_OK; ++n) {
      rc = coarse_of(p, E, viscous, order, lift_order, Un + sl * (n - 1), Un + sl * n, dT);
      if (rc == ORACLE_OK)
        for (size_t q = 0; q < sl; ++q) Un[sl * n + q] += D[sl * n + q];
    }
    if (rc) break;
    double err = 0.0;
    for (size_t q = 0; q < sl * (n_slices + 1); ++q) {
      double d = fabs(Un[q] - U[q]);
      if (d > err) err = d;
    }
    memcpy(U, Un, sl * (n_slices + 1) * sizeof(double));
    if (err_hist) err_hist[k] = err;
    kd = k + 1;
    if (err < tol) break;
  }
  if (k_done) *k_done = kd;
  if (rc == ORACLE_OK) memcpy(V_out, U, sl * (n_slices + 1) * sizeof(double));
  free(U); free(Un); free(D);
  return rc;
}

int bgk_oracle_parareal_iterate(const bgk_oracle_problem* p, const double* W0,
                                int32_t n_slices, double T, int32_t k_max,
                                double tol, double* V_out, double* err_hist,
                                int32_t* k_done) {
  return parareal_impl(p, NULL, 0, 0, 1, W0, n_slices, T, k_max, tol, V_out, err_hist, k_done);
}

int bgk_oracle_parareal_iterate_force(const bgk_oracle_problem* p, const double* E,
                                      const double* W0, int32_t n_slices, double T,
                                      int32_t k_max, double tol, double* V_out,
                                      double* err_hist, int32_t* k_done) {
  if (!E) return ORACLE_E_INVALID;
  return parareal_impl(p, E, 0, 0, 1, W0, n_slices, T, k_max, tol, V_out, err_hist, k_done);
}

int bgk_oracle_parareal_iterate_cns(const bgk_oracle_problem* p, const double* E,
                                    const double* W0, int32_t n_slices, double T,
                                    int32_t k_max, double tol, double* V_out,
                                    double* err_hist, int32_t* k_done) {
  return parareal_impl(p, E, 1, 0, 1, W0, n_slices, T, k_max, tol, V_out, err_hist, k_done);
}

/* The fine reference that parareal converges to: U^n = P F L(U^{n-1}). */
static int serial_impl(const bgk_oracle_problem* p, const double* E, int lift_order, int order,
                       const double* W0, int32_t n_slices, double T, double* V_out) {
  if (check_problem(p) || !W0 || !V_out || n_slices < 1 || !(T > 0.0))
    return ORACLE_E_INVALID;
  const size_t sl = 5 * (size_t)p->nx;
  for (int i = 0; i < p->nx; ++i) primitive_to_conserved(W0 + 5 * i, V_out + 5 * i);
  for (int n = 1; n <= n_slices; ++n) {
    int rc = propagate_impl(p, E, order, lift_order, V_out + sl * (n - 1), V_out + sl * n,
                            T / n_slices);
    if (rc) return rc;
  }
  return ORACLE_OK;
}

int bgk_oracle_serial_fine(const bgk_oracle_problem* p, const double* W0,
                           int32_t n_slices, double T, double* V_out) {
  return serial_impl(p, NULL, 0, 1, W0, n_slices, T, V_out);
}

int bgk_oracle_serial_fine_force(const bgk_oracle_problem* p, const double* E,
                                 const double* W0, int32_t n_slices, double T,
                                 double* V_out) {
  if (!E) return ORACLE_E_INVALID;
  return serial_impl(p, E, 0, 1, W0, n_slices, T, V_out);
}

/* --------------------------------------------------------------- adjoint -- */
/* One IMEX step is f^{n+1} = R(g), g = T f^n, with T the upwind transport
 * (linear) and R(g) = (g + lambda M[P g]) / (1 + lambda).  Its adjoint maps
 * fbar^{n+1} to fbar^n = T^t (dR/dg)^t fbar^{n+1}, by the chain rule through
 * the two-pass moments of Definition 1 and the Maxwellian of Section 1:
 *   w      = lambda/(1+lambda) fbar^{n+1}
 *   rhobar = sum_j w M / rho
 *   ubar   = sum_j w M (v-u) / theta
 *   thbar  = sum_j w M (|v-u|^2/(2 theta^2) - 3/(2 theta))
 *   gbar_j = fbar_j/(1+lambda)
 *            + dv3 [rhobar + ubar.(v_j-u)/rho + thbar (|v_j-u|^2 - 3 theta)/(3 rho)]
 * (d rho/dg_j = dv3, d u/dg_j = dv3 (v_j-u)/rho, d theta/dg_j =
 * dv3 (|v_j-u|^2 - 3 theta)/(3 rho), the u-derivative of the second sum
 * vanishing because u is the mean).  With d lambda/d log eps = -lambda and
 * dR/dlambda = (M - g)/(1+lambda)^2, the step adds
 *   -lambda sum_ij fbar^{n+1}_ij (M_ij - g_ij)/(1+lambda)^2  to dL/dlog eps. */
static int adjoint_step(const bgk_oracle_problem* p, const double* f_n,
                        const double* fbar_np1, double dt, double* fbar_n,
                        double* dlog_eps, double* g, double* gbar) {
  const int nx = p->nx;
  const long nv3 = nv3_of(p);
  const double dv3 = dv3_of(p);
  const double lambda = dt / p->eps;
  int rc = bgk_oracle_transport(p, f_n, dt, g);
  if (rc) return rc;
  int bad = 0;
  double* le_cell = (double*)calloc((size_t)nx, sizeof(double));
  if (!le_cell) return ORACLE_E_INVALID;
#pragma omp parallel for num_threads(NT) reduction(| : bad)
  for (int i = 0; i < nx; ++i) {
    const double* gi = g + (long)i * nv3;
    const double* fb = fbar_np1 + (long)i * nv3;
    double W5[5];
    if (moments_cell(p, gi, NULL, W5)) {
      bad = 1;
      continue;
    }
    double rho = W5[0], th = W5[4];
    double u[3] = {W5[1], W5[2], W5[3]};
    double rb = 0.0, ub[3] = {0.0, 0.0, 0.0}, tb = 0.0, le = 0.0;
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx)
      for (int jy = 0; jy < p->nv[1]; ++jy)
        for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
          double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
          double M = maxwellian(rho, u, th, v);
          double w = lambda / (1.0 + lambda) * fb[j];
          double d2 = 0.0;
          for (int a = 0; a < 3; ++a) d2 += (v[a] - u[a]) * (v[a] - u[a]);
          rb += w * M / rho;
          for (int a = 0; a < 3; ++a) ub[a] += w * M * (v[a] - u[a]) / th;
          tb += w * M * (d2 / (2.0 * th * th) - 1.5 / th);
          le += fb[j] * (M - gi[j]) / ((1.0 + lambda) * (1.0 + lambda));
        }
    le_cell[i] = -lambda * le;
    j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx)
      for (int jy = 0; jy < p->nv[1]; ++jy)
        for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
          double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
          double d2 = 0.0, ud = 0.0;
          for (int a = 0; a < 3; ++a) {
            d2 += (v[a] - u[a]) * (v[a] - u[a]);
            ud += ub[a] * (v[a] - u[a]);
          }
          gbar[(long)i * nv3 + j] =
              fb[j] / (1.0 + lambda) +
              dv3 * (rb + ud / rho + tb * (d2 - 3.0 * th) / (3.0 * rho));
        }
  }
  /* summed in cell order so that the result does not depend on threading */
  double dle = 0.0;
  for (int i = 0; i < nx; ++i) dle += le_cell[i];
  free(le_cell);
  if (bad) return ORACLE_E_NONPHYSICAL;
  *dlog_eps += dle;
  /* transpose of the transport stencil: every coefficient c of
   * g_i = sum_k c_{ik} f_{ghost(k)} is scattered back as fbar_ghost(k) += c gbar_i */
  const double r = dt / dx_of(p);
  memset(fbar_n, 0, (size_t)nx * nv3 * sizeof(double));
  for (int i = 0; i < nx; ++i) {
    int im = ghost(p, i - 1), ip = ghost(p, i + 1);
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx) {
      double vx = vc(p, 0, jx);
      double vp = vx > 0.0 ? vx : 0.0;
      double vm = vx < 0.0 ? vx : 0.0;
      /* g_i = f_i - r (vp f_i + vm f_{i+1} - vp f_{i-1} - vm f_i) */
      double c_self = 1.0 - r * vp + r * vm;
      double c_left = r * vp;
      double c_right = -r * vm;
      for (int jyz = 0; jyz < p->nv[1] * p->nv[2]; ++jyz, ++j) {
        double gb = gbar[(long)i * nv3 + j];
        fbar_n[(long)i * nv3 + j] += c_self * gb;
        fbar_n[(long)im * nv3 + j] += c_left * gb;
        fbar_n[(long)ip * nv3 + j] += c_right * gb;
      }
    }
  }
  return ORACLE_OK;
}

int bgk_oracle_fine_adjoint(const bgk_oracle_problem* p, const double* f_ckpt,
                            int32_t ckpt_every, int32_t n_steps, double dt,
                            const double* fbar_T, double* fbar_0,
                            double* dlog_eps) {
  if (check_problem(p) || !f_ckpt || !fbar_T || !fbar_0 || !dlog_eps ||
      ckpt_every < 1 || n_steps < 0 || !(dt > 0.0))
    return ORACLE_E_INVALID;
  const size_t n = (size_t)p->nx * nv3_of(p);
  double* states = (double*)malloc(n * (size_t)ckpt_every * sizeof(double));
  double* star = (double*)malloc(n * sizeof(double));
  double* g = (double*)malloc(n * sizeof(double));
  double* gbar = (double*)malloc(n * sizeof(double));
  double* fb = (double*)malloc(n * sizeof(double));
  double* fb2 = (double*)malloc(n * sizeof(double));
  if (!states || !star || !g || !gbar || !fb || !fb2) {
    free(states); free(star); free(g); free(gbar); free(fb); free(fb2);
    return ORACLE_E_INVALID;
  }
  memcpy(fb, fbar_T, n * sizeof(double));
  int rc = ORACLE_OK;
  int32_t n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
  for (int32_t c = n_seg - 1; c >= 0 && rc == ORACLE_OK; --c) {
    int32_t s0 = c * ckpt_every;
    int32_t s1 = s0 + ckpt_every < n_steps ? s0 + ckpt_every : n_steps;
    /* recompute the forward states s0..s1-1 of this segment */
    memcpy(states, f_ckpt + (size_t)c * n, n * sizeof(double));
    for (int32_t s = s0 + 1; s < s1 && rc == ORACLE_OK; ++s) {
      double* prev = states + (size_t)(s - 1 - s0) * n;
      double* next = states + (size_t)(s - s0) * n;
      rc = bgk_oracle_transport(p, prev, dt, star);
      if (rc == ORACLE_OK) rc = bgk_oracle_relax(p, star, dt, next);
    }
    for (int32_t s = s1 - 1; s >= s0 && rc == ORACLE_OK; --s) {
      rc = adjoint_step(p, states + (size_t)(s - s0) * n, fb, dt, fb2, dlog_eps,
                        g, gbar);
      double* t = fb;
      fb = fb2;
      fb2 = t;
    }
  }
  if (rc == ORACLE_OK) memcpy(fbar_0, fb, n * sizeof(double));
  free(states); free(star); free(g); free(gbar); free(fb); free(fb2);
  return rc;
}

/* Lifting adjoint in rho: M is linear in rho, so dM/drho = M/rho. */
int bgk_oracle_lift_adjoint_rho(const bgk_oracle_problem* p, const double* W,
                                const double* fbar, double* rhobar) {
  if (check_problem(p) || !W || !fbar || !rhobar) return ORACLE_E_INVALID;
  const long nv3 = nv3_of(p);
  for (int i = 0; i < p->nx; ++i) {
    const double* w = W + 5 * (long)i;
    if (!physical(w[0], w[4])) return ORACLE_E_NONPHYSICAL;
    double u[3] = {w[1], w[2], w[3]};
    double s = 0.0;
    long j = 0;
    for (int jx = 0; jx < p->nv[0]; ++jx)
      for (int jy = 0; jy < p->nv[1]; ++jy)
        for (int jz = 0; jz < p->nv[2]; ++jz, ++j) {
          double v[3] = {vc(p, 0, jx), vc(p, 1, jy), vc(p, 2, jz)};
          s += fbar[(long)i * nv3 + j] * maxwellian(w[0], u, w[4], v) / w[0];
        }
    rhobar[i] = s;
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------- options -- */
static int check_opts(int32_t lift_order, int32_t fine_order) {
  return ((lift_order != 0 && lift_order != 1) || (fine_order != 1 && fine_order != 2))
             ? ORACLE_E_INVALID
             : ORACLE_OK;
}

int bgk_oracle_transport_opts(const bgk_oracle_problem* p, const double* E,
                              int32_t fine_order, const double* f, double dt,
                              double* f_star) {
  if (check_opts(0, fine_order)) return ORACLE_E_INVALID;
  return transport_impl(p, E, fine_order, f, dt, f_star);
}

int bgk_oracle_fine_steps_opts(const bgk_oracle_problem* p, const double* E,
                               int32_t fine_order, const double* f_in, double* f_out,
                               double dt, int32_t n_steps) {
  if (check_opts(0, fine_order)) return ORACLE_E_INVALID;
  return fine_steps_impl(p, E, fine_order, f_in, f_out, dt, n_steps);
}

int bgk_oracle_fine_propagate_moments_opts(const bgk_oracle_problem* p,
                                           const double* E, int32_t lift_order,
                                           int32_t fine_order, const double* V_in,
                                           double* V_out, double t_span) {
  if (check_opts(lift_order, fine_order)) return ORACLE_E_INVALID;
  return propagate_impl(p, E, fine_order, lift_order, V_in, V_out, t_span);
}

int bgk_oracle_parareal_iterate_opts(const bgk_oracle_problem* p, const double* E,
                                     int32_t coarse, int32_t lift_order,
                                     int32_t fine_order, const double* W0,
                                     int32_t n_slices, double T, int32_t k_max,
                                     double tol, double* V_out, double* err_hist,
                                     int32_t* k_done) {
  if (coarse < 0 || coarse > 2 || check_opts(lift_order, fine_order))
    return ORACLE_E_INVALID;
  return parareal_impl(p, E, coarse, lift_order, fine_order, W0, n_slices, T, k_max, tol,
                       V_out, err_hist, k_done);
}

int bgk_oracle_serial_fine_opts(const bgk_oracle_problem* p, const double* E,
                                int32_t lift_order, int32_t fine_order,
                                const double* W0, int32_t n_slices, double T,
                                double* V_out) {
  if (check_opts(lift_order, fine_order)) return ORACLE_E_INVALID;
  return serial_impl(p, E, lift_order, fine_order, W0, n_slices, T, V_out);
}
