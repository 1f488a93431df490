/*
 * bgk_oracle.h -- plain FP64 CPU oracle for the multiscale kinetic/fluid
 * parareal method of Laidin & Rey, "A Parareal in time numerical method for
 * the collisional Vlasov equation in the hyperbolic scaling" (arXiv 2502.02704).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source, header, table or helper with the HIP library.
 *
 * Setting: 1D in x, 3D in v, hydrodynamic scaling (alpha = 0), no exterior
 * force (E = 0), BGK collision operator with tau = 1 so that the total
 * relaxation rate is 1/eps (the IMEX scheme of Section 3.1).
 *
 * Layouts (all row-major, last index fastest):
 *   f  : [nx][nvx][nvy][nvz]   phase-space cell values
 *   W  : [nx][5]  primitive moments  (rho, u_x, u_y, u_z, theta)
 *   V  : [nx][5]  conserved moments  (rho, rho u_x, rho u_y, rho u_z, E)
 *        with E = 1/2 rho |u|^2 + 3/2 rho theta (Section 1, energy relation)
 *
 * Every function returns 0 on success, -1 on invalid arguments and -2 when
 * a non-physical state (rho <= 0, theta <= 0 or NaN) is met.  Nothing is
 * clamped.
 */
#ifndef BGK_ORACLE_H
#define BGK_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_OK 0
#define ORACLE_E_INVALID (-1)
#define ORACLE_E_NONPHYSICAL (-2)

typedef struct {
  int32_t nx;          /* number of x cells                                  */
  int32_t nv[3];       /* velocity cells per axis                            */
  double x_lo, x_hi;   /* spatial domain                                     */
  double v_lo[3];      /* truncated velocity box, per axis                   */
  double v_hi[3];
  int32_t bc;          /* 0: Neumann (zero-gradient ghost), 1: periodic      */
  double eps;          /* Knudsen number; +inf means free transport          */
  double cfl;          /* Courant number for both fine and coarse steps      */
  double sound_gamma;  /* coarse sound speed c = sqrt(gamma * theta)         */
} bgk_oracle_problem;

/* Number of uniform fine steps for a span: dt_stab = cfl*dx/max|v_x| at the
 * velocity cell centres (Section 2.2, local step rule), n = ceil(span/dt_stab
 * - 1e-9), dt = span/n. */
int bgk_oracle_n_steps(const bgk_oracle_problem* p, double t_span,
                       int32_t* n_steps, double* dt);

/* Discrete lifting (Section 3.3): pointwise Maxwellian at velocity centres. */
int bgk_oracle_lift(const bgk_oracle_problem* p, const double* W, double* f);

/* Discrete projection (Definition 1, Section 3.3), literal two-pass form.
 * V (conserved) and/or W (primitive) may be NULL. */
int bgk_oracle_moments(const bgk_oracle_problem* p, const double* f,
                       double* V, double* W);

/* Upwind transport in x (Section 3.1 fluxes), f_star = f - dt/dx (F+ - F-). */
int bgk_oracle_transport(const bgk_oracle_problem* p, const double* f,
                         double dt, double* f_star);

/* Implicit BGK relaxation with explicit moments (Section 3.1):
 * f_out = (f_star + lambda M[P f_star]) / (1 + lambda), lambda = dt/eps. */
int bgk_oracle_relax(const bgk_oracle_problem* p, const double* f_star,
                     double dt, double* f_out);

/* n_steps IMEX steps of size dt. */
int bgk_oracle_fine_steps(const bgk_oracle_problem* p, const double* f_in,
                          double* f_out, double dt, int32_t n_steps);

/* Fine propagator over a span, step count from bgk_oracle_n_steps. */
int bgk_oracle_fine_step(const bgk_oracle_problem* p, const double* f_in,
                         double* f_out, double t_span, int32_t* n_steps_out);

/* P F L: lift conserved moments, fine-propagate over the span, project. */
int bgk_oracle_fine_propagate_moments(const bgk_oracle_problem* p,
                                      const double* V_in, double* V_out,
                                      double t_span);

/* Coarse propagator G: Euler equations, Rusanov finite volumes with adaptive
 * CFL substeps (Section 3.2). */
int bgk_oracle_euler_coarse_step(const bgk_oracle_problem* p,
                                 const double* V_in, double* V_out,
                                 double t_span, int32_t* n_sub_out);

/* Optimised parareal, Algorithm 2 (0-based k).  V_out: [n_slices+1][nx][5]
 * final iterate; err_hist: [k_max] successive errors. */
int bgk_oracle_parareal_iterate(const bgk_oracle_problem* p, const double* W0,
                                int32_t n_slices, double T, int32_t k_max,
                                double tol, double* V_out, double* err_hist,
                                int32_t* k_done);

/* Serial chained fine reference U^n = P F L (U^{n-1}); V_out [n_slices+1][nx][5]. */
int bgk_oracle_serial_fine(const bgk_oracle_problem* p, const double* W0,
                           int32_t n_slices, double T, double* V_out);

/* Adjoint of n_steps fine steps of size dt.  f_ckpt holds f at steps
 * 0, ckpt_every, 2*ckpt_every, ...  fbar_T is dL/df at the last step;
 * fbar_0 receives dL/df at step 0; *dlog_eps is incremented by dL/dlog(eps). */
int bgk_oracle_fine_adjoint(const bgk_oracle_problem* p, const double* f_ckpt,
                            int32_t ckpt_every, int32_t n_steps, double dt,
                            const double* fbar_T, double* fbar_0,
                            double* dlog_eps);

/* Adjoint of the lifting with respect to rho only:
 * rhobar_i = sum_j fbar_ij * dM_ij/drho_i. */
int bgk_oracle_lift_adjoint_rho(const bgk_oracle_problem* p, const double* W,
                                const double* fbar, double* rhobar);

/* Exterior force E_i along x at the cell centres (host [nx]; Section 3.1 with
 * E != 0): Rusanov fluxes in v_x with E_max = max_i |E_i|, zero flux through
 * the ends of the v_x range; the shared explicit step satisfies
 * dt (max|v_x|/dx + E_max/dv_x) <= cfl.  The coarse propagator adds the
 * source (0, rho E, 0, 0, rho u_x E).  Same contracts as the names without
 * _force. */
int bgk_oracle_n_steps_force(const bgk_oracle_problem* p, const double* E,
                             double t_span, int32_t* n_steps, double* dt);
int bgk_oracle_transport_force(const bgk_oracle_problem* p, const double* E,
                               const double* f, double dt, double* f_star);
int bgk_oracle_fine_steps_force(const bgk_oracle_problem* p, const double* E,
                                const double* f_in, double* f_out, double dt,
                                int32_t n_steps);
int bgk_oracle_fine_step_force(const bgk_oracle_problem* p, const double* E,
                               const double* f_in, double* f_out, double t_span,
                               int32_t* n_steps_out);
int bgk_oracle_fine_propagate_moments_force(const bgk_oracle_problem* p,
                                            const double* E, const double* V_in,
                                            double* V_out, double t_span);
int bgk_oracle_euler_coarse_step_force(const bgk_oracle_problem* p,
                                       const double* E, const double* V_in,
                                       double* V_out, double t_span,
                                       int32_t* n_sub_out);
int bgk_oracle_parareal_iterate_force(const bgk_oracle_problem* p, const double* E,
                                      const double* W0, int32_t n_slices, double T,
                                      int32_t k_max, double tol, double* V_out,
                                      double* err_hist, int32_t* k_done);
int bgk_oracle_serial_fine_force(const bgk_oracle_problem* p, const double* E,
                                 const double* W0, int32_t n_slices, double T,
                                 double* V_out);

/* Coarse propagator G as the compressible Navier-Stokes system (Section 1,
 * the Chapman-Enskog correction of Euler's equations) with the BGK transport
 * coefficients mu = rho theta, kappa = (5/2) rho theta: Rusanov convective
 * fluxes plus central viscous and heat fluxes, explicit, with the convective
 * and diffusive step limits.  E (host [nx]) may be NULL (no force).  Needs a
 * finite eps.  The parareal variant uses it as G; its fixed point is the
 * same serial fine chain. */
int bgk_oracle_cns_coarse_step(const bgk_oracle_problem* p, const double* E,
                               const double* V_in, double* V_out, double t_span,
                               int32_t* n_sub_out);
int bgk_oracle_parareal_iterate_cns(const bgk_oracle_problem* p, const double* E,
                                    const double* W0, int32_t n_slices, double T,
                                    int32_t k_max, double tol, double* V_out,
                                    double* err_hist, int32_t* k_done);

/* Lifting of order one (Definition 3, L = 1): Maxwellian times
 * (1 - eps P), P the first Chapman-Enskog correction of the BGK operator
 * (its stress and heat flux are the Navier-Stokes ones with mu = rho theta,
 * kappa = 5/2 rho theta), x-derivatives of the primitive moments W by central
 * differences with the boundary condition's ghost cells.  Finite eps only. */
int bgk_oracle_lift_ce(const bgk_oracle_problem* p, const double* W, double* f);

/* General forms: E (host [nx]) may be NULL; coarse 0 = Euler, 1 =
 * Navier-Stokes, 2 = the fine propagator itself as G (a check of the
 * correction: with G = F one iteration reproduces the serial fine chain);
 * lift_order 0 = Maxwellian (Definition 2), 1 = the lifting
 * above; fine_order 1 = the upwind transport of Section 3.1, 2 = with the
 * van Leer limited Lax-Wendroff correction (second order where smooth, TVD).
 * The serial fine chain with the same lifting and order is parareal's fixed
 * point. */
int bgk_oracle_transport_opts(const bgk_oracle_problem* p, const double* E,
                              int32_t fine_order, const double* f, double dt,
                              double* f_star);
int bgk_oracle_fine_steps_opts(const bgk_oracle_problem* p, const double* E,
                               int32_t fine_order, const double* f_in, double* f_out,
                               double dt, int32_t n_steps);
int bgk_oracle_fine_propagate_moments_opts(const bgk_oracle_problem* p,
                                           const double* E, int32_t lift_order,
                                           int32_t fine_order, const double* V_in,
                                           double* V_out, double t_span);
int bgk_oracle_parareal_iterate_opts(const bgk_oracle_problem* p, const double* E,
                                     int32_t coarse, int32_t lift_order,
                                     int32_t fine_order, const double* W0,
                                     int32_t n_slices, double T, int32_t k_max,
                                     double tol, double* V_out, double* err_hist,
                                     int32_t* k_done);
int bgk_oracle_serial_fine_opts(const bgk_oracle_problem* p, const double* E,
                                int32_t lift_order, int32_t fine_order,
                                const double* W0, int32_t n_slices, double T,
                                double* V_out);

void bgk_oracle_set_threads(int n);
int bgk_oracle_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
