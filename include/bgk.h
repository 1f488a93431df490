/*
 * bgk.h -- C ABI of libbgk.so, the MI355X (gfx950) fine kinetic propagator of
 * the multiscale kinetic/fluid parareal method for the collisional Vlasov-BGK
 * equation in the hyperbolic scaling (Laidin & Rey, arXiv 2502.02704).
 *
 * Model (Section 1, Section 3.1): 1D in x, 3D in v, alpha = 0, BGK operator
 * relaxing at rate 1/eps (tau = 1), IMEX scheme with explicit upwind
 * transport in x and implicit relaxation whose n+1 moments come from
 * conservation.  The calls without a suffix have no exterior force; the
 * _force calls add one along x (the Test 3 setting of Section 5.3), the
 * _cns and _opts calls the Navier-Stokes coarse model, the order-one lifting
 * and second-order transport.
 *
 * Conventions shared by every entry point
 *  - Pointers marked [device] are HIP device pointers; [host] are host
 *    pointers.  The caller owns every array and the workspace.  The library
 *    never allocates or frees device memory on these calls.
 *  - Layouts are row-major with the last index fastest:
 *      f : [nx][nv0][nv1][nv2]  FP64 phase-space cell values (v_z fastest)
 *      W : [nx][5]  primitive moments (rho, u_x, u_y, u_z, theta)
 *      V : [nx][5]  conserved moments (rho, rho u_x, rho u_y, rho u_z, E),
 *                   E = rho |u|^2 / 2 + 3 rho theta / 2 (Section 1).
 *    A batch of B arrays of one problem is stored back to back.
 *  - Velocity points are the cell centres v_a(j) = v_lo[a] + (j + 1/2) dv_a of
 *    a uniform truncated box (Section 3); x cells are uniform on [x_lo, x_hi].
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls are enqueued on
 *    it and return without waiting, except where stated.
 *  - `ws`/`ws_bytes`: caller-owned device workspace of at least
 *    bgk_workspace_bytes(prob, op, batch) bytes, 256-byte aligned.  A
 *    workspace may be reused by successive calls on the same stream; calls
 *    that overlap in time on different streams need separate workspaces.
 *  - Return value: BGK_OK or a negative status.  Arguments are validated on
 *    the host before anything is enqueued; then nothing is launched.
 *    Non-physical states met on the device (rho <= 0, theta <= 0, NaN) raise
 *    a sticky flag in the workspace; bgk_check(stream) reads and clears the
 *    flags of every workspace used on a stream, bgk_status(ws) one of them.
 *  - Caches between calls (captured HIP graphs, tuned tile shapes, the
 *    workspaces each stream used since its last check) live in a plan:
 *    the library's default plan, or one the caller creates and selects with
 *    bgk_plan_use (see "plans" below).
 */
#ifndef BGK_H
#define BGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BGK_OK 0
#define BGK_E_INVALID (-1)     /* bad argument: null, nx < 2, nv < 1, eps <= 0 or
                                  NaN, cfl outside (0,1], empty box, aliasing */
#define BGK_E_NONPHYSICAL (-2) /* rho <= 0, theta <= 0 or NaN met on the device */
#define BGK_E_WORKSPACE (-3)   /* ws NULL, misaligned or smaller than required */
#define BGK_E_HIP (-4)         /* a HIP runtime call failed; see bgk_last_error */

/* Problem statement (Section 1 and Section 3): Knudsen number, spatial
 * domain with its boundary condition, truncated velocity grid.  Must match
 * the oracle's field order. */
typedef struct bgk_problem {
  int32_t nx;          /* x cells, >= 2                                        */
  int32_t nv[3];       /* velocity cells per axis, 1..256                     */
  double x_lo, x_hi;   /* spatial domain                                      */
  double v_lo[3];      /* velocity box per axis                               */
  double v_hi[3];
  int32_t bc;          /* 0: Neumann zero-gradient ghost cells, 1: periodic   */
  double eps;          /* Knudsen number in (0, +inf]; +inf = free transport  */
  double cfl;          /* Courant number of both propagators, in (0, 1]       */
  double sound_gamma;  /* coarse sound speed c = sqrt(sound_gamma * theta)    */
} bgk_problem;

/* Operation selectors for bgk_workspace_bytes. */
#define BGK_OP_FINE_STEP 0    /* bgk_fine_step / bgk_fine_steps               */
#define BGK_OP_MOMENTS 1      /* bgk_moments                                   */
#define BGK_OP_LIFT 2         /* bgk_lift                                      */
#define BGK_OP_COARSE 3       /* euler_coarse_step                             */
#define BGK_OP_PROPAGATE 4    /* bgk_fine_propagate_moments (batch = slices)   */
#define BGK_OP_PARAREAL 5     /* parareal_iterate / bgk_serial_fine (batch =
                                 number of slices)                             */
#define BGK_OP_ADJOINT 6      /* bgk_fine_adjoint (batch = ckpt_every)         */

/* Workspace size in bytes for `op` on `prob` with `batch` members (>= 1).
 * Returns 0 on invalid arguments. */
size_t bgk_workspace_bytes(const bgk_problem* prob, int32_t op, int32_t batch);

/* Fine step count for a span (Section 2.2, local step rule): dt_stab =
 * cfl * dx / max_j |v_x(j)|, n = ceil(t_span / dt_stab - 1e-9), dt = t_span/n.
 * Independent of the data and of eps (the relaxation is implicit).
 * [host] n_steps, dt. */
int bgk_n_steps(const bgk_problem* prob, double t_span, int32_t* n_steps,
                double* dt);

/* Discrete lifting (Definition 2, Section 3.3): f_ij = M[W_i](v_j), the
 * pointwise Maxwellian rho (2 pi theta)^{-3/2} exp(-|v - u|^2 / (2 theta)).
 * [device] W [nx][5] primitive, f [nx][nv3] output. */
int bgk_lift(const bgk_problem* prob, const double* W, double* f, void* ws,
             size_t ws_bytes, void* stream);

/* Discrete projection (Definition 1, Section 3.3), first-order quadrature:
 * rho = sum_j f dv^3, rho u = sum_j v f dv^3, E = sum_j |v|^2/2 f dv^3.
 * [device] f [nx][nv3]; V [nx][5] conserved output (nullable); W [nx][5]
 * primitive output (nullable), theta = (2E/rho - |u|^2)/3. */
int bgk_moments(const bgk_problem* prob, const double* f, double* V, double* W,
                void* ws, size_t ws_bytes, void* stream);

/* n_steps IMEX steps of size dt (Section 3.1):
 *   f* = f - dt/dx (F_{i+1/2} - F_{i-1/2}),
 *   F_{i+1/2,j} = max(v_x,0) f_ij + min(v_x,0) f_{i+1,j},
 *   f^{n+1} = (f* + lambda M[P f*]) / (1 + lambda),  lambda = dt / eps.
 * Ghost cells per prob->bc.  [device] f_in, f_out [nx][nv3]; they must not
 * overlap.  n_steps >= 0 (0 copies f_in). */
int bgk_fine_steps(const bgk_problem* prob, const double* f_in, double* f_out,
                   double dt, int32_t n_steps, void* ws, size_t ws_bytes,
                   void* stream);

/* Fine propagator over t_span with the step count of bgk_n_steps.
 * [host] n_steps_out (nullable). */
int bgk_fine_step(const bgk_problem* prob, const double* f_in, double* f_out,
                  double t_span, int32_t* n_steps_out, void* ws,
                  size_t ws_bytes, void* stream);

/* Uneven batch of independent problems, batched launches over the instances
 * still stepping: instance q advances f_in[q] -> f_out[q] by t_span[q] with
 * its own grid, eps and step count.  With two or more steps per pass set
 * (bgk_set_step_fusion), every instance takes its first step alone and then
 * two steps per pass (one step where one is left) on paired lanes: those
 * with even nv[2] in place (f_in[q], f_out[q] 16-byte aligned, else on
 * unpaired lanes), those with odd nv[2] on a copy in the workspace whose z
 * rows carry one extra point above the box with a zero Maxwellian factor
 * (f stays zero there; f_out[q] receives the live points only).  With one
 * step per pass set, one step per launch.  The results equal one step per
 * launch to rounding.  [host] probs[n], f_in[n], f_out[n] (arrays of
 * [device] pointers), t_span[n], n_steps_out[n] (nullable).  ws: at least
 * bgk_workspace_bytes_batched(probs, n) (two padded fields per instance with
 * odd nv[2], one field per other instance, and per-cell scratch). */
size_t bgk_workspace_bytes_batched(const bgk_problem* probs, int32_t n);
int bgk_fine_step_batched(const bgk_problem* probs, int32_t n,
                          const double* const* f_in, double* const* f_out,
                          const double* t_span, int32_t* n_steps_out, void* ws,
                          size_t ws_bytes, void* stream);

/* Steps 5-7 of Algorithm 2 for a batch of slices: V_out[b] =
 * P F L(V_in[b]) over t_span (lift, fine propagation, projection), all
 * members in one launch per pass.  From the Maxwellian lift (order 0), with
 * no exterior force and first-order transport, the last steps are not
 * written out as f: under triples two for n = 2 mod 3, n >= 5 (after a first
 * three-step pass from the lift), else (n - 2) mod 3 for n >= 4 (after a
 * first two-step pass); under quads (n - 4) mod 4; one for odd n >= 3 under
 * pairs.  Their moments, and the projection, follow from moment sums of the
 * last stored field weighted by 1 and powers of max(+-nu,0) (transport
 * being linear); V_out equals advancing f through every step to rounding.
 * The same holds for parareal_iterate and bgk_serial_fine.  [device] V_in,
 * V_out [batch][nx][5] conserved; may not overlap. */
int bgk_fine_propagate_moments(const bgk_problem* prob, int32_t batch,
                               const double* V_in, double* V_out, double t_span,
                               void* ws, size_t ws_bytes, void* stream);

/* Coarse propagator G (Section 3.2): Euler equations in conserved variables
 * with Rusanov fluxes H = (h_L + h_R)/2 - S/2 (V_R - V_L), S = max(|u_x| + c),
 * c = sqrt(sound_gamma theta), adaptive substeps dt = min(cfl dx / max(|u_x|+c),
 * remaining span).  [device] V_in, V_out [batch][nx][5] (may alias);
 * n_sub_out [batch] substep counts (nullable). */
int euler_coarse_step(const bgk_problem* prob, int32_t batch, const double* V_in,
                      double* V_out, double t_span, int32_t* n_sub_out, void* ws,
                      size_t ws_bytes, void* stream);

/* Optimised parareal, Algorithm 2 (iterations counted from 0): coarse guess
 * U^{n,0} = G(U^{n-1,0}); iteration k computes the jumps
 * Delta^n = P F L(U^{n-1,k}) - G(U^{n-1,k}) for n = k+1..N in one batched
 * fine launch per step, then the sequential correction
 * U^{n,k+1} = G(U^{n-1,k+1}) + Delta^n (slices n <= k are frozen), and the
 * successive error max_{n,i,c} |U^{n,k+1} - U^{n,k}|.  Stops after k_max
 * iterations or when the error is below tol.
 * [device] W0 [nx][5] primitive initial moments; V_out [n_slices+1][nx][5]
 * conserved final iterate.  [host] err_hist [k_max], k_done.
 * Synchronises `stream` once per iteration (error readback). */
int parareal_iterate(const bgk_problem* prob, const double* W0,
                     int32_t n_slices, double T, int32_t k_max, double tol,
                     double* V_out, double* err_hist, int32_t* k_done, void* ws,
                     size_t ws_bytes, void* stream);

/* The fine reference that parareal converges to (Section 2.2: N iterations
 * reproduce it): U^n = P F L(U^{n-1}), one slice at a time with the same
 * kernels.  [device] W0 [nx][5]; V_out [n_slices+1][nx][5]. */
int bgk_serial_fine(const bgk_problem* prob, const double* W0, int32_t n_slices,
                    double T, double* V_out, void* ws, size_t ws_bytes,
                    void* stream);

/* ------------------------------------------------------ exterior force --
 * Section 3.1 with E != 0: the step also transports in v_x under an exterior
 * force E_i per x cell,
 *   f* -= dt/dv_x (G_{i,j+1/2} - G_{i,j-1/2}),
 *   G_{i,j+1/2} = E_i/2 (f_ij + f_i,j+1) - e_max/2 (f_i,j+1 - f_ij),
 * j+1 the next v_x point at the same (v_y, v_z), no flux through the ends of
 * the v_x range (mass is conserved); the printed dissipation term is read as
 * this Rusanov one.  The explicit step satisfies
 * dt (max|v_x|/dx + e_max/dv_x) <= cfl.  The coarse propagator adds the
 * source (0, rho E, 0, 0, rho u_x E) to the Euler system (Section 3.2).
 * [device] E [nx] at the x-cell centres, read during the call (and by the
 * replays of captured sequences: keep it alive and unchanged while a
 * workspace is reused with it).  e_max: host scalar, the Rusanov coefficient,
 * which must be >= max_i |E_i| (checked on the device: a violation or a
 * non-finite E_i makes bgk_status return BGK_E_INVALID).  Steps run one per
 * pass on the generic lane mapping.  Arguments, workspaces (same BGK_OP_*
 * sizes) and errors otherwise as the functions without _force. */
int bgk_n_steps_force(const bgk_problem* prob, double e_max, double t_span,
                      int32_t* n_steps, double* dt);
/* The Rusanov coefficient e_max = max_i |E_i| of a force (NaN if an E_i is
 * NaN).  E [device] when E_on_device is nonzero (read on `stream`, which is
 * synchronised), else [host]; [host] e_max. */
int bgk_force_bound(const bgk_problem* prob, const double* E, int32_t E_on_device,
                    double* e_max, void* stream);
int bgk_fine_steps_force(const bgk_problem* prob, const double* E, double e_max,
                         const double* f_in, double* f_out, double dt,
                         int32_t n_steps, void* ws, size_t ws_bytes, void* stream);
int bgk_fine_step_force(const bgk_problem* prob, const double* E, double e_max,
                        const double* f_in, double* f_out, double t_span,
                        int32_t* n_steps_out, void* ws, size_t ws_bytes,
                        void* stream);
int bgk_fine_propagate_moments_force(const bgk_problem* prob, const double* E,
                                     double e_max, int32_t batch,
                                     const double* V_in, double* V_out,
                                     double t_span, void* ws, size_t ws_bytes,
                                     void* stream);
int euler_coarse_step_force(const bgk_problem* prob, const double* E,
                            int32_t batch, const double* V_in, double* V_out,
                            double t_span, int32_t* n_sub_out, void* ws,
                            size_t ws_bytes, void* stream);
int parareal_iterate_force(const bgk_problem* prob, const double* E, double e_max,
                           const double* W0, int32_t n_slices, double T,
                           int32_t k_max, double tol, double* V_out,
                           double* err_hist, int32_t* k_done, void* ws,
                           size_t ws_bytes, void* stream);
int bgk_serial_fine_force(const bgk_problem* prob, const double* E, double e_max,
                          const double* W0, int32_t n_slices, double T,
                          double* V_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------- Navier-Stokes coarse model --
 * The compressible Navier-Stokes system of Section 1 (the first-order
 * Chapman-Enskog correction of Euler's equations) with the BGK transport
 * coefficients of the relaxation rate 1/eps: viscosity eps*mu, mu = rho
 * theta, heat conductivity eps*kappa, kappa = (5/2) rho theta (Prandtl number
 * 1); in 1D-3V sigma_xx = (4/3) du_x/dx, sigma_xy = du_y/dx, sigma_xz =
 * du_z/dx.  Rusanov convective fluxes plus central viscous and heat face
 * fluxes (face coefficients the mean of the two cells), explicit, with
 * dt = min(cfl dx / max(|u_x| + c), cfl dx^2 / (2 eps (5/3) max theta)).  A
 * finer coarse propagator for parareal (Section 3.2): same fixed point (the
 * serial fine chain), fewer iterations where viscosity matters.  E may be
 * NULL (no force; e_max ignored) or an exterior force as in the _force calls.
 * BGK_E_INVALID for an infinite eps.  Workspaces: BGK_OP_COARSE and
 * BGK_OP_PARAREAL sizes; arguments otherwise as euler_coarse_step and
 * parareal_iterate. */
int euler_coarse_step_cns(const bgk_problem* prob, const double* E, int32_t batch,
                          const double* V_in, double* V_out, double t_span,
                          int32_t* n_sub_out, void* ws, size_t ws_bytes,
                          void* stream);
int parareal_iterate_cns(const bgk_problem* prob, const double* E, double e_max,
                         const double* W0, int32_t n_slices, double T,
                         int32_t k_max, double tol, double* V_out,
                         double* err_hist, int32_t* k_done, void* ws,
                         size_t ws_bytes, void* stream);

/* ------------------------------------------------------ general options --
 * Lifting of order one (Definition 3 with L = 1) for the BGK operator with
 * relaxation rate 1/eps:
 *   f = M[rho,u,theta] (1 - eps P),  c = v - u,
 *   P = (u_x'/theta)(c_x^2 - |c|^2/3) + (u_y'/theta) c_x c_y
 *       + (u_z'/theta) c_x c_z + (theta'/theta) c_x (|c|^2/(2 theta) - 5/2),
 * the first Chapman-Enskog correction (its stress and heat flux are the
 * Navier-Stokes ones with mu = rho theta, kappa = 5/2 rho theta); x-derivatives
 * of the primitive moments by central differences with the boundary
 * condition's ghost cells.  bgk_lift_ce: [device] W [nx][5] primitive, f
 * [nx][nv3] output; BGK_OP_LIFT workspace; BGK_E_INVALID for an infinite eps.
 *
 * bgk_options selects, for the propagate / parareal / serial-fine calls, an
 * exterior force (E device [nx] or NULL, e_max as in the _force calls), the
 * coarse model (BGK_COARSE_EULER: Section 3.2; BGK_COARSE_NAVIER_STOKES: the
 * Navier-Stokes model above) and the lifting order (0: Definition 2's
 * Maxwellian; 1: the order-one lifting, which the fine propagator then starts
 * from; the serial fine chain with the same order is parareal's fixed point).
 * fine_order 2 gives the fine propagator second order in x: the upwind flux
 * with the Lax-Wendroff correction limited by van Leer's limiter (the flux
 * limiters Section 3.1 names as the natural improvement),
 *   v_x > 0: F_{i+1/2} = v_x [f_i + (1-nu)/2 L(f_i - f_{i-1}, f_{i+1} - f_i)],
 *   v_x < 0: F_{i+1/2} = v_x [f_{i+1} - (1-|nu|)/2 L(f_{i+2} - f_{i+1}, f_{i+1} - f_i)],
 * L(a, b) = 2ab/(a+b) if ab > 0 else 0, nu = v_x dt/dx, ghost cells two deep;
 * TVD for |nu| <= 1; it runs one step per pass on the generic lane mapping
 * (2 or 4 velocities per lane: a tile override of 8 runs as 4), or with the
 * exterior force on v_x columns.  bgk_fine_steps_opts is bgk_fine_steps with
 * these options (the coarse and lift fields are ignored there).
 * A NULL options pointer means no force, Euler, order 0 lift, order 1
 * transport.  Workspaces and the other arguments as bgk_fine_steps,
 * bgk_fine_propagate_moments, parareal_iterate and bgk_serial_fine. */
enum { BGK_COARSE_EULER = 0, BGK_COARSE_NAVIER_STOKES = 1 };
typedef struct {
  const double* E;    /* exterior force at the x centres, or NULL */
  double e_max;       /* Rusanov coefficient >= max |E_i| (ignored without E) */
  int32_t coarse;     /* BGK_COARSE_EULER or BGK_COARSE_NAVIER_STOKES */
  int32_t lift_order; /* 0 or 1 */
  int32_t fine_order; /* x transport: 1 (or 0) upwind; 2 van Leer limited */
  int32_t reserved;   /* 0 */
} bgk_options;

int bgk_lift_ce(const bgk_problem* prob, const double* W, double* f, void* ws,
                size_t ws_bytes, void* stream);
int bgk_fine_steps_opts(const bgk_problem* prob, const bgk_options* opts,
                        const double* f_in, double* f_out, double dt,
                        int32_t n_steps, void* ws, size_t ws_bytes, void* stream);
int bgk_fine_propagate_moments_opts(const bgk_problem* prob, const bgk_options* opts,
                                    int32_t batch, const double* V_in,
                                    double* V_out, double t_span, void* ws,
                                    size_t ws_bytes, void* stream);
int parareal_iterate_opts(const bgk_problem* prob, const bgk_options* opts,
                          const double* W0, int32_t n_slices, double T,
                          int32_t k_max, double tol, double* V_out,
                          double* err_hist, int32_t* k_done, void* ws,
                          size_t ws_bytes, void* stream);
int bgk_serial_fine_opts(const bgk_problem* prob, const bgk_options* opts,
                         const double* W0, int32_t n_slices, double T,
                         double* V_out, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of n_steps IMEX steps of size dt (the transpose of the step's
 * Jacobian: transposed upwind stencil, adjoint of moments -> Maxwellian ->
 * relaxation).  [device] f_ckpt [ceil(n_steps/ckpt_every)][nx][nv3] forward
 * states at steps 0, ckpt_every, ...; fbar_T [nx][nv3] dL/df(final);
 * fbar_0 [nx][nv3] output dL/df(0) (must not overlap fbar_T);
 * dlog_eps [1] incremented by dL/dlog(eps).  Recomputes each segment of
 * ckpt_every forward states (ws sized with batch = ckpt_every). */
int bgk_fine_adjoint(const bgk_problem* prob, const double* f_ckpt,
                     int32_t ckpt_every, int32_t n_steps, double dt,
                     const double* fbar_T, double* fbar_0, double* dlog_eps,
                     void* ws, size_t ws_bytes, void* stream);

/* Adjoint of the lifting in rho (Definition 2: M is linear in rho):
 * rhobar_i = sum_j fbar_ij M[W_i](v_j) / rho_i.  [device] W [nx][5],
 * fbar [nx][nv3], rhobar [nx]. */
int bgk_lift_adjoint_rho(const bgk_problem* prob, const double* W,
                         const double* fbar, double* rhobar, void* ws,
                         size_t ws_bytes, void* stream);

/* Adjoint of the density of the discrete projection (Definition 1):
 * rho_i = sum_j f_ij dv^3, so fbar_ij = rhobar_i dv^3.
 * [device] rhobar [nx], fbar [nx][nv3] output.  Needs no workspace. */
int bgk_density_adjoint(const bgk_problem* prob, const double* rhobar,
                        double* fbar, void* stream);

/* ---------------------------------------------- allocation-free variant --
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  bgk_fine_propagate_moments (same V_in, V_out, batch, t_span
 * and results, bitwise) with its workspace in a static device array of
 * BGK_NOALLOC_SCRATCH_BYTES per device, held from the library's first call
 * on that device until the process ends.  The call allocates nothing and
 * records no timing events.  Limit: bgk_workspace_bytes(prob,
 * BGK_OP_PROPAGATE, batch) <= BGK_NOALLOC_SCRATCH_BYTES (for 64 x 16^3
 * cells, up to 14 members), else BGK_E_WORKSPACE before anything is enqueued.
 * status [device] (nullable): after the call's kernels, receives BGK_OK or
 * BGK_E_NONPHYSICAL for the states this call met (the sticky word is cleared
 * at the start of every call).  All calls on one device share its array:
 * calls that overlap in time on one device (different streams, threads or
 * replays in flight together) race and must be serialised by the caller. */
#define BGK_NOALLOC_SCRATCH_BYTES (64u << 20)
int bgk_fine_propagate_moments_noalloc(const bgk_problem* prob, int32_t batch,
                                       const double* V_in, double* V_out,
                                       double t_span, int32_t* status, void* stream);

/* Synchronises `stream`, returns and clears the sticky device status in ws:
 * BGK_OK, BGK_E_NONPHYSICAL, or BGK_E_INVALID for an exterior force that
 * exceeds e_max or is not finite. */
int bgk_status(void* ws, void* stream);

/* Synchronises `stream`, then reads and clears the sticky status of every
 * workspace that calls of the calling thread's plan enqueued on `stream`
 * since the last bgk_check(stream), and returns the first non-OK one
 * (statuses as bgk_status).  Those workspaces must still be allocated: call
 * it before freeing a workspace that calls on the stream used. */
int bgk_check(void* stream);

/* ------------------------------------------------------------------ plans --
 * A plan holds what the library keeps between calls: the HIP graphs captured
 * for launch-bound sequences (parareal iterations, the serial fine chain,
 * the uneven batch, the adjoint), the tile shapes bgk_autotune chose, and
 * the workspaces bgk_check will read.  Every thread starts on the library's
 * default plan, which lives until the library is unloaded.
 * bgk_plan_create: a new, empty plan ([host] *plan receives it).
 * bgk_plan_use: makes `plan` the one the calling thread's later calls use
 *   (NULL: the default plan again).
 * bgk_plan_destroy: synchronises the device, destroys the plan's graphs and
 *   frees it; the calling thread returns to the default plan if it used it;
 *   other threads must have stopped using it.  NULL is a no-op.
 * bgk_plan_info: [host] graphs and tuned tile shapes a plan holds (plan NULL:
 *   the calling thread's plan); outputs nullable.
 * bgk_plan_save_tiles / bgk_plan_load_tiles: the tuned tile shapes as a JSON
 *   file, entries keyed by (device architecture, nv[3], nx and batch rounded
 *   up to powers of two, steps per pass); load merges the entries measured
 *   on the current device's architecture into the plan (plan NULL: the
 *   calling thread's plan).  BGK_E_INVALID for a file that cannot be opened
 *   or parsed. */
typedef struct bgk_plan bgk_plan;
int bgk_plan_create(bgk_plan** plan);
int bgk_plan_use(bgk_plan* plan);
int bgk_plan_destroy(bgk_plan* plan);
int bgk_plan_info(const bgk_plan* plan, int32_t* n_graphs, int32_t* n_tiles);
int bgk_plan_save_tiles(const bgk_plan* plan, const char* path);
int bgk_plan_load_tiles(bgk_plan* plan, const char* path);

const char* bgk_status_string(int status);

/* Message of the last failing call on this thread ("" if none). */
const char* bgk_last_error(void);

/* Tile shape of the fused step kernel: velocity elements per lane (2, 4 or 8)
 * and x cells per work item (1..64); 0 restores the built-in choice.  pair:
 * 1 = lanes own pairs of adjacent v_z cells (used only when nv[2] is even and
 * f is 16-byte aligned), 0 = one velocity per lane slot, -1 = built-in,
 * 2 = the exterior-force step on v_x columns (a lane owns one (v_y, v_z)
 * point and elems consecutive v_x points) even where nv[1] nv[2] < 64, 3 =
 * the same with two adjacent (v_y, v_z) points per lane (even nv[1] nv[2],
 * 16-byte aligned f, elems 2 or 4); the built-in choice takes columns, paired
 * where it can, when nv[1] nv[2] >= 64, and 0 keeps that step on the flat
 * mapping. */
int bgk_set_tiles(int32_t elems_per_lane, int32_t x_chunk, int32_t pair);

/* Times candidate tile shapes on `prob` with `batch` members (nine fine
 * steps from a lift: whole two- and three-step passes; uses ws of
 * BGK_OP_PROPAGATE size; synchronises) and keeps the fastest in the calling
 * thread's plan for problems of the same velocity grid, nx and batch
 * rounded up to powers of two, and steps per pass.  The candidates are the
 * built-in choice, 2, 4 or 8 velocities per lane by 1 to 48-cell chunks,
 * paired or not, and the longest three-step chunks the LDS holds; shapes
 * whose passes need more than 160 KB of LDS are skipped.  [host]
 * best_elems, best_chunk, best_pair (nullable). */
int bgk_autotune(const bgk_problem* prob, int32_t batch, void* ws,
                 size_t ws_bytes, void* stream, int32_t* best_elems,
                 int32_t* best_chunk, int32_t* best_pair);

/* IMEX steps per pass over f: 2 runs pairs of steps in one
 * read-write pass (8 bytes per update instead of 16; the second step's
 * moments follow by linearity of the transport from moment sums of the
 * previous field weighted by max(nu,0) and max(-nu,0), nu = v_x dt/dx);
 * 3 (default) runs triples (16/3 bytes per update; the third step's moments need the
 * sums weighted by max(nu,0)^2 and max(-nu,0)^2 too) where every velocity tile
 * lies in one v_x plane (nv[1] nv[2] a multiple of 64 times the velocities
 * per lane), nx >= 3 and the paired lane mapping is used (even nv[2],
 * 16-byte aligned f), else pairs (paired or unpaired lanes); 4 runs quads
 * (4 bytes per update; sums weighted to the third power) on grids where
 * nv[1] nv[2] is a multiple of 128, nx >= 4 and lanes are paired, with one
 * velocity pair per lane, else as 3; a call that returns moments closes the
 * n - 4 mod 4 steps after its last quad on the moments.  1 runs one step per
 * pass.  The exterior-force step and the second-order transport always run
 * one step per pass; the uneven batch (bgk_fine_step_batched) runs pairs
 * under 2, 3 and 4. */
int bgk_set_step_fusion(int32_t steps_per_pass);

/* Launch-bound sequences (each parareal iteration, the serial chain of
 * bgk_serial_fine) are captured as HIP graphs on first use and replayed;
 * 0 turns this off (every kernel launched on the stream directly), 1 on
 * (default).  Kernel timing (bgk_prof_enable) always launches directly. */
int bgk_set_graphs(int32_t on);

/* Destroys every graph cached in the calling thread's plan, after
 * synchronising the device (none cached: returns at once, no device call).
 * Graphs are keyed by the workspace, the problem, the launch parameters and
 * the device pointers they read, so later calls capture again; call it
 * before freeing workspaces to give the graphs' resources back.  [host] */
int bgk_release_graphs(void);

/* Kernel timing of the step kernels: when on, every launch of one is
 * bracketed by HIP events on its stream and tagged with its kind:
 *   BGK_PROF_TWO_STEP       two IMEX steps per pass, reading and writing f
 *                           (16 algorithmic bytes per cell per pass)
 *   BGK_PROF_TWO_STEP_LIFT  two steps from the lifted Maxwellian (writes f
 *                           only: 8 bytes per cell per pass)
 *   BGK_PROF_ONE_STEP       one step per pass (16 bytes per cell; 8 for the
 *                           first step of a slice, which computes the lifted
 *                           Maxwellian instead of reading it)
 *   BGK_PROF_THREE_STEP     three IMEX steps per pass, reading and writing f
 *                           (16 algorithmic bytes per cell per pass)
 *   BGK_PROF_THREE_STEP_LIFT three steps from the lifted Maxwellian (8)
 *   BGK_PROF_FOUR_STEP      four IMEX steps per pass, reading and writing f (16)
 *   BGK_PROF_FOUR_STEP_LIFT four steps from the lifted Maxwellian (8)
 * bgk_prof_read synchronises and returns, over the launches of `kind`
 * (BGK_PROF_ALL: every kind) since the last bgk_prof_enable(1), the summed
 * milliseconds, the launch count, the phase-space updates (cells times steps)
 * and the algorithmic bytes moved.  [host] outputs, each nullable.
 * BGK_E_INVALID for an unknown kind. */
enum {
  BGK_PROF_ALL = 0,
  BGK_PROF_TWO_STEP = 1,
  BGK_PROF_TWO_STEP_LIFT = 2,
  BGK_PROF_ONE_STEP = 3,
  BGK_PROF_THREE_STEP = 4,
  BGK_PROF_THREE_STEP_LIFT = 5,
  BGK_PROF_FOUR_STEP = 6,
  BGK_PROF_FOUR_STEP_LIFT = 7
};
int bgk_prof_enable(int32_t on);
int bgk_prof_read(int32_t kind, double* total_ms, int64_t* launches, double* updates,
                  double* bytes);

#ifdef __cplusplus
}
#endif
#endif
