/*
 * fvib -- one time step of an incompressible finite-volume solver with
 * immersed-boundary fluid-structure coupling, and its discrete adjoint,
 * for AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Fan, Liu, Wang & Wang, "Diff-FlowFSI: A
 * GPU-Optimized Differentiable CFD Platform for High-Fidelity Turbulence
 * and FSI Simulations" (arXiv 2505.23940):
 *   - staggered finite volumes on a rectangular, uniform or stretched grid
 *     (Sec. 2.3.1), periodic / Dirichlet / Neumann boundaries (Sec. 2.5,
 *     Table 1);
 *   - forward-Euler predictor with central or upwind convection and central
 *     diffusion (Eq. 4), direct-forcing IBM (Eq. 5);
 *   - modified pressure Poisson equation (Eq. 9) and correction (Eq. 10);
 *   - 4-point-kernel transfers between markers and the grid (Eqs. 18-22);
 *   - rigid spring-damper body integrated with RK4 (Eq. 12);
 *   - one weakly coupled step = Alg. 1 with N = 1;
 *   - reverse-mode gradients (Sec. 2.4.1), here as a hand-written discrete
 *     adjoint of every sub-step with the Poisson adjoint taken through the
 *     implicit function theorem (Eq. 24).
 *
 * Conventions common to every call
 * --------------------------------
 * Layout.  Velocity component c (0 = u, 1 = v, 2 = w) lives on the faces
 * normal to axis c; the face with index i along axis c is the low face of
 * cell i.  Arrays are dense and C-contiguous in (z, y, x) order, x fastest.
 * Along its own axis a component has n[c] faces on a periodic axis and
 * n[c] + 1 faces otherwise; along the other axes it has n[a] entries.
 * Pressure is cell-centred, shape (n[2], n[1], n[0]).  2D grids use
 * dim = 2, n[2] = 1 and two components.  fvib_field_layout() returns the
 * exact shapes.
 *
 * Precision.  FVIB_PREC_FP64: velocities, forcing fields and all
 * arithmetic are double.  FVIB_PREC_FP32_MIXED: velocities and forcing
 * fields are float and the stencils run in float, while the Poisson
 * residual, its iterative-refinement correction, the pressure and every
 * global reduction are double.  Pressure and body state are always double.
 *
 * Memory.  Pointers in fvib_fields / fvib_adjoint / fvib_step_info are
 * device pointers owned by the caller; the library never frees them.  The
 * library owns the handle and its workspace.  Host pointers in the
 * descriptors are read during the call only.
 *
 * Streams.  All device work is enqueued on the HIP stream given at
 * creation.  fvib_step / fvib_step_adjoint synchronise that stream only to
 * poll the convergence of the Poisson solve (every check_every
 * iterations); results are ready when the stream is.
 *
 * Errors.  Every call returns FVIB_OK (0) or a negative status.  Invalid
 * arguments are reported before any work is enqueued.  Device-side
 * conditions (no convergence, non-finite residual) are reported in the
 * returned status and in info->status, and the message is available from
 * fvib_last_error().  A handle must not be used from two threads at once.
 */
#ifndef FVIB_H
#define FVIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fvib_grid fvib_grid;   /* opaque handle owned by the library */

enum {
  FVIB_OK = 0,
  FVIB_EINVAL = -1,      /* invalid argument or descriptor               */
  FVIB_ENOMEM = -2,      /* device or host allocation failed             */
  FVIB_EHIP = -3,        /* a HIP runtime call failed                    */
  FVIB_ENOCONV = -4,     /* Poisson solve did not reach poisson_tol      */
  FVIB_ENONFINITE = -5,  /* NaN / Inf met in a global reduction          */
  FVIB_ESTATE = -6       /* call out of order (e.g. no body set)         */
};

/* Boundary kinds (Table 1 of the paper).  The velocity vector of each
 * boundary is given in fvib_grid_desc.bc_vel. */
enum {
  FVIB_BC_PERIODIC = 0,           /* must be paired on both sides of an axis   */
  FVIB_BC_NOSLIP = 1,             /* Dirichlet wall, wall velocity bc_vel      */
  FVIB_BC_FREESLIP = 2,           /* zero normal velocity, zero shear          */
  FVIB_BC_INFLOW = 3,             /* Dirichlet velocity bc_vel                 */
  FVIB_BC_OUTFLOW_CONVECTIVE = 4, /* du/dt + U_conv du/dn = 0 on normal faces  */
  FVIB_BC_OUTFLOW_NEUMANN = 5     /* du/dn = 0                                 */
};

enum { FVIB_CONV_CENTRAL2 = 0, FVIB_CONV_UPWIND1 = 1 };
enum { FVIB_PREC_FP64 = 0, FVIB_PREC_FP32_MIXED = 1 };
enum { FVIB_BODY_STATIC = 0, FVIB_BODY_RIGID_SPRING = 1 };
/* Pressure solver.  CG: conjugate gradients (the paper's solver; double
 * CG, or float CG inside double iterative refinement).  FDM: exact fast
 * diagonalisation of the separable operator (per-axis eigenbases applied as
 * dense contractions on the matrix cores) inside the same double-residual
 * refinement; both stop on the same double-precision divergence test. */
enum { FVIB_SOLVER_CG = 0, FVIB_SOLVER_FDM = 1 };
enum { FVIB_DTYPE_F32 = 0, FVIB_DTYPE_F64 = 1 };
/* Time schemes of fvib_step_rk (Sec. 2.3.1, Table 1: forward Euler or an
 * explicit Runge-Kutta scheme), in Shu-Osher form over the forward-Euler
 * step S(v) = P(v + dt R(v)): v_0 = u^n, v_s = a_s u^n + b_s S(v_{s-1}),
 * u^{n+1} = v_S.  FE: (0, 1).  RK2 (Heun): (0, 1), (1/2, 1/2).  RK3 (third
 * order, strong-stability preserving): (0, 1), (3/4, 1/4), (1/3, 2/3). */
enum { FVIB_TIME_FE = 0, FVIB_TIME_RK2 = 1, FVIB_TIME_RK3 = 2 };

/* Grid and solver description (Sec. 2.5 of the paper). */
typedef struct {
  int32_t dim;              /* 2 or 3                                          */
  int32_t n[3];             /* cells per axis; n[2] = 1 when dim = 2           */
  const double *faces[3];   /* host: n[a] + 1 increasing face coordinates;
                               periodic axes must be uniform                   */
  int32_t bc[3][2];         /* boundary kind per axis and side (0 low, 1 high) */
  double bc_vel[3][2][3];   /* velocity vector of each boundary                */
  double nu;                /* kinematic viscosity, > 0                        */
  double rho;               /* density, > 0                                    */
  double dt;                /* time step, > 0                                  */
  double u_conv;            /* convective outflow speed                        */
  int32_t convection;       /* FVIB_CONV_*                                     */
  int32_t precision;        /* FVIB_PREC_*                                     */
  double poisson_tol;       /* stop when max over cells of |div u^{n+1}|,
                               evaluated in double before any rounding to the
                               storage type, is <= poisson_tol (units 1/time) */
  int32_t poisson_maxit;    /* max CG iterations per solve (per refinement
                               sweep in mixed mode)                            */
  int32_t ir_maxit;         /* max refinement sweeps (mixed mode)              */
  double inner_rtol;        /* residual reduction of each float inner solve    */
  int32_t check_every;      /* iterations between convergence polls, >= 1     */
  int32_t solver;           /* FVIB_SOLVER_*: inner solve of the refinement   */
} fvib_grid_desc;

/* Immersed rigid body: a closed polygon of Lagrangian markers (2D only). */
typedef struct {
  int32_t kind;             /* FVIB_BODY_STATIC or FVIB_BODY_RIGID_SPRING      */
  int32_t n_markers;        /* M >= 3                                          */
  const double *X0;         /* host, M x 2 marker positions at zero
                               displacement, counter-clockwise                 */
  const double *ds;         /* host, M arc-length elements                     */
  int32_t free_dof[3];      /* 1 where the translational DOF is free           */
  double m;                 /* body mass (Eq. 12), > 0 for a spring body       */
} fvib_body_desc;

/* Per-step fields (device pointers).  body = [d_x, d_y, d_z, v_x, v_y, v_z]
 * (displacement and velocity, double).  kc = [k_x, k_y, k_z, c_x, c_y, c_z]
 * (double) are the spring stiffness and damping of Eq. 12; fb is an
 * external body force per face (e.g. a driving pressure gradient), may be
 * NULL for zero. */
typedef struct {
  void *u[3];               /* velocity components (dtype per precision)       */
  double *p;                /* pressure; on input the initial guess            */
  const void *fb[3];        /* body-force components or NULL                   */
  double *body;             /* body state (6 doubles), may be NULL w/o body    */
  const double *kc;         /* spring constants (6 doubles), may be NULL       */
} fvib_fields;

/* Adjoint fields (device pointers), same layouts as fvib_fields. */
typedef struct {
  void *u[3];               /* adjoint velocity                                */
  void *fb[3];              /* adjoint body force (accumulated), may be NULL   */
  double *body;             /* adjoint body state (6 doubles)                  */
  double *kc;               /* adjoint spring constants (accumulated, 6)       */
  double *mu;               /* adjoint pressure (cells, like p), may be NULL:  */
                            /* in bar_in, the initial guess of the step's      */
                            /* adjoint Poisson solve on input and its solution */
                            /* on output; NULL starts from zero in workspace   */
} fvib_adjoint;

/* Step diagnostics, written on the stream into device (or host-mapped)
 * memory. 64 bytes. */
typedef struct {
  int32_t status;           /* FVIB_OK or a negative status                    */
  int32_t cg_iters;         /* total CG iterations of the step                 */
  int32_t ir_iters;         /* refinement sweeps (mixed mode), else 0          */
  int32_t flags;            /* bit 0: body window clamped; bits 8-23: coupling
                               sub-iterations of a strongly coupled step (Alg. 1),
                               0 for a weakly coupled one                       */
  double res;               /* final max |div| estimate of the Poisson solve   */
  double div_max;           /* max |D u^{n+1}| in double before storage        */
  double force[3];          /* fluid force on the body F^n (Eq. 20, summed)    */
  double xi;                /* coupling error of the last sub-iteration
                               (strongly coupled step), else 0                 */
} fvib_step_info;

/* Create a grid handle.  Validates the descriptor (paired periodic sides,
 * uniform periodic axes, increasing faces, positive nu / rho / dt), uploads
 * the per-axis metrics and allocates the workspace.  hip_stream is a
 * hipStream_t (NULL = default stream).  On success *out receives the
 * handle; on failure *out is NULL.  The handle also takes one word of
 * coherent pinned host memory, through which the device reports each
 * convergence check of the refinement (Sec. 2.5's Poisson solve) and the
 * host polls it; with FVIB_NO_POLL=1 in the environment at creation (or if
 * that allocation fails) the checks wait on a HIP event instead.  Both
 * take the same decisions and give the same results. */
int fvib_create_grid(const fvib_grid_desc *desc, void *hip_stream, fvib_grid **out);

/* Destroy a handle and release its workspace (synchronises its stream). */
int fvib_destroy_grid(fvib_grid *g);

/* Shape and element strides (z, y, x order) of component comp (0..2) or of
 * the pressure (comp = 3) / a cell field, and its dtype (FVIB_DTYPE_*). */
int fvib_field_layout(const fvib_grid *g, int comp, int64_t shape[3],
                      int64_t strides[3], int *dtype);

/* Attach an immersed body (Sec. 2.2, Fig. 2; Sec. 2.3.3, Eqs. 18-22); NULL removes it.  2D
 * grids with equal uniform spacing h in x and y only.  The body must stay
 * at least four cells away from the domain boundary.  Point classes are
 * rebuilt inside fvib_step from the displacement in the body state. */
int fvib_ib_set_body(fvib_grid *g, const fvib_body_desc *body);

/* Attach a static immersed box to a 3D grid (the cubic roughness elements
 * standing on the channel wall of Sec. 3.4.2, with the direct forcing of
 * Sec. 2.3.1, Eq. 5, and the point classes of Sec. 2.2, Fig. 2); lo = NULL
 * removes it.  lo, hi (host, 3 doubles): the box [lo, hi) per axis; it may
 * reach through a wall.  Point classes per velocity component on its own
 * face points: solid in the half-open box, immersed-boundary point when a
 * six-neighbour is solid; both forced to zero velocity (the body is at
 * rest), except boundary-normal faces of bounded axes, which keep their
 * boundary condition.  The force reported in fvib_step_info.force is the
 * momentum the forcing removes from the fluid, -rho sum f dv over the
 * forced faces (a 3D body has no Lagrangian markers); fvib_step_adjoint's
 * dF is its adjoint.  On a periodic axis the box either spans the axis or
 * stays off its seam (face points 0 and n-1).  No body state: fields.body may be
 * NULL.  FVIB_ESTATE if a marker body is attached (and
 * fvib_ib_set_body fails while a box is). */
int fvib_ib_set_box(fvib_grid *g, const double *lo, const double *hi);

/* Large-eddy simulation model (Sec. 2.5, Table 1; Sec. 3.4.5, Eqs. 27-29). */
typedef struct {
  double cs;                /* Smagorinsky constant C_s >= 0                    */
  int32_t wall_model;       /* 1: equilibrium wall-stress model on the y walls  */
  int32_t reserved;         /* 0                                                */
  double kappa, B;          /* Spalding-law constants (the paper: 0.4, 5)       */
  double eps;               /* Eq. 28 regulariser (the paper: 1e-6)             */
} fvib_les_desc;

/* Enable the subgrid model on a 3D grid whose axes are all periodic or
 * no-slip wall pairs; d = NULL disables it.  Every later step (fvib_step,
 * fvib_step_rk) adds the divergence of the subgrid stress 2 nu_t S to the
 * momentum right-hand side on the evolved faces, nu_t = (C_s Delta)^2 |S|
 * at cell centres (Delta = (dx dy dz)^(1/3), |S| = sqrt(2 S_ij S_ij)),
 * shear stresses on cell edges with the four-cell mean of nu_t and zero
 * viscosity on wall edges; fvib_step_adjoint differentiates it.  With
 * wall_model = 1 (walls normal to y, x and z periodic, n[1] >= 2) the wall
 * edges of u and w get the viscosity of Eq. 28 from the Spalding law
 * (Eq. 27) at the half height of the wall cell, tau_w = u_tau^2 split by
 * Eq. 29 (kinematic stress), the other tangential component averaged from
 * its four nearest faces.  FVIB_EINVAL for a grid or a descriptor outside
 * these rules; allocates its workspace (about 25 cell-sized arrays). */
int fvib_les_set(fvib_grid *g, const fvib_les_desc *d);

/* One weakly coupled time step (Alg. 1 with N = 1): classification and
 * target velocities, predictor with direct forcing (Eqs. 4-5), boundary
 * faces, modified PPE (Eq. 9) solved by conjugate gradients (double, or
 * float inner solves inside double iterative refinement), correction
 * (Eq. 10), loads on the body (Eq. 20) and RK4 body update (Eq. 12).
 * out may alias in (in-place step).  info may be NULL. */
int fvib_step(fvib_grid *g, const fvib_fields *in, fvib_fields *out,
              fvib_step_info *info);

/* Discrete adjoint of fvib_step at the state fwd_in (the masks of the step
 * are frozen).  Its Poisson solve stops at a max-norm residual of 1e-10
 * (double) or 1e-7 (mixed) relative to its right-hand side.  Given the adjoints of the step outputs -- bar_out->u
 * (u^{n+1}), bar_out->body (body state^{n+1}) and dF (3 doubles, device:
 * the direct derivative of the loss with respect to the force F^n reported
 * by the step, may be NULL) -- it writes bar_in->u (u^n) and
 * bar_in->body (body state^n) and adds into bar_in->fb and bar_in->kc.
 * bar_in may not alias bar_out.  The pressure of fwd_in is not used.
 * bar_in->mu (optional) warm-starts the adjoint solve, e.g. with the
 * previous adjoint step's solution along a rollout; a warm start that
 * does not converge within the sweeps its first check allows is dropped
 * and the solve restarts from zero, so the stopping test is the same. */
int fvib_step_adjoint(fvib_grid *g, const fvib_fields *fwd_in,
                      const fvib_adjoint *bar_out, const double *dF,
                      fvib_adjoint *bar_in, fvib_step_info *info);

/* One strongly coupled time step (Alg. 1 with N = max_iters, Sec. 2.3.3):
 * the structural iterate starts at the time level w^n = in->body; each
 * coupling sub-iteration advances the fluid from u^n with the body placed
 * and moving as the current iterate (point classes, target velocities,
 * predictor with direct forcing, Eqs. 4-5, 18-23), takes its loads
 * (Eq. 20) and advances the structure from w^n under them (Eq. 12, RK4)
 * to the next iterate; the coupling error xi = |w_k - w_{k-1}|^2 /
 * max(|w_{k-1}|^2, 1e-30) ends the sub-iterations once xi < tol, or after
 * max_iters (1 <= max_iters <= 65535; max_iters = 1 is fvib_step).  The
 * modified PPE (Eq. 9) and the correction (Eq. 10) do not feed the loads
 * and run once, with the body at the last iterate the fluid saw.  out->body
 * receives the last structural update; omega (device, 6 doubles, may be
 * NULL, may not alias a body state) receives the iterate the fluid saw
 * last, which fvib_step_strong_adjoint needs.  info->flags bits 8-23 hold
 * the sub-iteration count, info->xi the last coupling error.  The host
 * reads the coupling error after each sub-iteration (one stream
 * synchronisation per sub-iteration).  Needs a body (FVIB_ESTATE). */
int fvib_step_strong(fvib_grid *g, const fvib_fields *in, fvib_fields *out, int32_t max_iters,
                     double tol, double *omega, fvib_step_info *info);

/* Adjoint of fvib_step_strong by implicit differentiation of the coupling
 * fixed point (Eq. 24, Sec. 2.4.1), at the iterate omega the forward step
 * returned (point classes frozen at omega).  With Phi(w) the structural
 * update from w^n under the loads of the fluid seen with the body at w,
 * the fixed-point adjoint lam solves (I - dPhi/dw^T) lam = bar_out->body +
 * dL/domega (6 x 6, on the device); u^n, f_b, w^n, k and c then receive the
 * partial derivatives of L + lam . Phi at fixed omega.  Arguments and
 * outputs as in fvib_step_adjoint. */
int fvib_step_strong_adjoint(fvib_grid *g, const fvib_fields *fwd_in, const double *omega,
                             const fvib_adjoint *bar_out, const double *dF,
                             fvib_adjoint *bar_in, fvib_step_info *info);

/* One explicit Runge-Kutta step of the fluid (Sec. 2.3.1 and Table 1; the
 * schemes are listed at FVIB_TIME_*), each stage a forward-Euler step with
 * its own modified PPE solve and correction, the correction writing the
 * stage combination a_s u^n + b_s S(v_{s-1}) itself.  Every stage is
 * divergence free.  Grids without a body (FVIB_ESTATE otherwise: a stage
 * combination would not hold the forced faces at the body velocity).  out
 * may alias in; out->p receives the last stage's pressure (each stage's
 * solve starts from the previous one's).  info: the last stage's record.
 * The first call allocates the Runge-Kutta workspace (six velocity sets and
 * one cell array). */
int fvib_step_rk(fvib_grid *g, const fvib_fields *in, fvib_fields *out, int scheme,
                 fvib_step_info *info);

/* Discrete adjoint of fvib_step_rk at fwd_in (Sec. 2.4.1): the stage inputs
 * are recomputed from fwd_in->u (fwd_in->p, may be NULL, is the solves'
 * initial guess), then each stage's forward-Euler adjoint is applied in
 * reverse order.  Writes bar_in->u, adds into bar_in->fb; bar_in->mu as in
 * fvib_step_adjoint.  bar_in may not alias bar_out. */
int fvib_step_rk_adjoint(fvib_grid *g, const fvib_fields *fwd_in, const fvib_adjoint *bar_out,
                         fvib_adjoint *bar_in, int scheme, fvib_step_info *info);

/* Change the time step of the handle (every later step and adjoint step
 * uses it; Sec. 2.5: fixed or CFL-adaptive time steps). */
int fvib_set_dt(fvib_grid *g, double dt);

/* CFL-adaptive time step from the instantaneous maximum velocity (Sec. 2.5):
 * *dt (host) = min(dt_max, cfl h_min / max |u|), the maximum over every face
 * value of every component (a device reduction) and h_min the smallest cell
 * width; dt_max when u is zero.  Synchronises the stream.  Does not change
 * the handle's time step (fvib_set_dt does). */
int fvib_cfl_dt(fvib_grid *g, const void *const u[3], double cfl, double dt_max, double *dt);

/* Mean wall shear J = (nu/2) [ <u>_lo / (yc_0 - y_0) + <u>_hi / (y_N - yc_{N-1}) ]
 * of the streamwise velocity at the two wall-adjacent rows (walls normal
 * to y, at rest).  Writes J (1 double, device) and, if ubar is not NULL,
 * adds dJ/du into ubar[0] (dtype of the velocity). */
int fvib_loss_wall_shear(fvib_grid *g, const void *u0, double *J, void *ubar0);

/* Allocation-free variant of fvib_loss_wall_shear, for callers that
 * cannot allocate device memory while they run (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results (bit for bit) as fvib_loss_wall_shear;
 * its block partial sums live in a static device array of the library
 * (2 x 2048 doubles, 32 KiB per device, held until the process ends)
 * instead of the handle's workspace, and the call allocates nothing.
 * The launch is capped at 2048 blocks, so every wall plane fits; a launch
 * that would need more slots than the array holds returns FVIB_EINVAL.
 * The array is shared by every call on one device and keeps the last
 * call's partial sums: calls that overlap on one device (different
 * streams or threads) race.  FVIB_ESTATE if the array's address was not
 * set up for the handle's device (done by fvib_create_grid). */
int fvib_loss_wall_shear_noalloc(fvib_grid *g, const void *u0, double *J, void *ubar0);

/* Root-mean-square lift coefficient of a force history:
 * J = sqrt(mean_n C_L^2), C_L = 2 F_y / (rho U^2 D).  Fh: nsteps rows of
 * `stride` doubles with F at offset `offset` (device).  Writes J (device)
 * and, if dFh is not NULL, dJ/dF into the same row layout of dFh. */
int fvib_loss_rms_lift(fvib_grid *g, const double *Fh, int nsteps, int stride,
                       int offset, double u_ref, double diameter, double *J,
                       double *dFh);

/* Message of the last error on this handle ("" if none). */
const char *fvib_last_error(const fvib_grid *g);

/* Device-side failures are sticky (the error behaviour the paper's solver
 * loop needs when a step of Alg. 2 fails): once a step or adjoint step has
 * met one -- FVIB_ENOCONV, FVIB_ENONFINITE, or FVIB_EINVAL for a body that
 * left its window -- that call and every later fvib_step /
 * fvib_step_adjoint on the handle return it without enqueuing work.  With
 * deferred status the step record's kernel also stores a failed status in
 * a pinned word that the next step call reads, so a failure the host has
 * not yet looked at stops the calls that follow it once the failed step
 * has run.  fvib_clear_error synchronises the stream and resets the state
 * (the fields of the failed step are not restored). */
int fvib_clear_error(fvib_grid *g);

/* ---------------------------------------------------------------------
 * Sub-step entry points for parity tests.  Same layouts as above; every
 * pointer is a device pointer.
 * ------------------------------------------------------------------- */

/* Eq. 4 right-hand side R = -div(u (x) u) + nu lap u + fb on the faces the
 * momentum equation advances (other faces receive 0). */
int fvib_test_momentum(fvib_grid *g, const void *const u[3], const void *const fb[3],
                       void *R[3]);

/* Volume-integrated PPE right-hand side b of Eq. 9 (double, mean not
 * removed) from a predicted field ustar (no forcing mask). */
int fvib_test_ppe_rhs(fvib_grid *g, const void *const ustar[3], double *b);

/* Solve A p = b - mean(b) with the step's solver (double or mixed);
 * p is the initial guess on input.  iters may be NULL. */
int fvib_test_poisson(fvib_grid *g, const double *b, double *p, int32_t *iters);

/* Matrix-free A p of the volume-integrated PPE operator (double). */
int fvib_test_apply_A(fvib_grid *g, const double *p, double *Ap);

/* Velocity correction of Eq. 10: u = ustar - (dt/rho) G p on the faces the
 * correction acts on (boundary-normal faces of bounded axes keep ustar);
 * *div_max (device, may be NULL) = max over cells of |D u| in double before
 * rounding to the velocity type (Eq. 8).  u may not alias ustar. */
int fvib_test_project(fvib_grid *g, const void *const ustar[3], const double *p, void *u[3],
                      double *div_max);

/* Adjoint of fvib_test_project with respect to the pressure (Sec. 2.4.1):
 * pbar = -(dt/rho) G^T ubar (cells, double); the adjoint with respect to
 * ustar is ubar itself. */
int fvib_test_project_adjoint(fvib_grid *g, const void *const ubar[3], double *pbar);

/* Target velocity of Eqs. 18-19 and 23 of the attached body at state body
 * (6 doubles): u_s on every forced face (solid and immersed-boundary
 * points) of component c written into the full face array us[c], 0 on the
 * other faces. */
int fvib_test_ib_target(fvib_grid *g, const double *body, void *us[3]);

/* Adjoint of fvib_test_ib_target: adds into bodybar[3 + c] the sum of
 * usbar[c] over the forced faces (the normalised interpolation returns the
 * rigid velocity exactly, so the marker positions do not enter). */
int fvib_test_ib_target_adjoint(fvib_grid *g, const double *body, const void *const usbar[3],
                                double *bodybar);

/* Loads of Eq. 20 summed as in Eq. 12: F (3 doubles) = rho sum_k q_k dV_k of
 * the forcing field f (full face arrays; only the forced faces of the body
 * at state body are read). */
int fvib_test_ib_loads(fvib_grid *g, const double *body, const void *const f[3], double *F);

/* Adjoint of fvib_test_ib_loads for a force adjoint Fbar (3 doubles):
 * writes fbar (full face arrays, 0 off the forced faces) and adds the
 * marker-position part into bodybar[0..1]. */
int fvib_test_ib_loads_adjoint(fvib_grid *g, const double *body, const void *const f[3],
                               const double *Fbar, void *fbar[3], double *bodybar);

/* Rigid-body update of Eq. 12: one classic RK4 step of the body state under
 * a force F (3 doubles) held over the step; kc = [k(3), c(3)] (NULL = 0);
 * fixed degrees of freedom keep their values. */
int fvib_test_body_rk4(fvib_grid *g, const double *body, const double *F, const double *kc,
                       double *body_out);

/* Adjoint of fvib_test_body_rk4: writes bodybar_in (6) and Fbar (3) and adds
 * into kcbar (6, may be NULL). */
int fvib_test_body_rk4_adjoint(fvib_grid *g, const double *body, const double *F,
                               const double *kc, const double *bodybar_out, double *bodybar_in,
                               double *Fbar, double *kcbar);

/* Point classes of the current body at displacement body[0..2]: writes
 * one byte per face (0 fluid, 1 solid, 2 immersed-boundary point) into
 * cls[c] (full face arrays). */
int fvib_test_ib_classify(fvib_grid *g, const double *body, uint8_t *cls[3]);

/* ---------------------------------------------------------------------
 * Kernel timing for measurement.  While enabled, every launch of the
 * classes below is bracketed by HIP events recorded on the handle's stream
 * (the stream the kernels run on); totals accumulate until re-enabled.
 * ------------------------------------------------------------------- */
enum {
  FVIB_K_PREDICTOR = 0,   /* Eqs. 4-5 predictor with direct forcing        */
  FVIB_K_BOUNDARY = 1,    /* boundary-normal faces and outflow correction  */
  FVIB_K_PPE_RHS = 2,     /* Eq. 9 right-hand side                         */
  FVIB_K_RESIDUAL = 3,    /* double residual / refinement sweep            */
  FVIB_K_CG_DIR = 4,      /* CG search direction + p.Ap                    */
  FVIB_K_CG_UPDATE = 5,   /* CG iterate / residual update + r.r            */
  FVIB_K_IR_CORRECT = 6,  /* refinement correction                         */
  FVIB_K_PROJECT = 7,     /* Eq. 10 correction + divergence check          */
  FVIB_K_IB = 8,          /* point classes, targets, loads, RK4            */
  FVIB_K_ADJOINT = 9,     /* other adjoint stencils (boundary faces)       */
  FVIB_K_FDM_X = 10,      /* fast-diagonalisation contraction along x      */
  FVIB_K_FDM_Y = 11,      /* ... along y                                   */
  FVIB_K_FDM_Z = 12,      /* ... along z                                   */
  FVIB_K_ADJ_MOMENTUM = 13, /* transposed momentum stencil (all components) */
  FVIB_K_FDM_LAST = 14,   /* last axis: forward, division and inverse in one */
  FVIB_K_FFT = 15,        /* real FFT along a uniform periodic axis          */
  FVIB_K_FFT_ACC = 16,    /* last inverse FFT of a sweep, adding into p      */
  FVIB_K_ADJ_RHS = 17,    /* adjoint Poisson right-hand side G^T ubar        */
  FVIB_K_ADJ_USTAR = 18,  /* adjoint predicted velocity from the solution    */
  FVIB_K_RHS_RES = 19,    /* Eq. 9 right-hand side with the first residual   */
  FVIB_K_ADJ_RHS_RES = 20, /* adjoint right-hand side with the first residual */
  FVIB_K_LES = 21,        /* subgrid viscosity, wall model, stress divergence */
  FVIB_K_ADJ_LES = 22,    /* their adjoint                                   */
  FVIB_K_NCLASSES = 23
};

/* Start (enable != 0, totals cleared) or stop recording.  A recorded
 * launch is timed from the start of its first kernel to the end of its
 * last (kernel execution only). */
int fvib_timing_enable(fvib_grid *g, int enable);

/* Restrict recording to the classes whose bit (1u << class) is set in
 * class_mask (default: all).  Fewer events keep the host's launch rate
 * close to that of an untimed run. */
int fvib_timing_select(fvib_grid *g, uint32_t class_mask);

/* Record one launch in `every` (>= 1, default 1) of each class.  Each
 * recorded launch carries timestamp events in its dispatch, which idles
 * the device for a few microseconds around it; sampling keeps a timed run
 * close to an untimed one. */
int fvib_timing_sample(fvib_grid *g, int every);

/* Total device time (ms) and launch count of one kernel class since the
 * last enable; synchronises the stream.  Launches of refinement sweeps
 * that the device skipped (queued ahead of the convergence check and found
 * the solve converged) are not included. */
int fvib_timing_read(fvib_grid *g, int kclass, double *total_ms, int64_t *launches);

/* The same for the skipped launches alone (each returns at once). */
int fvib_timing_read_skipped(fvib_grid *g, int kclass, double *total_ms, int64_t *launches);

/* Deferred status (on != 0): fvib_step and fvib_step_adjoint return as soon
 * as the step's work is enqueued instead of waiting for it, so the host can
 * enqueue the next step while this one runs.  A Poisson solve that exhausts
 * its refinement budget is still reported at once (the solve polls its
 * convergence); every other device-side condition (body window left,
 * non-finite reduction) is reported only in info->status, which the caller
 * reads after synchronising the stream.  Off by default. */
int fvib_defer_status(fvib_grid *g, int on);

/* Build version string. */
const char *fvib_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FVIB_H */
