/*
 * ibr.h -- C ABI of the MI355X solver for the rigidly constrained
 * immersed-boundary Stokes / Navier-Stokes system of Kallemov, Bhalla,
 * Griffith & Donev, "An immersed boundary method for rigid bodies".
 *
 * One context owns every device buffer of one problem size: the MAC grid
 * state, the multigrid hierarchy, the Krylov bases and the factored per-body
 * mobility blocks.  They stay resident between calls, so consecutive solves
 * (time steps, warm starts) reuse them.  The caller owns every pointer it
 * passes; the library copies what it needs during the call and keeps no
 * caller pointer afterwards.  Calls on one context are not thread-safe; use
 * one context per host thread.  Every call returns an ibr_status; on failure
 * ibr_last_error() holds a message.  No exception crosses the ABI.
 *
 * Layouts (all host arrays are row-major, double precision):
 *   grid      periodic box [0, n h)^dim, cells indexed (k, j, i) with i (x)
 *             fastest; cell centres at ((i+1/2)h, (j+1/2)h, (k+1/2)h).  With
 *             walls = IBR_WALLS_NOSLIP the last axis (z in 3D, y in 2D) ends
 *             at no-slip walls at 0 and n h instead of wrapping; with
 *             IBR_WALLS_BOX every axis does.  Along a walled axis the faces
 *             of the velocity component normal to it with index 0 lie on the
 *             wall and hold 0.
 *   velocity  u[dim][n^dim]: component a of cell c lives on the a-face half a
 *             cell below the centre along a (the MAC grid of Sec. 3).
 *   pressure  p[n^dim] at cell centres, returned with zero mean.
 *   markers   R[N][dim], grouped contiguously by body; offsets[nb+1].
 *   Lambda    lambda[N][dim], the force each marker applies to the fluid
 *             (the +S Lambda forcing of eq. semi_continuum).
 *   bodies    centres X[nb][dim]; U[nb][dim]; Omega[nb][3] (3D) or [nb][1] (2D).
 *             Marker velocities V_i = U_p + Omega_p x (R_i - X_p) (minimum
 *             image); force F_p = sum_i Lambda_i, torque
 *             T_p = sum_i (R_i - X_p) x Lambda_i (Sec. 2).
 */
#ifndef IBR_H
#define IBR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ibr_ctx ibr_ctx;

typedef enum {
  IBR_OK = 0,
  IBR_EINVAL = 1,      /* an argument is out of range; nothing was changed */
  IBR_ENOMEM = 2,      /* device allocation failed */
  IBR_ENOCONV = 3,     /* max_iters reached; the last iterate is kept */
  IBR_EBREAKDOWN = 4,  /* Krylov breakdown with the residual above target */
  IBR_EFACTOR = 5,     /* a mobility block could not be factored even shifted */
  IBR_ENUMERIC = 6,    /* NaN or Inf in the residual */
  IBR_EDEVICE = 7,     /* a HIP call failed */
  IBR_ESTATE = 8       /* call out of order (e.g. solve before set_bodies) */
} ibr_status;

typedef enum { IBR_FP64 = 0, IBR_MIXED = 1 } ibr_precision;
typedef enum { IBR_PC_LOWER = 0, IBR_PC_FULL = 1 } ibr_pc;
/* Boundaries: periodic; no-slip walls at both ends of the last axis (the
 * slit channel of Sec. 7); or no-slip walls on every side (the closed box of
 * the non-periodic runs of Sec. 7.1 and of Sec. 7.3).  Boundary rules of the
 * appendix on physical boundary conditions. */
typedef enum { IBR_WALLS_NONE = 0, IBR_WALLS_NOSLIP = 1, IBR_WALLS_BOX = 2 } ibr_walls;
/* Explicit advection of the unsteady step (Sec. 3; the paper cites an upwind
 * scheme without stating it).  CENTRED: the second-order advective form on
 * the MAC grid with Adams-Bashforth 2.  SL: semi-Lagrangian transport, each
 * face's value taken from the departure point x - dt u(x) by multilinear
 * interpolation; unconditionally bounded, first order. */
typedef enum { IBR_ADVECT_CENTRED = 0, IBR_ADVECT_SL = 1 } ibr_advection;
/* Approximate mobility M~ of the preconditioner (Sec. 4).  ANALYTIC: the RPY
 * tensor with the periodic shift (steady 3D), the Brinkmanlet with a blended
 * self term (finite beta), regularised logarithms (2D).  FITTED: the forms
 * of Appendix A (3D) and Appendix B (2D) fitted to pair mobilities of the
 * four-point kernel measured with this solver (the Sec. 4.2 procedure); at
 * viscous CFL number beta = eta dt / (rho h^2) the forms of the two table
 * rows around beta, both evaluated at beta, are blended linearly in log
 * beta; beta above the last row uses the steady fit; an unsteady periodic
 * box adds its mean mode dt / (rho l^d).  AUTO: FITTED where the library
 * holds a table for the dimension, else ANALYTIC. */
typedef enum { IBR_MOB_ANALYTIC = 0, IBR_MOB_FITTED = 1, IBR_MOB_AUTO = 2 } ibr_mobility;

/* Problem and solver parameters.  Sec. 3.2 (eq. A_def) defines
 * A = (rho/dt) I - eta h^-2 L; rho == 0 selects steady Stokes, where the
 * periodic system becomes eq. constrained_periodic (S' = S - vol^-1 1 1^T,
 * <v> = 0).  Sec. 5 defines the solver knobs. */
typedef struct {
  int dim;            /* 2 or 3 */
  int n;              /* cells per direction: power of two, 2D 16..4096, 3D 8..512 */
  double h;           /* grid spacing (> 0); the box side is n*h */
  double rho;         /* density; 0 = steady Stokes */
  double eta;         /* viscosity (> 0) */
  double dt;          /* time step (> 0 unless steady) */
  int precision;      /* IBR_FP64, or IBR_MIXED: fp32 preconditioner, fp64 outer */
  int pc;             /* IBR_PC_LOWER (default) or IBR_PC_FULL, Sec. 5.1 */
  int n_s;            /* inner Stokes GMRES iterations N_s (default 2), Sec. 5.2 */
  int restart;        /* FGMRES restart length (default 100, Sec. 7.1) */
  int max_iters;      /* cap on FGMRES iterations (default 1000) */
  double rtol;        /* stop when ||b - K x||_2 <= rtol ||b||_2 (default 1e-8) */
  int mg_pre;         /* red-black sweeps before coarsening (default 2) */
  int mg_post;        /* red-black sweeps after prolongation (default 2) */
  int mg_coarse;      /* red-black sweeps on the 4^dim coarsest grid (default 4) */
  int device;         /* HIP device ordinal */
  void* stream;       /* hipStream_t to run on, or NULL for a library stream */
  int graphs;         /* 1 (default): replay each outer iteration as a captured
                         HIP graph; 0: plain stream launches (same kernels) */
  int walls;          /* IBR_WALLS_NONE (default); IBR_WALLS_NOSLIP: no-slip
                         walls at both ends of the last axis, periodic along the
                         others; IBR_WALLS_BOX: no-slip walls on every side.
                         Along a walled axis the tangential velocity's ghost
                         values beyond
                         a wall are its mirror image with the sign reversed,
                         the pressure's (inside the preconditioner) with the
                         sign kept; interpolation and spreading fold kernel taps
                         beyond a wall the same way (J = J0 E, S = E^T S0).
                         Steady Stokes then needs no mean-velocity condition
                         and uses S as is.  Markers must lie strictly between
                         the walls (ibr_set_bodies returns IBR_EINVAL
                         otherwise); ibr_step's advection uses the same
                         mirror rules, and it returns IBR_EINVAL (moving
                         nothing) when a body would cross a wall.  Between
                         walls P_S^-1 approximates the Stokes block less well
                         (Sec. 7.1): n_s = 4 is the robust choice for many
                         markers.  The walls are at rest unless
                         ibr_set_wall_velocity gives them a velocity. */
  int advection;      /* IBR_ADVECT_CENTRED (default) or IBR_ADVECT_SL.
                         CENTRED: N(v) = sum_b vbar^b (v^a_{c+e_b} -
                         v^a_{c-e_b}) / 2h with vbar^b the average of the four
                         b-faces around the a-face, and g = (rho/dt) v -
                         rho (3/2 N^n - 1/2 N^{n-1}) (forward Euler on the
                         first step); it needs viscous damping per step (cell
                         Reynolds number |u| h rho / eta of a few) and grows
                         without bound otherwise.  SL: v_d = v^a interpolated
                         at x - dt vbar(x) on the a-face lattice (periodic
                         wrap, E's mirror rules between walls), N = (v - v_d)/dt
                         so that g = (rho/dt) v_d; stable at any cell Reynolds
                         number and CFL number.  ibr_advect returns the
                         selected form's N. */
  int mobility;       /* IBR_MOB_AUTO (default), IBR_MOB_ANALYTIC or
                         IBR_MOB_FITTED (IBR_EINVAL without a table for the
                         dimension).  It changes the preconditioner, hence
                         iteration counts, not the converged solution. */
} ibr_params;

/* Per-solve report.  ps_applications counts P_S^-1 applications, the cost
 * unit of Sec. 7.1. */
typedef struct {
  int iters;              /* FGMRES iterations (all restart cycles) */
  int restarts;           /* restart cycles started */
  int ps_applications;    /* applications of P_S^-1 */
  int vcycles;            /* scalar V-cycles (a 3-field batched cycle counts 3) */
  int status;             /* ibr_status of the solve */
  double rel_residual;    /* ||b - K x|| / ||b|| recomputed in fp64 at exit */
  double ms;              /* device time of the solve, milliseconds */
  double max_mobility_shift; /* largest shift s used to factor a block (0 = none) */
} ibr_info;

/* Fill p with the defaults listed above (3D, n = 32, h = 1/32, steady, eta = 1). */
void ibr_default_params(ibr_params* p);

/* Static string for a status code. */
const char* ibr_status_string(int status);

/* Create a context for one grid size; allocates the grid state and multigrid
 * hierarchy on params->device.  *out is set only on IBR_OK. */
ibr_status ibr_create(const ibr_params* params, ibr_ctx** out);

/* Free every device buffer of the context (NULL is accepted). */
void ibr_destroy(ibr_ctx* ctx);

/* Message of the last failed call on this context ("" if none). */
const char* ibr_last_error(const ibr_ctx* ctx);

/* Device bytes a context with these parameters would hold after
 * ibr_set_bodies with nbodies bodies of markers_per_body[b] markers each (the
 * per-body mobility blocks are sized from each body's count, as the library
 * allocates them, plus an allowance for the allocator's rounding), for
 * admission control before ibr_create.  Not included: the one-time device
 * memory of the HIP runtime and the library's code, taken by the process's
 * first context and kept until the process ends (about 150 MiB).  0 if params
 * is NULL or invalid, nbodies < 0, or markers_per_body is NULL with nbodies > 0
 * or holds a negative count.  The caller keeps markers_per_body. */
size_t ibr_footprint_bytes(const ibr_params* params, int nbodies, const int* markers_per_body);

/* Set the rigid bodies (Sec. 2): nbodies >= 1, offsets[nbodies+1] increasing
 * from 0, R[N][dim] markers inside [0, n h) (wrapped otherwise), centres
 * X[nb][dim].  Builds the marker bins, assembles and factors each body's
 * approximate mobility block (Sec. 4, Sec. 5.3).  Velocities reset to zero. */
ibr_status ibr_set_bodies(ibr_ctx* ctx, int nbodies, const int* offsets, const double* R,
                          const double* centres);

/* Prescribed rigid velocities U[nb][dim] and Omega[nb][3 or 1] (Sec. 2). */
ibr_status ibr_set_velocities(ibr_ctx* ctx, const double* U, const double* Omega);

/* Walls moving with a prescribed velocity (inhomogeneous Dirichlet data of
 * the appendix on physical boundary conditions; Sec. 7.3's box moves with the
 * cavity).  lo[dim], hi[dim]: the velocities of the walls at coordinate 0 and
 * n h of the last axis.  Slit channel (IBR_WALLS_NOSLIP): the walls slide in
 * their planes, lo[dim-1] = hi[dim-1] = 0 (Couette flow between them).  Box
 * (IBR_WALLS_BOX): every wall moves with one velocity, lo == hi (a box
 * translating with the fluid it holds).  The library solves for u - u_b,
 * u_b the flow those walls carry without bodies (linear along the last axis,
 * an exact solution of the discrete homogeneous equations: its Laplacian
 * and divergence vanish and it meets the mirror rules), with the markers'
 * prescribed velocities reduced by u_b there and, with inertia, the
 * momentum right-hand side by (rho/dt) u_b; ibr_get_solution(_dev) returns
 * u itself, the normal components' wall faces holding the wall velocity.
 * NULL lo and hi put the walls back at rest.  IBR_EINVAL for a periodic box,
 * for data outside these two cases, and later from ibr_solve with free bodies
 * and from ibr_step (advection is not linear in u). */
ibr_status ibr_set_wall_velocity(ibr_ctx* ctx, const double* lo, const double* hi);

/* Fluid right-hand sides g[dim][n^dim] and h[n^dim] of eq. constrained_Stokes
 * (NULL = zero).  For steady periodic problems the mean of g is removed (the
 * paper's consistency assumption <g> = 0, Sec. 3.4). */
ibr_status ibr_set_rhs(ibr_ctx* ctx, const double* g, const double* hp);

/* ibr_set_rhs with device pointers (double, same layouts) on the context's
 * GPU, e.g. the data of torch tensors: the right-hand side never crosses
 * PCIe.  The copies run on the context's stream and are complete on return.
 * IBR_EINVAL if a non-NULL pointer is not device memory of that GPU. */
ibr_status ibr_set_rhs_dev(ibr_ctx* ctx, const void* g, const void* hp);

/* Solve eq. constrained_Stokes (eq. constrained_periodic when steady) by
 * FGMRES with the Schur-complement preconditioner of Sec. 5.1.  warm_start
 * != 0 starts from the context's previous solution.  info may be NULL. */
ibr_status ibr_solve(ibr_ctx* ctx, int warm_start, ibr_info* info);

/* One unsteady step (rho > 0): explicit advection right-hand side in the
 * form params.advection selects (centred with Adams-Bashforth 2, forward
 * Euler on the first step; or semi-Lagrangian transport, g = (rho/dt) v_d),
 * markers moved by dt U_p, constrained solve warm-started from the previous
 * step's solution (Sec. 3).
 * Bodies translate only: IBR_EINVAL if some Omega is nonzero.  With walls,
 * IBR_EINVAL (nothing moved) if a body's markers would reach a wall. */
ibr_status ibr_step(ibr_ctx* ctx, ibr_info* info);

/* Free kinematics (Sec. 2 poses it; Sec. 8 names the enlarged system and its
 * body mobility (K* M^-1 K)^-1, approximated here per body): free[p] != 0
 * makes body p move under the applied force F[p][dim] and torque
 * T[p][1 or 3] instead of its prescribed velocity (which is ignored); its
 * linear and angular velocities become unknowns of the solve, and at the
 * solution the body hands exactly (F_p, T_p) to the fluid.  The stacked
 * vector of ibr_apply_operator and ibr_precondition then gains a body block
 * after lambda: U[nb][dim], then Omega[nb][1 or 3] (identity rows for the
 * prescribed bodies).  free == NULL (or all zero) returns every body to
 * prescribed motion.  Call after ibr_set_bodies, which resets it.  Steady or
 * unsteady ibr_solve only: ibr_step refuses free bodies (IBR_EINVAL).
 * IBR_EFACTOR if a body's approximate body mobility is not positive definite
 * (the bodies are then all prescribed again).  Allocates device memory. */
ibr_status ibr_set_free_bodies(ibr_ctx* ctx, const int* free, const double* F, const double* T);

/* Rigid velocities of every body: U[nb][dim], Omega[nb][1 or 3] (either may
 * be NULL).  Free bodies: the velocities of the last solve; prescribed
 * bodies: the ones set by ibr_set_velocities. */
ibr_status ibr_get_velocities(ibr_ctx* ctx, double* U, double* Omega);

/* Start a new unsteady run (Sec. 7.6): the fluid at rest (v, pi and lambda
 * zero) and no advection history, so the next ibr_step is the first step of
 * a simulation (forward Euler advection).  Bodies, their current positions
 * and velocities are kept.  No device allocation; IBR_EINVAL for NULL. */
ibr_status ibr_reset(ibr_ctx* ctx);

/* Copy the current solution to host arrays (any pointer may be NULL):
 * u[dim][n^dim], p[n^dim], lambda[N][dim], F[nb][dim], T[nb][3 or 1]. */
ibr_status ibr_get_solution(ibr_ctx* ctx, double* u, double* p, double* lambda, double* F,
                            double* T);

/* ibr_get_solution into device arrays of the context's GPU (any may be
 * NULL), complete on return; IBR_EINVAL if a pointer is not device memory of
 * that GPU. */
ibr_status ibr_get_solution_dev(ibr_ctx* ctx, void* u, void* p, void* lambda, void* F, void* T);

/* Current marker positions R[N][dim] and centres X[nb][dim] (they move in ibr_step). */
ibr_status ibr_get_markers(ibr_ctx* ctx, double* R, double* centres);

/* ---- single-operator entry points (same layouts; used for kernel parity) ---- */

/* y = K x for the stacked vector x = [u (dim n^dim), p (n^dim), lambda (N dim)],
 * K the matrix of eq. constrained_Stokes (S' when steady); with free bodies
 * (ibr_set_free_bodies) x and y end with the body block, and K is the
 * enlarged free-kinematics matrix. */
ibr_status ibr_apply_operator(ibr_ctx* ctx, const double* x, double* y);

/* f = S lambda (Sec. 3.1, eq. S_unweighted; no mean removal): f[dim][n^dim]. */
ibr_status ibr_spread(ibr_ctx* ctx, const double* lambda, double* f);

/* V = J u (Sec. 3.1): V[N][dim]. */
ibr_status ibr_interp(ibr_ctx* ctx, const double* u, double* V);

/* One V-cycle (Sec. 5.2) for (c0 - c1 L) x = b on nfields independent
 * fields b[nfields][n^dim], x[nfields][n^dim]; c0 == 0 is the restricted
 * (mean-zero) inverse.  Runs in the context's precision.  With walls,
 * nfields == dim is the velocity cycle (field a is component a: normal to the
 * walls of axis a, its wall faces pinned to 0, and tangential to any other
 * walls) and nfields == 1 the pressure cycle (mirror with the sign kept;
 * c0 == 0 is then the mean-zero inverse); other counts return IBR_EINVAL. */
ibr_status ibr_vcycle(ibr_ctx* ctx, double c0, double c1, int nfields, const double* b,
                      double* x);

/* z = P r: one application of the Schur-complement preconditioner of
 * Sec. 5.1 to a stacked vector r (layout of ibr_apply_operator). */
ibr_status ibr_precondition(ibr_ctx* ctx, const double* r, double* z);

/* Approximate mobility block of one body (Sec. 4) as assembled on the device,
 * M[(dim Np)^2] row-major, and the shift s used to factor it. */
ibr_status ibr_mobility_block(ibr_ctx* ctx, int body, double* M, double* shift);

/* Inverse of the (possibly shifted) block as used by the preconditioner,
 * Minv[(dim Np)^2] row-major (Sec. 5.3 dense mobility solve). */
ibr_status ibr_mobility_inverse(ibr_ctx* ctx, int body, double* Minv);

/* Advection term N(u) of the unsteady step on the MAC grid, host arrays
 * u[dim][n^dim] in and N[dim][n^dim] out, in the form params.advection
 * selects (the semi-Lagrangian one uses params.dt; IBR_EINVAL when the
 * context is steady).  Resets the Adams-Bashforth history of ibr_step. */
ibr_status ibr_advect(ibr_ctx* ctx, const double* u, double* N);

/* ---- allocation-free spreading ---- */

/* Size of the library's static device scratch array (per GPU, held until the
 * process ends) used by ibr_spread_noalloc. */
#define IBR_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * f = S lambda as ibr_spread (Sec. 3.1, eq. S_unweighted, no mean removal),
 * without a context: from params only dim, n, h, walls, device and stream are
 * read.  R[nmarkers][dim] (marker positions, wrapped into the box as in
 * ibr_set_bodies) and lambda[nmarkers][dim] are device arrays of
 * params->device; f[dim][n^dim] is a device array that receives the field
 * (it is overwritten, not accumulated).  Asynchronous on params->stream (NULL
 * = the device's null stream): f is complete when the stream reaches the
 * call, and R and lambda must stay valid until then.  Every temporary (kernel
 * taps, tile bins) lives in the static scratch array of
 * IBR_NOALLOC_SCRATCH_BYTES: no call allocates or frees device memory.  That
 * array is shared by all calls on one GPU and keeps the last call's contents,
 * so calls that overlap on one GPU (other streams or host threads) race.
 * Sizes beyond the scratch (88 469 markers at n = 512 in 3D, 104 850 on
 * grids of one tile) return IBR_EINVAL with the largest marker count
 * that fits in msg.  msg (may be NULL) receives a message of at most msg_len
 * - 1 characters on failure, "" on success.  No device work runs unless every
 * argument is valid. */
ibr_status ibr_spread_noalloc(const ibr_params* params, int nmarkers, const void* R, const void* lambda,
                              void* f, char* msg, size_t msg_len);

/* ---- live kernel timing (measurement support) ---- */

/* Bracket every stride-th launch of one kernel class with HIP events on its
 * stream and accumulate that launch's algorithmic bytes (stride 0 = off).
 * Classes: "rb_fine" (red-black half sweeps and first sweeps on the finest
 * multigrid level), "rb_red_prolong" (the finest level's first post-smoothing
 * red half sweep, which also forms the prolonged correction of its black
 * neighbours), "ortho_dot" and "ortho_axpy" (the reduction and update passes
 * of the outer Arnoldi step), "stokes_apply" (the MAC stencil of the outer
 * operator), "vcycle" (whole V-cycle calls), "wall_rb_fine" (finest-level half
 * sweeps of the walled V-cycle).
 * Process-wide; enabling resets the class's counters.  While any class is
 * enabled the solver launches its kernels directly on the stream instead of
 * replaying captured iteration graphs, so every launch can be bracketed.
 * IBR_EINVAL for an unknown class or a negative stride. */
int ibr_timer_enable(const char* kernel, int stride);

/* Total event time in ms, number of timed launches and summed algorithmic
 * bytes of the timed launches since enabling (waits for the recorded events). */
int ibr_timer_read(const char* kernel, double* ms, long* launches, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* IBR_H */
