/*
 * nc.h -- C ABI of the MI355X (gfx950) natural-convection state / adjoint solver.
 *
 * The library solves the stabilised trilinear-hexahedron discretisation of the
 * Darcy / Boussinesq / convection-diffusion model of Pollini, Sigmund, Andreasen and
 * Alexandersen (arXiv 1904.00182): the Darcy velocity of Sec. 2.1 (eq. finaldarcy)
 * inserted into incompressibility and the energy equation (Sec. 2.2, eq. goveq), in
 * the weak form of App. A (eq. weakstable) with the Tezduyar SUPG weight, posed as
 * R(s) = M(s) s - f = 0 (eq. finalsyseq).  Conductivity and permeability are RAMP
 * interpolated (Sec. 5.2, eqs. condRAMP, permRAMP) from a filtered density.  The
 * state is solved by damped Newton (Sec. 5.4) with matrix-free Jacobian applies,
 * flexible GMRES and a geometric-multigrid preconditioner; design sensitivities
 * follow from the adjoint (Sec. 5.1, eq. optprob and the adjoint analysis).
 *
 * Unknowns: five per node, node-interleaved (u, v, w, P, T).  The P and T rows are
 * the paper's two-field system; the u, v, w rows are the lumped L2 projection of the
 * Darcy velocity, which does not feed back into the P and T rows.
 *
 * Grid numbering (all arrays):
 *   node    n = i + (nx+1) * (j + (ny+1) * k)      state arrays are [n][5] float64
 *   element e = i + nx * (j + ny * k)              design arrays are [e] float64
 *   z is vertical, gravity (0, 0, -g0).
 * Boundary conditions of the cavity (Sec. 6.1): T = 0 on x = 0, x = Lx, y = 0,
 * y = Ly and z = Lz; the bottom is insulated except for a heat flux q_h entering
 * through a rectangular patch; u.n = 0 on all walls (natural); the pressure level
 * is fixed by P = 0 at node (0, 0, nz).
 *
 * Memory ownership: every pointer whose name ends in _dev is a device pointer owned
 * by the caller.  The library never allocates device memory: all of its persistent
 * device buffers live in the single caller-provided workspace sized by
 * nc_workspace_bytes().  A context is bound to one HIP stream (passed as void*),
 * is not thread-safe, and is independent of every other context.
 *
 * Errors: every int-returning function returns NC_OK (0) on success, a positive
 * value for a non-fatal outcome (NC_NOT_CONVERGED: the best iterate is left in the
 * output and the info struct is filled) and a negative value on error.  Functions
 * that return host-visible values synchronise the context's stream; the others only
 * enqueue work.  No C++ exception crosses this interface.
 */
#ifndef NC_H
#define NC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NC_OK               0
#define NC_NOT_CONVERGED    1
#define NC_EINVAL         (-1)
#define NC_ENOMEM         (-2)
#define NC_EHIP           (-3)
#define NC_ENAN           (-4)

#define NC_FP64   0   /* everything in float64                                          */
#define NC_MIXED  1   /* float32 inner Krylov / multigrid / operator, float64 outer loop */

#define NC_DENSE_MAX 2000   /* largest coarsest-grid system solved by a dense inverse */

#define NC_FILTER_CONE 0  /* normalised cone weights max(0, R - |c_e - c_j| / h)              */
#define NC_FILTER_PDE  1  /* PDE (Helmholtz) filter of Sec. 5.1: -r^2 lap y + y = x, Neumann
                             walls, r = R h / (2 sqrt 3), Q1 consistent mass, gamma_e = mean
                             of y over the element                                          */

typedef struct nc_problem {
  int    nx, ny, nz;          /* elements per axis; at most 2^31 / 5 nodes in all and    *
                               * (nx+1)(ny+1) < 2^32 / 40 nodes in one z-layer           */
  double h;                   /* element edge; <= 0 means 1/nx                           */
  double rho0, mu, cp, g0;    /* reference density, viscosity, heat capacity, gravity    */
  double alpha;               /* thermal expansion coefficient (= Gr with unit constants)*/
  double k_f, k_s;            /* fluid / solid conductivity                              */
  double kappa_f, kappa_s;    /* fluid / solid permeability                              */
  double q_c, q_p;            /* RAMP penalties of k and kappa                           */
  double q_h;                 /* heat flux through the bottom patch                      */
  double patch_x0, patch_x1, patch_y0, patch_y1; /* patch: bottom faces with centre inside */
  double Q;                   /* volumetric heat source (on q_box, else everywhere)      */
  double filter_radius;       /* density filter radius R in element lengths; 0 = none    */
  int    precision;           /* NC_FP64 or NC_MIXED                                     */
  int    levels;              /* multigrid levels; 0 = choose automatically              */
  double newton_step_rtol;    /* stop when a full step, or the error predicted to remain after
                                 it, is <= rtol |s_f| per field                           */
  double krylov_rtol;         /* relative tolerance of each linear solve (NC_FP64)       */
  double adjoint_rtol;        /* relative residual of the adjoint solve                  */
  int    newton_maxit, krylov_restart, krylov_maxit;
  int    smooth_pre, smooth_post; /* block-Jacobi sweeps before / after the coarse-grid
                                    correction on the finest level (pre >= 1)             */
  double smooth_omega;        /* block-Jacobi damping                                    */
  int    smooth_pre_coarse, smooth_post_coarse; /* the same on the coarser levels        */
  double krylov_rtol_mixed;   /* relative tolerance of each float32 inner solve (NC_MIXED) */
  int    gs_passes;           /* classical Gram-Schmidt passes per FGMRES step, 1 or 2   */
  int    coarse_tail;         /* 1: the last smoothed level and the dense coarsest level of
                                 each V-cycle run in one workgroup when they fit; 0: one
                                 launch per step everywhere (same operators and order)   */
  double newton_eta0;         /* linear tolerance of the first Newton step; later steps use
                                 0.9 (|R_k| / |R_k-1|)^2 between the Krylov tolerance and
                                 this (Eisenstat-Walker); 0: the Krylov tolerance always   */
  int    filter_kind;         /* NC_FILTER_CONE or NC_FILTER_PDE                          */
  /* The benchmark of Sec. 6.1: a quarter of the symmetric cavity, a heat-source block and
   * a design domain.  A box (x0, x1, y0, y1, z0, z1) is in use when x1 > x0, y1 > y0 and
   * z1 > z0; an element belongs to it when its centre lies in the closed box.           */
  int    sym_x, sym_y;        /* 1: the wall x = Lx (y = Ly) is a symmetry plane: insulated,
                                 u.n = 0 (the normal velocity unknowns there are held at 0) */
  double q_box[6];            /* elements carrying Q; unused box: Q everywhere            */
  double solid_box[6];        /* passive solid: gamma = 1 whatever the design              */
  double design_box[6];       /* design domain; elements outside it and outside solid_box
                                 are passive fluid (gamma = 0); unused box: all design     */
  double smooth_omega_fallback; /* block-Jacobi damping used for good, in this context, once
                                 an FGMRES solve has stalled (its first restart cycle did not
                                 halve the residual: undamped block Jacobi diverges on
                                 strongly convective blocks); the stalled solve is redone.
                                 Only a stronger damping than the current one is taken over.
                                 0: no fallback                                          */
  int    f64_krylov_fallback; /* NC_MIXED, 1: the workspace also holds a float64 Krylov basis
                                 (krylov_restart + 1 vectors and as many preconditioned ones);
                                 a float32 Krylov solve that ends unconverged is redone with
                                 float64 vectors and operator, preconditioned by the float32
                                 V-cycle, and the context keeps that for good (nc_info
                                 krylov_f64).  Where the V-cycle amplifies a few directions by
                                 orders of magnitude (a solid region whose permeability is far
                                 below the fluid's, in the convective regime) float32 rounding
                                 of the basis and of the operator reaches the size of the
                                 residual.  0: no reserve, no fallback; ignored in NC_FP64  */
} nc_problem;

#define NC_HIST_MAX 32  /* Newton steps / refinement sweeps recorded in nc_info */

typedef struct nc_info {
  int    newton_its;          /* Newton steps taken                                      */
  int    krylov_its;          /* total FGMRES iterations (state or adjoint)              */
  int    refine_its;          /* outer refinement sweeps (adjoint)                       */
  int    levels;              /* multigrid levels used                                   */
  double res0[5];             /* residual 2-norm per field (u, v, w, P, T) before the first
                                 step: R~(s0) for the state, the masked rhs for the adjoint */
  double res[5];              /* final residual 2-norm per field                         */
  double rel_res;             /* final relative residual of the last linear solve        */
  double t_setup;             /* seconds of device time spent rebuilding the multigrid
                                 hierarchy (state injection, node-block inverses, coarsest
                                 inverse), summed over rebuilds; it partly overlaps the
                                 first V-cycle, which runs beside it on the solver's stream */
  double t_solve;             /* t_total - t_setup                                       */
  double t_total;             /* seconds, host wall clock of the call                    */
  int    hist_len;            /* entries filled in hist_krylov / hist_res (<= NC_HIST_MAX) */
  int    hist_krylov[NC_HIST_MAX];   /* FGMRES iterations of each Newton step (state) or
                                        refinement sweep (adjoint)                        */
  double hist_res[NC_HIST_MAX][5];   /* residual 2-norm per field after that step / sweep */
  int    krylov_f64;          /* NC_MIXED with f64_krylov_fallback: 1 once a float32 Krylov
                                 solve of this context has ended unconverged; from then on
                                 (until nc_set_problem) its Krylov vectors and operator are
                                 float64, preconditioned by the float32 V-cycle.  0 otherwise */
} nc_info;

typedef struct nc_ctx nc_ctx;

/* Fill *p with the defaults of the paper's unit-constant cavity (Sec. 3 and Sec. 6.1:
 * rho0 = mu = c_p = g0 = 1, k_f = 1, k_s = 100) for an nx*ny*nz grid; alpha 1e3 with
 * the Table tab:2 permeability 0.00513, kappa_s 1e-4, q_c = q_p = 8, unit flux on the
 * centred patch [0.375, 0.625] x [0.125, 0.375]. */
void   nc_problem_default(nc_problem* p, int nx, int ny, int nz);

/* Bytes of device workspace a context for *p needs (also the admission footprint).
 * Returns 0 for an invalid problem. */
size_t nc_workspace_bytes(const nc_problem* p);

/* Create a context.  workspace_dev: caller-owned device buffer of >= bytes
 * (nc_workspace_bytes), 256-byte aligned; stream: hipStream_t or NULL for the
 * default stream.  NC_EINVAL for bad sizes, NC_ENOMEM if bytes is too small. */
int    nc_create(const nc_problem* p, void* workspace_dev, size_t bytes, void* stream, nc_ctx** out);
int    nc_destroy(nc_ctx* ctx);
const char* nc_status_string(int status);

/* Design chain: gamma = F_R x (the density filter of Sec. 5.1: the cone filter or the
 * PDE filter of filter_kind, radius filter_radius element lengths, identity if 0; the PDE
 * filter is solved by a fixed number of Chebyshev steps planned from closed-form spectrum
 * bounds, to a relative error below 1e-15), gamma set to 1 on passive solid and 0 on
 * passive fluid elements (Sec. 6.1), then the RAMP conductivity and
 * permeability of Sec. 5.2 (eqs. condRAMP, permRAMP) and their derivatives, on the
 * finest level and averaged onto the coarser multigrid levels.
 * x_dev: [E] float64 in [0, 1].  Enqueue only. */
int    nc_set_design(nc_ctx* ctx, const double* x_dev);
/* Copy the filtered density gamma [E] into gamma_dev. */
int    nc_get_gamma(nc_ctx* ctx, double* gamma_dev);
/* The context's density filter on its own (Sec. 5.1): y = F_R x, or y = F_R^T x when
 * transpose != 0 (the map of element sensitivities back to the raw design; the PDE filter
 * is symmetric, so both are the same there).  x_dev, y_dev: [E] float64, distinct.  The
 * identity for radius 0.  Enqueue only. */
int    nc_filter_apply(nc_ctx* ctx, int transpose, const double* x_dev, double* y_dev);

/* Nonlinear residual R~(s) = M(s) s - f of App. A (eq. finalsyseq, assembled from the
 * element integrals of eq. weakstable with the SUPG weight N* of App. A), [N][5] ->
 * [N][5]; the velocity rows are the lumped projection of the Darcy velocity of Sec. 2.1
 * (eq. finaldarcy).  Constrained rows hold s - s_bar (s_bar = 0).  Enqueue only. */
int    nc_residual(nc_ctx* ctx, const double* s_dev, double* r_dev);

/* Store the linearisation state (P, T of s) used by the Jacobian applies. */
int    nc_linearize(nc_ctx* ctx, const double* s_dev);
/* y = J~ v and y = J~^T w at the stored linearisation: J~ = dR/ds, the exact Newton
 * Jacobian of eq. finalsyseq (Sec. 5.4), including the derivatives of the SUPG weight
 * and tau of App. A through the centroid velocity, with constrained rows and columns
 * replaced by the identity; J~^T is the operator of the adjoint problem of Sec. 5.1.
 * Matrix-free, element by element.  Float64 and float32 variants ([N][5] each; the
 * float32 ones use the float32 copy of the state and coefficients).  Enqueue only. */
int    nc_jac_apply(nc_ctx* ctx, const double* v_dev, double* y_dev);
int    nc_jacT_apply(nc_ctx* ctx, const double* w_dev, double* y_dev);
int    nc_jac_apply_f32(nc_ctx* ctx, const float* v_dev, float* y_dev);
int    nc_jacT_apply_f32(nc_ctx* ctx, const float* w_dev, float* y_dev);

/* State solve R~(s) = 0 by damped Newton (Sec. 5.4: full steps, damped when the
 * residual norm grows), each linear step solved by flexible GMRES (Sec. 5.4) with a
 * geometric-multigrid preconditioner; constraints of Sec. 6.1 (T = 0 walls, one pressure
 * pin) fused into every kernel.  s_dev [N][5]: in = initial guess (zeros for a cold start,
 * a previous solution for a warm start; constrained entries are overwritten), out =
 * solution.  Synchronises; fills *info if non-NULL.  NC_NOT_CONVERGED leaves the last
 * iterate; NC_ENAN on a non-finite residual. */
int    nc_solve_state(nc_ctx* ctx, double* s_dev, nc_info* info);

/* Objective: the thermal compliance of Sec. 5.1 (eq. objdiscr), f = sum_e f_tQ,e^T t_e
 * with the volumetric load f_tQ,e = int N*^T Q of App. A (its SUPG weight N* depends on
 * the state), plus f_qh^T t for the boundary-flux load of the patch, to *f_host.
 * Synchronises. */
int    nc_objective(nc_ctx* ctx, const double* s_dev, double* f_host);
/* d f / d s at the state s_dev, [N][5]: f_qh on the T entries of the patch nodes plus the
 * derivative of the volumetric part (P and T entries of the source elements' nodes), 0 on
 * constrained entries.  s_dev may be NULL when Q = 0 (the gradient is then the constant
 * flux load); NC_EINVAL otherwise.  Enqueue only. */
int    nc_objective_grad(nc_ctx* ctx, const double* s_dev, double* g_dev);

/* Adjoint solve J~^T lambda = rhs at the state s (the adjoint sensitivity analysis of
 * Sec. 5.1; rhs = df/ds, e.g. from nc_objective_grad, Sec. 5.1 eq. objdiscr).  rhs_dev,
 * lam_dev [N][5]; the rhs is zeroed on constrained dofs, so lambda is 0 there.  In
 * NC_MIXED the float32 Krylov solves are refined in float64 to adjoint_rtol.
 * Synchronises; fills *info if non-NULL. */
int    nc_solve_adjoint(nc_ctx* ctx, const double* s_dev, const double* rhs_dev, double* lam_dev, nc_info* info);

/* Adjoint term of the design sensitivities of Sec. 5.1 for any objective whose d f / d s
 * was the adjoint's right-hand side: dfdgamma_e = -lambda_e^T dR_e/dgamma_e through the
 * RAMP derivatives of Sec. 5.2 (zero on passive elements), then dfdx = F_R^T dfdgamma (the
 * chain rule through the density filter; zero off the design domain).  An objective with
 * an explicit dependence on gamma adds it (nc_objective_sensitivity does for
 * nc_objective).  dfdx_dev [E] (required), dfdgamma_dev [E] (may be NULL).  Enqueue
 * only. */
int    nc_sensitivity(nc_ctx* ctx, const double* s_dev, const double* lam_dev, double* dfdx_dev, double* dfdgamma_dev);

/* d f / d x of nc_objective (Sec. 5.1): the adjoint term of nc_sensitivity plus the
 * objective's explicit dependence on gamma (the volumetric load's SUPG weight depends on
 * the permeability), for lam_dev from nc_solve_adjoint with rhs = nc_objective_grad.
 * Passive elements have zero dfdgamma, and dfdx is zero off the design domain.  Enqueue
 * only. */
int    nc_objective_sensitivity(nc_ctx* ctx, const double* s_dev, const double* lam_dev, double* dfdx_dev,
                                double* dfdgamma_dev);

/* Volume constraint of Sec. 5.1 (eq. constr) without its bound g*: the solid fraction
 * sum_D gamma_e v_e / sum_D v_e of the filtered design over the design domain D (the
 * design box minus the solid box), to *frac_host, and, when dgdx_dev [E] is not NULL, its
 * gradient with respect to the raw design through the filter (zero off D).  NC_EINVAL
 * for an empty design domain.  Synchronises. */
int    nc_volume(nc_ctx* ctx, double* frac_host, double* dgdx_dev);

/* Changes the parameters of a context in place (continuation of the penalties and of the
 * solid permeability, Sec. 5.3 eq. contsch1; a ramp of the heat source, Sec. 5.4; or a new
 * request on a pooled context).  The new problem must give the same workspace layout:
 * the same grid, multigrid levels, precision, Krylov restart and filter work; NC_EINVAL
 * otherwise.  The design must be set again (nc_set_design) before the next solve.  Host
 * only (waits for the context's setup streams). */
int    nc_set_problem(nc_ctx* ctx, const nc_problem* p);

/* One iteration of the Method of Moving Asymptotes (Sec. 5.1, Svanberg's method; the move
 * limit of Sec. 6.1) for min f subject to g <= 0 and 0 <= x <= 1, over the design elements
 * of the context (the raw design of passive elements is left as it is).  iter: 1 for the
 * first update of a run, then 2, 3, ... (the asymptotes start from x in the first two
 * iterations and then widen or narrow with the sign pattern of the last two steps);
 * x_dev [E]: in the current design, out the update; dfdx_dev, dgdx_dev [E]: derivatives of
 * the objective and of the constraint; g: the constraint value (e.g. volume fraction -
 * g*); state_dev: caller-owned NC_MMA_ROWS x E doubles kept between iterations (the last
 * two iterates and the asymptotes; the rest is scratch).  The subproblem is solved
 * through its dual (one multiplier, written to *lambda_host when not NULL; infinite when
 * no point within the move limit satisfies the constraint's approximation, and the update
 * then reduces it most).  Synchronises. */
#define NC_MMA_ROWS 10
int    nc_mma_update(nc_ctx* ctx, int iter, double* x_dev, const double* dfdx_dev, double g, const double* dgdx_dev,
                     double move, double* state_dev, double* lambda_host);

/* Optional per-context timing of the solver's kernels with HIP events on the context's
 * stream (a tracing aid; adds one event pair per timed launch).  nc_set_timing(ctx, 1)
 * creates the events (once) and zeroes the counters; 0 turns timing off.
 * nc_get_timing synchronises, then fills ms[k] (summed milliseconds), counts[k]
 * (launches) and, when bytes is non-NULL, bytes[k] (the algorithmic bytes of those
 * launches: every input read once, every output written once) for k < n over the kernel
 * classes 0 residual, 1 J v and 2 J^T w of the (P, T) Krylov solve, 3 smoothing sweep on the
 * finest grid, 4 transposed sweep on the finest grid, 5 multigrid residual on the finest
 * grid, 6 node-block diagonal, 7 velocity coupling, 8 grid transfers, 9 coarsest solve (and
 * the bottom of the V-cycle where it runs in one workgroup),
 * 10 Krylov multi-dot, 11 Krylov multi-axpy, 12 other vector kernels, 13 preconditioner
 * setup, 14 smoothing sweeps on coarser levels, 15 multigrid residuals on coarser levels;
 * returns the number of classes (16) or an error code. */
int    nc_set_timing(nc_ctx* ctx, int enable);
int    nc_get_timing(nc_ctx* ctx, double* ms, long* counts, double* bytes, int n);

/* One application of the multigrid preconditioner of the (P, T) Krylov solves (the
 * paper's F-GMRES of Sec. 5.4 leaves the preconditioner to its references): the hierarchy is
 * rebuilt at the linearisation state s_dev [N][5] (state injection, node-block
 * inverses, coarsest inverse), then z = M^-1 v, or M^-T v when transpose != 0, by one
 * V-cycle in the working precision.  v_dev, z_dev: [N][2] float64 (P, T) pairs; the
 * constrained entries of z are zero.  A diagnostic of the solver's building block.
 * Enqueue only. */
int    nc_precondition(nc_ctx* ctx, int transpose, const double* s_dev, const double* v_dev, double* z_dev);

/* Stand-alone cone density filter (Sec. 5.1 regularises the design by filtering; the
 * normalised cone weights max(0, R - |c_e - c_j| / h)) on an nx*ny*nz element grid:
 * y = F_R x.  transpose != 0 with radius > 0 is NC_EINVAL here (the transpose needs a
 * temporary; nc_sensitivity applies it).  Used to build filtered designs.  Enqueued on
 * stream. */
int    nc_cone_filter(int nx, int ny, int nz, double radius, const double* x_dev, double* y_dev, int transpose, void* stream);

/* Coarsest-grid solve of the multigrid preconditioner, exposed on its own (the paper
 * leaves the preconditioner to its references; the hierarchy here inverts the coarsest
 * (P, T) operator densely): in-place Gauss-Jordan inversion with partial pivoting of a
 * dense n x n float64 matrix, 1 <= n <= NC_DENSE_MAX.  a_dev holds 2 n^2 doubles: on
 * entry the first n^2 are A (row-major); on return they are A^-1 and the next n^2 are
 * (A^-1)^T (the second half is overwritten as scratch).  iwork_dev (2 n ints, returns the
 * pivot rows in order first) and dwork_dev (2 n doubles) are scratch.  A singular A (a
 * zero pivot) leaves non-finite entries; nothing is checked on the device.  NC_EINVAL for
 * a bad n or NULL pointer.  Enqueued on stream. */
int    nc_dense_inverse(double* a_dev, int n, int* iwork_dev, double* dwork_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): nc_dense_inverse without the two
 * scratch arguments.  The pivot rows and step columns live in a library-owned static
 * device buffer of NC_DENSE_NOALLOC_SCRATCH bytes per GPU (enough for n = NC_DENSE_MAX),
 * held until the process ends; nothing is allocated.  The buffer of the device current
 * at the call is used, so stream must belong to that device.  Every call on one GPU
 * shares that buffer and leaves its contents behind: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.  Results are
 * those of nc_dense_inverse.  NC_EINVAL for n outside [1, NC_DENSE_MAX] or a NULL a_dev;
 * NC_EHIP if the buffer's device address cannot be obtained.  Enqueued on stream. */
#define NC_DENSE_NOALLOC_SCRATCH 49152
int    nc_dense_inverse_noalloc(double* a_dev, int n, void* stream);

/* ---------------------------------------------------------------------------------
 * Navier-Stokes / Brinkman flow model: the full-flow model of the paper's hybrid
 * strategy (Sec. 6.4), for the same five unknowns per node and the same design chain,
 * objective and adjoint machinery.  Governing equations: the steady incompressible
 * momentum equation of Sec. 2.1 (eq. app_NS) with the modified pressure and Boussinesq
 * buoyancy of Sec. 2.1, a Brinkman friction a(gamma) u, the incompressibility condition and the energy equation of eq. goveq.  Equal-order
 * trilinear elements with SUPG and PSPG stabilisation: streamline weight W = N + tau_m
 * u0 . grad N on the momentum rows, tau_m / rho0 grad N . r_m added to the continuity
 * rows, tau_m = (4|u0|^2/h_e^2 + 16 nu^2/h_e^4 + (a/rho0)^2)^(-1/2), the energy rows as in
 * App. A.  Boundary conditions: no slip on the walls (only u.n = 0 on a symmetry plane), T
 * and the pressure level as in the Darcy model.
 *
 * Brinkman coefficient: in this model kappa_s is the solid's impermeability and q_p its
 * RAMP penalty, a(gamma) = kappa_s q_p gamma / (1 + q_p - gamma), zero in the fluid (the
 * roles the paper gives them in the Navier-Stokes stage of its hybrid continuation,
 * eq. contsch2: kappa_s = 1e5, q_p = 8); kappa_f is unused.
 *
 * The other fields of nc_problem keep their meaning; the solver uses precision (NC_MIXED: a
 * float32 multigrid preconditioner inside float64 Krylov solves on the float64 Jacobian),
 * levels, the Newton and
 * Krylov controls (newton_step_rtol, newton_eta0, krylov_rtol as the smallest linear
 * tolerance, krylov_restart, krylov_maxit, adjoint_rtol) and the smoother's sweeps and
 * damping.  The Krylov residuals are those of the row-equilibrated system (each field's
 * rows divided by the root mean square of its diagonal entries); the adjoint pressure
 * then carries about 100 times the adjoint's relative residual, so an adjoint_rtol of
 * 1e-12 gives multipliers accurate to about 1e-10.  Undamped node-block Jacobi
 * (smooth_omega 1) diverges on these saddle-point blocks beyond small grids; 0.7 suits
 * them, and smooth_omega_fallback takes over as in the Darcy model when a first restart
 * cycle stalls.  krylov_rtol_mixed, gs_passes and coarse_tail are ignored.  The Jacobian is assembled (27 neighbours x 5 x 5 per node) by forward-mode
 * differentiation of the element rows; the workspace holds it on every multigrid level
 * (about 5.4 KB per node in float64, plus 2.7 KB per node in float32 with NC_MIXED).
 * Errors, ownership and synchronisation as for the Darcy model's entry points.
 * --------------------------------------------------------------------------------- */
typedef struct nc_ns_ctx nc_ns_ctx;

/* Workspace bytes of a Navier-Stokes context for *p (0 for an invalid problem). */
size_t nc_ns_workspace_bytes(const nc_problem* p);
int    nc_ns_create(const nc_problem* p, void* workspace_dev, size_t bytes, void* stream, nc_ns_ctx** out);
int    nc_ns_destroy(nc_ns_ctx* ctx);
/* Parameters changed in place (the continuation of eq. contsch2, a ramp of the heat
 * source), under the conditions of nc_set_problem: same grid, levels, precision, Krylov
 * restart and filter work, NC_EINVAL otherwise; the design must be set again.  Host only
 * (synchronises). */
int    nc_ns_set_problem(nc_ns_ctx* ctx, const nc_problem* p);
/* The design chain of nc_set_design (filter, passive regions, RAMP of Sec. 5.2), with the
 * permeability turned into the Brinkman coefficient.  Enqueue only. */
int    nc_ns_set_design(nc_ns_ctx* ctx, const double* x_dev);
int    nc_ns_get_gamma(nc_ns_ctx* ctx, double* gamma_dev);
/* Residual R~(s) of the model above, [N][5] -> [N][5] (s_dev and r_dev distinct);
 * constrained rows hold s.  Enqueue only. */
int    nc_ns_residual(nc_ns_ctx* ctx, const double* s_dev, double* r_dev);
/* Assemble the Jacobian J~ = dR~/ds at s (exact, including the derivatives of tau_m and
 * of the streamline weights) on every multigrid level.  Synchronises. */
int    nc_ns_linearize(nc_ns_ctx* ctx, const double* s_dev);
/* y = J~ v, y = J~^T w with the float64 Jacobian of the last nc_ns_linearize (or solve);
 * NC_EINVAL before any.  Enqueue only. */
int    nc_ns_jac_apply(nc_ns_ctx* ctx, const double* v_dev, double* y_dev);
int    nc_ns_jacT_apply(nc_ns_ctx* ctx, const double* w_dev, double* y_dev);
/* One V-cycle of the preconditioner at the last linearisation: z = M^-1 v (M^-T v when
 * transpose != 0), [N][5] float64.  Enqueue only. */
int    nc_ns_precondition(nc_ns_ctx* ctx, int transpose, const double* v_dev, double* z_dev);
/* Damped Newton (Sec. 5.4) with FGMRES on the assembled Jacobian: s_dev in = initial
 * guess, out = solution, as nc_solve_state.  Synchronises. */
int    nc_ns_solve_state(nc_ns_ctx* ctx, double* s_dev, nc_info* info);
/* The compliance of nc_objective (Sec. 5.1 eq. objdiscr, the volumetric load weighted by
 * the energy rows' streamline weight at the element's centroid velocity) and its state
 * derivative (patch load on T; the volumetric part on T and on the velocity unknowns of
 * the source elements' nodes; 0 on constrained entries). */
int    nc_ns_objective(nc_ns_ctx* ctx, const double* s_dev, double* f_host);
int    nc_ns_objective_grad(nc_ns_ctx* ctx, const double* s_dev, double* g_dev);
/* J~^T lambda = rhs at s (rhs zeroed on constrained dofs), to adjoint_rtol.  Synchronises. */
int    nc_ns_solve_adjoint(nc_ns_ctx* ctx, const double* s_dev, const double* rhs_dev, double* lam_dev, nc_info* info);
/* dfdgamma_e = -lambda_e^T dR_e/dgamma_e through the conductivity and the Brinkman
 * coefficient (zero on passive elements), dfdx = F_R^T dfdgamma (zero off the design
 * domain).  The compliance has no explicit dependence on gamma in this model, so this is
 * its full gradient.  Enqueue only. */
int    nc_ns_sensitivity(nc_ns_ctx* ctx, const double* s_dev, const double* lam_dev, double* dfdx_dev,
                         double* dfdgamma_dev);

#ifdef __cplusplus
}
#endif
#endif /* NC_H */
