/*
 * erem.h - C ABI of the MI355X exponential Rosenbrock-Euler (EREM) library.
 *
 * The library advances the semi-discrete energy equation dT/dt = G(T) of a
 * two-point-flux (TPFA) finite-volume discretisation with upwind advection
 * (Tambue, Berre, Nordbotten, Sec. 3.1) by the EREM step
 *
 *     T^{n+1} = T^n + h phi1(h J_n) G(T^n),   J_n = D_T G(T^n)   (Eq. EERM)
 *
 * with phi1(h J) v evaluated by Newton interpolation at real Leja points
 * (Sec. 4.2, Eqs. lejaa, approle, newt) or by an Arnoldi projection
 * (Sec. 4.1, Eq. approphi, Alg. alg:al2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Cells of an nx x ny x nz Cartesian grid (nz = 1 in 2D) are stored flat,
 *   index x + nx*(y + ny*z).  All field arrays are FP64 unless stated.
 * - Pointers named d_* are DEVICE pointers (HIP global memory on the device
 *   that was current at erem_create).  The caller owns them; the library
 *   reads or writes them only during the call's stream-ordered work and keeps
 *   no reference afterwards (inputs are copied into context storage).
 * - Pointers named h_* or plain out/in are HOST pointers.
 * - Every call enqueues its device work on the stream given to erem_create
 *   (a hipStream_t passed as void*; NULL = the null stream).  Calls that fill
 *   an erem_stats or return host data synchronise that stream before
 *   returning.
 * - Return value: EREM_OK (0) or a negative error code; on error a message is
 *   available from erem_last_error(ctx) and, for erem_step, T is unmodified.
 *   No C++ exception crosses the ABI.
 * - Units are SI; temperatures in degrees C.
 */
#ifndef EREM_H
#define EREM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EREM_OK = 0,
    EREM_EINVAL = -1,      /* invalid argument (sizes, NULL, state order) */
    EREM_ENOMEM = -2,      /* device or host allocation failed */
    EREM_EDEVICE = -3,     /* a HIP runtime call failed */
    EREM_ENOCONV = -4,     /* phi1 or pressure solve did not converge within limits */
    EREM_ENONFINITE = -5   /* NaN or Inf met in a norm */
};

enum { EREM_METHOD_LEJA = 0, EREM_METHOD_KRYLOV = 1 };
enum { EREM_PREC_FP64 = 0, EREM_PREC_MIXED = 1 };
enum { EREM_LAW_CONSTANT = 0, EREM_LAW_WATER = 1 };

typedef struct erem_ctx erem_ctx;

/* Cartesian grid: dim is 2 or 3 (dim 2 requires nz == 1); cell sizes in m. */
typedef struct {
    int32_t dim;
    int64_t nx, ny, nz;
    double dx, dy, dz;
} erem_grid;

/* Options of one phi1 evaluation / EREM step.
 * tol_a, tol_r: absolute / relative tolerance of the scaled error norm
 *   sqrt(1/N sum (e_i / scal)^2), scal = tol_a + tol_r * ||T^n||_inf
 *   (Sec. 4.2).  For erem_phi1_apply, ||T^n||_inf is replaced by h*||v||_inf.
 * p_order: the stop test is 10^p_order * (mean of the last five estimates) < 1.
 * m_max: maximum Leja degree per substep (<= 1024).
 * max_substeps: maximum number of substeps the step may be split into.
 * krylov_m: Arnoldi dimension of the Krylov method.
 * rho_max: a-priori substep rule, substeps s = ceil(h (beta - alpha) / rho_max)
 *   where [alpha, beta] is the Gershgorin interval of J (<= 0 disables).  With
 *   precision MIXED a rho_max above 32 is taken as 32: on an interval of width
 *   rho the Newton terms grow to about e^(rho/10) times the result before they
 *   cancel, and in FP32 that growth is lost accuracy (at 64, about 3e-5 of
 *   the step on the 128^3 layered workload; at 32, below 1e-5).
 * chunk: Leja terms enqueued before the host polls the device stop flag
 *   (0 = automatic). */
typedef struct {
    int32_t method;
    int32_t precision;
    double tol_a, tol_r;
    int32_t p_order, m_max, max_substeps, krylov_m, chunk;
    double rho_max;
} erem_opts;

/* Statistics of the last call that fills them. */
typedef struct {
    int32_t m_total;       /* Leja terms (or Arnoldi steps) summed over substeps */
    int32_t substeps;      /* substeps actually used */
    int32_t iterations;    /* PCG iterations (erem_solve_pressure) */
    int32_t restarts;      /* step restarts after non-convergence */
    double alpha, beta;    /* Gershgorin interval of J */
    double est_err;        /* last scaled error estimate (Leja) / residual (PCG) */
} erem_stats;

/* Fill *opts with the defaults: Leja, FP64, tol_a 0, tol_r 1e-12, p 2,
 * m_max 256, max_substeps 64, krylov_m 10, chunk 0, rho_max 64. */
void erem_default_opts(erem_opts* opts);

/* Create a context for one grid on the current HIP device.  Allocates all
 * device storage the path needs (about 20 FP64 words per cell).  stream is a
 * hipStream_t (or NULL).  Errors: EINVAL for non-positive sizes, dim not in
 * {2,3}, dim 2 with nz != 1; ENOMEM; EDEVICE. */
int erem_create(const erem_grid* grid, void* stream, erem_ctx** out);
int erem_destroy(erem_ctx* ctx);
const char* erem_last_error(const erem_ctx* ctx);

/* Rock: d_logk natural log of the permeability [m^2] and d_poro porosity,
 * both N cells; lambda bulk thermal conductivity [W/m/K]; rhoc_s rock
 * volumetric heat capacity [J/m^3/K].  The arrays are copied (Sec. 2). */
int erem_set_rock(erem_ctx* ctx, const double* d_logk, const double* d_poro,
                  double lambda, double rhoc_s);

/* Fluid: law EREM_LAW_CONSTANT (rho = rho0, mu = mu0) or EREM_LAW_WATER
 * (rho = 1000 (1 - 3e-4 (T - 20)), mu = 2.414e-5 * 10^(247.8/(T + 133)));
 * c_f specific heat [J/kg/K].  The heat capacity of a cell is
 * C = phi rho(T) c_f + (1 - phi) rhoc_s (Sec. 2, local equilibrium). */
int erem_set_fluid(erem_ctx* ctx, int32_t law, double c_f, double mu0, double rho0);

/* Boundary conditions: pressure Dirichlet p_left on the x = 0 face and
 * p_right on the x = nx face (no flow elsewhere); temperature Dirichlet
 * T_left on x = 0 (half-cell conduction when dirichlet_left != 0, and
 * advective inflow), advective outflow on x = nx (inflow there enters at
 * T_right), no heat flux elsewhere (Sec. 3.1 boundary fluxes and upwind
 * rule). */
int erem_set_bc(erem_ctx* ctx, double p_left, double p_right, double T_left, double T_right,
                int32_t dirichlet_left);

/* TPFA transmissibilities of the mass mobility rho(T) K / mu(T) with the
 * harmonic mean |s| k_i k_j / (k_i d_j + k_j d_i) on interior faces and the
 * Dirichlet half-cell |s| k_i / d_i on x faces (Sec. 3.1).  d_T gives the
 * cell temperatures for the fluid laws (NULL: use T = 20 C). */
int erem_assemble_transmissibilities(erem_ctx* ctx, const double* d_T);

/* Steady pressure of the TPFA system sum_s tau_s (p_i - p_nb) = 0 by
 * preconditioned conjugate gradients to relative residual rtol (at most
 * max_iter iterations), then the face mass fluxes F = tau (p_i - p_j)
 * (Darcy's law, Eq. darcy, g = 0).  d_p (N, may be NULL) is read as the
 * initial guess when warm != 0 and receives the pressure; with warm != 0 and
 * d_p NULL the context's own (double-double) pressure of the last solve is
 * the initial guess, and no copy is made; with warm == 2 and d_p NULL the
 * guess is the linear extrapolation 2 p^n - p^(n-1) of the context's last two
 * solutions when the previous call also kept the context's pressure (else
 * p^n, as with warm == 1).  stats (may be NULL) gets iterations and the
 * final relative residual.  ENOCONV if rtol is not reached. */
int erem_solve_pressure(erem_ctx* ctx, double rtol, int32_t max_iter, int32_t warm,
                        double* d_p, erem_stats* stats);

/* Preconditioner of the pressure conjugate gradients: EREM_PRECOND_JACOBI
 * (diagonal) or EREM_PRECOND_MULTIGRID (default: a symmetric V-cycle of
 * 2 x 2 (x 2) cell aggregation with damped-Jacobi smoothing, Galerkin
 * coarse operators, over-relaxed coarse correction).  Both give the same
 * pressure up to the requested tolerance. */
enum { EREM_PRECOND_JACOBI = 0, EREM_PRECOND_MULTIGRID = 1 };
int erem_set_pressure_preconditioner(erem_ctx* ctx, int32_t kind);

/* Set the face mass fluxes [kg/s] directly, replacing the pressure solve:
 * d_fx (nz, ny, nx+1), d_fy (nz, ny+1, nx), d_fz (nz+1, ny, nx; NULL in 2D),
 * positive along +x/+y/+z, boundary faces included. */
int erem_set_face_fluxes(erem_ctx* ctx, const double* d_fx, const double* d_fy,
                         const double* d_fz);

/* Copy the face mass fluxes (same layouts as erem_set_face_fluxes) and the
 * x/y/z face transmissibilities of the last assembly (same layouts; NULL
 * pointers are skipped). */
int erem_get_faces(erem_ctx* ctx, double* d_fx, double* d_fy, double* d_fz,
                   double* d_tx, double* d_ty, double* d_tz);

/* Form the Jacobian J = D_T G (Eq. linear) as a 5-point (2D) or 7-point (3D)
 * stencil and F = G(T) at d_T, with the current face fluxes:
 * G_i = R_i(T) / (V C_i(T)), R_i = sum of the TPFA conductive and upwind
 * advective face terms (Sec. 3.1). */
int erem_form_jacobian(erem_ctx* ctx, const double* d_T);

/* Copy the stencil of J to d_coef (ndir x N, ndir = 5 in 2D, 7 in 3D,
 * direction order centre, -x, +x, -y, +y, -z, +z; a coefficient toward a
 * missing neighbour is 0) and F = G(T) to d_F (N).  Either may be NULL. */
int erem_get_jacobian(erem_ctx* ctx, double* d_coef, double* d_F);

/* Replace J and F by a caller-given stencil (same layout as
 * erem_get_jacobian; coefficients toward missing neighbours must be 0) and
 * F (N values), e.g. for a matrix that does not come from the TPFA model.
 * The Gershgorin interval (Sec. 4.2) is recomputed from the rows. */
int erem_set_jacobian(erem_ctx* ctx, const double* d_coef, const double* d_F);

/* d_out = phi1(h J) d_v for the J of the last erem_form_jacobian
 * (Sec. 4.2 Newton-Leja or Sec. 4.1 Krylov, per opts->method).  d_v and
 * d_out hold N values and must not alias. */
int erem_phi1_apply(erem_ctx* ctx, double h, const double* d_v, double* d_out,
                    const erem_opts* opts, erem_stats* stats);

/* One EREM step in place: forms J and G at d_T with the current fluxes and
 * sets d_T <- d_T + h phi1(h J) G(d_T) (Eq. EERM).  Substeps (Sec. 4.2,
 * splitting when the degree is too large) integrate the linearised problem
 * u' = J u + G(T^n) exactly up to the tolerance: u <- u + delta phi1(delta J)
 * (G + J u).  After a first Leja step on the context (and for budgets of at
 * most 31 terms) the Newton passes are enqueued behind the assembly without
 * a host synchronisation: the substep count is predicted from the previous
 * step's interval width and confirmed afterwards (a failed prediction runs
 * the step again on the interval read back); the result is the same bit for
 * bit.  The call returns after the step has completed on the stream. */
int erem_step(erem_ctx* ctx, double h, double* d_T, const erem_opts* opts, erem_stats* stats);

/* As erem_step but with the J and F already held by the context (from
 * erem_set_jacobian or erem_form_jacobian): d_T <- d_T + h phi1(h J) F. */
int erem_step_frozen(erem_ctx* ctx, double h, double* d_T, const erem_opts* opts,
                     erem_stats* stats);

/* One step of the non-autonomous EREM scheme (Sec. 3.2.3, Eq. nEERMg) in
 * place, for boundary temperatures that change in time: T_left on x = 0 and
 * T_right on x = nx (the values at t_n), changing at the rates dT_left_dt and
 * dT_right_dt [K/s] at t_n.  Sets the context's boundary temperatures to
 * T_left and T_right (they stay so), forms J and G at d_T with the current
 * fluxes, D_t G (b is linear in the boundary temperatures, so D_t G is the
 * boundary vector with the rates in their place, over V C(T)), and sets
 *   d_T <- d_T + h phi1(h J) G + h^2 phi2(h J) D_t G.
 * With s substeps of delta = h / s (the rule of erem_step) it integrates
 * u' = J u + G + t D_t G exactly up to the tolerance:
 *   u <- u + delta phi1(delta J) (G + t_j D_t G + J u) + delta^2 phi2(delta J) D_t G,
 * the last term one Newton-Leja pass with the divided differences of phi2,
 * computed once per step.  Leja method only (EREM_EINVAL for Krylov);
 * EREM_EINVAL for non-finite temperatures or rates.  stats->m_total counts
 * the Newton terms of every pass, the phi2 pass included. */
int erem_step_nonautonomous(erem_ctx* ctx, double h, double T_left, double T_right,
                            double dT_left_dt, double dT_right_dt, double* d_T,
                            const erem_opts* opts, erem_stats* stats);

/* ---- transient (compressible) pressure, Eq. masscon4 / spaceheat3 ----
 *
 * With a slightly compressible fluid and rock the pressure obeys, per cell,
 *   dp/dt = G4 = (b - A p) / (V rho(T) S) + (phi alpha_f / S) G2,
 *   S = phi (beta_f + alpha_b),  alpha_f = -rho'(T) / rho(T),
 * A p = b the TPFA pressure system of the current transmissibilities (Dirichlet
 * x faces at p_left, p_right), G2 = dT/dt.  The sequential scheme (Sec. 3.2.2)
 * takes, per step: transmissibilities at T^n, the face fluxes of p^n
 * (erem_face_fluxes_from_pressure), the EREM temperature step (erem_step,
 * which leaves G2 = G(T^n, p^n) in the context), then the EREM pressure step
 * (Eq. EERM1, erem_step_pressure) with the T^n the caller kept. */

/* Face fluxes F = t (p_i - p_j) of the given pressure d_p (N values, device)
 * with the current transmissibilities, Dirichlet x faces included. */
int erem_face_fluxes_from_pressure(erem_ctx* ctx, const double* d_p);

/* d_p <- d_p + h phi1(h J_p) G4 (Eq. EERM1) with J_p = -diag(1/(V rho S)) A
 * (G2 held fixed in p), at the temperature d_T (T^n; rho, alpha_f and the
 * storage are evaluated there) and the G2 = F of the context's last
 * erem_form_jacobian / erem_step.  alpha_b (rock) and beta_f (fluid
 * compressibility) in 1/Pa, >= 0, not both 0.  phi1 by opts->method (the
 * paper pairs Krylov for the pressure with Leja for the temperature); the
 * error scale is tol_a + tol_r max|p|.  With the Leja method, after a first
 * pressure step and for budgets of at most 31 terms, the Newton passes are
 * enqueued as in erem_step (substep count predicted from the previous
 * pressure step's interval, confirmed afterwards).  Afterwards the context's J and F are
 * J_p and G4: until the next erem_form_jacobian, erem_step or
 * erem_set_jacobian, this call (which needs G2) and erem_get_jacobian,
 * erem_phi1_apply, erem_step_frozen and erem_shifted_solve (which need the
 * heat Jacobian) return EREM_EINVAL and leave their outputs unchanged. */
int erem_step_pressure(erem_ctx* ctx, double h, double* d_p, const double* d_T, double alpha_b, double beta_f,
                       const erem_opts* opts, erem_stats* stats);

/* ---- comparison schemes: Rosenbrock-type methods and theta-Euler ----
 *
 * The linear systems of these schemes, (I/(tau gamma) - J) k = rhs, are
 * solved by BiCGSTAB (the paper's solver, Sec. 3.2.3) with Jacobi right
 * preconditioning, M = diag(sigma - J_ii), from x = 0 to the relative
 * residual rtol (recursive residual).  EREM_ENOCONV on breakdown or when
 * the iteration limit is reached. */

/* x = (sigma I - J)^{-1} b for the J of the last erem_form_jacobian or
 * erem_set_jacobian; sigma > 0, rtol in (0, 1), max_iter >= 1.  d_b and d_x
 * (N values each, device) must not alias.  stats->iterations: BiCGSTAB
 * iterations. */
int erem_shifted_solve(erem_ctx* ctx, double sigma, const double* d_b, double* d_x, double rtol,
                       int32_t max_iter, erem_stats* stats);

#define EREM_ROSM_1 0     /* ROSM(1), Eq. ROS with gamma = 1 */
#define EREM_ROSM_HALF 1  /* ROSM(1/2), Eq. ROS with gamma = 1/2 */
#define EREM_ROS2 2       /* ROS2(1), Eq. ROSMh with Table ros2 */
#define EREM_ROS3P 3      /* ROS3p, Eq. ROSMh with Table ros3 */

/* One Rosenbrock-type step in place on d_T for the autonomous heat model
 * with the current fluxes (Eq. ROSMh, D_t f = 0): J and G are formed at d_T,
 * then for each stage i
 *   (I/(h gamma) - J) k_i = G(T + sum_{j<i} a_ij k_j) - sum_{j<i} (c_ij / h) k_j
 * and d_T <- d_T + sum_i b_i k_i; ROSM(gamma) is the one-stage case
 * T + h (I - h gamma J)^{-1} G(T) (Eq. ROS).  lin_rtol: relative residual of
 * every stage solve.  stats->substeps: stages; stats->iterations: BiCGSTAB
 * iterations summed over the stages.  The context keeps J and G of the
 * start of the step. */
int erem_step_rosenbrock(erem_ctx* ctx, double h, int32_t scheme, double* d_T, double lin_rtol,
                         erem_stats* stats);

/* The same step for boundary temperatures that change in time (Eq. ROSf,
 * Eq. ROSMh with D_t f): T_left_stage[i], T_right_stage[i] (host arrays, one
 * value per stage) are the boundary temperatures at the stage times
 * t_n + alpha_i h (alpha = (0) for ROSM, (0, 1) for ROS2(1), (0, 1, 1) for
 * ROS3p), dT_left_dt and dT_right_dt their rates at t_n.  J and G are formed
 * at t_n, D_t f at t_n as in erem_step_nonautonomous, G of stage i at its
 * stage time, and stage i adds h gamma_i D_t f to its right-hand side.  The
 * context's boundary temperatures are left at the stage-0 values. */
int erem_step_rosenbrock_nonautonomous(erem_ctx* ctx, double h, int32_t scheme, const double* T_left_stage,
                                       const double* T_right_stage, double dT_left_dt, double dT_right_dt,
                                       double* d_T, double lin_rtol, erem_stats* stats);

/* One theta-Euler step in place (Eq. temscheme): X = T^{n+1} solves
 *   X - h theta G(X) - h (1 - theta) G(T^n) - T^n = 0
 * by Newton's method from X_0 = T^n, (I - h theta J(X_k)) dX = -F(X_k), until
 * max|dX| <= newton_rtol max|T^n| (at most max_newton iterations, else
 * EREM_ENOCONV with d_T unchanged).  theta in [0, 1]; theta = 0 is the
 * explicit Euler step.  stats->substeps: Newton iterations;
 * stats->iterations: BiCGSTAB iterations summed over them. */
int erem_step_theta(erem_ctx* ctx, double h, double theta, double* d_T, double newton_rtol,
                    double lin_rtol, int32_t max_newton, erem_stats* stats);

/* ---- sequential coupled step and its adjoint (2D grids) ----
 *
 * The coupled step of Sec. 3.2.2 (pressure first, then temperature): TPFA
 * transmissibilities of rho(T) K / mu(T) at T^n, steady pressure, face mass
 * fluxes, J and G at T^n, then the EREM step T^{n+1} = T^n + h phi1(h J) G
 * (Eq. EERM) by Newton-Leja substeps (Sec. 4.2).  The discrete choices of the
 * step -- Gershgorin interval, substep count and the Newton-Leja degree of
 * every substep -- form its tape.  Replaying a tape evaluates exactly the
 * same polynomial in J without stop tests, so the step becomes a smooth map
 * of (T^n, log K) near the recorded point; the adjoint differentiates that
 * map. */
#define EREM_TAPE_MAX_SUBSTEPS 256
typedef struct {
    int32_t substeps;                    /* s; 0 marks a step without Leja terms */
    int32_t m[EREM_TAPE_MAX_SUBSTEPS];   /* Newton-Leja terms applied in substep j */
    double alpha, beta;                  /* Gershgorin interval of J used by the step */
} erem_tape;

/* One coupled step in place on d_T (N values).  The pressure is solved from
 * a zero initial guess to relative residual p_rtol (erem_solve_pressure).
 * tape_in == NULL: the step chooses as erem_step does; otherwise it replays
 * tape_in (method Leja, FP64).  tape_out (may be NULL) receives the choices
 * used (Leja, FP64 only).  EINVAL for 3D grids, a Krylov or mixed-precision
 * opts with a tape, or a tape whose substeps are outside [1, 256] or whose
 * degrees are outside [1, m_max]. */
int erem_coupled_step(erem_ctx* ctx, double h, double* d_T, double p_rtol, const erem_opts* opts,
                      const erem_tape* tape_in, erem_tape* tape_out, erem_stats* stats);

/* Adjoint of erem_coupled_step with the choices of `tape`: given T^n in d_T
 * (unchanged) and Tbar = d phi / d T^{n+1} in d_Tbar, overwrite d_Tbar with
 * d phi / d T^n and ADD d phi / d log K to d_logk_bar (N values each, device).
 * The step is recomputed from T^n; the Leja iterates q_k of every substep are
 * kept on the device when ckpt_stride is 1, or every ckpt_stride-th of them
 * with the others recomputed segment by segment during the reverse sweep.
 * The reverse Newton recurrence runs with the transposed stencil of J; the
 * pressure adjoint is a second solve with the same symmetric matrix to
 * relative residual max(p_rtol, 1e-12).  Errors as erem_coupled_step, plus EINVAL for
 * ckpt_stride < 1 and ENOMEM if the iterate store does not fit. */
int erem_coupled_step_adjoint(erem_ctx* ctx, double h, const double* d_T, double p_rtol,
                              const erem_opts* opts, const erem_tape* tape, int32_t ckpt_stride,
                              double* d_Tbar, double* d_logk_bar, erem_stats* stats);

/* ---- batched form: many independent linear problems in one graph launch ----
 *
 * Each problem is a 2D grid with fixed face fluxes and constant heat capacity
 * (constant fluid law), so G_p(T) = J_p T + g_p with constant J_p and the EREM
 * step (Eq. EERM) uses a fixed Gershgorin interval, substep count and set of
 * divided differences per problem (Sec. 4.2).  erem_batch_run advances all
 * problems by nsteps steps.  The problems are cut into 64 x rows tiles that
 * form one list; a run is a sequence of phases, and each phase is one work
 * launch over the whole list - every problem that is not done takes one step
 * of its own schedule: a substep's start pass (q_0, p = d_0 q_0), four Newton
 * terms (Eq. newt) staged in LDS, or the last step's T update - followed by a
 * control launch that reduces each problem's tile partials in a fixed order
 * (so runs are bit-for-bit reproducible), applies the stop test of Sec. 4.2
 * and picks the problem's next phase.  With use_graph the whole sequence is
 * one hipGraph, captured on first use with the number of phases a
 * calibration run on a copy of T needed plus a margin; a run that needs more
 * continues with launches from the host.  Temperatures are packed: problem i
 * owns cells [off_i, off_i + nx_i ny_i) of the caller's array
 * (erem_batch_offsets). */
typedef struct erem_batch erem_batch;

typedef struct {
    int64_t terms_total;   /* Newton-Leja terms summed over problems and steps */
    int32_t terms_min, terms_max;  /* per problem, over the run */
    int32_t failed;        /* problems that stopped on an error (see the return code) */
    int32_t tile_shape;    /* 0: 64 x 8 tiles on 512 threads, 1: 64 x 16 on 1024 threads,
                              2: 64 x 8 on 512 threads, 3: 64 x 16 on 512, 4: 64 x 32 on
                              512, all with four Newton terms per pass; 5: 64 x 16 and
                              6: 64 x 8 and 7: 64 x 32 on 512 threads with eight terms per
                              pass; each XCD takes a contiguous range of tiles in 2-7.  The stop test is
                              evaluated term by term after each pass and all terms of the
                              pass are kept (the applied degree is the first multiple of
                              the pass width at which the test holds) */
    int32_t graph;         /* 1 if the run was replayed from a hipGraph */
    int32_t grid;          /* workgroups of a work launch (tiles) */
    double ms;             /* device time of the run (HIP events) */
    double leja_bytes;     /* algorithmic bytes of the Newton terms: sum over
                              problems of terms x cells x (72 B FP64, 36 B FP32) */
    int32_t phases;        /* work passes the longest problem needed */
    int32_t work_timed;    /* work launches timed (erem_batch_profile) */
    int64_t passes;        /* work launches of the run (graph budget included) */
    double work_ms;        /* summed device time of the timed work launches */
} erem_batch_stats;

/* nprob 2D grids (dim 2, nz 1).  Errors: EINVAL, ENOMEM, EDEVICE. */
int erem_batch_create(int32_t nprob, const erem_grid* grids, void* stream, erem_batch** out);
int erem_batch_destroy(erem_batch* b);
const char* erem_batch_last_error(const erem_batch* b);
/* Host array of nprob + 1 cell offsets of the packed layout. */
int erem_batch_offsets(const erem_batch* b, int64_t* out);
/* Problem i: rock, constant fluid law, boundary conditions as for the
 * single-problem context; computes the steady pressure, the face fluxes, the
 * Jacobian stencil and g at d_T0 (device, N_i values). */
int erem_batch_set_problem(erem_batch* b, int32_t i, const double* d_logk, const double* d_poro,
                           double lambda, double rhoc_s, double c_f, double mu0, double rho0,
                           double p_left, double p_right, double T_left, double T_right,
                           const double* d_T0);
/* Fix the step h and the options for every problem: Gershgorin interval,
 * substeps s = ceil(h (beta - alpha) / rho_max) (at most max_substeps),
 * divided differences up to m_max; opts->precision selects FP64 or FP32
 * Newton passes.  EINVAL for a problem whose interval is degenerate
 * (beta - alpha <= 1e-14 max(|alpha|, |beta|), e.g. one cell: J = c I), for
 * the Krylov method, m_max outside [5, 1024] or bad tolerances. */
int erem_batch_prepare(erem_batch* b, double h, const erem_opts* opts);
/* Time every tile shape on a copy of d_T (nsteps steps) and keep the fastest;
 * *chosen receives its index.  d_T is not modified. */
int erem_batch_autotune(erem_batch* b, const double* d_T, int32_t nsteps, int32_t* chosen);
/* Select a tile shape by index (0 .. 7, see erem_batch_stats.tile_shape)
 * instead of timing them.  EINVAL for another index. */
int erem_batch_set_tile_shape(erem_batch* b, int32_t shape);
/* Time every stride-th work launch of the following runs by the start and
 * stop events of its own dispatch; 0 turns it off.  While it is on, runs are
 * enqueued from the host (use_graph is ignored: a graph cannot carry the
 * dispatch events).  The sums go to erem_batch_stats.work_ms / work_timed.
 * EINVAL for stride < 0. */
int erem_batch_profile(erem_batch* b, int32_t stride);
/* Advance the packed temperatures d_T by nsteps EREM steps; use_graph != 0
 * replays one hipGraph (captured on first use per nsteps, tile shape and T
 * array).  Synchronises the batch's stream.  ENOCONV / ENONFINITE (EINVAL for
 * a zero error scale) if a problem failed: the others are still advanced and
 * a failed problem's cells hold the T of its last completed step. */
int erem_batch_run(erem_batch* b, double* d_T, int32_t nsteps, int32_t use_graph, erem_batch_stats* st);

/* ---- allocation-free evaluation ----
 *
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): out = phi1(h J) v, the operation of
 * erem_set_jacobian(J) followed by erem_phi1_apply, without a context.
 * d_coef is J as a 5-point (2D) or 7-point (3D) stencil in the context's
 * layout (ndir x N, SoA: centre, -x, +x, -y, +y, -z, +z; 0 toward missing
 * neighbours), d_v and d_out N values; all device pointers owned by the
 * caller, d_out distinct from d_v.  FP64, Leja method only; opts as for
 * erem_phi1_apply (the term budget starts at opts->chunk if > 0, else m_max).
 * Every device buffer of the evaluation lives in one statically sized array
 * of the library (13.1 MB per GPU, held until the process ends); the first
 * call on a device looks up that device's copy and, once per process,
 * computes the Leja points; after that set-up a call allocates nothing,
 * host or device.
 * Limits: N <= 262144 cells, at most 16384 blocks of 64 x 4 cells
 * (ceil(nx/64) ceil(ny/4) nz), m_max <= 256, at most 64 substeps; beyond
 * them EREM_EINVAL.  The call enqueues on `stream` and synchronises it.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the
 * caller.  Returns EREM_OK, EREM_EINVAL (bad arguments or limits),
 * EREM_ENOCONV, EREM_ENONFINITE (non-finite J or v), EREM_EDEVICE; d_out is
 * written only on EREM_OK.  stats (may be NULL) as for erem_phi1_apply. */
int erem_phi1_apply_noalloc(const erem_grid* grid, const double* d_coef, double h, const double* d_v,
                            double* d_out, const erem_opts* opts, void* stream, erem_stats* stats);

/* ---- measurement support ---- */

/* Accumulated device time of the hot kernels while profiling is on,
 * measured with a HIP event before and after each launch on the context's
 * stream.  Only launches that did work are counted (a Leja term launch
 * after the stop test passed, or a PCG iteration after convergence,
 * returns at entry and is left out). */
typedef struct {
    double leja_term_ms;        /* Newton-Leja term kernels (Eq. newt) */
    int64_t leja_term_launches;
    double pcg_a_ms;            /* PCG: search direction + operator apply */
    int64_t pcg_a_launches;
    double pcg_b_ms;            /* PCG: iterate / residual / preconditioner update */
    int64_t pcg_b_launches;
    double mg_ms;               /* multigrid preconditioner (all its kernels) */
    int64_t mg_cycles;
    double adj_rev_ms;          /* reverse Newton-Leja term kernel (adjoint) */
    int64_t adj_rev_launches;
    double bicg_ms;             /* BiCGSTAB iteration (its three kernels) */
    int64_t bicg_iterations;
} erem_kernel_times;

/* Per-launch event timing: enable = 0 turns it off, enable = n > 0 times one
 * launch in n (Newton terms whose index is a multiple of n, CG iterations
 * whose index is a multiple of n: a sample that keeps the event overhead
 * small), and resets the counters.  Synchronises the stream.  Up to 8
 * substeps per evaluation are timed.  The averages are per timed launch. */
int erem_profile(erem_ctx* ctx, int32_t enable);
int erem_profile_read(erem_ctx* ctx, erem_kernel_times* out);

/* ---- host-side numerics (no device work; callable without a GPU) ---- */

/* The first n real Leja points of [-2, 2] (Eq. lejaa): xi_0 = 2, then each
 * new point maximises prod_k |xi - xi_k| over the interval; ties take the
 * larger point.  n <= 1024. */
int erem_leja_points(int32_t n, double* out);

/* Newton divided differences d_k = g[xi_0..xi_k], k < n, of
 * g(xi) = phi1(hc + hg xi) at the points xi (host array of n values),
 * computed as the first column of phi1(hc I + hg L) with L lower bidiagonal
 * (diagonal xi, subdiagonal 1) (Sec. 4.2), through the exponential of the
 * augmented lower-bidiagonal matrix by Taylor scaling-and-squaring. */
int erem_phi1_divided_differences(double hc, double hg, const double* xi, int32_t n,
                                  double* out);

/* The same for g(xi) = phi2(hc + hg xi), phi2(z) = (e^z - 1 - z) / z^2
 * (Sec. 3.2.3): the first column of phi2(hc I + hg L), read off the
 * exponential of the bidiagonal matrix augmented by two leading rows and
 * columns.  Same argument rules as erem_phi1_divided_differences. */
int erem_phi2_divided_differences(double hc, double hg, const double* xi, int32_t n,
                                  double* out);

#ifdef __cplusplus
}
#endif
#endif /* EREM_H */
