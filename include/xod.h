/*
 * xod.h -- C ABI of the implicit photochemical column solver (libxod).
 *
 * The library integrates the coupled species-continuity equations of a 1-D
 * atmospheric column (Section 2.1, Eq. continuity):
 *
 *     dn_y/dt = P_y - L_y - d(phi_y)/dz ,   y = 1..S
 *
 * with the transport flux of Eq. transportflux (eddy + molecular diffusion),
 * discretised on N layers (Eq. discrete_continuity, Eq. dzz) with zero-flux
 * boundaries (Section 2.5), chemistry from two-body (Kooij / modified
 * Arrhenius), three-body (Lindemann) and photolysis reactions with reverse
 * rates from NASA-7 Gibbs energies (Section 2.3), by linearly implicit
 * backward-Euler steps (Section 2.1 lists backward Euler among the implicit
 * integrators).  Each step solves the block-tridiagonal system
 *
 *     a_k * x_{k-1} + B_k x_k + c_k * x_{k+1} = F_k(n),   B_k = I/dt - dF_k/dn_k
 *
 * (S x S dense diagonal blocks, diagonal off-diagonal blocks a_k, c_k) by a
 * block Thomas elimination whose Schur complements are inverted on the GPU.
 *
 * Conventions
 *   - Every function returns xod_status; XOD_OK == 0.  No exception crosses
 *     the ABI.  xod_last_error() returns a thread-local message naming the
 *     failing column / layer / row where that applies.
 *   - Units are CGS (cm^-3, s, K); pressures are given in bar.
 *   - Layer k = 0 is the bottom of the column.  Arrays are layer-major:
 *     n[k*S + y], kf[k*R + r], B[(k*ld + i)*ld + j].
 *   - Host arrays passed to *_create are copied; the caller keeps ownership.
 *     The library owns every device allocation inside a handle and frees it
 *     in *_destroy.
 *   - Pointers passed to the hot-path calls (xod_rates .. xod_btd_solve) are
 *     DEVICE pointers owned by the caller (e.g. torch tensors' data_ptr());
 *     the library never frees them.  Work is enqueued on the column's HIP
 *     stream and is asynchronous unless stated otherwise.
 *   - After an error no partial result is promised; the column state of
 *     xod_step / steady-state calls is left unchanged on a rejected step.
 */
#ifndef XOD_H
#define XOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  XOD_OK = 0,
  XOD_EINVAL = 1,         /* bad argument: null pointer, size, index range  */
  XOD_ENOMEM = 2,         /* device allocation failed                        */
  XOD_ESINGULAR = 3,      /* zero / non-finite pivot in a Schur complement   */
  XOD_ENOTCONVERGED = 4,  /* step rejected too often / refinement stalled    */
  XOD_ENONFINITE = 5,     /* NaN or Inf in a state or right-hand side        */
  XOD_EHIP = 6,           /* HIP runtime error                               */
  XOD_ENOTIMPL = 7,       /* size outside the supported range                */
  XOD_EBUSY = 8           /* serving: no slot or memory free right now       */
} xod_status;

typedef enum {
  XOD_FP64 = 0,   /* every kernel in FP64                                      */
  XOD_MIXED = 1   /* Schur complements and their inverses in FP32 with row
                     scaling, FP64 rates / residuals / pivot blocks and FP64
                     iterative refinement of every solve                       */
} xod_precision;

/* How a column's step system (block tridiagonal, Section 2.1) is factored.
 * Both give the solution of the same block system; they differ only in the
 * elimination order and hence in rounding. */
typedef enum {
  XOD_SOLVER_THOMAS = 0,  /* block Thomas: layers eliminated bottom to top,
                             N dependent block inversions                     */
  XOD_SOLVER_CR = 1       /* block cyclic reduction: odd-indexed layers of
                             each level eliminated together (both ends when
                             three remain), at most ceil(log2 N)+1 dependent
                             batched inversions (8 for N = 150) plus dense
                             block products on the matrix cores; needs about
                             2N further ld x ld blocks of workspace         */
} xod_solver;

enum { XOD_MAX_REAC = 3, XOD_MAX_PROD = 3 };
enum { XOD_RT_BIMOL = 0, XOD_RT_TERMOL = 1, XOD_RT_PHOTO = 2 };

typedef struct xod_network xod_network;   /* opaque, device-resident */
typedef struct xod_column xod_column;     /* opaque, owns state + workspace */
typedef struct xod_batch xod_batch;       /* set of columns stepped together */
typedef struct xod_server xod_server;     /* continuous-batching request loop */

/* Reaction network (Section 2.2-2.3).  Host arrays, copied at create.
 *   elem_comp [E*S]    atom counts a_{e,y} (diagnostics only)
 *   mass_amu  [S]      molecular masses
 *   nasa7     [S*2*7]  NASA-7 sets, low range then high range per species
 *                      (Appendix A); the high range is used iff T >= t_mid
 *   rtype     [R]      XOD_RT_BIMOL | XOD_RT_TERMOL | XOD_RT_PHOTO
 *   reac,prod [R*3]    species ids, -1 padded; a repeated id is a power;
 *                      the third body M is never listed
 *   reversible[R]      1: k_r = k_f / K_c from Gibbs energies (Section
 *                      2.3.4); ignored for photolysis (always irreversible)
 *   tb_kooij  [R]      1: T_b = T/300 (Kooij), 0: T_b = T (mod. Arrhenius)
 *   params    [R*6]    two-body (ln alpha, beta, gamma, -, -, -);
 *                      three-body (ln alpha0, beta0, gamma0, ln alpha_inf,
 *                      beta_inf, gamma_inf); photolysis (ln J0, -, ...).   */
typedef struct {
  int32_t S, R, E;
  const int32_t *elem_comp;
  const double *mass_amu;
  const double *nasa7;
  double t_mid;
  const int32_t *rtype;
  const int32_t *reac;
  const int32_t *prod;
  const int32_t *reversible;
  const int32_t *tb_kooij;
  const double *params;
} xod_network_desc;

/* Column profile.  Host arrays, copied at create.
 *   P_bar, T_K, Kzz [N]   bottom (k = 0) to top; P strictly decreasing
 *   Dmol  [N*S] or NULL   molecular-diffusion coefficients (NULL = 0)
 *   alphaT [S] or NULL    thermal-diffusion factors (NULL = 0)
 *   mbar_amu, g_cgs       mean molecular mass and gravity (hydrostatic grid)
 *   sigma_tau             gray cross section: tau_k = sigma_tau times the
 *                         total-gas column above the layer midpoint
 *                         (Section 2.3.3, with t_f = mu = 1).              */
typedef struct {
  int32_t N;
  const double *P_bar, *T_K, *Kzz;
  const double *Dmol;
  const double *alphaT;
  double mbar_amu, g_cgs, sigma_tau;
} xod_profile;

/* ---- lifecycle -------------------------------------------------------- */

/* Validates the description (species ids in range, S >= 1, R >= 0, S <=
 * 1024), builds the incidence and Jacobian-pattern tables on the host and
 * uploads everything.  XOD_EINVAL on a bad description. */
xod_status xod_network_create(const xod_network_desc *desc, xod_network **out);
xod_status xod_network_destroy(xod_network *net);
xod_status xod_network_sizes(const xod_network *net, int32_t *S, int32_t *R,
                             int32_t *ld);

/* Allocates the column's device state and workspace (dense blocks: N*ld*ld
 * doubles, or floats in XOD_MIXED, ld = S rounded up to 32), runs the grid
 * set-up kernel (number densities, half levels, hydrostatic heights, optical
 * depths, transport coefficients, Gibbs energies) and uploads n0 (host,
 * [N*S] cm^-3).  hip_stream may be NULL (default stream).  The network
 * must outlive the column. */
xod_status xod_column_create(const xod_network *net, const xod_profile *prof,
                             const double *n0, xod_precision prec,
                             void *hip_stream, xod_column **out);
xod_status xod_column_destroy(xod_column *col);

/* State transfer (synchronous).  n is a HOST pointer [N*S]; t and dt may be
 * NULL.  The state (n, t, dt) is the whole checkpoint of a column; setting
 * it also clears the step history (BDF2's previous step, the mixed-precision
 * step size that fell back to FP64). */
xod_status xod_column_get_state(const xod_column *col, double *n, double *t,
                                double *dt);
xod_status xod_column_set_state(xod_column *col, const double *n, double t,
                                double dt);
/* Device pointer of the column's state n [N*S] (owned by the column). */
xod_status xod_column_state_ptr(xod_column *col, double **n_dev);
/* Grid quantities (host copies, any pointer may be NULL): n_gas [N],
 * tau [N], dz [N]; mix_time = max over half levels and species of
 * dzh^2 / (K + D). */
xod_status xod_column_grid(const xod_column *col, double *ngas, double *tau,
                           double *dz, double *mix_time);

/* Select the factorisation used by xod_step and
 * xod_integrate_to_steady_state on this column (default XOD_SOLVER_THOMAS).
 * XOD_SOLVER_CR allocates its workspace on first selection (XOD_ENOMEM if
 * it does not fit).  The explicit-block calls xod_btd_factor / xod_btd_solve
 * use the column's solver too.  The FP64 fallback of a mixed-precision solve
 * uses the column's solver in FP64 (a mixed column with XOD_SOLVER_CR holds
 * FP64 and FP32 cyclic-reduction workspaces). */
xod_status xod_column_set_solver(xod_column *col, xod_solver solver);

/* ---- hot-path calls (device pointers, asynchronous on the column stream) */

/* Rate coefficients (Section 2.3): kf, kr [N*R].  Two-body:
 * alpha T_b^beta exp(-gamma/T); three-body: Lindemann with [M] = n_gas,k;
 * photolysis: J0 exp(-tau_k); reverse: k_r = k_f exp(dg - dnu ln(P0/kT)),
 * i.e. k_f / K_c with K_c = exp(-dg) (P0/kT)^dnu. */
xod_status xod_rates(xod_column *col, double *kf, double *kr);

/* Right-hand side F(n) = P - L - d(phi)/dz [N*S] for the given rate
 * coefficients (from xod_rates) and state n [N*S]. */
xod_status xod_rhs(xod_column *col, const double *kf, const double *kr,
                   const double *n, double *f);

/* Step matrix blocks of M = I/dt - dF/dn at state n:
 *   B [N*ld*ld] dense diagonal blocks (rows/columns >= S padded with the
 *   identity), a, c [N*ld] sub/super-diagonal coupling (zero padded;
 *   a_0 = c_{N-1} = 0).  ld must be >= S and a multiple of 32. */
xod_status xod_jacobian(xod_column *col, const double *kf, const double *kr,
                        const double *n, double dt, double *B, double *a,
                        double *c, int32_t ld);

/* Factorisation of the block-tridiagonal system M = (B, a, c) of
 * xod_jacobian (Section 2.1: the step matrix I/dt - dF/dn, S x S diagonal
 * blocks, diagonal couplings; B padded with the identity), in precision
 * `prec` with the column's solver (xod_column_set_solver):
 *   XOD_FP64 + block Thomas: in place.  For k = 0..N-1 the Schur complement
 *     D'_k = B_k - diag(a_k) D'_{k-1}^{-1} diag(c_{k-1}) is inverted by
 *     Gauss-Jordan elimination with partial pivoting (implicit row pivoting:
 *     the unused row of largest magnitude, compared to 42 mantissa bits,
 *     lowest row among equals).  On return block k holds W_k and
 *     piv[k*ld+j] the row chosen as pivot for column j, such that
 *     (D'_k^{-1})[j][i] = W_k[piv[j]][q(i)], q = inverse permutation of piv.
 *   XOD_FP64 + cyclic reduction, and XOD_MIXED with either solver: B, a, c
 *     are read only and piv is not used (may be NULL).  The factors are held
 *     in the column's own workspace until its next factor, step, solver
 *     switch or batch: FP64 factors of a copy of the system, or, in
 *     XOD_MIXED, FP32 factors of the row-scaled system (each row of B, a, c
 *     divided by its largest magnitude), the FP64 B, a, c serving the
 *     refinement of xod_btd_solve (the caller keeps them unchanged until
 *     then).  A column created in FP64 allocates its FP32 blocks (N ld^2
 *     floats) on the first mixed factorisation.
 * XOD_ESINGULAR (layer and column in xod_last_error) on a zero or
 * non-finite pivot.  Synchronises the stream to read the singular flag. */
xod_status xod_btd_factor(xod_column *col, double *B, const double *a,
                          const double *c, int32_t ld, int32_t *piv,
                          xod_precision prec);

/* Solve M x = rhs with the factorisation of xod_btd_factor (same column and
 * the same B, a, c, piv pointers), rhs [N*S] overwritten by x:
 *   block Thomas FP64: g'_k = g_k - a_k * D'^{-1}_{k-1} g'_{k-1};
 *     x_k = D'^{-1}_k (g'_k - c_k * x_{k+1}) with the factors in B, piv;
 *   cyclic reduction FP64: substitution through the held levels;
 *   XOD_MIXED: x from the FP32 factors, then up to max_refine refinements
 *     x += M32^{-1} (rhs - M x) with the residual in FP64 from the caller's
 *     B, a, c, stopping once no component moves by more than rtol of |x_i|
 *     or atol of its layer's largest |x| (the rule and options of xod_step);
 *     if the corrections stall above ten times that, or max_refine runs
 *     out first, the system is refactored and solved in FP64 (max_refine 0:
 *     the FP32 solution as it is).
 * max_refine in 0..100 (ignored in FP64).  XOD_EINVAL when the column holds
 * no factorisation of these B, a, c (cyclic reduction and mixed precision
 * need xod_btd_factor first).  Mixed solves synchronise the stream. */
xod_status xod_btd_solve(xod_column *col, const double *B, const double *a,
                         const double *c, int32_t ld, const int32_t *piv,
                         double *rhs, int32_t max_refine);

/* Refinements, FP64 fallback (0/1) and the last componentwise correction
 * size of the column's last xod_btd_solve (0 for FP64 solves); any pointer
 * may be NULL. */
xod_status xod_btd_solve_info(const xod_column *col, int32_t *refine_iters,
                              int32_t *fp64_fallback, double *correction);

/* One linearly implicit backward-Euler step of the column state:
 * solve (I/dt - J(n)) delta = F(n), n <- n + delta (no clipping).  In
 * XOD_MIXED each refinement solves for the FP64 residual (computed from the
 * reaction list and the transport coefficients) with the FP32 factors and
 * adds the correction d; it stops once every component whose new mixing
 * ratio exceeds 1e-30 moved by at most rtol of its new density or by atol of
 * its layer's largest increment, |d_i| <= rtol |n_i + delta_i| + atol
 * max_k |delta_k| (rtol 1e-7, atol 1e-14: options "refine_tol_exp",
 * "refine_atol_exp"), or, once the corrections stop halving or after 10
 * refinements, if they are within ten times that; otherwise the step is
 * refactored and solved in FP64.  After such a fallback at step size dt_f,
 * the column's next steps of size >= dt_f go to FP64 directly (option
 * "mixed_sticky", default 16 steps; fp64_fallback 1, refine_iters 0), then
 * FP32 is tried again; one that converges at a size >= dt_f clears dt_f.
 * The larger steps' FP32 factors would not converge either: along a
 * steady-state solve of the 594-species column every step from dt ~ 2 s on
 * fell back.  Synchronous (reads the statistics). */
typedef struct {
  double max_rel_change;   /* max |delta| / |n_new| over n_new/n_gas > 1e-30 */
  double min_ratio;        /* min n_new / n_gas                               */
  double resid_inf;        /* final correction ratio (mixed) or 0            */
  int32_t refine_iters;    /* refinement iterations used (mixed)              */
  int32_t fp64_fallback;   /* 1 if the mixed solve fell back to FP64          */
  int32_t nonfinite;       /* 1 if the new state holds NaN / Inf              */
  int32_t pad_;
} xod_step_stats;
xod_status xod_step(xod_column *col, double dt, xod_step_stats *stats);

/* One backward-Euler step with the step matrix of the last xod_step
 * frozen (the factor-reusing family of stiff integrators): solve
 * (I/dt - J(n_f)) Delta = F(n) with the factorisation xod_step left for the
 * state n_f it started from, at the current state n, then n <- n + Delta.
 * Rates and F are those of n (spectral photolysis too).  Costs the rates,
 * F, the solve and the update, no Jacobian and no factorisation.  FP64
 * columns; dt must equal the dt of that factorisation (XOD_EINVAL
 * otherwise, or when no factorisation is held: after creation, a solver
 * switch, a boundary change or a mixed-precision step).  The factorisation
 * may also come from xod_step_ros2 (of gamma dt), xod_step_bdf2 (of
 * h = (1+w)/(1+2w) dt, w the step ratio; 2dt/3 at constant step) or
 * xod_step_newton.  A column that joined a batch holds none.  st as for
 * xod_step (resid_inf, refine_iters 0). */
xod_status xod_step_frozen(xod_column *col, double dt, xod_step_stats *st);

/* One step of the two-stage, second-order, L-stable Rosenbrock method ROS2
 * (Verwer, Spee, Blom and Hundsdorfer 1999; Section 2.1 names Rosenbrock
 * solvers among the stiff integrators for this problem) on the same step
 * matrix and block-tridiagonal solver as xod_step: with g = 1 + 1/sqrt 2,
 * M = I/(g dt) - J(n) is factored once and solved twice,
 *   M d1 = F(n),  M d2 = F(n + d1/g) - 2 d1/(g dt),  n <- n + (3 d1 + d2)/(2g).
 * Rates (spectral photolysis too) are those of n for both stages.  FP64
 * columns (XOD_EINVAL for mixed), dt > 0.  Leaves the factorisation of
 * g dt held, so xod_step_frozen(col, g*dt) may follow.  st as for xod_step
 * (resid_inf, refine_iters 0); XOD_ENONFINITE leaves the state unchanged. */
xod_status xod_step_ros2(xod_column *col, double dt, xod_step_stats *st);

/* One backward-Euler step solved by modified Newton (the corrector of the
 * DLSODES family Section 2.1 names): the linearised step Delta = M^-1 F(n),
 * M = I/dt - J(n), then iters - 1 corrections reusing M's factorisation,
 *   Delta += M^-1 (F(n + Delta) - Delta/dt),
 * toward the solution of n1 - n - dt F(n1) = 0.  iters = 1 is xod_step.
 * The corrections converge only while the stale M is close enough (small
 * dt or near steady state): there is no convergence test, and a diverging
 * iteration ends in XOD_ENONFINITE with the state unchanged.  FP64 columns,
 * iters in 1..64 (XOD_EINVAL otherwise).  st as for xod_step, refine_iters
 * = iters - 1.  Leaves the factorisation of dt held. */
xod_status xod_step_newton(xod_column *col, double dt, int32_t iters, xod_step_stats *st);

/* One step of the second-order backward differentiation formula BDF2 (the
 * BDF family of the DLSODES solver Section 2.1 names) with variable step,
 * linearised about the current state n (one Newton iteration from n).  With
 * w = dt/dt_prev, dt_prev the previous step's size:
 *   n_new - (1+w)^2/(1+2w) n + w^2/(1+2w) n_prev = (1+w)/(1+2w) dt F(n_new)
 * becomes, with h = (1+w)/(1+2w) dt,
 *   (I/h - J(n)) Delta = F(n) + w^2/(1+2w) (n - n_prev)/h,  n <- n + Delta
 * (w = 1: h = 2dt/3, history term (n - n_prev)/(2 dt)).  n_prev is the
 * state the previous step started from; that step must be a completed
 * xod_step, xod_step_frozen, xod_step_ros2, xod_step_bdf2 or
 * xod_step_newton on this column (XOD_EINVAL otherwise: after creation,
 * xod_column_set_state, a failed step, a batch step or the steady-state
 * driver).  Ratios w above 1 + sqrt 2 make the formula unstable over many
 * steps; they are not refused.  FP64 and mixed columns (the mixed solve
 * refines against the same right-hand side).  Leaves the factorisation of
 * h held.  st as for xod_step. */
xod_status xod_step_bdf2(xod_column *col, double dt, xod_step_stats *st);

/* Adaptive driver to steady state; each step is a backward-Euler step, or
 * with method 1 a ROS2 step (xod_step_ros2), or with method 2 a
 * backward-Euler step on a step matrix kept across steps (below), under the
 * same control:
 *   reject (dt /= 2) if the step is not finite or a species whose mixing
 *   ratio exceeded y_sig falls below mixing ratio -y_neg; accept otherwise,
 *   clip negatives to zero (so a clipped overshoot adds at most y_neg of the
 *   layer's gas to a species per step) and set dt *= 2 / 1.2 / 0.7 for a
 *   control change c < 0.5 / < 0.9 /
 *   otherwise, c = max |n1 - n0| / max(n0, n1) over mixing ratios > y_sig;
 *   converged when max |dn| / n over mixing ratios > y_floor is < tol_rel
 *   with dt >= the mixing time (Section 3.2), or when t >= t_end.
 * Method 2 (FP64 columns) amortises factorisations after the corrector of
 * the DLSODES family Section 2.1 names: a step of size dt solves
 * n1 - n - dt F(n1) = 0.  With a fresh factorisation of M = I/dt - J(n) it
 * takes the first Newton iterate (the plain linearly implicit step); with
 * a held one, factored at an earlier state and step dt_f, it iterates
 * Delta += M_f^-1 (F(n + Delta) - Delta/dt) from Delta = 0 until a
 * correction is at most 1e-3 of every new density with mixing ratio above
 * y_floor (at most 4 corrections; one not below 0.3 of the previous ends
 * the attempt, which is retried with a fresh factorisation, not rejected).
 * A factorisation serves while dt/dt_f is in [1/1.3, 1.3], for at most 20
 * accepted steps.  res->factorizations counts them (every attempt for
 * methods 0 and 1), res->newton_iters the corrections on held ones.
 * Zero fields take the defaults in brackets. */
typedef struct {
  double tol_rel;    /* [1e-4]  */
  double y_floor;    /* [1e-30] */
  double y_sig;      /* [1e-10] */
  double t_end;      /* [1e12 s] */
  double dt0;        /* [1e-8 s] */
  int32_t max_steps; /* [5000]  */
  int32_t max_consec_rejects; /* [30] */
  int32_t use_mix_rule;       /* 0/1 [1 if the struct is NULL] */
  int32_t method;             /* 0 backward Euler [0], 1 ROS2, 2 backward
                                 Euler with factorisations kept across steps
                                 (1 and 2: FP64 columns) */
  double y_neg;      /* [1e-6]; a tiny value such as 1e-300 rejects any
                        negative of a species above y_sig */
} xod_ss_opts;
typedef struct {
  double t, dt, clipped;
  int64_t steps, rejects;
  int32_t converged;
  int32_t factorizations;     /* step-matrix factorisations */
  int64_t newton_iters;       /* method 2: corrections on held factorisations */
} xod_ss_result;
xod_status xod_integrate_to_steady_state(xod_column *col,
                                         const xod_ss_opts *opts,
                                         xod_ss_result *res);

/* nsteps backward-Euler steps of one size dt (no clipping, no rejection)
 * keeping the step matrix across steps when reuse = 1: the chord /
 * modified-Newton corrector of the DLSODES family Section 2.1 names.  A
 * step on a fresh factorisation of M = I/dt - J(n) takes the first Newton
 * iterate (the linearly implicit step of xod_step); a step on the held
 * factorisation (of an earlier state) solves n1 - n - dt F(n1) = 0 by
 * Delta += M_f^-1 (F(n + Delta) - Delta/dt) from Delta = 0 until a
 * correction is at most 1e-3 of every new density with mixing ratio above
 * 1e-10; a correction not below half the previous one, a non-finite iterate
 * or 4 corrections without convergence make the step start again on a
 * fresh factorisation, as does a factorisation that has served 20 steps.
 * reuse = 0: every step is an xod_step.  reuse = 1 needs an FP64 column.
 * XOD_ENONFINITE stops at the first step whose result is not finite (the
 * state is that of the steps before it).  st may be NULL. */
typedef struct {
  int64_t steps;            /* steps taken                                  */
  int64_t factorizations;   /* step-matrix factorisations                   */
  int64_t newton_iters;     /* corrections on held factorisations           */
} xod_reuse_stats;
xod_status xod_integrate_fixed_dt(xod_column *col, double dt, int32_t nsteps,
                                  int32_t reuse, xod_reuse_stats *st);

/* One global iteration of the Lagrangian parcel scheme (the paper's own
 * model: Section 2, an air parcel tracked from the bottom of the atmosphere
 * to the top and back; Section 2.1, molecular diffusion as a
 * pseudo-reaction) on the column's state, which is the profile and is
 * updated in place.  The parcel visits layers 0, 1, ..., N-1, N-2, ..., 0;
 * at layer k it takes the layer's temperature and gas density (its mixing
 * ratios carried over), stays for the layer's eddy mixing time
 * dz_k^2 / K_k (eddy mixing is the parcel's motion, so K appears nowhere
 * else), and evolves by the layer's chemistry plus molecular diffusion: the
 * molecular-diffusion part of the column's transport (K = 0), its
 * self-coefficient removing the molecule from the parcel where negative,
 * every gain (the profile's neighbours, a positive self-coefficient on the
 * profile's own density) entering as a fixed source.  The integration is by
 * linearly implicit backward-Euler steps on the layer's dense S x S system
 * under the steady-state driver's control (xod_integrate_to_steady_state)
 * inside the residence time, the first step of size dt0, each later visit
 * starting with the step size the previous one ended on; the parcel's
 * composition at the end of a visit becomes the profile at that layer.
 * dt_last (may be NULL) receives the step size the last visit ended on.
 * FP64, closed columns with gray photolysis and K > 0 in every layer
 * (XOD_EINVAL otherwise); XOD_ENOTCONVERGED if a visit's step size
 * collapses (more than 30 rejections in a row).  Synchronous. */
typedef struct {
  int64_t steps, rejects;   /* backward-Euler steps taken and rejected        */
  double clipped;           /* negative density clipped to zero (sum)         */
  int32_t visits;           /* layer visits (2N - 1)                          */
  int32_t pad_;
} xod_parcel_stats;
xod_status xod_parcel_pass(xod_column *col, double dt0, double *dt_last,
                           xod_parcel_stats *st);

/* Copy of the last error message of this thread (always NUL-terminated). */
xod_status xod_last_error(char *buf, size_t len);

/* Spectral photolysis rate coefficients (Section 2.3.3: the actinic flux
 * J = J0 exp(-tau/mu) with no diffuse part, the optical depth as the sum of
 * the absorbers' extinction cross sections times their columns, and the rate
 * integral over wavelength bins), FP64:
 *   Ncol[k][a] = n[k][absorbers[a]] dz[k]/2 + sum_{j>k} n[j][absorbers[a]] dz[j]
 *   tau[k][b]  = sum_a Ncol[k][a] sig_ext[a*L + b]
 *   kph[k*P+p] = t_f sum_b J0[b] exp(-tau[k][b]/mu) sig_ph[p*L + b] dlam[b]
 * N layers (0 at the bottom), S species, A absorbers (A = 0: no
 * attenuation), L wavelength bins, P photolysis reactions.  n [N*S] and dz
 * [N] as for the column; absorbers [A] species indices in 0..S-1;
 * sig_ext [A*L], J0 [L], dlam [L], sig_ph [P*L], kph [N*P] out; all DEVICE
 * pointers owned by the caller, row-major.  work: device scratch of at
 * least xod_photolysis_workspace(N, A, L, P) bytes.  Enqueued on `stream`
 * (a hipStream_t, NULL for the default stream), asynchronous.  XOD_EINVAL
 * for sizes out of range (N, S, L > 0; A, P >= 0), mu <= 0, a null pointer
 * the sizes need, or a short workspace; absorber indices are not checked
 * against S on the device. */
size_t xod_photolysis_workspace(int32_t N, int32_t A, int32_t L, int32_t P);
/* Exchange through the column's ends (Section 2.4 escape, Section 2.5
 * boundary conditions), in the flux divergence of the bottom and top layers
 * (upward flux positive):
 *   top:    phi = v_top,y n_{y,N-1}                (escape)
 *   bottom: phi = phi_surf,y - v_dep,y n_{y,0}     (emission, deposition)
 * so df_{y,N-1} -= v_top n_{y,N-1} / dz_{N-1} and df_{y,0} += (phi_surf -
 * v_dep n_{y,0}) / dz_0, and the step matrix gains v/dz on those diagonals.
 * v_top,y = V_lim,y for species flagged in escape_diff_limited, V_lim =
 * D (1/H_0 - 1/H_y) with H_0 = k_B T/(mbar g), H_y = k_B T/(m_y g) and the
 * top layer's D and T, clamped at 0 (no escape for heavier-than-mean
 * species), plus v_top[y] when given (set velocities).  Each member is a
 * HOST array [S] or NULL (none of that kind): flags 0/1; v_top, v_dep cm/s,
 * finite, >= 0; phi_surf cm^-2 s^-1, finite.  Copied; b == NULL (or all
 * members NULL) closes the column again.  XOD_EINVAL for invalid entries
 * (nothing changed) or a column in a batch.  Synchronous; a held
 * factorisation is dropped (xod_step_frozen needs a new xod_step). */
typedef struct {
  const int32_t *escape_diff_limited;
  const double *v_top;
  const double *v_dep;
  const double *phi_surf;
} xod_boundary;
xod_status xod_column_set_boundary(xod_column *col, const xod_boundary *b);

/* Use spectral photolysis rates in this column's steps: every xod_step (and
 * xod_rates) first computes kph from the column's state at that moment, as
 * xod_photolysis_spectral does with the column's layer thicknesses, and the
 * photolysis reactions take k_f = kph[k][p] (p = the reaction's index among
 * the network's photolysis reactions, in reaction order) instead of
 * J0 exp(-tau_k).  Within a step the rates stay those of its starting state
 * (lagged: the Jacobian holds them fixed).  The tables are DEVICE pointers
 * the caller keeps valid while the setting is in force: absorbers [A],
 * sig_ext [A*L], J0 [L], dlam [L], sig_ph [nph*L] for the network's nph
 * photolysis reactions.  L = 0 returns to the gray law.  Batches reject
 * columns with a spectrum (XOD_EINVAL at xod_batch_create). */
xod_status xod_column_set_photolysis_spectrum(xod_column *col, int32_t A, int32_t L,
                                              const int32_t *absorbers, const double *sig_ext,
                                              const double *J0, const double *dlam,
                                              const double *sig_ph, double t_f, double mu);
xod_status xod_photolysis_spectral(int32_t N, int32_t S, int32_t A, int32_t L, int32_t P,
                                   const double *n, const double *dz,
                                   const int32_t *absorbers, const double *sig_ext,
                                   const double *J0, const double *dlam, const double *sig_ph,
                                   double t_f, double mu, void *work, size_t work_bytes,
                                   double *kph, void *stream);

/* xod_photolysis_spectral without a workspace argument and without any
 * device allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, results and checks otherwise.  The workspace is a fixed 64 MiB
 * device array, one per GPU the library runs on, held until the process
 * ends: sizes whose xod_photolysis_workspace(N, A, L, P) exceeds 64 MiB are
 * refused with XOD_EINVAL (the 150-layer, 463-absorber, 10,000-bin,
 * 772-reaction workload needs 36.6 MB).  `stream` must belong to the
 * current device.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller. */
xod_status xod_photolysis_spectral_noalloc(int32_t N, int32_t S, int32_t A, int32_t L,
                                           int32_t P, const double *n, const double *dz,
                                           const int32_t *absorbers, const double *sig_ext,
                                           const double *J0, const double *dlam,
                                           const double *sig_ph, double t_f, double mu,
                                           double *kph, void *stream);

/* Kernel options (process-wide; for tests and tuning).
 *   "gemm": 0 = VALU FMA Schur update, 1 = MFMA Schur update (default).
 *   "update32": 1 = MFMA trailing update in 32-column strips by four-wave
 *            work-groups when a launch updates many blocks (default);
 *            0 = always 16-column strips by 16-wave work-groups.
 *   "update32_min": "many" above: at least this many (block, 32-column
 *            strip) pairs in the launch (default 200).
 *   "gemm_large": 1 = cyclic-reduction block products of large batches use
 *            128 x 128 output tiles (default); 0 = always 64 x 64.
 *   "gemm_lib": 0 = the cyclic-reduction block products run in the
 *            hand-written MFMA kernel, which gathers the permuted rows as it
 *            stages them (default); 1 = as rocBLAS batched GEMMs, after a
 *            gather kernel copies each product's row-permuted operand into
 *            scratch blocks.  The two sum in different orders (same to
 *            rounding).
 *   "gemm_waves": waves per work-group of the 128 x 128 block-product
 *            tiles, 16 (default: 2 x 2 MFMA tiles per wave) or 8 (4 x 2,
 *            each LDS fragment of A feeding two MFMAs and of B four); same
 *            K order, same bits;
 *   "gemm_k": K step of the block products staged through LDS, 16 or 32
 *            (default 32); every element sums its K terms in the same order
 *            with either.
 *   "refine_tol_exp": e in 3..15: a mixed-precision solve has converged
 *            once no component with mixing ratio above 1e-30 moves by more
 *            than 10^-e of its new density (default 7), or by more than the
 *            absolute floor below;
 *   "refine_atol_exp": e in 8..17: that floor, 10^-e times the layer's
 *            largest increment (default 14);
 *   "mixed_sticky": 0..1000 (default 16): the number of steps a
 *            mixed-precision column takes in FP64 directly after a fallback
 *            (see xod_step); 0 = always try FP32 first;
 *   "refine64": 0..10 corrections of every FP64 solve of a step with its
 *            own factors (residual in FP64 from the reaction list), a fixed
 *            number with no host round trip; a layer whose last correction
 *            exceeds 1e5 times the mixed-precision tolerance keeps the
 *            unrefined solution.  Default 0: the explicit inverses make the
 *            FP64 solve forward stable only, and one correction brings the
 *            trace components to the residual's rounding (30 times closer to
 *            the oracle on the 594-species column), but the adaptive drivers'
 *            negativity test then sees the linearised step's own negative
 *            trace densities, which the unrefined solve happens to miss;
 *            the 90-species steady state then stalls with block Thomas;
 *   "fused_max_ld": FP64 block Thomas of columns with padded blocks up to
 *            this size (0, 32, 64 (default), 96 or 128; 0 = never) runs in
 *            two persistent launches per column, one work-group each, for
 *            the factorisation and for the solve, instead of per-layer panel
 *            launches; the solve reads either kind of factors;
 *   "outer": Gauss-Jordan outer panel width, 32 (default), 64, 96 or 128:
 *            with a width above 32 the 32-column panels of an outer panel
 *            update only its own columns, then one rank-width update covers
 *            the rest of the block (fewer passes over the block, more
 *            launches); 32 = every panel updates the whole block.
 *   "panel_sync": barriers per Gauss-Jordan pivot column, 2 (default: the
 *            wave keys, then the winning row alone) or 1 (every wave's best
 *            row published before one barrier); same pivots, same bits.
 *   "outer_nmat": the outer panel width applies to launches of at least
 *            this many blocks (default 1); smaller launches use 32.
 *   "graph": 1 = the cyclic-reduction factor and solve launch sequences of a
 *            column are captured once into HIP graphs (kernel nodes only)
 *            and replayed (default); 0 = launched one by one.  Graphs are
 *            not used while "profile" is on.
 *   "profile": 1 = record HIP events on the launching stream around each
 *              profiled kernel launch (default 0).
 *   "profile_every": profile layer k only when k % value == 0 (default 1). */
xod_status xod_set_option(const char *name, int64_t value);

/* Current value of a kernel option above (refine_tol_exp: the exponent e of
 * the current tolerance 10^-e, rounded).  XOD_EINVAL for an unknown name or a
 * null pointer. */
xod_status xod_get_option(const char *name, int64_t *value);

/* Sum of the recorded launch durations (ms) and the launch count of one
 * kernel kind: "panel", "update", "prologue", "solve", "jacobian", "rates",
 * "rhs", "gemm", "photolysis" (the spectral-photolysis product).  Waits for the recorded events.  xod_profile_reset() drops them. */
xod_status xod_profile_read(const char *kernel, double *total_ms, int64_t *launches);
xod_status xod_profile_reset(void);

/* ---- batches ---------------------------------------------------------- */

/* A batch steps many columns together with block Thomas: columns with the
 * same block size share every launch (their layer chains advance in lock
 * step; a column with fewer layers idles once its chain ends).  Columns keep
 * ownership of their state; a column may belong to one batch at a time; all
 * columns of a batch have one precision.  Mixed-precision columns of a block
 * size are refined together until the group's largest correction ratio meets
 * the single-column stopping rule (a group that stalls is refactored in
 * FP64); stats report each column's group refinements and fallback. */
xod_status xod_batch_create(xod_column *const *cols, int32_t ncols,
                            xod_batch **out);
xod_status xod_batch_destroy(xod_batch *b);
/* One BE step of every column with its own dt (host array [ncols]); stats
 * (host array [ncols]) may be NULL.  Synchronous. */
xod_status xod_batch_step(xod_batch *b, const double *dt_per_col,
                          xod_step_stats *stats);

/* ---- tile-shape autotuner for the block factorisations ---------------- */

/* The factorisations' tile options ("fused_max_ld", "outer", "update32",
 * "gemm_large", "gemm_k", "panel_sync" of xod_set_option) have settings
 * that differ in speed with the block size, the precision, the
 * factorisation, the number of blocks a launch covers and the GPU.  The
 * tuner times candidate settings on the caller's own work and keeps the
 * fastest per (GPU architecture, padded block size, precision,
 * factorisation, single column or batch) in a process-wide table; from then
 * on, factorisations of that kind of column (steps, drivers, batches,
 * serving) run with it, and other kinds keep the xod_set_option values.
 * Every candidate computes the same factorisation up to the order of
 * rounding.  Candidates: block Thomas: the persistent small-block kernels
 * (blocks up to 128, FP64), or the panel kernels with outer panels of 32,
 * 64 or 128 columns and 16- or 32-column strip updates; cyclic reduction:
 * block-product tiles 128 (16 or 8 waves) or 64, K step 32 or 16, one or
 * two barriers per pivot column.  The first candidate is always the current xod_set_option
 * setting (default_ms). */
typedef struct {
  char key[96];          /* "arch/ldN/precision/factorisation/column|batch" */
  int32_t candidates;    /* settings timed */
  int32_t fused_max_ld, outer, update32, gemm_large, gemm_k, panel_sync,
          gemm_waves;    /* the chosen setting */
  double best_ms;        /* its time (one step's solve, or one group's step) */
  double default_ms;     /* the first candidate's time */
} xod_tune_result;

/* Tune for columns like col: each candidate runs one untimed and `trials`
 * timed linearised steps of size dt (rates, F, Jacobian, factorisation,
 * solve, mixed refinement; the state is not advanced), HIP events on the
 * column's stream.  The column's held factorisation is dropped.  trials in
 * 1..100; XOD_EINVAL for a column in a batch or dt <= 0. */
xod_status xod_autotune(xod_column *col, double dt, int32_t trials,
                        xod_tune_result *res);

/* Tune every group (padded block size, precision) of a batch: each
 * candidate runs one untimed and `trials` timed batch steps with the dts
 * given (states not advanced), and a group's time is its own device time
 * (events on its stream).  res has room for max_results groups; *nresults
 * receives their number.  trials in 1..20. */
xod_status xod_batch_autotune(xod_batch *b, const double *dt_per_col, int32_t trials,
                              xod_tune_result *res, int32_t max_results,
                              int32_t *nresults);

/* Forget every tuned setting. */
xod_status xod_autotune_clear(void);

/* ---- serving: continuous batching of steady-state solves -------------- */

/* hbm_budget_bytes bounds the device memory held by resident requests;
 * max_slots bounds their number.  With the default solver (block cyclic
 * reduction) each slot owns a HIP stream created here (default priority);
 * with block Thomas all work goes to hip_stream. */
xod_status xod_serve_create(size_t hbm_budget_bytes, int32_t max_slots,
                            xod_precision prec, void *hip_stream,
                            xod_server **out);
xod_status xod_serve_destroy(xod_server *srv);
/* Factorisation used for the requests (default XOD_SOLVER_CR).  Only before
 * the first submit (XOD_EINVAL afterwards).  XOD_SOLVER_THOMAS steps all
 * resident FP64 requests in shared batched launches. */
xod_status xod_serve_set_solver(xod_server *srv, xod_solver solver);
/* Device bytes one request of this network and layer count occupies with
 * the default solver (column state and blocks plus the cyclic-reduction
 * workspace; an upper bound for block Thomas). */
xod_status xod_serve_footprint(const xod_network *net, int32_t N,
                               xod_precision prec, size_t *bytes);
/* Queue a steady-state solve (host arrays copied; opts as for
 * xod_integrate_to_steady_state, NULL = defaults; requests are stepped with
 * backward Euler, so opts->method must be 0; the columns are closed: no
 * boundary exchange, gray photolysis).  Never blocks: a request
 * waits in the queue until a slot and memory are free.  XOD_EINVAL if the
 * request could never fit the budget or asks for another method. */
xod_status xod_serve_submit(xod_server *srv, const xod_network *net,
                            const xod_profile *prof, const double *n0,
                            const xod_ss_opts *opts, uint64_t *req_id);
/* One iteration: admit queued requests (arrival order) while a slot is free
 * and the footprint fits, advance every resident request by one adaptive BE
 * step (cyclic reduction: FP64 requests' steps are enqueued on their slot
 * streams before any is awaited, so they overlap on the device; block
 * Thomas: FP64 requests share batched launches), retire converged / failed
 * ones (state copied to the host, slot and memory freed).  Synchronous. */
xod_status xod_serve_step(xod_server *srv, int32_t *n_active, int32_t *n_queued);
/* state: 0 queued, 1 running, 2 converged, 3 failed.  n_out (host [N*S],
 * may be NULL) and latency_s (completion - submission, seconds) are valid
 * once state >= 2.  Returns the failure status for state 3. */
xod_status xod_serve_poll(xod_server *srv, uint64_t req_id, int32_t *state,
                          double *n_out, xod_ss_result *res, double *latency_s);
/* Forget a finished request. */
xod_status xod_serve_release(xod_server *srv, uint64_t req_id);
xod_status xod_serve_usage(const xod_server *srv, size_t *used_bytes,
                           int32_t *active, int32_t *queued, int64_t *iterations);

#ifdef __cplusplus
}
#endif

#endif /* XOD_H */
