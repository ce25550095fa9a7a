/*
 * sph.h -- C ABI of the MI355X (gfx950) semi-implicit SPH viscous solver.
 *
 * The library solves the implicit viscous system of Bilotta et al., "A
 * numerically robust, parallel-friendly variant of BiCGSTAB for the
 * semi-implicit integration of the viscous term in Smoothed Particle
 * Hydrodynamics" (arXiv 2206.14780), Section "Shared formulation":
 *
 *     A(dt) V = B,   A: N x N (one row per particle),  V, B: N x 3,
 *
 * three systems (one per velocity component) sharing one matrix, solved by
 * the paper's restructured ("robust") BiCGSTAB (Section "Restructuring the
 * stabilized biconjugate gradient method"), by the textbook BiCGSTAB, or,
 * when the system is symmetric, by the paper's rotated Conjugate Gradient
 * (Section "Restructuring the Conjugate Gradient").
 *
 * Conventions for every call:
 *   - Pointers inside sph_particles and the x/y/rhs arrays are DEVICE pointers
 *     owned by the caller, in the caller's (original) particle order, unless
 *     the comment says "host".  The library never frees them.
 *   - Work is issued on the context's HIP stream.  sph_visc_apply and
 *     sph_visc_papanastasiou are asynchronous; sph_build_neighbors,
 *     sph_neighbors_export and sph_visc_solve return after the stream work
 *     they issued has finished.
 *   - Negative status = failure, outputs undefined.  Positive status = the
 *     outputs are valid and the report says why the solve stopped.
 *   - A context is not thread-safe; use one context per host thread.
 *   - Matrix rows, taking the diffusive sign of eq. kab (the printed sign would
 *     make the fluid rows lose diagonal dominance): with pair weight w_ba = -2 mubar_ab m_a F(r_ab)/(rho_a rho_b)
 *       fluid row b:        A_bb = 1 + dt sum_a w_ba,  A_ba = -dt w_ba     (eqs. diag, offdiag)
 *       dynamic wall row b: identity                          (eq. implicit-system-dyn-full)
 *       dummy wall row b:   A_bb = 1, A_ba = W_ba / sum_{a' fluid} W_ba' for fluid a,
 *                           identity if b has no fluid neighbour
 *                                                             (eq. implicit-system-dummy-full)
 *     W, F: Wendland psi_{3,1} kernel of radius 2h (Section "Smoothing kernel choice").
 *     Neighbours: a != b with |r_a - r_b|^2 < (2h)^2, minimum image on periodic axes.
 */
#ifndef SPH_H
#define SPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx; /* device, stream binding, workspace */
typedef struct sph_nbr sph_nbr; /* cell-linked lists of one particle configuration */

typedef enum {
    SPH_OK = 0,
    SPH_STALLED = 1,        /* no component progressing, at least one stalled */
    SPH_NOT_CONVERGED = 2,  /* max_iter reached with a component still progressing */
    SPH_E_ARG = -1,         /* invalid argument (null pointer, size, enum, geometry) */
    SPH_E_OOM = -2,         /* device allocation failed */
    SPH_E_HIP = -3,         /* HIP runtime error (message via sph_last_error) */
    SPH_E_OVERFLOW = -4,    /* output capacity too small (sph_neighbors_export) */
    SPH_E_NONFINITE = -5    /* non-finite right-hand side */
} sph_status;

/* Precision.  SPH_F64 and SPH_F32: operator, vectors and the caller's arrays
 * in that precision (inner products and scalars are always FP64).
 * SPH_MIXED (sph_visc_solve only): FP32 operator and Krylov vectors, the
 * solution accumulated in FP64, and the caller's rhs, x and warm_u arrays in
 * FP64.  An FP32 solution cannot carry a scaled residual much below
 * 2^-24 A_rr relative to b, so for stiff rows only SPH_MIXED reaches tight
 * tolerances with the FP32 operator. */
enum { SPH_F64 = 0, SPH_F32 = 1, SPH_MIXED = 2 };
enum { SPH_FLUID = 0, SPH_WALL = 1 };              /* particle type */
/* Smoothing kernel (Section "Smoothing kernel choice"): the Wendland psi_{3,1}
 * of radius 2, or the normalised truncated Gaussian of radius 3,
 * w(q) = (e^{-q^2} - e^{-9}) / w_G with w_G = pi^{3/2} erf(3) - 2 pi e^{-9} 21/3
 * and F = (1/r) dW/dr = -2 e^{-q^2} / (w_G h^5) (the printed f has the
 * opposite sign; the derivative's is used, as for the Wendland kernel).  It is
 * chosen with the domain of the neighbour build and holds for every operator,
 * solve and viscosity update on that handle. */
enum { SPH_KERNEL_WENDLAND = 0, SPH_KERNEL_GAUSSIAN = 1 };
enum { SPH_WALL_DYNAMIC = 0, SPH_WALL_DUMMY = 1 }; /* boundary model (Section "Boundary conditions") */
enum { SPH_AVG_ARITH = 0, SPH_AVG_HARMONIC = 1 };  /* pairwise viscosity mean (Section "Discretized equations") */
enum { SPH_ROBUST = 0, SPH_STANDARD = 1, SPH_CG = 2 }; /* solver: robust / textbook BiCGSTAB, rotated CG */
enum { SPH_OP_CACHED = 0, SPH_OP_ONTHEFLY = 1, SPH_OP_PAPER32 = 2 }; /* operator evaluation (see sph_visc_params) */
enum { SPH_CONVERGED = 0, SPH_STATE_STALLED = 1, SPH_PROGRESSING = 2 }; /* per-component state */

/* One particle configuration.  n >= 1; all arrays have n entries. */
typedef struct {
    int64_t n;
    const double *x, *y, *z;       /* positions */
    const double *mass, *rho, *mu; /* mass, density, DYNAMIC viscosity (mu = nu rho) */
    const uint8_t *type;           /* SPH_FLUID or SPH_WALL */
} sph_particles;

/* Domain box.  On a periodic axis the period is hi - lo (> 0) and
 * distances use the minimum image, so each pair counts once; on other axes
 * particles outside [lo, hi] are binned into the edge cells (still exact,
 * only slower). */
typedef struct {
    double lo[3], hi[3];
    int32_t periodic[3];
    double h;       /* smoothing length */
    int32_t kernel; /* SPH_KERNEL_WENDLAND (support 2h) or SPH_KERNEL_GAUSSIAN (support 3h) */
} sph_domain;

/* Parameters of A(dt).
 *   jacobi: 1 = left Jacobi scaling, the operator and solver use D^-1 A and
 *           D^-1 B with D = diag(A) (appendix "Implementation notes").
 *   op_mode: SPH_OP_CACHED evaluates every pair coefficient once per call in
 *           FP64 and keeps the matrix in HBM (sliced ELLPACK, rounded to the
 *           vector precision) for all applications of that call;
 *           SPH_OP_ONTHEFLY re-evaluates the coefficients from positions in
 *           every application (the paper's matrix-free gemv);
 *           SPH_OP_PAPER32 (SPH_F32 and the Wendland kernel only, else
 *           SPH_E_ARG) is the paper's single-precision arithmetic (appendix
 *           "Implementation notes", appendix on relative positions): every
 *           pair weight evaluated in FP32 from FP32 positions relative to the
 *           centres of the neighbour cells, the displacement of a pair grouped
 *           as o' + (r'_b - r'_a) with o' = l (c_b - c_a) the FP32 offset of
 *           the two cells (l the cell side); the diagonal 1 + dt sum w and the
 *           dummy-wall normalisation sum W as compensated (Kahan) FP32 sums;
 *           the matrix cached in FP32; the gemv y_r = A_rr x_r + sum A_ra x_a
 *           with every product rounded to FP32 and the terms summed by Kahan's
 *           compensation.  In sph_visc_solve it also makes every inner
 *           product a compensated FP32 sum of FP32 products and every scalar
 *           of the recurrences FP32 (as fp32_scalars); the true residual of
 *           the library's final check stays FP64. */
typedef struct {
    double dt;
    int32_t wall;    /* SPH_WALL_DYNAMIC / SPH_WALL_DUMMY */
    int32_t avg;     /* SPH_AVG_ARITH / SPH_AVG_HARMONIC */
    int32_t jacobi;  /* 0 / 1 */
    int32_t op_mode; /* SPH_OP_CACHED / SPH_OP_ONTHEFLY / SPH_OP_PAPER32 */
} sph_visc_params;

/* Solver options.
 *   variant: SPH_ROBUST, SPH_STANDARD or SPH_CG.  The CG needs a symmetric
 *          system (Section "Linear system properties and resolution"):
 *          dynamic walls (dummy walls: SPH_E_ARG) and uniform particle mass
 *          (not checked; with unequal masses it may stall or not converge).
 *          It starts the wall rows at their exact value (b), so that the
 *          iteration runs on the symmetric fluid block, and with jacobi it
 *          takes its inner products weighted by D = diag(A), the form in
 *          which D^-1 A is self-adjoint (Jacobi-preconditioned CG).  One
 *          operator pass per iteration (the BiCGSTAB takes two).
 *          restart_drop does not apply to it; force_stall_iter treats
 *          p . A p as zero.
 *   tol:   relative tolerance eps; component c converges when r.r < tau2_c,
 *          tau2_c = max(eps^2 b.b, floor) on the (scaled) system
 *          (Section "Restructuring the Conjugate Gradient", stopping criterion).
 *   floor: lower bound of tau2; < 0 selects FLT_MIN (SPH_F32) or DBL_MIN (SPH_F64).
 *   true_res_period: every that many iterations, and whenever no component
 *          is progressing, the residual b - A x is recomputed in FP64 with the
 *          on-the-fly operator; a converged component that fails it is
 *          restarted from that residual.  0 = only when no component progresses.
 *   x0_given: 1 = x holds the initial guess on entry, 0 = start from zero.
 *   poll_every: most iterations issued between two host reads of the device
 *          control block (0 = library default, 8).  Batches grow 2, 4, ... up
 *          to it, and shrink to what the residual history predicts is left,
 *          so that few iterations are issued past the halt.  Does not change
 *          the result.
 *   force_stall_iter / force_stall_comp: test hook; at that iteration that
 *          component's delta is treated as zero.  -1 = off.
 *   profile: k > 0 = bracket the second operator launch (A r_star and its
 *          dot products; the CG's only one) of every k-th iteration with HIP events on the
 *          context stream and report the total time of the executed ones
 *          (apply_ms, apply_launches); 0 = off.  Each event pair leaves a
 *          gap of a few microseconds in the stream, so k > 1 keeps the
 *          measurement from slowing the solve it measures.
 *   restart_drop: at each periodic true-residual check, a progressing
 *          component whose true r.r has fallen below restart_drop times its
 *          r.r at the last (re)start restarts from the true residual
 *          (r0hat = r = r_true, alpha' = beta = 0): a restarted BiCGSTAB
 *          whose shadow vector follows the residual, which also keeps FP32
 *          recurrences commensurate with it.  < 0 selects 0.1; 0 = never
 *          (the paper's unrestarted iteration).  With true_res_period = 20
 *          this default cut iterations by a third on stiff cases.
 *   warm_params: device, SPH_MLP_NPARAM floats, or null.  Non-null: the
 *          solve also forms the learned initial guess of sph_mlp_warmstart
 *          from the current velocity u and, per component, starts from
 *          whichever of the learned guess and the plain start (x on entry if
 *          x0_given, else zero) has the smaller FP64 true residual.  The
 *          tolerance and stopping test are unchanged.
 *   fp32_scalars: 1 = FP32 scalars with FP64-accumulated inner products
 *          (SPH_F32 only, else SPH_E_ARG): every reduced inner product, the
 *          FP64 sum of the FP32 products, and every scalar of the recurrences
 *          (alpha, beta, omega, gamma, delta, tau^2) is rounded to FP32; the
 *          vectors and the operator are FP32 as in SPH_F32.  The inner
 *          products are more accurate than the paper's single precision (an
 *          FP64 sum keeps the low bits of products that cancel); the paper's
 *          own arithmetic, compensated FP32 sums of FP32 products, is
 *          params->op_mode = SPH_OP_PAPER32, which implies FP32 scalars.  Set
 *          true_res_period = 0 and restart_drop = 0 for the paper's
 *          unrestarted iteration.
 *   warm_u: device, n values of the caller's precision each: u.  A null
 *          component takes the initial guess (x0_given; the usual case of a
 *          previous-step start, which also saves one operator pass) or rhs. */
typedef struct {
    double tol;
    int32_t max_iter;
    int32_t variant; /* SPH_ROBUST / SPH_STANDARD / SPH_CG */
    double floor;
    int32_t true_res_period;
    int32_t x0_given;
    int32_t poll_every;
    int32_t force_stall_iter;
    int32_t force_stall_comp;
    int32_t profile;
    double restart_drop;
    const float *warm_params;
    const void *warm_u[3];
    int32_t fp32_scalars;
} sph_solve_opts;

/* Solve report (host memory).  history, if non-null, is a host buffer of
 * history_cap x 3 doubles that receives r.r per component at the end of
 * each iteration (row 0 = initial residual).  Residuals are reported as
 * squared norms, as the stopping test compares them (r.r < tau^2, Section
 * "Restructuring the Conjugate Gradient"): the relative residual of
 * component c is sqrt(rr[c] / bb[c]) (recursive) and sqrt(true_rr[c] /
 * bb[c]) (FP64 true residual), both of the (scaled) system solved. */
typedef struct {
    int32_t iters;
    int32_t status;
    int32_t state[3];       /* SPH_CONVERGED / SPH_STATE_STALLED / SPH_PROGRESSING */
    int32_t stall_count[3]; /* iterations in which the component broke down (a
                               component with a zero right-hand side, converged at
                               the start, breaks down in every iteration) */
    double rr[3];           /* final recursive r.r of the scaled system */
    double bb[3];           /* b.b of the scaled right-hand side */
    double tau2[3];
    double true_rr[3];      /* final FP64 (b - A x).(b - A x) of the scaled system */
    int32_t n_true_checks;
    int32_t n_replaced;     /* restarts from the true residual (both kinds) */
    double *history;        /* host, may be null */
    int32_t history_cap;
    int32_t history_len;
    double setup_ms;        /* device time: gathers, matrix build, initial residual */
    double iterate_ms;      /* device time of the iterations and residual checks */
    int32_t launches;       /* kernel launches issued by the solve */
    int64_t mat_nnz;        /* off-diagonal entries of the cached matrix (SPH_OP_CACHED) */
    int64_t mat_slots;      /* stored entries including slice padding (SPH_OP_CACHED) */
    double apply_ms;        /* with opts->profile: summed duration of the timed launches */
    int32_t apply_launches; /* with opts->profile: number of timed launches */
    /* learned initial guess (opts->warm_params non-null) */
    int32_t warm_used[3];   /* 1: the component started from the learned guess */
    double warm_rr[3];      /* true r.r of the learned guess (scaled system) */
    double plain_rr[3];     /* true r.r of the plain start */
    double warm_scale;      /* U, the normalisation of the features */
    double warm_ms;         /* device time of forming the learned guess and both residuals */
    int32_t issued_iters;   /* iterations queued by the host; those past the halt
                               (issued_iters - iters) return at once */
} sph_solve_report;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; null = the device's null stream).  *ctx receives the handle. */
sph_status sph_create(sph_ctx **ctx, int32_t device, void *hip_stream);
/* Release the context and all its device workspace. */
sph_status sph_destroy(sph_ctx *ctx);
/* Re-bind the context to another stream of the same device. */
sph_status sph_set_stream(sph_ctx *ctx, void *hip_stream);
/* Message of the last failure on this context (static storage of the context). */
const char *sph_last_error(const sph_ctx *ctx);
const char *sph_status_str(sph_status s);

/* Cell-linked lists by counting sort (Section "Smoothing kernel choice" for
 * the support radius; appendix on relative positions for the cell grid):
 * cells of side >= 2h, particles ordered by cell and, inside a cell, by
 * original index.  Positions are copied; the handle stays valid after the
 * caller's arrays change.  *out receives a new handle (free it with
 * sph_neighbors_free).  Only the positions of `p` are read.  The handle holds
 * the cell lists only, never an explicit per-particle neighbour list (there
 * is no option for one): every operator build scans the cells itself and
 * keeps its lists for that build, so a list in the handle would be a second
 * copy of data that each solve renews anyway. */
sph_status sph_build_neighbors(sph_ctx *ctx, const sph_particles *p, const sph_domain *dom,
                               sph_nbr **out);
/* Number of particles and of (directed) neighbour pairs of the handle. */
sph_status sph_neighbors_info(sph_ctx *ctx, const sph_nbr *nb, int64_t *n, int64_t *nnz);
/* Neighbour lists in canonical form (the neighbour set of Section
 * "Smoothing kernel choice": b != a, |r_a - r_b| < 2h, or 3h for the
 * truncated Gaussian, minimum image on periodic axes): CSR over original
 * particle indices, columns ascending.  row_ptr: device, n + 1 entries;
 * cols: device, cap entries (both device arrays, so that checks of large
 * systems need no host copy; the caller copies what it wants on the host).
 * *nnz (host) receives the pair count; SPH_E_OVERFLOW if cap < nnz. */
sph_status sph_neighbors_export(sph_ctx *ctx, const sph_nbr *nb, int64_t *row_ptr,
                                int32_t *cols, int64_t cap, int64_t *nnz);
sph_status sph_neighbors_free(sph_nbr *nb);

/* y = A x (or D^-1 A x when params->jacobi) for the three components: the
 * viscous matrix of eqs. diag, offdiag (fluid rows) and
 * implicit-system-dyn-full / implicit-system-dummy-full (wall rows), the
 * paper's gemv (appendix "Implementation notes").
 * x[c], y[c]: device arrays of n doubles (prec SPH_F64) or floats (SPH_F32).
 * x and y must not overlap.  Coefficients are evaluated in FP64 in both
 * precisions; SPH_OP_CACHED rounds them to the vector precision. */
sph_status sph_visc_apply(sph_ctx *ctx, const sph_nbr *nb, const sph_particles *p,
                          const sph_visc_params *params, int32_t prec, const void *const x[3],
                          void *const y[3]);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight time-stepping loops, harnesses that forbid hipMalloc.
 * ------------------------------------------------------------------------ */
#define SPH_NOALLOC_MAX_N 262144 /* particles; 97 bytes each of staging, 25.4 MB per device */
/* sph_visc_apply with the on-the-fly operator, allocating nothing: the
 * cell-order staging of the particle properties, x and y lives in one static
 * device array of the library (SPH_NOALLOC_MAX_N x 97 bytes, held by each
 * device the library runs on until the process ends) instead of the
 * context's workspace.  Arguments, layouts and results are those of
 * sph_visc_apply (the same kernels, so the same bits); params->op_mode must
 * be SPH_OP_ONTHEFLY (the cached matrix needs storage that grows with the
 * system) and nb->n <= SPH_NOALLOC_MAX_N, else SPH_E_ARG.  Asynchronous on
 * the context stream.  All calls on one device share its array: calls that
 * overlap on one device (other contexts, other streams) race. */
sph_status sph_visc_apply_noalloc(sph_ctx *ctx, const sph_nbr *nb, const sph_particles *p,
                                  const sph_visc_params *params, int32_t prec, const void *const x[3],
                                  void *const y[3]);

/* Solve A V = B.  nb may be null, then dom must be given and the lists are
 * built inside the call.  rhs[c]: device, n values of the precision (FP64
 * for SPH_MIXED); x[c]: device, n values of the same; initial guess on
 * entry if opts->x0_given, solution on exit.  Vector updates and operator
 * run in `prec`; every inner product and every scalar of the recurrences is
 * FP64 in all precisions.  With the dummy model the wall rows of V are the
 * viscous velocities. */
sph_status sph_visc_solve(sph_ctx *ctx, const sph_nbr *nb, const sph_domain *dom,
                          const sph_particles *p, const sph_visc_params *params, int32_t prec,
                          const void *const rhs[3], void *const x[3], const sph_solve_opts *opts,
                          sph_solve_report *report);

/* Apparent viscosity of the Papanastasiou regularised Bingham law from a
 * velocity field (Section "Non-Newtonian viscosity", eq. papa), the update
 * the paper makes between solves with the viscosity lagged one step:
 *   G_b   = sum_a (m_a / rho_a) F(r_ab) r_ab u_ab^T over the neighbours a of
 *           b (fluid and wall, with the velocities given for them), r_ab =
 *           r_a - r_b by minimum image, u_ab = u_a - u_b, F as in eq. kab;
 *   S_b   = (G_b + G_b^T) / 2, D_b = sqrt(2 S_b : S_b) (equal to the rate in
 *           simple shear);
 *   mu_b  = tau0 Ybar(D_b) + mu0 on fluid rows, Ybar(D) = (1 - e^{-m D}) / D,
 *           replaced for m D < (9! 2^-23)^(1/8) = 0.675 by m times its
 *           Maclaurin series cut after 8 terms (Horner form), the D -> 0
 *           limit being m; wall rows keep p->mu.
 * Everything in FP64.  u[c]: device, n values of precision prec (SPH_F64 or
 * SPH_F32), caller order.  mu_out: device, n doubles, caller order; may be
 * p->mu itself (updated in place).  shear_out: device, n doubles receiving
 * D, or null.  tau0, mu0 finite and >= 0, m finite and > 0, else SPH_E_ARG.
 * Asynchronous on the context stream, like sph_visc_apply. */
sph_status sph_visc_papanastasiou(sph_ctx *ctx, const sph_nbr *nb, const sph_particles *p, int32_t prec,
                                  const void *const u[3], double tau0, double m, double mu0,
                                  double *mu_out, double *shear_out);

/* Parameters of one semi-implicit step (sph_semi_implicit_step). */
typedef struct {
    double g[3];           /* body force per unit mass: the inviscid acceleration of this path */
    int32_t papanastasiou; /* 1 = update the fluid viscosity with the law of sph_visc_papanastasiou */
    double tau0, m, mu0;   /* its parameters (read when papanastasiou = 1) */
} sph_step_params;

/* One step of the semi-implicit predictor/corrector (Section "Semi-implicit
 * integration scheme") with the body force as the whole inviscid
 * acceleration and the density held fixed (pressure and continuity belong to
 * the weakly compressible solver around this one):
 *   half step: A(r^n, mu^n; dt/2) V* = u^n + (dt/2) g, started from u^n;
 *              u* = V* on fluid rows; r* = r^n + (dt/2) u^n; mu* = mu(r*, u*)
 *   full step: A(r*, mu*; dt) V = u^n + dt g, started from u*;
 *              u^{n+1} = V on fluid rows; r^{n+1} = r^n + (dt/2)(u^n + u^{n+1});
 *              mu^{n+1} = mu(r^{n+1}, u^{n+1})  (the viscosity lags one step)
 * Wall particles keep their position and velocity (u on wall rows is the
 * prescribed wall velocity u_w; their right-hand side is u_w for dynamic and
 * 2 u_w for dummy walls) and their viscosity.  Positions are wrapped into
 * the box on periodic axes.  The neighbour lists are rebuilt at r^n, r* and
 * (with the viscosity update) r^{n+1}.
 *   p: positions, mass, rho, mu and type at step n (device, caller order).
 *   params: dt = the full step; wall, avg, jacobi, op_mode as for a solve.
 *   prec: SPH_F64 or SPH_MIXED (the velocities are FP64 arrays).
 *   opts: options of both solves; x0_given is set by the step (each solve
 *         starts from the previous velocity: u^n, then u*), and a learned
 *         start (warm_params) takes that velocity as its u (warm_u unused).
 *   pos_out[c]: device, n doubles: r^{n+1}; may be p->x, p->y, p->z.
 *   u[c]: device, n doubles: u^n on entry, u^{n+1} on exit.
 *   mu_out: device, n doubles: mu^{n+1} (a copy of p->mu without the
 *         update); may be p->mu.
 *   reports: host, two reports (half step, full step) or null.
 * Returns after the step's work has finished; the status is the worse of
 * the two solves' (negative on failure, when the outputs are undefined). */
sph_status sph_semi_implicit_step(sph_ctx *ctx, const sph_domain *dom, const sph_particles *p,
                                  const sph_visc_params *params, int32_t prec, const sph_step_params *sp,
                                  const sph_solve_opts *opts, double *const pos_out[3], double *const u[3],
                                  double *mu_out, sph_solve_report *reports);

/* ------------------------------------------------------------------------
 * Learned initial guess.  Not part of the paper, which names better initial
 * guesses as future work (Sections "Conclusions and future work" and
 * "Implementation notes"): a per-particle MLP
 *   x[4] -> 64 -> 64 -> 64 -> o[3] (ReLU), pred = o . B,
 * one sample per fluid particle and velocity component, with
 *   features x = (u_c / U, d_c / U, log10 nu - L, log10(dt nu / h^2)),
 *   basis    B = (b_c / U, u_c / U, d_c / U),  target t = V_c / U,
 * d = D^-1 (u - A u) (the viscous increment of u scaled by the row's
 * diagonal D = A_rr: one Jacobi correction), A the unscaled matrix of
 * sph_visc_params, u the current velocity, b the right-hand side,
 * nu = mu / rho, L the mean of log10 nu over fluid rows (the viscosity
 * feature is relative to the geometric-mean viscosity: scale-free), U the
 * RMS of b over fluid rows and components.  The initial guess is x0_c = U pred on fluid rows; wall rows
 * take b (dynamic model) or satisfy their own row exactly, x0_w = b_w -
 * sum_a W x0_a / sum_a W (dummy model).
 * Parameters: one FP32 vector of SPH_MLP_NPARAM values (W1 [4][64], b1,
 * W2 [64][64], b2, W3 [64][64], b3, W4 [64][3], b4; matrices [in][out]).
 * The weights enter every product as BF16; accumulation is FP32.
 * ------------------------------------------------------------------------ */
#define SPH_MLP_NPARAM 8835
#define SPH_MLP_SAMPLE 8 /* floats per sample: x[4], B[3], t */

/* Samples of one configuration, for training: samples (device, FP32,
 * 3 n x SPH_MLP_SAMPLE) receives sample 3 k + c for particle k (original
 * order) and component c; wall particles get all-zero samples.  u[c],
 * rhs[c], target[c]: device, n doubles each (target may be null: t = 0).
 * *U (host) receives the normalisation.  A u is evaluated in FP64.
 * samples must be 16-byte aligned (else SPH_E_ARG). */
sph_status sph_mlp_samples(sph_ctx *ctx, const sph_nbr *nb, const sph_particles *p,
                           const sph_visc_params *params, const double *const u[3],
                           const double *const rhs[3], const double *const target[3],
                           float *samples, double *U);
/* The learned initial guess alone (no fallback): x0[c] (device, n values of
 * the precision, original order) = U (o . B) on fluid rows, rhs on dynamic
 * wall rows, and on dummy wall rows the value that satisfies the row
 * exactly.  u[c], rhs[c]: device, n values of the precision each;
 * mlp_params: device, SPH_MLP_NPARAM floats: the FP32 master parameters that
 * training updates; every block rounds them to BF16 (nearest even) as it
 * loads them, so no separate BF16 copy has to be kept in step with them.
 * *U (host, may be null) receives the normalisation. */
sph_status sph_mlp_warmstart(sph_ctx *ctx, const sph_nbr *nb, const sph_particles *p,
                             const sph_visc_params *params, int32_t prec, const void *const u[3],
                             const void *const rhs[3], const float *mlp_params, void *const x0[3],
                             double *U);
/* out (device, n x 4) = (o0, o1, o2, pred) of samples (device, n x SPH_MLP_SAMPLE).
 * samples and out must be 16-byte aligned (else SPH_E_ARG). */
sph_status sph_mlp_forward(sph_ctx *ctx, const float *samples, int64_t n, const float *params,
                           float *out);
/* Gradient (device, SPH_MLP_NPARAM) of the mean squared error of the batch
 * samples[idx[0 .. batch)] (idx: device int32); *loss (host) = that error. */
sph_status sph_mlp_grad(sph_ctx *ctx, const float *samples, const int32_t *idx, int64_t batch,
                        const float *params, float *grad, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1)
 * on the FP32 master parameters (device) with moment buffers adam_m, adam_v
 * (device, SPH_MLP_NPARAM each, zero before step 1); *loss (host, may be
 * null) = mean squared error of the batch before the step.  The batch is
 * given as indices idx (device int32, batch entries) into the sample array
 * of sph_mlp_samples (device, FP32, SPH_MLP_SAMPLE values each: features,
 * basis and target together), so that one sample array built once serves
 * every step; the BF16 weights are rounded from params inside the kernels,
 * as in sph_mlp_warmstart. */
sph_status sph_mlp_train_step(sph_ctx *ctx, const float *samples, const int32_t *idx,
                              int64_t batch, float *params, float *adam_m, float *adam_v,
                              int32_t step, double lr, double *loss);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
