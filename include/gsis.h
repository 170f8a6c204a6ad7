/*
 * gsis.h -- C-ABI of the MI355X (gfx950) steady gray GSIS / source-iteration
 * solver library (libgsis.so).
 *
 * Problem (Sec. 2.1 Eq. RTE_g without the time derivative and the material
 * equation; Sec. 4.1 Eq. RTE_d with dt -> infinity):
 *     Omega . grad I + sigma_t I = (sigma_s phi + q) / (4 pi),
 *     phi = sum_k w_k I_k (Eq. def_rho),  F = sum_k w_k Omega_k I_k (Eq. def_F),
 * discretised by the cell-centred finite-volume scheme of Sec. 4.1
 * (second-order upwind faces from an adaptive least-squares gradient, Sec. 5,
 * and an optional Barth-Jespersen limiter) on a uniform Cartesian grid, and
 * solved by source iteration (Eq. SI_update) or by GSIS (Eqs. GSIS_HoT,
 * GSIS_dse, GSIS_update) with the synthetic equation of Sec. 4.2 solved on
 * the GPU by conjugate gradients preconditioned with geometric multigrid.
 * Convergence is Err(phi) of Eq. Err_W.
 *
 * Conventions shared by every call:
 *  - cell c = j*nx + i (x fastest); cell (i,j) covers [i*dx,(i+1)*dx] x
 *    [j*dy,(j+1)*dy];
 *  - boundary faces are numbered W side (j = 0..ny-1), E side (ny + j),
 *    S side (2*ny + i), N side (2*ny + nx + i);
 *  - every floating-point array is IEEE double;
 *  - the caller owns every buffer it passes; the library keeps no caller
 *    pointer after a call returns (plans copy what they need);
 *  - a context, and every plan made from it, must not be used by two host
 *    threads at once.
 *
 * Errors: every call returns a gsis_status. On GSIS_E_* the call has no
 * effect on its outputs and gsis_last_error() names the first offending
 * argument (field and index) or the HIP error. GSIS_NOT_CONVERGED and
 * GSIS_DIVERGED still write the last iterate and the full history.
 */
#ifndef GSIS_H
#define GSIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GSIS_OK = 0,
  GSIS_NOT_CONVERGED = 1,   /* max_iter reached with Err >= tol */
  GSIS_DIVERGED = 2,        /* Err became non-finite, or the change
                               ||phi^{m+1} - phi^m||_V grew above 1e3 times
                               its smallest value in the solve so far
                               (floored at 1e-9 ||phi^{m+1}||_V): the outer
                               iteration is unstable (GSIS at strong opacity
                               jumps needs the pseudo-time shift of Sec.
                               4.3, options.beta) */
  GSIS_E_INVALID_ARG = -1,  /* argument check failed; see gsis_last_error */
  GSIS_E_DEVICE = -2,       /* a HIP call failed */
  GSIS_E_OOM = -3,          /* device or host allocation failed */
  GSIS_E_UNSUPPORTED = -4   /* option combination not implemented */
} gsis_status;

/* Opaque handles. A context binds one GPU; a plan holds one problem's
 * device state (angular intensities, coefficients, multigrid hierarchy). */
typedef struct gsis_ctx gsis_ctx;
typedef struct gsis_plan gsis_plan;

/* Create a context on HIP device `device` (ordinal). */
gsis_status gsis_ctx_create(int32_t device, gsis_ctx **out);
/* Destroy a context (NULL is a no-op). Plans made from it must be destroyed
 * first. */
void gsis_ctx_destroy(gsis_ctx *ctx);
/* Message of the last failed call on ctx (or of the last failed
 * gsis_ctx_create when ctx is NULL). Valid until the next call on ctx. */
const char *gsis_last_error(const gsis_ctx *ctx);

/* Problem statement (Sec. 4.1, Sec. 4.4). */
typedef struct {
  int32_t nx, ny;          /* cells per direction, >= 1, with nx*ny at most
                              GSIS_MAX_CELLS (GSIS_E_INVALID_ARG otherwise,
                              before anything is read or allocated) */
  double dx, dy;           /* cell sizes, > 0 */
  int32_t K;               /* number of ordinates, >= 1 */
  const double *mu;        /* [K] x direction cosine of Omega_k */
  const double *eta;       /* [K] y direction cosine; mu^2 + eta^2 <= 1 */
  const double *w;         /* [K] quadrature weights, sum = 4 pi (1e-12 rel.) */
  const double *sigma_a;   /* [nx*ny] absorption cross section, >= 0 */
  const double *sigma_s;   /* [nx*ny] scattering cross section, >= 0;
                              sigma_a + sigma_s > 0 in every cell */
  const double *q;         /* [nx*ny] isotropic volumetric source integrated
                              over the sphere (the transport source is
                              q/(4 pi) per steradian) */
  const double *bnd_in;    /* [2*(nx+ny)][K] incoming intensity per boundary
                              face and ordinate (Eq. micro_bc, no
                              reflection); entries with Omega_k . n_out >= 0
                              are ignored; NULL = vacuum */
} gsis_problem;

/* Largest nx*ny: the transport kernels address a quadrant's 48-byte
 * per-cell records with 32-bit byte offsets, so 48 nx ny < 2^32. */
#define GSIS_MAX_CELLS 89478485

enum { GSIS_SI = 0, GSIS_GSIS = 1 };
enum { GSIS_FP64 = 0, GSIS_FP32_MIXED = 1 };
enum { GSIS_HOT_CENTRAL = 0, GSIS_HOT_TRANSPORT = 1 };

typedef struct {
  int32_t method;        /* GSIS_SI or GSIS_GSIS (default) */
  int32_t precision;     /* GSIS_FP64 (default) or GSIS_FP32_MIXED: FP32
                            intensities (stored as deviations from
                            phi/(4 pi)), FP32 wavefront recurrence and
                            FP32 sums of the deviations' moments; FP64
                            residual, phi^m part of the moments, synthetic
                            solve, update and Err */
  int32_t order;         /* 1 = first-order upwind, 2 = second order (default) */
  int32_t limiter;       /* Barth-Jespersen limiter on (1, default) or off */
  int32_t alsm;          /* 1 = adaptive least squares (Sec. 5.2, default),
                            0 = plain least squares (Sec. 5.1) */
  int32_t hot_face;      /* GSIS_HOT_CENTRAL (default): face average of the
                            cell higher-order terms (Eq. Fij_d);
                            GSIS_HOT_TRANSPORT: on every interior face the
                            transport flux sum_k w_k (Omega_k . n) I_f,k of
                            the swept intensity (second-order upwind face
                            values, as in the residual) minus the compact
                            diffusion flux Gamma_f (phi_c - phi_nb), the full
                            form of Sec. 3.1 (Eq. DSA_Alcouffe), whose fixed
                            point is the source-iteration one. Single plans
                            only (a batch returns GSIS_E_UNSUPPORTED), not
                            with synth_form 1 or the adjoint */
  double tol;            /* stop when Err(phi) < tol (Eq. Err_W); default 1e-6 */
  int32_t max_iter;      /* outer iteration cap, >= 1; default 1000 */
  double synth_rtol;     /* synthetic CG stops at ||r|| <= synth_rtol ||r0||
                            (r0: residual of the warm start, the previous
                            phi) or at ||r|| <= 1e-14 ||b||; default 0.1.
                            The fixed point does not depend on it (at the
                            fixed point r0 = 0); it trades V-cycles per outer
                            iteration against outer iterations */
  int32_t synth_max_iter;/* CG iteration cap per outer iteration; default 50 */
  const double *I0;      /* optional warm start [nx*ny][K] (cell-major, the
                            caller's ordinate order); NULL = zero */
  void *stream;          /* hipStream_t to run on; NULL = default stream */
  int32_t device_ptrs;   /* 1: every array in gsis_problem, I0 and
                            gsis_result is device memory; 0: host memory */
  int32_t profile;       /* 1: record HIP events around each phase so that
                            gsis_plan_phase_times() can report them */
  double cfl_p;          /* global pseudo-time number CFL_p (Sec. 4.3, Eq.
                            cfl_pse): adds 1/(CFL_p dx_ref) to the diagonal
                            of every cell's increment solve; 0 = off
                            (default). dx_ref = min(dx, dy) */
  double beta;           /* local pseudo-time parameter beta (Eq. tau_pse):
                            adds max over face neighbours j of
                            |sigma_t,i r^L_ij - sigma_t,j r^R_ij| / (beta
                            dx_ref) to cell i's increment-solve diagonal,
                            which damps the increments of thin cells beside
                            thick ones; 0 = off (default). Neither shift
                            changes the fixed point (Eq. elem_main_shifted) */
  int32_t graph;         /* batches only: 1 (default) captures one outer
                            iteration in a hipGraph at gsis_batch_create and
                            replays it; 0 enqueues kernels one by one */
  int32_t synth_form;    /* synthetic balance (GSIS): 0 (default) takes the
                            compact diffusion flux Gamma_f (phi_c - phi_nb)
                            on interior faces; 1 takes the face average of
                            the cells' diffusive fluxes, -(grad phi_c /
                            (3 sigma_t,c) + grad phi_nb / (3 sigma_t,nb)) .
                            n / 2 (Eq. Fij_d), reached by synth_sub
                            defect-correction sub-iterations with the
                            compact matrix (Eqs. MSE_d1, Gamma_ij_def,
                            MSE_d_mtx1) from phi^{m+1/2}, each a CG +
                            multigrid solve. Single plans only (a batch
                            returns GSIS_E_UNSUPPORTED), not with the
                            adjoint, and with central HoT faces */
  int32_t synth_sub;     /* sub-iterations for synth_form 1 (>= 1); default 4 */
} gsis_options;

/* Fill *o with the defaults listed above. */
gsis_status gsis_options_default(gsis_options *o);

typedef struct {
  double *phi;           /* [nx*ny] out: phi at the last iterate */
  double *Fx, *Fy;       /* [nx*ny] out: radiative flux of the last iterate */
  double *err_hist;      /* [max_iter] out: Err after each iteration (Eq.
                            Err_W; may be NULL) */
  double *tres_hist;     /* [max_iter] out (may be NULL): relative transport
                            residual of the iterate I^m that iteration m
                            starts from, ||r(I^m)||_V / ||(sigma_s phi^m +
                            q)/(4 pi)||_V with r of Eq. RTE_d_res and
                            ||x||_V^2 = sum_c V sum_k w_k x_ck^2. It is 0
                            only where I^m solves the discrete transport
                            equation, so it exposes a source iteration that
                            meets Err < tol without having converged (Sec.
                            5.2.1); GSIS with central HoT faces keeps a
                            small nonzero value at its fixed point. (With the
                            test-only environment switch
                            GSIS_SWEEP_REFERENCE the history reads 0.) */
  int32_t n_iter;        /* out: iterations performed */
  double final_err;      /* out: Err of the last iteration */
} gsis_result;

/* One-shot solve: plan, iterate until Err < tol or max_iter, read, destroy. */
gsis_status gsis_solve(gsis_ctx *ctx, const gsis_problem *p,
                       const gsis_options *o, gsis_result *r);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * same solve as gsis_solve, with every piece of device state (intensities,
 * coefficients, multigrid hierarchy, CG vectors, flags) carved from one
 * library-owned scratch region of 256 MiB per GPU, a static device array
 * that each GPU the library runs on holds until the process ends. The call
 * makes no hipMalloc, hipHostMalloc or hipFree (its host-side set-up uses
 * ordinary heap memory) and profiling is off. The caller still passes the
 * problem and result buffers (host or device memory as options.device_ptrs
 * says). A problem whose state does not fit returns GSIS_E_INVALID_ARG with
 * a message naming the sizes (about 16 N K + 800 N + 64 K (nx + ny) bytes
 * for N = nx ny cells and K ordinates in FP64, 8 N K in place of 16 N K in
 * FP32-mixed: 256 x 256 x 128 in FP64 takes about 190 MB).
 * Every call on a GPU reuses that GPU's region, which keeps the last call's
 * contents; each call initialises what it reads. Calls that overlap on one
 * GPU (two host threads, or two streams) race on the region and must not
 * be made. */
gsis_status gsis_solve_noalloc(gsis_ctx *ctx, const gsis_problem *p,
                               const gsis_options *o, gsis_result *r);

/* Plans: set up once, then enqueue iterations. */
gsis_status gsis_plan_create(gsis_ctx *ctx, const gsis_problem *p,
                             const gsis_options *o, gsis_plan **out);
void gsis_plan_destroy(gsis_plan *plan);
/* Enqueue n more outer iterations on the plan's stream. Iterations after
 * convergence (Err < tol), divergence or max_iter do no work, so the
 * iterate stops exactly where a synchronous loop would. SI plans return
 * without waiting. GSIS plans wait for the device once per outer iteration:
 * the host reads the synthetic CG's device stop flag (after the CG update
 * of the iteration at which the previous solve stopped, the end of the
 * outer iteration already in the stream behind it) so that it launches no
 * V-cycle past convergence, and stops enqueueing once an iteration has
 * ended the solve. */
gsis_status gsis_plan_iterate(gsis_plan *plan, int32_t n);
/* Wait for the plan's stream, then report progress: iterations done and
 * whether Err < tol was reached (converged = 1) or the iteration diverged
 * (converged = -1, see GSIS_DIVERGED). Returns GSIS_E_DEVICE if the workgroups that share one
 * ordinate's wavefront recurrence (its rows are spread over up to 4 of them
 * when ny > 256 or when the ordinates alone would fill under half the CUs;
 * GSIS_CHAIN_PARTS=1..4 in the environment at plan creation fixes the
 * count) stopped waiting for each other: the iterate is then not
 * valid until gsis_plan_reset. */
gsis_status gsis_plan_status(gsis_plan *plan, int32_t *n_iter,
                             int32_t *converged, double *last_err);
/* Wait for the plan's stream and copy phi, F and the history into r (host or
 * device pointers as the plan's device_ptrs says). */
gsis_status gsis_plan_read(gsis_plan *plan, gsis_result *r);
/* Reset the iterate to the warm start (or zero) and the history. */
gsis_status gsis_plan_reset(gsis_plan *plan);

enum {
  GSIS_PHASE_RESIDUAL = 0, /* transport residual of every cell-ordinate (Eq. RTE_d_res),
                              written as the recurrence's right-hand side */
  GSIS_PHASE_SWEEP = 1,    /* exact first-order-upwind increment solve on the
                              wavefront (Eqs. RTE_d_increment..elem_mtx) */
  GSIS_PHASE_MOMENTS = 2,  /* phi and F of the swept intensity, boundary fluxes */
  GSIS_PHASE_HOT = 3,      /* HoT */
  GSIS_PHASE_SYNTH = 4,    /* synthetic right-hand side, CG + multigrid solve */
  GSIS_PHASE_UPDATE = 5,   /* correction, Err and the next source */
  GSIS_NUM_PHASES = 6
};
/* Wait for the plan's stream; *vcycles receives the number of multigrid
 * V-cycles (preconditioner applications: one after the warm start of each
 * synthetic solve, one per CG iteration) of all synthetic solves since the
 * plan was created or reset (with synth_form 1, of the last sub-iteration's
 * solve of each outer iteration). 0 for source iteration. */
gsis_status gsis_plan_synth_vcycles(gsis_plan *plan, int64_t *vcycles);
/* The transport step a plan runs: the residual of every cell-ordinate (Eq.
 * RTE_d_res) and the exact first-order-upwind increment solve on the
 * wavefront (Eqs. RTE_d_increment..elem_mtx). *form receives
 * GSIS_TRANSPORT_SPLIT (a residual launch, then the recurrence) or
 * GSIS_TRANSPORT_PIPELINED (one launch: workgroups of *bands bands of 64
 * rows, *parts workgroups per ordinate); the two give the same bits. The
 * choice is made at plan creation (FP64 problems of at least 2^26
 * cell-ordinates run pipelined) and the environment variable
 * GSIS_SWEEP_REFERENCE (0 split, 3 pipelined) overrides it. bands and parts
 * may be NULL. No device work. */
enum { GSIS_TRANSPORT_SPLIT = 0, GSIS_TRANSPORT_PIPELINED = 3 };
gsis_status gsis_plan_transport_form(gsis_plan *plan, int32_t *form, int32_t *bands,
                                     int32_t *parts);
/* Wait for the plan's stream; ms[GSIS_NUM_PHASES] receives the summed
 * duration of each phase over all profiled iterations (HIP events on the
 * plan's stream), *n_iter the number of profiled iterations. Needs
 * options.profile = 1. Clears the accumulated samples. */
gsis_status gsis_plan_phase_times(gsis_plan *plan, double *ms, int32_t *n_iter);

/* ------------------------------------------------------------------ batches
 * Many independent problems of uneven size (grid, ordinates, media) solved
 * together with shared options. Each keeps its own state and stops on its
 * own Err < tol; finished problems turn their kernels into no-ops. One outer
 * iteration runs the transport sweeps of all problems in one persistent
 * launch (work items = (problem, ordinate), longest first; the launch
 * configuration is chosen at creation by timing each compiled one on the
 * batch), and every other step, including each CG and multigrid step of the
 * synthetic solves, as one launch over all problems, each problem with its
 * own hierarchy, scalars and stop flag. The synthetic CG runs a fixed number
 * of iterations per outer iteration (the most any problem needed on the
 * first outer iteration, plus 2, at most synth_max_iter), each problem
 * stopping on its own test. options.I0 must be NULL; options.stream NULL
 * makes the batch create its own stream (graph capture cannot use the
 * default stream). */
typedef struct gsis_batch gsis_batch;

gsis_status gsis_batch_create(gsis_ctx *ctx, int32_t n, const gsis_problem *p /* [n] */,
                              const gsis_options *o, gsis_batch **out);
void gsis_batch_destroy(gsis_batch *b);
/* Enqueue n outer iterations (graph replays, or eager launches). */
gsis_status gsis_batch_iterate(gsis_batch *b, int32_t n);
/* Wait, then report per problem (arrays of length n, each may be NULL) the
 * iterations done, converged flag (1 / -1 / 0 as in gsis_plan_status) and
 * last Err, and how many problems have stopped (converged, diverged or at
 * max_iter). */
gsis_status gsis_batch_status(gsis_batch *b, int32_t *n_iter, int32_t *converged,
                              double *last_err, int32_t *n_finished);
/* Results of problem i, as gsis_plan_read. */
gsis_status gsis_batch_read(gsis_batch *b, int32_t i, gsis_result *r);
/* Every problem back to its initial state. */
gsis_status gsis_batch_reset(gsis_batch *b);

typedef struct {
  int32_t rows, prefetch;  /* chosen sweep configuration: rows per pass
                              (workgroup size) and prefetch depth */
  int32_t grid;            /* persistent workgroups launched */
  int32_t cg_iters;        /* CG iterations per outer iteration */
  int32_t n_configs;       /* compiled configurations timed (<= 8) */
  int32_t config_rows[8], config_prefetch[8];
  double config_ms[8];     /* measured sweep time of each (-1: did not fit) */
} gsis_batch_tuning;
gsis_status gsis_batch_get_tuning(gsis_batch *b, gsis_batch_tuning *t);

/* One-shot: create, iterate until every problem stops, read r[0..n-1],
 * destroy. Returns the worst per-problem status. */
gsis_status gsis_solve_batch(gsis_ctx *ctx, int32_t n, const gsis_problem *p,
                             const gsis_options *o, gsis_result *r /* [n] */);

/* ------------------------------------------------------------------ adjoint
 * Gradients of J = <g_phi, phi*> + <g_Fx, Fx*> + <g_Fy, Fy*> at the fixed
 * point of a plan with respect to sigma_a, sigma_s and q of every cell. With
 * the limiter off an outer iteration is affine in the intensity,
 * I' = G I + c(sigma_a, sigma_s, q); the adjoint lambda = G^T lambda + M^T g
 * (M: the moments of I) is iterated (each step one reverse pass of an outer
 * iteration: unweighted ordinate sum, synthetic solve with D1, transposed
 * right-hand side and HoT, transposed wall reconstruction, the increment
 * solve swept downstream-first, transposed residual) until Err of
 * sum_k lambda_k / (4 pi) < tol, and dJ/dp = lambda^T dT(I*)/dp is collected
 * cell by cell. Any explicit dependence of an objective on the parameters
 * is the caller's. Needs limiter = 0, precision FP64, central HoT faces and
 * no pseudo-time shift (GSIS_E_UNSUPPORTED otherwise), and a plan that has
 * converged (GSIS_E_INVALID_ARG otherwise); tighter forward tolerances give
 * more accurate gradients (about the forward Err, relative). */
typedef struct {
  int32_t n_iter;         /* adjoint iterations */
  double final_err;       /* Err of the ordinate sum at the last check */
  int32_t forward_iter;   /* outer iterations of the forward solve */
} gsis_adjoint_info;

/* Cotangents g_* and gradients g_sigma_a, g_sigma_s, g_q are [nx*ny] in the
 * caller's cell order, host or device memory as the plan's device_ptrs says;
 * a NULL cotangent is zero, a NULL gradient is not written. The plan keeps
 * three [nx*ny][K] adjoint arrays from the first call on. */
gsis_status gsis_plan_adjoint(gsis_plan *plan, const double *g_phi, const double *g_Fx,
                              const double *g_Fy, double tol, int32_t max_iter,
                              double *g_sigma_a, double *g_sigma_s, double *g_q,
                              gsis_adjoint_info *info /* may be NULL */);
/* One-shot: plan, forward solve to options.tol, optional forward results
 * (fwd may be NULL), adjoint to options.tol within options.max_iter. */
gsis_status gsis_adjoint(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                         const double *g_phi, const double *g_Fx, const double *g_Fy,
                         double *g_sigma_a, double *g_sigma_s, double *g_q, gsis_result *fwd,
                         gsis_adjoint_info *info);

/* ------------------------------------------------------- time-dependent form
 * The gray RTE with the material energy equation (Sec. 2.1 Eqs. RTE_g,
 * Tm_g; emission phi = a c T^4, isotropic), backward Euler in time with a
 * fixed step (Eqs. RTE_d, Tm_d), opacities constant in time. Each step
 * n -> n+1 runs inner iterations from (I^n, T^n) until max(Err(rho),
 * Err(T)) < options.tol (the criterion after Eq. Err_W) or options.max_iter:
 *  - the transport residual and increment solve take the 1/(c dt) terms
 *    (Eqs. RTE_d_res, RTE_d_increment, elem_mtx) and the emission of T^m;
 *  - source iteration: rho^{m+1} = rho^{m+1/2}, then sub_iter steps
 *    T <- T + R2 / D2 of the material equation with rho fixed (Eqs. MSE_d2,
 *    R2_def, MSE_d_mtx2, elem_mtx_M);
 *  - GSIS: sub_iter sub-iterations of the synthetic and material equations
 *    (Eq. GSIS_dse), each D1 d_rho = R1 (D1 with 1/(c dt) on the diagonal,
 *    Eqs. MSE_d1, R1_def, MSE_d_mtx1; compact diffusion flux plus the face
 *    HoT as in the steady form, walls F_T . n + kappa (rho - rho^{m+1/2}))
 *    and D2 d_T = R2 from the same sub-iterate, then the correction of Eq.
 *    GSIS_update.
 * FP64 only, synth_form 0, single plans (no batch, no adjoint). */
typedef struct {
  double c;            /* speed of light, > 0 */
  double a;            /* radiation constant, >= 0 */
  double dt;           /* time step, > 0 */
  const double *cv;    /* [nx*ny] volume specific heat, > 0 */
  const double *T0;    /* [nx*ny] initial material temperature, >= 0 */
  int32_t sub_iter;    /* macroscopic sub-iterations per inner iteration, >= 1 */
} gsis_material;

/* A plan of the time-dependent form: options.I0 is the initial intensity
 * (NULL = 0); cv and T0 host or device memory as options.device_ptrs says
 * (copied). Destroy it with gsis_plan_destroy; gsis_plan_status and
 * gsis_plan_read report the current step's inner iterations. */
gsis_status gsis_td_create(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                           const gsis_material *m, gsis_plan **out);
/* Advance n_steps time steps; inner_iters[n_steps] and last_err[n_steps]
 * (may be NULL) receive each step's inner iterations and final Err. Waits
 * for the device. Returns GSIS_NOT_CONVERGED if a step stopped at
 * options.max_iter (the steps after it still run), GSIS_DIVERGED at the
 * first step that diverged (no later step runs). */
gsis_status gsis_td_advance(gsis_plan *plan, int32_t n_steps, int32_t *inner_iters,
                            double *last_err);
/* rho = phi, T, Fx, Fy [nx*ny] of the current state (host or device memory
 * as the plan's device_ptrs says). */
gsis_status gsis_td_read(gsis_plan *plan, double *rho, double *T, double *Fx, double *Fy);

/* Library build string (compiler, target, options). */
const char *gsis_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GSIS_H */
