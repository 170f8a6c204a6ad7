/*
 * gsis_oracle.h -- plain FP64 CPU oracle of the steady gray GSIS / SI method.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this file; only tests, the smoke check and the CPU-baseline leg of the
 * benchmark do. It shares no code with the HIP library.
 *
 * Problem (Sec. 2.1 Eq. RTE_g, steady, no material coupling; Sec. 4.1):
 *   Omega . grad I + sigma_t I = (sigma_s phi + q) / (4 pi),
 *   phi = sum_k w_k I_k (zeroth moment, Eq. def_rho), F = sum_k w_k Omega_k I_k
 *   (Eq. def_F), on a uniform nx x ny Cartesian grid, cell c = j*nx + i.
 *
 * Boundary faces are numbered W side (j = 0..ny-1), E side (ny + j),
 * S side (2ny + i), N side (2ny + nx + i); bnd_in[f*K + k] is the incoming
 * intensity (Eq. micro_bc with alpha_w = 0), NULL means vacuum.
 */
#ifndef GSIS_ORACLE_H
#define GSIS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny;
  double dx, dy;
  int K;
  const double *mu, *eta, *w;            /* [K] */
  const double *sig_a, *sig_s, *q;       /* [nx*ny] */
  const double *bnd_in;                  /* [2(nx+ny)][K] or NULL */
} ora_problem;

typedef struct {
  int method;     /* 0 = source iteration, 1 = GSIS */
  int order;      /* 1 = first-order upwind, 2 = second-order upwind */
  int limiter;    /* Barth-Jespersen limiter on/off */
  int alsm;       /* 1 = adaptive least squares (shifted points), 0 = plain LSQ */
  int hot_face;   /* 0 = central average of cell HoT, 1 = transport face flux */
  double tol;     /* stop when Err(phi) < tol */
  int max_iter;
  double cfl_p;   /* global pseudo-time number (Eq. cfl_pse); 0 = off */
  double beta;    /* local pseudo-time parameter (Eq. tau_pse); 0 = off */
  int synth_form; /* 0 = compact diffusion flux Gamma (x_c - x_nb) in the
                     synthetic balance; 1 = the face average of the cells'
                     diffusive fluxes (Eq. Fij_d), reached by synth_sub
                     defect-correction sub-iterations with the compact
                     matrix D1 (Eqs. MSE_d1, Gamma_ij_def, MSE_d_mtx1) from
                     phi^{m+1/2}; central HoT faces only */
  int synth_sub;  /* sub-iterations of synth_form 1 (>= 1) */
} ora_options;

/* ALSM / LSQ cell gradient of a cell field U[nx*ny] (Sec. 5, Eqs. LSF,
 * LSM_mtx, shifted_j, new_vector, LSF_mdf). */
void ora_gradient(const ora_problem *p, int alsm, const double *U,
                  double *Gx, double *Gy);

/* Barth-Jespersen limiter value per cell (Sec. 4.1 Eq. Ii,k). */
void ora_bj_limiter(const ora_problem *p, const double *U, const double *Gx,
                    const double *Gy, double *psi);

/* Synthetic-equation face coefficients: Gamma on interior x faces
 * [(nx-1)*ny] (face right of cell (i,j) at index j*(nx-1)+i) and y faces
 * [nx*(ny-1)] (face above (i,j) at j*nx+i) (Eq. Gamma_ij_com2); kappa per
 * boundary face [2(nx+ny)] (Eqs. macro_bc_delta_flux, macro_bc_delta_flux2). */
void ora_plant_kappa(int mode);   /* test hook, see gsis_oracle.c */
void ora_face_coeffs(const ora_problem *p, double *gam_x, double *gam_y,
                     double *kappa);

/* Mesoscopic residual r[c*K+k] of I[c*K+k] (Eq. RTE_d_res, steady). */
void ora_residual(const ora_problem *p, const ora_options *o, const double *I,
                  double *r);

/* Exact first-order-upwind increment solve per ordinate (Eqs.
 * RTE_d_increment, delta_Iij, RTE_d_mtx, elem_mtx, steady). */
void ora_sweep(const ora_problem *p, const ora_options *o, const double *r,
               double *dI);

/* Pseudo-time shift of the increment-solve diagonal per cell (Eq.
 * elem_main_shifted without the physical time term); 0 when o is NULL or
 * both parameters are 0. */
double ora_pseudo_shift(const ora_problem *p, const ora_options *o, int c);

/* One outer iteration: I_in -> I_out (Eqs. SI_update or GSIS_update).
 * phi_out receives phi^{m+1}. Returns 0 on success. */
int ora_iterate(const ora_problem *p, const ora_options *o, const double *I_in,
                double *I_out, double *phi_out);

/* Full solve from I0 (NULL = 0). Outputs phi, Fx, Fy [nx*ny]; err_hist
 * [max_iter] (may be NULL): Err(phi) after iteration m (Eq. Err_W);
 * tres_hist [max_iter] (may be NULL): the relative transport residual
 * ||r(I^m)||_V / ||(sigma_s phi^m + q)/(4 pi)||_V of the iterate I^m that
 * iteration m starts from (||x||_V^2 = sum_c V sum_k w_k x_ck^2);
 * I_final [nx*ny*K] (may be NULL).
 * Returns 0 if converged, 1 if max_iter was reached, 2 if the iteration
 * diverged (Err not finite, or ||phi^{m+1} - phi^m||_V above 1e3 times its
 * smallest value so far, floored at 1e-9 ||phi^{m+1}||_V), <0 on error. */
int ora_solve(const ora_problem *p, const ora_options *o, const double *I0,
              double *phi, double *Fx, double *Fy, double *err_hist,
              double *tres_hist, int *n_iter, double *final_err, double *I_final);

/* Solve the synthetic system D1 x = b exactly (banded Cholesky) or, above a
 * size limit, by CG to a relative residual of 1e-14 (Eqs. MSE_d_mtx1,
 * elem_mtx_M, steady). Exposed for tests. */
int ora_synthetic_solve(const ora_problem *p, const double *b, double *x);

/* Apply D1 (for tests). */
void ora_synthetic_apply(const ora_problem *p, const double *x, double *y);

/* The synthetic balance with the face-averaged diffusive flux of Eq. Fij_d
 * differs from the compact one (D1 x = b) on interior faces only:
 *   D1 x = b + corr(x),  corr_c = sum over interior faces f of c of
 *   A_f [Gamma_f (x_c - x_nb) + (w_c + w_nb) . n_f / 2],
 * w = grad(x) / (3 sigma_t) with the ALSM (alsm = 1) or LSQ gradient. */
void ora_wide_correction(const ora_problem *p, int alsm, const double *x, double *corr);

/* n_sub sub-iterations x <- D1^{-1} (b + corr(x)) from the given x, each an
 * exact solve: the defect correction D1 dx = R1(x) of Eqs. MSE_d1 and
 * MSE_d_mtx1, R1 the residual of the face-averaged balance. */
int ora_synthetic_wide(const ora_problem *p, int alsm, const double *b, int n_sub, double *x);

/* Time-dependent gray RTE with the material energy equation (Sec. 2.1 Eqs.
 * RTE_g, Tm_g; emission phi = a c T^4), backward Euler in time (Eqs. RTE_d,
 * Tm_d) with opacities constant in time, and inner iterations per step (SI,
 * or GSIS with the synthetic and material equations of Eq. GSIS_dse solved
 * by sub_iter sub-iterations of Eqs. MSE_d1, MSE_d2). */
typedef struct {
  double c;          /* speed of light, > 0 */
  double a;          /* radiation constant, >= 0 */
  double dt;         /* time step, > 0 */
  const double *cv;  /* [nx*ny] volume specific heat, > 0 */
  int sub_iter;      /* macroscopic sub-iterations per inner iteration, >= 1 */
} ora_material;

/* n_steps time steps from I0 [nx*ny*K] (NULL = 0) and T0 [nx*ny]; each step
 * iterates until max(Err(rho), Err(T)) < o->tol or o->max_iter inner
 * iterations. Outputs I_out (may be NULL), T_out, rho, Fx, Fy of the last
 * step; inner_iters and err_last [n_steps] (may be NULL). Returns 0 if every
 * step converged, 1 if a step reached max_iter, 2 on divergence, <0 on
 * error (-1: invalid material data or synth_form 1). */
int ora_td_solve(const ora_problem *p, const ora_options *o, const ora_material *mt,
                 const double *I0, const double *T0, int n_steps, double *I_out,
                 double *T_out, double *rho, double *Fx, double *Fy, int *inner_iters,
                 double *err_last);

/* Adjoint of the fixed point I* of the iteration (limiter off, central HoT
 * faces, no pseudo time; method SI or GSIS): lambda = G^T lambda + M^T g for
 * the output J = <g_phi, phi*> + <g_Fx, Fx*> + <g_Fy, Fy*> (any cotangent may
 * be NULL), iterated until Err of sum_k lambda_k/(4 pi) < tol; then
 * dJ/dsigma_a, dJ/dsigma_s, dJ/dq per cell (any output may be NULL) and,
 * optionally, lambda [N][K]. Returns 0, 1 (not converged), <0 on error
 * (-4: unsupported options). */
int ora_adjoint(const ora_problem *p, const ora_options *o, const double *I_star,
                const double *g_phi, const double *g_Fx, const double *g_Fy, double tol,
                int max_iter, double *g_sa, double *g_ss, double *g_q, double *lam_out,
                int *n_iter, double *err_hist);

#ifdef __cplusplus
}
#endif
#endif
