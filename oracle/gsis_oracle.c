/*
 * gsis_oracle.c -- plain FP64 CPU oracle of the steady gray source iteration
 * (SI) and general synthetic iterative scheme (GSIS).
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
 * the benchmark call it; the product path never does. It shares no code,
 * header, table or helper with the HIP library.
 *
 * Everything is written out per cell, per face and per ordinate, in the order
 * the paper states the steps, with no blocking or fusion. OpenMP only splits
 * independent ordinates (or independent rows of a factorisation); every sum
 * is taken in a fixed order, so results do not depend on the thread count.
 *
 * Readings of the paper that this file fixes (the paper is silent there):
 *  - steady state: the 1/(c dt) terms and the material equation are dropped;
 *    the emission term sigma_a*phi_emit is the isotropic source q, so the
 *    transport source is (sigma_s*phi + q)/(4 pi) and the synthetic source q;
 *  - the transport increment system (Eq. RTE_d_mtx) is solved exactly, once
 *    per outer iteration, by visiting cells in upwind order per ordinate;
 *  - the synthetic equation uses the compact flux Gamma_f (phi_c - phi_nb)
 *    for the diffusion part (its own Jacobian, Eq. Gamma_ij_def) and the
 *    face average of the cell higher-order terms (Eq. Fij_d, second term);
 *    the resulting SPD system is solved exactly;
 *  - least squares use the existing face neighbours only, unweighted;
 *  - the Barth-Jespersen limiter takes the extrema over the cell and its
 *    face neighbours and checks all four faces;
 *  - an upwind tie (Omega.n = 0) takes the cell's own value.
 */
#include "gsis_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FOUR_PI (4.0 * M_PI)

/* Face directions of a Cartesian cell: 0 = east (+x), 1 = west (-x),
 * 2 = north (+y), 3 = south (-y). */
static const double NX_[4] = {1.0, -1.0, 0.0, 0.0};
static const double NY_[4] = {0.0, 0.0, 1.0, -1.0};
static const int OPP_[4] = {1, 0, 3, 2};

static int neighbour(const ora_problem *p, int i, int j, int f) {
  int ii = i + (f == 0) - (f == 1);
  int jj = j + (f == 2) - (f == 3);
  if (ii < 0 || ii >= p->nx || jj < 0 || jj >= p->ny) return -1;
  return jj * p->nx + ii;
}

/* Boundary-face index of cell (i,j) on side f (only valid if no neighbour). */
static int bface(const ora_problem *p, int i, int j, int f) {
  switch (f) {
    case 1: return j;                         /* west  */
    case 0: return p->ny + j;                 /* east  */
    case 3: return 2 * p->ny + i;             /* south */
    default: return 2 * p->ny + p->nx + i;    /* north */
  }
}

/* x_f - x_c for face f (face centres sit midway on a uniform grid). */
static double face_ox(const ora_problem *p, int f) { return 0.5 * p->dx * NX_[f]; }
static double face_oy(const ora_problem *p, int f) { return 0.5 * p->dy * NY_[f]; }
/* Face area over cell volume. */
static double area_over_vol(const ora_problem *p, int f) {
  return (f < 2) ? 1.0 / p->dx : 1.0 / p->dy;
}
static double face_area(const ora_problem *p, int f) { return (f < 2) ? p->dy : p->dx; }

static double sig_t(const ora_problem *p, int c) { return p->sig_a[c] + p->sig_s[c]; }

/* ------------------------------------------------------------------------ */
/* Gradient: least squares over face neighbours (Eqs. Uj-Ui, LSF, LSM_mtx);  */
/* with alsm=1 each neighbour centre x_j is replaced by the shifted point     */
/* x'_j = x_ij + (sigma_t,j / sigma_t,i) r^R_ij (Eqs. shifted_j, new_vector,  */
/* LSF_mdf).                                                                   */
/* ------------------------------------------------------------------------ */
static void gradient_cell(const ora_problem *p, int alsm, const double *U,
                          int i, int j, double *gx, double *gy) {
  const int c = j * p->nx + i;
  double Mxx = 0, Mxy = 0, Myy = 0, bx = 0, by = 0;
  for (int f = 0; f < 4; ++f) {
    int nb = neighbour(p, i, j, f);
    if (nb < 0) continue;
    /* x_j - x_i */
    double ex = NX_[f] * p->dx, ey = NY_[f] * p->dy;
    if (alsm) {
      /* face midpoint x_ij = x_i + (x_j - x_i)/2, r^R = x_j - x_ij */
      double fx = 0.5 * ex, fy = 0.5 * ey;
      double rx = ex - fx, ry = ey - fy;
      double ratio = sig_t(p, nb) / sig_t(p, c);
      ex = fx + ratio * rx;      /* x'_j - x_i */
      ey = fy + ratio * ry;
    }
    double du = U[nb] - U[c];
    Mxx += ex * ex; Mxy += ex * ey; Myy += ey * ey;
    bx += ex * du;  by += ey * du;
  }
  if (Mxx > 0 && Myy > 0) {
    double det = Mxx * Myy - Mxy * Mxy;
    *gx = (bx * Myy - by * Mxy) / det;
    *gy = (by * Mxx - bx * Mxy) / det;
  } else if (Mxx > 0) {
    *gx = bx / Mxx; *gy = 0.0;
  } else if (Myy > 0) {
    *gx = 0.0; *gy = by / Myy;
  } else {
    *gx = 0.0; *gy = 0.0;
  }
}

void ora_gradient(const ora_problem *p, int alsm, const double *U, double *Gx,
                  double *Gy) {
  for (int j = 0; j < p->ny; ++j)
    for (int i = 0; i < p->nx; ++i)
      gradient_cell(p, alsm, U, i, j, &Gx[j * p->nx + i], &Gy[j * p->nx + i]);
}

/* Barth-Jespersen limiter (Sec. 4.1, Eq. Ii,k and its reference). */
static double bj_cell(const ora_problem *p, const double *U, int i, int j,
                      double gx, double gy) {
  const int c = j * p->nx + i;
  double umax = U[c], umin = U[c];
  for (int f = 0; f < 4; ++f) {
    int nb = neighbour(p, i, j, f);
    if (nb < 0) continue;
    if (U[nb] > umax) umax = U[nb];
    if (U[nb] < umin) umin = U[nb];
  }
  double psi = 1.0;
  for (int f = 0; f < 4; ++f) {
    double delta = gx * face_ox(p, f) + gy * face_oy(p, f);
    double pf = 1.0;
    if (delta > 0) pf = fmin(1.0, (umax - U[c]) / delta);
    else if (delta < 0) pf = fmin(1.0, (umin - U[c]) / delta);
    if (pf < psi) psi = pf;
  }
  return psi;
}

void ora_bj_limiter(const ora_problem *p, const double *U, const double *Gx,
                    const double *Gy, double *psi) {
  for (int j = 0; j < p->ny; ++j)
    for (int i = 0; i < p->nx; ++i) {
      int c = j * p->nx + i;
      psi[c] = bj_cell(p, U, i, j, Gx[c], Gy[c]);
    }
}

/* Linear reconstruction of a cell field at the centre of face f of cell c
 * (Eq. Ii,k): U_c + psi_c G_c . (x_f - x_c). With order 1 the gradient is
 * absent and the face takes the cell value. */
typedef struct {
  const double *U, *Gx, *Gy, *psi;
  int order;
} recon;

static double rec_face(const ora_problem *p, const recon *R, int c, int f) {
  if (R->order < 2) return R->U[c];
  return R->U[c] + R->psi[c] * (R->Gx[c] * face_ox(p, f) + R->Gy[c] * face_oy(p, f));
}

/* Build gradient and limiter of one ordinate field U (scratch: Gx, Gy, psi). */
static void build_recon(const ora_problem *p, const ora_options *o,
                        const double *U, double *Gx, double *Gy, double *psi,
                        recon *R) {
  R->U = U; R->Gx = Gx; R->Gy = Gy; R->psi = psi; R->order = o->order;
  if (o->order < 2) return;
  ora_gradient(p, o->alsm, U, Gx, Gy);
  if (o->limiter) ora_bj_limiter(p, U, Gx, Gy, psi);
  else for (int c = 0; c < p->nx * p->ny; ++c) psi[c] = 1.0;
}

/* Face value of ordinate k on face f of cell (i,j), upwinded (Eqs. Iij,
 * micro_bc with alpha_w = 0). */
static double face_value(const ora_problem *p, const recon *R, int i, int j,
                         int f, int k) {
  const int c = j * p->nx + i;
  const double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
  int nb = neighbour(p, i, j, f);
  if (on >= 0) return rec_face(p, R, c, f);
  if (nb >= 0) return rec_face(p, R, nb, OPP_[f]);
  return p->bnd_in ? p->bnd_in[(size_t)bface(p, i, j, f) * p->K + k] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Moments (Sec. 4.1 quadrature; Eqs. def_rho, def_F).                        */
/* ------------------------------------------------------------------------ */
static void moments(const ora_problem *p, const double *I, double *phi,
                    double *Fx, double *Fy) {
  const int N = p->nx * p->ny, K = p->K;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < N; ++c) {
    double s0 = 0, sx = 0, sy = 0;
    for (int k = 0; k < K; ++k) {
      double v = p->w[k] * I[(size_t)c * K + k];
      s0 += v; sx += p->mu[k] * v; sy += p->eta[k] * v;
    }
    phi[c] = s0;
    if (Fx) Fx[c] = sx;
    if (Fy) Fy[c] = sy;
  }
}

/* ------------------------------------------------------------------------ */
/* Mesoscopic residual (Eq. RTE_d_res, steady):                               */
/*   r = (sigma_s phi + q)/(4 pi) - sigma_t I - (1/V) sum_f (Omega.n_f) A_f I_f */
/* ------------------------------------------------------------------------ */
/* The same with the backward-Euler time terms of Eq. RTE_d_res:
 *   r = S_c - (sigma_t + tdiag) I + tdiag I^n - (1/V) sum_f (Omega.n_f) A_f I_f,
 * tdiag = 1/(c dt), I^n [N][K] the previous time level (NULL: no term) and
 * S_c [N] the isotropic source per steradian (NULL: (sigma_s phi + q)/(4 pi)
 * from the moments of I, the steady case). */
static void residual_t(const ora_problem *p, const ora_options *o, const double *I,
                       const double *S_iso, double tdiag, const double *I_n, double *r);

void ora_residual(const ora_problem *p, const ora_options *o, const double *I,
                  double *r) {
  residual_t(p, o, I, NULL, 0.0, NULL, r);
}

static void residual_t(const ora_problem *p, const ora_options *o, const double *I,
                       const double *S_iso, double tdiag, const double *I_n, double *r) {
  const int N = p->nx * p->ny, K = p->K;
  double *phi = (double *)malloc(sizeof(double) * N);
  moments(p, I, phi, NULL, NULL);
#pragma omp parallel
  {
    double *U = (double *)malloc(sizeof(double) * N * 4);
    double *Gx = U + N, *Gy = U + 2 * N, *psi = U + 3 * N;
#pragma omp for schedule(dynamic, 1)
    for (int k = 0; k < K; ++k) {
      for (int c = 0; c < N; ++c) U[c] = I[(size_t)c * K + k];
      recon R;
      build_recon(p, o, U, Gx, Gy, psi, &R);
      for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
          const int c = j * p->nx + i;
          double div = 0.0;
          for (int f = 0; f < 4; ++f) {
            double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
            div += on * area_over_vol(p, f) * face_value(p, &R, i, j, f, k);
          }
          const double src = S_iso ? S_iso[c] : (p->sig_s[c] * phi[c] + p->q[c]) / FOUR_PI;
          double rv = src - (sig_t(p, c) + tdiag) * U[c] - div;
          if (I_n) rv += tdiag * I_n[(size_t)c * K + k];
          r[(size_t)c * K + k] = rv;
        }
    }
    free(U);
  }
  free(phi);
}

/* ------------------------------------------------------------------------ */
/* Pseudo-time diagonal shift (Sec. 4.3, Eqs. cfl_pse, tau_pse,               */
/* elem_main_shifted). The speed of light cancels in 1/(c dt_p):              */
/*   1/(c dt_p)  = 1 / (CFL_p dx_ref),                                        */
/*   1/(c tau_p) = max_{j in N(i)} |sig_i r^L_ij - sig_j r^R_ij| / (beta dx_ref)*/
/* with dx_ref = min(dx, dy). Only the increment solve sees the shift, so the */
/* fixed point is unchanged.                                                  */
/* ------------------------------------------------------------------------ */
double ora_pseudo_shift(const ora_problem *p, const ora_options *o, int c) {
  if (!o) return 0.0;
  const double dref = p->dx < p->dy ? p->dx : p->dy;
  double s = 0.0;
  if (o->cfl_p > 0) s += 1.0 / (o->cfl_p * dref);
  if (o->beta > 0) {
    const int i = c % p->nx, j = c / p->nx;
    double m = 0.0;
    for (int f = 0; f < 4; ++f) {
      const int nb = neighbour(p, i, j, f);
      if (nb < 0) continue;
      const double rLx = -face_ox(p, f), rLy = -face_oy(p, f);
      const double rRx = face_ox(p, f), rRy = face_oy(p, f);
      const double vx = sig_t(p, c) * rLx - sig_t(p, nb) * rRx;
      const double vy = sig_t(p, c) * rLy - sig_t(p, nb) * rRy;
      const double v = sqrt(vx * vx + vy * vy);
      if (v > m) m = v;
    }
    s += m / (o->beta * dref);
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Increment solve (Eqs. RTE_d_increment, delta_Iij, RTE_d_mtx, elem_mtx):    */
/*   d_ii dI_i + sum_{inflow faces} (Omega.A_ij / V_i) dI_j = r_i,            */
/*   d_ii = sigma_t + sum_{outflow faces} Omega.A_ij / V_i (+ pseudo shift),  */
/* first-order upwind increments, zero increments on inflow boundary faces.   */
/* Cells are visited in upwind order, which makes the solve exact.            */
/* ------------------------------------------------------------------------ */
/* The increment solve with tdiag = 1/(c dt) on the diagonal (Eq. elem_mtx). */
static void sweep_t(const ora_problem *p, const ora_options *o, double tdiag, const double *r,
                    double *dI);

void ora_sweep(const ora_problem *p, const ora_options *o, const double *r, double *dI) {
  sweep_t(p, o, 0.0, r, dI);
}

static void sweep_t(const ora_problem *p, const ora_options *o, double tdiag, const double *r,
                    double *dI) {
  const int nx = p->nx, ny = p->ny, K = p->K;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < K; ++k) {
    const int i0 = p->mu[k] >= 0 ? 0 : nx - 1, di = p->mu[k] >= 0 ? 1 : -1;
    const int j0 = p->eta[k] >= 0 ? 0 : ny - 1, dj = p->eta[k] >= 0 ? 1 : -1;
    for (int jj = 0, j = j0; jj < ny; ++jj, j += dj)
      for (int ii = 0, i = i0; ii < nx; ++ii, i += di) {
        const int c = j * nx + i;
        double d = sig_t(p, c) + tdiag + ora_pseudo_shift(p, o, c), rhs = r[(size_t)c * K + k];
        for (int f = 0; f < 4; ++f) {
          double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
          if (on > 0) {
            d += on * area_over_vol(p, f);
          } else if (on < 0) {
            int nb = neighbour(p, i, j, f);
            if (nb >= 0) rhs -= on * area_over_vol(p, f) * dI[(size_t)nb * K + k];
          }
        }
        dI[(size_t)c * K + k] = rhs / d;
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Synthetic-equation coefficients.                                           */
/* Gamma_ij = -((sig_i r^L - sig_j r^R) . n) / (3 |sig_i r^L - sig_j r^R|^2)  */
/* (Eq. Gamma_ij_com2), r^L = x_i - x_ij, r^R = x_j - x_ij.                   */
/* kappa_iw = (x_iw - x_i).n / (3 sig_i |x_iw - x_i|^2) + 1/4                  */
/* (normal part of Eq. macro_bc_delta_flux with Eq. macro_bc_delta_flux2).    */
/* ------------------------------------------------------------------------ */
static double gamma_face(const ora_problem *p, int c, int nb, int f) {
  double rLx = -face_ox(p, f), rLy = -face_oy(p, f);       /* x_i - x_ij */
  double rRx = face_ox(p, f), rRy = face_oy(p, f);         /* x_j - x_ij */
  double vx = sig_t(p, c) * rLx - sig_t(p, nb) * rRx;
  double vy = sig_t(p, c) * rLy - sig_t(p, nb) * rRy;
  return -(vx * NX_[f] + vy * NY_[f]) / (3.0 * (vx * vx + vy * vy));
}

/* Test hook: ora_plant_kappa(m) replaces kappa by a misreading (1: escape
 * term only, 2: diffusion term only, 3: the two terms in series, 4: none) so
 * that the pins can show they catch it; 0 restores the paper's form. */
static int kappa_plant = 0;
void ora_plant_kappa(int mode) { kappa_plant = mode; }

static double kappa_face(const ora_problem *p, int c, int f) {
  double ox = face_ox(p, f), oy = face_oy(p, f);
  const double kd = (ox * NX_[f] + oy * NY_[f]) / (3.0 * sig_t(p, c) * (ox * ox + oy * oy));
  switch (kappa_plant) {
    case 1: return 0.25;
    case 2: return kd;
    case 3: return 1.0 / (1.0 / kd + 4.0);
    case 4: return 0.0;
    default: return kd + 0.25;
  }
}

void ora_face_coeffs(const ora_problem *p, double *gam_x, double *gam_y,
                     double *kappa) {
  const int nx = p->nx, ny = p->ny;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i + 1 < nx; ++i)
      gam_x[j * (nx - 1) + i] = gamma_face(p, j * nx + i, j * nx + i + 1, 0);
  for (int j = 0; j + 1 < ny; ++j)
    for (int i = 0; i < nx; ++i)
      gam_y[j * nx + i] = gamma_face(p, j * nx + i, (j + 1) * nx + i, 2);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int f = 0; f < 4; ++f)
        if (neighbour(p, i, j, f) < 0)
          kappa[bface(p, i, j, f)] = kappa_face(p, j * nx + i, f);
}

/* D1 x (Eqs. MSE_d_mtx1, elem_mtx_M, steady, multiplied by V):               */
/*   V sig_a x_c + sum_int A Gamma (x_c - x_nb) + sum_bnd A kappa x_c.         */
/* D1 x with tdiag = 1/(c dt) added to sigma_a on the diagonal (Eq.
 * elem_mtx_M; tdiag = 0 in steady state). */
static void synthetic_apply_t(const ora_problem *p, double tdiag, const double *x, double *y) {
  const int nx = p->nx, ny = p->ny;
  const double V = p->dx * p->dy;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      double s = V * (p->sig_a[c] + tdiag) * x[c];
      for (int f = 0; f < 4; ++f) {
        int nb = neighbour(p, i, j, f);
        if (nb >= 0) s += face_area(p, f) * gamma_face(p, c, nb, f) * (x[c] - x[nb]);
        else s += face_area(p, f) * kappa_face(p, c, f) * x[c];
      }
      y[c] = s;
    }
}

void ora_synthetic_apply(const ora_problem *p, const double *x, double *y) {
  synthetic_apply_t(p, 0.0, x, y);
}

/* Dense-band entry of D1: row c, column c - d (d = 0, 1 or nx). */
typedef struct {
  int N, bw;          /* bandwidth */
  double *L;          /* band of L: L[c*(bw+1) + d] = L(c, c-d) */
  int use_cg;
  double tdiag;       /* 1/(c dt) on the diagonal (0: steady) */
} synth_factor;

#define BAND_LIMIT (1L << 31)   /* doubles (16 GiB); above this CG is used */

static int synth_factor_build(const ora_problem *p, double tdiag, synth_factor *S) {
  const int nx = p->nx, ny = p->ny, N = nx * ny;
  const int bw = ny > 1 ? nx : 1;
  S->N = N; S->bw = bw; S->L = NULL; S->tdiag = tdiag;
  S->use_cg = ((long)N * (bw + 1) > BAND_LIMIT);
  if (S->use_cg) return 0;
  double *L = (double *)calloc((size_t)N * (bw + 1), sizeof(double));
  if (!L) return -3;
  const double V = p->dx * p->dy;
  /* assemble the lower band of D1 */
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      double diag = V * (p->sig_a[c] + tdiag);
      for (int f = 0; f < 4; ++f) {
        int nb = neighbour(p, i, j, f);
        if (nb >= 0) {
          double a = face_area(p, f) * gamma_face(p, c, nb, f);
          diag += a;
          if (nb < c) L[(size_t)c * (bw + 1) + (c - nb)] = -a;
        } else {
          diag += face_area(p, f) * kappa_face(p, c, f);
        }
      }
      L[(size_t)c * (bw + 1)] = diag;
    }
  /* banded Cholesky, left-looking: L(i,j) = (A(i,j) - sum_k L(i,k)L(j,k))/L(j,j) */
  const size_t ld = bw + 1;
  for (int jc = 0; jc < N; ++jc) {
    double s = L[(size_t)jc * ld];
    int k0 = jc - bw > 0 ? jc - bw : 0;
    for (int k = k0; k < jc; ++k) {
      double v = L[(size_t)jc * ld + (jc - k)];
      s -= v * v;
    }
    if (!(s > 0)) { free(L); return -1; }
    const double djj = sqrt(s);
    L[(size_t)jc * ld] = djj;
    int iend = jc + bw < N - 1 ? jc + bw : N - 1;
#pragma omp parallel for schedule(dynamic, 16) if (bw >= 64)
    for (int i = jc + 1; i <= iend; ++i) {
      double t = L[(size_t)i * ld + (i - jc)];
      int kk0 = i - bw > 0 ? i - bw : 0;
      double acc = 0.0;
#pragma omp simd reduction(+ : acc)
      for (int k = kk0; k < jc; ++k)
        acc += L[(size_t)i * ld + (i - k)] * L[(size_t)jc * ld + (jc - k)];
      t -= acc;
      L[(size_t)i * ld + (i - jc)] = t / djj;
    }
  }
  S->L = L;
  return 0;
}

static void synth_factor_free(synth_factor *S) { free(S->L); S->L = NULL; }

static int synth_cg(const ora_problem *p, double tdiag, const double *b, double *x) {
  const int N = p->nx * p->ny;
  double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N),
         *pp = malloc(sizeof(double) * N), *Ap = malloc(sizeof(double) * N),
         *dg = malloc(sizeof(double) * N), *e = calloc(N, sizeof(double));
  /* Jacobi preconditioner: the diagonal of D1 */
  for (int c = 0; c < N; ++c) e[c] = 1.0;
  /* diag(D1) = D1 applied to unit vectors would be O(N^2); assemble directly */
  {
    const int nx = p->nx, ny = p->ny;
    const double V = p->dx * p->dy;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = j * nx + i;
        double d = V * (p->sig_a[c] + tdiag);
        for (int f = 0; f < 4; ++f) {
          int nb = neighbour(p, i, j, f);
          d += face_area(p, f) * (nb >= 0 ? gamma_face(p, c, nb, f) : kappa_face(p, c, f));
        }
        dg[c] = d;
      }
  }
  double bn = 0;
  for (int c = 0; c < N; ++c) { x[c] = 0; r[c] = b[c]; bn += b[c] * b[c]; }
  bn = sqrt(bn);
  int ret = 1;
  if (bn == 0) ret = 0;
  double rz = 0;
  for (int c = 0; c < N; ++c) { z[c] = r[c] / dg[c]; pp[c] = z[c]; rz += r[c] * z[c]; }
  for (int it = 0; it < 200000 && ret; ++it) {
    synthetic_apply_t(p, tdiag, pp, Ap);
    double pAp = 0;
    for (int c = 0; c < N; ++c) pAp += pp[c] * Ap[c];
    double a = rz / pAp, rn = 0;
    for (int c = 0; c < N; ++c) { x[c] += a * pp[c]; r[c] -= a * Ap[c]; rn += r[c] * r[c]; }
    if (sqrt(rn) <= 1e-14 * bn) { ret = 0; break; }
    double rz2 = 0;
    for (int c = 0; c < N; ++c) { z[c] = r[c] / dg[c]; rz2 += r[c] * z[c]; }
    double bb = rz2 / rz;
    rz = rz2;
    for (int c = 0; c < N; ++c) pp[c] = z[c] + bb * pp[c];
  }
  free(r); free(z); free(pp); free(Ap); free(dg); free(e);
  return ret == 0 ? 0 : -2;
}

/* x = (L L^T)^{-1} b by forward and backward substitution in the band. */
static void band_substitute(const synth_factor *S, const double *b, double *x) {
  const int N = S->N, bw = S->bw;
  const size_t ld = bw + 1;
  const double *L = S->L;
  /* L y = b */
  for (int i = 0; i < N; ++i) {
    double t = b[i];
    int k0 = i - bw > 0 ? i - bw : 0;
    for (int k = k0; k < i; ++k) t -= L[(size_t)i * ld + (i - k)] * x[k];
    x[i] = t / L[(size_t)i * ld];
  }
  /* L^T x = y */
  for (int i = N - 1; i >= 0; --i) {
    double t = x[i];
    int k1 = i + bw < N - 1 ? i + bw : N - 1;
    for (int k = i + 1; k <= k1; ++k) t -= L[(size_t)k * ld + (k - i)] * x[k];
    x[i] = t / L[(size_t)i * ld];
  }
}

/* D1 x = b by the Cholesky factor and one step of iterative refinement
 * (r = b - D1 x, x += (L L^T)^{-1} r): on the high-contrast media D1's
 * condition number reaches 1e9, where the refinement takes the solution
 * from about 1e-10 to about 1e-12 of the exact solve the method asks for. */
static int synth_solve_with(const ora_problem *p, const synth_factor *S,
                            const double *b, double *x) {
  if (S->use_cg) return synth_cg(p, S->tdiag, b, x);
  const int N = S->N;
  band_substitute(S, b, x);
  double *r = malloc(sizeof(double) * N), *dx = malloc(sizeof(double) * N);
  if (!r || !dx) { free(r); free(dx); return -3; }
  synthetic_apply_t(p, S->tdiag, x, r);
  for (int c = 0; c < N; ++c) r[c] = b[c] - r[c];
  band_substitute(S, r, dx);
  for (int c = 0; c < N; ++c) x[c] += dx[c];
  free(r); free(dx);
  return 0;
}

int ora_synthetic_solve(const ora_problem *p, const double *b, double *x) {
  synth_factor S;
  int e = synth_factor_build(p, 0.0, &S);
  if (e) return e;
  e = synth_solve_with(p, &S, b, x);
  synth_factor_free(&S);
  return e;
}

/* ------------------------------------------------------------------------ */
/* Face-averaged diffusive flux (Eq. Fij_d): the synthetic balance            */
/*   V sig_a x + sum_int A [-(w_c + w_nb) . n / 2 + h_f]                       */
/*             + sum_bnd A [F_T . n + kappa (x_c - phi_half_c)] = V q,         */
/* w = grad(x) / (3 sig_t), is D1 x = b + corr(x) with the compact b; its     */
/* defect correction D1 dx = R1(x) (Eqs. MSE_d1, Gamma_ij_def, MSE_d_mtx1)    */
/* reads x^{s+1} = D1^{-1} (b + corr(x^s)).                                   */
/* ------------------------------------------------------------------------ */
void ora_wide_correction(const ora_problem *p, int alsm, const double *x, double *corr) {
  const int nx = p->nx, ny = p->ny, N = nx * ny;
  double *gx = malloc(sizeof(double) * N * 2), *gy = gx + N;
  ora_gradient(p, alsm, x, gx, gy);
  for (int c = 0; c < N; ++c) {
    gx[c] /= 3.0 * sig_t(p, c);
    gy[c] /= 3.0 * sig_t(p, c);
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      double s = 0.0;
      for (int f = 0; f < 4; ++f) {
        int nb = neighbour(p, i, j, f);
        if (nb < 0) continue;
        double wn = 0.5 * ((gx[c] + gx[nb]) * NX_[f] + (gy[c] + gy[nb]) * NY_[f]);
        s += face_area(p, f) * (gamma_face(p, c, nb, f) * (x[c] - x[nb]) + wn);
      }
      corr[c] = s;
    }
  free(gx);
}

static int synth_wide_with(const ora_problem *p, const synth_factor *S, int alsm,
                           const double *b, int n_sub, double *x) {
  const int N = p->nx * p->ny;
  double *bs = malloc(sizeof(double) * N * 2), *corr = bs + N;
  int e = 0;
  for (int s = 0; s < n_sub && e == 0; ++s) {
    ora_wide_correction(p, alsm, x, corr);
    for (int c = 0; c < N; ++c) bs[c] = b[c] + corr[c];
    e = synth_solve_with(p, S, bs, x);
  }
  free(bs);
  return e;
}

int ora_synthetic_wide(const ora_problem *p, int alsm, const double *b, int n_sub, double *x) {
  synth_factor S;
  int e = synth_factor_build(p, 0.0, &S);
  if (e) return e;
  e = synth_wide_with(p, &S, alsm, b, n_sub, x);
  synth_factor_free(&S);
  return e;
}

/* ------------------------------------------------------------------------ */
/* Transport face fluxes F_T,f . n_f = sum_k w_k (Omega_k . n_f) I_f,k from   */
/* an intensity field (boundary faces: the initial synthetic boundary flux,   */
/* Sec. 4.4; interior faces: only for the transport-face variant).            */
/* bflux[2(nx+ny)] uses the outward normal; fx[(nx-1)*ny] uses +x, fy uses +y. */
/* ------------------------------------------------------------------------ */
static void transport_face_fluxes(const ora_problem *p, const ora_options *o,
                                  const double *I, double *bflux, double *fx,
                                  double *fy) {
  const int nx = p->nx, ny = p->ny, N = nx * ny, K = p->K;
  const int nb_f = 2 * (nx + ny);
  const int nfx = (nx - 1) * ny, nfy = nx * (ny - 1);
  double *cb = calloc((size_t)nb_f * K, sizeof(double));
  double *cx = fx ? calloc((size_t)(nfx > 0 ? nfx : 1) * K, sizeof(double)) : NULL;
  double *cy = fy ? calloc((size_t)(nfy > 0 ? nfy : 1) * K, sizeof(double)) : NULL;
#pragma omp parallel
  {
    double *U = (double *)malloc(sizeof(double) * N * 4);
    double *Gx = U + N, *Gy = U + 2 * N, *psi = U + 3 * N;
#pragma omp for schedule(dynamic, 1)
    for (int k = 0; k < K; ++k) {
      for (int c = 0; c < N; ++c) U[c] = I[(size_t)c * K + k];
      recon R;
      build_recon(p, o, U, Gx, Gy, psi, &R);
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
          for (int f = 0; f < 4; ++f) {
            double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
            if (neighbour(p, i, j, f) < 0) {
              cb[(size_t)bface(p, i, j, f) * K + k] =
                  p->w[k] * on * face_value(p, &R, i, j, f, k);
            } else if (f == 0 && cx) {
              cx[(size_t)(j * (nx - 1) + i) * K + k] = p->w[k] * on * face_value(p, &R, i, j, f, k);
            } else if (f == 2 && cy) {
              cy[(size_t)(j * nx + i) * K + k] = p->w[k] * on * face_value(p, &R, i, j, f, k);
            }
          }
    }
    free(U);
  }
  for (int b = 0; b < nb_f; ++b) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += cb[(size_t)b * K + k];
    bflux[b] = s;
  }
  if (cx) for (int f = 0; f < nfx; ++f) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += cx[(size_t)f * K + k];
    fx[f] = s;
  }
  if (cy) for (int f = 0; f < nfy; ++f) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += cy[(size_t)f * K + k];
    fy[f] = s;
  }
  free(cb); free(cx); free(cy);
}

/* ------------------------------------------------------------------------ */
/* One outer iteration.                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  const ora_problem *p;
  const ora_options *o;
  synth_factor S;
  int have_S;
  double tdiag;     /* 1/(c dt) of a time step (0: steady) */
} ora_ctx;

/* Relative transport residual of the iterate I (whose residual is r):
 *   ||r||_V / ||(sigma_s phi + q) / (4 pi)||_V,  phi = sum_k w_k I_k,
 * with ||x||_V^2 = sum_c V_c sum_k w_k x_{c,k}^2 (cells weighted by volume,
 * ordinates by their quadrature weights; the denominator is the isotropic
 * source of the same iterate). It is zero exactly when I solves the
 * discrete transport equation, whatever the outer method, so it shows a
 * method that stops on Err (Eq. Err_W) before the transport has converged. */
static double transport_residual_norm(const ora_problem *p, const double *I, const double *r) {
  const int N = p->nx * p->ny, K = p->K;
  const double V = p->dx * p->dy;
  double num = 0.0, den = 0.0;
  for (int c = 0; c < N; ++c) {
    double phi = 0.0;
    for (int k = 0; k < K; ++k) phi += p->w[k] * I[(size_t)c * K + k];
    const double s = (p->sig_s[c] * phi + p->q[c]) / FOUR_PI;
    for (int k = 0; k < K; ++k) {
      const double rk = r[(size_t)c * K + k];
      num += V * p->w[k] * rk * rk;
      den += V * p->w[k] * s * s;
    }
  }
  if (den == 0) return num == 0 ? 0.0 : INFINITY;
  return sqrt(num / den);
}

static int iterate_ctx(ora_ctx *X, const double *I_in, double *I_out,
                       double *phi_out, double *tres) {
  const ora_problem *p = X->p;
  const ora_options *o = X->o;
  const int nx = p->nx, ny = p->ny, N = nx * ny, K = p->K;
  const size_t NK = (size_t)N * K;
  double *r = malloc(sizeof(double) * NK);
  double *dI = malloc(sizeof(double) * NK);
  if (!r || !dI) { free(r); free(dI); return -3; }

  /* residual and exact increment solve */
  ora_residual(p, o, I_in, r);
  if (tres) *tres = transport_residual_norm(p, I_in, r);
  ora_sweep(p, o, r, dI);
  free(r);
  /* I^{m+1/2} = I^m + dI */
#pragma omp parallel for schedule(static)
  for (size_t t = 0; t < NK; ++t) I_out[t] = I_in[t] + dI[t];
  free(dI);

  double *ph = malloc(sizeof(double) * N * 3);
  double *Fxh = ph + N, *Fyh = ph + 2 * N;
  moments(p, I_out, ph, Fxh, Fyh);

  if (o->method == 0) {
    /* SI (Eq. SI_update) */
    memcpy(phi_out, ph, sizeof(double) * N);
    free(ph);
    return 0;
  }

  /* GSIS: boundary (and, for the transport-face variant, interior) fluxes */
  const int nb_f = 2 * (nx + ny);
  double *bflux = malloc(sizeof(double) * nb_f);
  double *fx = NULL, *fy = NULL;
  if (o->hot_face == 1) {
    fx = malloc(sizeof(double) * ((nx - 1) * ny + 1));
    fy = malloc(sizeof(double) * (nx * (ny - 1) + 1));
  }
  transport_face_fluxes(p, o, I_out, bflux, fx, fy);

  /* HoT_c = F_c + grad(phi)_c / (3 sigma_t) (Eq. GSIS_HoT), ALSM gradient */
  double *gpx = malloc(sizeof(double) * N * 2), *gpy = gpx + N;
  ora_gradient(p, o->alsm, ph, gpx, gpy);
  double *hx = malloc(sizeof(double) * N * 2), *hy = hx + N;
  for (int c = 0; c < N; ++c) {
    hx[c] = Fxh[c] + gpx[c] / (3.0 * sig_t(p, c));
    hy[c] = Fyh[c] + gpy[c] / (3.0 * sig_t(p, c));
  }
  /* right-hand side: V q - sum_int A h_f - sum_bnd A (F_T.n - kappa phi_half) */
  const double V = p->dx * p->dy;
  double *b = malloc(sizeof(double) * N);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      double s = V * p->q[c];
      for (int f = 0; f < 4; ++f) {
        int nb = neighbour(p, i, j, f);
        double A = face_area(p, f);
        if (nb >= 0) {
          double h;
          if (o->hot_face == 0) {
            /* central average of cell HoT (Eq. Fij_d, second term) */
            h = 0.5 * ((hx[c] + hx[nb]) * NX_[f] + (hy[c] + hy[nb]) * NY_[f]);
          } else {
            /* transport face flux minus the implicit diffusion part */
            double ft;
            if (f == 0) ft = fx[j * (nx - 1) + i];
            else if (f == 1) ft = -fx[j * (nx - 1) + i - 1];
            else if (f == 2) ft = fy[j * nx + i];
            else ft = -fy[(j - 1) * nx + i];
            h = ft - gamma_face(p, c, nb, f) * (ph[c] - ph[nb]);
          }
          s -= A * h;
        } else {
          s -= A * (bflux[bface(p, i, j, f)] - kappa_face(p, c, f) * ph[c]);
        }
      }
      b[c] = s;
    }

  /* synthetic solve D1 phi' = b */
  int e = 0;
  if (!X->have_S) {
    e = synth_factor_build(p, X->tdiag, &X->S);
    if (e == 0) X->have_S = 1;
  }
  if (e == 0) {
    if (o->synth_form == 1) {
      /* sub-iterations from phi^{m+1/2} */
      memcpy(phi_out, ph, sizeof(double) * N);
      e = synth_wide_with(p, &X->S, o->alsm, b, o->synth_sub, phi_out);
    } else {
      e = synth_solve_with(p, &X->S, b, phi_out);
    }
  }

  /* GSIS correction I^{m+1} = I^{m+1/2} + (phi' - phi_half)/(4 pi)
   * (Eq. GSIS_update) */
  if (e == 0) {
#pragma omp parallel for schedule(static)
    for (int c = 0; c < N; ++c) {
      double dl = (phi_out[c] - ph[c]) / FOUR_PI;
      for (int k = 0; k < K; ++k) I_out[(size_t)c * K + k] += dl;
    }
  }
  free(b); free(hx); free(gpx); free(bflux); free(fx); free(fy); free(ph);
  return e;
}

int ora_iterate(const ora_problem *p, const ora_options *o, const double *I_in,
                double *I_out, double *phi_out) {
  ora_ctx X = {p, o, {0, 0, NULL, 0, 0.0}, 0, 0.0};
  int e = iterate_ctx(&X, I_in, I_out, phi_out, NULL);
  if (X.have_S) synth_factor_free(&X.S);
  return e;
}

/* Err(W) = sqrt( sum V (W^m - W^{m-1})^2 / sum V (W^m)^2 ) (Eq. Err_W);
 * *dnorm receives the numerator's root ||W^m - W^{m-1}||_V, *wnorm the
 * denominator's ||W^m||_V. */
static double err_w(const double *Wn, const double *Wo, int N, double V, double *dnorm,
                    double *wnorm) {
  double num = 0, den = 0;
  for (int c = 0; c < N; ++c) {
    double d = Wn[c] - Wo[c];
    num += V * d * d;
    den += V * Wn[c] * Wn[c];
  }
  *dnorm = sqrt(num);
  *wnorm = sqrt(den);
  if (den == 0) return num == 0 ? 0.0 : INFINITY;
  return sqrt(num / den);
}

int ora_solve(const ora_problem *p, const ora_options *o, const double *I0,
              double *phi, double *Fx, double *Fy, double *err_hist,
              double *tres_hist, int *n_iter, double *final_err, double *I_final) {
  const int N = p->nx * p->ny, K = p->K;
  const size_t NK = (size_t)N * K;
  const double V = p->dx * p->dy;
  double *Ia = malloc(sizeof(double) * NK), *Ib = malloc(sizeof(double) * NK);
  double *phi_old = malloc(sizeof(double) * N), *phi_new = malloc(sizeof(double) * N);
  if (!Ia || !Ib || !phi_old || !phi_new) return -3;
  if (I0) memcpy(Ia, I0, sizeof(double) * NK);
  else memset(Ia, 0, sizeof(double) * NK);
  if (o->synth_form == 1 && (o->hot_face != 0 || o->synth_sub < 1)) {
    free(Ia); free(Ib); free(phi_old); free(phi_new);
    return -1;
  }

  ora_ctx X = {p, o, {0, 0, NULL, 0, 0.0}, 0, 0.0};
  int status = 1, m = 0;
  double err = INFINITY, dmin = INFINITY;
  for (m = 0; m < o->max_iter; ++m) {
    moments(p, Ia, phi_old, NULL, NULL);          /* phi^m */
    double tres = 0.0;
    int e = iterate_ctx(&X, Ia, Ib, phi_new, &tres);   /* phi^{m+1} */
    if (e) { status = e; break; }
    double dn, pn;
    err = err_w(phi_new, phi_old, N, V, &dn, &pn);
    if (err_hist) err_hist[m] = err;
    if (tres_hist) tres_hist[m] = tres;
    double *t = Ia; Ia = Ib; Ib = t;
    /* divergence (an unstable outer iteration, e.g. GSIS at strong opacity
     * jumps without the pseudo-time shift of Sec. 4.3): Err not finite, or
     * the change ||phi^{m+1} - phi^m||_V above 1e3 times its smallest value
     * so far (floored at 1e-9 ||phi^{m+1}||_V, far above rounding). Err
     * itself cannot show a geometric blow-up: it tends to |1 - 1/g| for a
     * growth factor g. */
    if (!isfinite(err) || dn > 1e3 * fmax(dmin, 1e-9 * pn)) { status = 2; ++m; break; }
    if (dn < dmin) dmin = dn;
    if (err < o->tol) { status = 0; ++m; break; }
  }
  if (n_iter) *n_iter = m;
  if (final_err) *final_err = err;
  /* outputs: phi^{final} and F of the final intensity */
  memcpy(phi, phi_new, sizeof(double) * N);
  {
    double *tmp = malloc(sizeof(double) * N);
    moments(p, Ia, tmp, Fx, Fy);
    free(tmp);
  }
  if (I_final) memcpy(I_final, Ia, sizeof(double) * NK);
  if (X.have_S) synth_factor_free(&X.S);
  free(Ia); free(Ib); free(phi_old); free(phi_new);
  return status;
}

/* ======================================================================== */
/* Time-dependent gray RTE with the material energy equation (Sec. 2.1 Eqs.   */
/* RTE_g, Tm_g), backward Euler in time (Eqs. RTE_d, Tm_d), inner iterations  */
/* per time step (Sec. 4.1, 4.2).                                             */
/*                                                                            */
/* One inner iteration m of step n -> n+1, from (I^m, T^m):                   */
/*  1. residual of Eq. RTE_d_res with phi^m = a c (T^m)^4 and the time terms  */
/*     -(I^m - I^n)/(c dt); increment solve with 1/(c dt) on the diagonal     */
/*     (Eqs. RTE_d_increment, elem_mtx); I^{m+1/2} = I^m + dI;                */
/*  2. SI: rho^{m+1} = rho^{m+1/2}, and the material equation (Eq. Tm_d) with  */
/*     rho fixed at rho^{m+1/2} by sub_iter steps of dT = R2 / D2 (Eqs. MSE_d2,*/
/*     R2_def, MSE_d_mtx2, elem_mtx_M);                                       */
/*  3. GSIS: the synthetic and material equations (Eq. GSIS_dse) by sub_iter   */
/*     sub-iterations s from (rho^{m+1/2}, T^m), each solving D1 d_rho = R1    */
/*     and D2 d_T = R2 with the residuals of iteration s (Eqs. MSE_d1, MSE_d2, */
/*     R1_def, R2_def, MSE_d_mtx1, MSE_d_mtx2, elem_mtx_M); the face flux of   */
/*     R1 is the compact diffusion flux plus the face HoT as in the steady    */
/*     synthetic equation, and on walls F_T . n + kappa (rho - rho^{m+1/2});   */
/*     then I^{m+1} = I^{m+1/2} + (rho^{m+1} - rho^{m+1/2})/(4 pi) (Eq.        */
/*     GSIS_update);                                                          */
/*  4. Err = max(Err(rho), Err(T)) (Eq. Err_W and the criterion after it).    */
/* ======================================================================== */
static int td_iterate(ora_ctx *X, const ora_material *mt, const double *I_n,
                      const double *rho_n, const double *T_n, const double *I_in,
                      const double *T_in, double *I_out, double *T_out, double *rho_out) {
  const ora_problem *p = X->p;
  const ora_options *o = X->o;
  const int nx = p->nx, ny = p->ny, N = nx * ny, K = p->K;
  const size_t NK = (size_t)N * K;
  const double V = p->dx * p->dy, dt = mt->dt, cl = mt->c, ar = mt->a;
  const double tdiag = 1.0 / (cl * dt);
  double *r = malloc(sizeof(double) * NK), *dI = malloc(sizeof(double) * NK);
  double *wk = malloc(sizeof(double) * N * 8);
  if (!r || !dI || !wk) { free(r); free(dI); free(wk); return -3; }
  double *rho_m = wk, *Siso = wk + N, *ph = wk + 2 * N, *Fxh = wk + 3 * N, *Fyh = wk + 4 * N;
  double *rs = wk + 5 * N, *Ts = wk + 6 * N, *R = wk + 7 * N;

  /* 1. transport step */
  moments(p, I_in, rho_m, NULL, NULL);
  for (int c = 0; c < N; ++c) {
    const double T = T_in[c];
    Siso[c] = (p->sig_s[c] * rho_m[c] + p->sig_a[c] * ar * cl * T * T * T * T + p->q[c]) / FOUR_PI;
  }
  residual_t(p, o, I_in, Siso, tdiag, I_n, r);
  sweep_t(p, o, tdiag, r, dI);
  free(r);
#pragma omp parallel for schedule(static)
  for (size_t t = 0; t < NK; ++t) I_out[t] = I_in[t] + dI[t];
  free(dI);
  moments(p, I_out, ph, Fxh, Fyh);

  /* material residual R2 and diagonal D2 of (rho_s, T_s): one step of T */
  #define TD_T_STEP(RHO)                                                          \
    for (int c = 0; c < N; ++c) {                                              \
      const double T = Ts[c], sa = p->sig_a[c], cv = mt->cv[c];                \
      const double R2 = -cv * (T - T_n[c]) / dt + sa * ((RHO)[c] - ar * cl * T * T * T * T); \
      const double D2 = cv / dt + 4.0 * ar * cl * T * T * T * sa;              \
      R[c] = T + R2 / D2;                                                      \
    }                                                                          \
    memcpy(Ts, R, sizeof(double) * N);

  memcpy(Ts, T_in, sizeof(double) * N);
  if (o->method == 0) {
    /* 2. source iteration: rho^{m+1} = rho^{m+1/2}; material equation */
    for (int s = 0; s < mt->sub_iter; ++s) { TD_T_STEP(ph) }
    memcpy(rho_out, ph, sizeof(double) * N);
    memcpy(T_out, Ts, sizeof(double) * N);
    free(wk);
    return 0;
  }

  /* 3. GSIS: wall (and, for the transport-face variant, interior) fluxes, HoT */
  const int nb_f = 2 * (nx + ny);
  double *bflux = malloc(sizeof(double) * nb_f);
  double *fx = NULL, *fy = NULL;
  if (o->hot_face == 1) {
    fx = malloc(sizeof(double) * ((nx - 1) * ny + 1));
    fy = malloc(sizeof(double) * (nx * (ny - 1) + 1));
  }
  transport_face_fluxes(p, o, I_out, bflux, fx, fy);
  double *gpx = malloc(sizeof(double) * N * 2), *gpy = gpx + N;
  ora_gradient(p, o->alsm, ph, gpx, gpy);
  double *hx = malloc(sizeof(double) * N * 2), *hy = hx + N;
  for (int c = 0; c < N; ++c) {
    hx[c] = Fxh[c] + gpx[c] / (3.0 * sig_t(p, c));
    hy[c] = Fyh[c] + gpy[c] / (3.0 * sig_t(p, c));
  }
  int e = 0;
  if (!X->have_S) {
    e = synth_factor_build(p, tdiag, &X->S);
    if (e == 0) X->have_S = 1;
  }
  double *drho = malloc(sizeof(double) * N), *R1 = malloc(sizeof(double) * N);
  memcpy(rs, ph, sizeof(double) * N);
  for (int s = 0; s < mt->sub_iter && e == 0; ++s) {
    /* R1 (Eq. R1_def) times V, at (rho_s, T_s) */
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = j * nx + i;
        const double T = Ts[c];
        double v = V * (-(rs[c] - rho_n[c]) / (cl * dt) +
                        p->sig_a[c] * (ar * cl * T * T * T * T - rs[c]) + p->q[c]);
        for (int f = 0; f < 4; ++f) {
          const int nb = neighbour(p, i, j, f);
          const double A = face_area(p, f);
          if (nb >= 0) {
            const double g = gamma_face(p, c, nb, f);
            double h;
            if (o->hot_face == 0) {
              h = 0.5 * ((hx[c] + hx[nb]) * NX_[f] + (hy[c] + hy[nb]) * NY_[f]);
            } else {
              double ft;
              if (f == 0) ft = fx[j * (nx - 1) + i];
              else if (f == 1) ft = -fx[j * (nx - 1) + i - 1];
              else if (f == 2) ft = fy[j * nx + i];
              else ft = -fy[(j - 1) * nx + i];
              h = ft - g * (ph[c] - ph[nb]);
            }
            v -= A * (g * (rs[c] - rs[nb]) + h);
          } else {
            v -= A * (bflux[bface(p, i, j, f)] + kappa_face(p, c, f) * (rs[c] - ph[c]));
          }
        }
        R1[c] = v;
      }
    e = synth_solve_with(p, &X->S, R1, drho);
    if (e) break;
    TD_T_STEP(rs)                       /* T_{s+1} from (rho_s, T_s) */
    for (int c = 0; c < N; ++c) rs[c] += drho[c];
  }
  #undef TD_T_STEP
  if (e == 0) {
    memcpy(rho_out, rs, sizeof(double) * N);
    memcpy(T_out, Ts, sizeof(double) * N);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < N; ++c) {
      const double dl = (rs[c] - ph[c]) / FOUR_PI;
      for (int k = 0; k < K; ++k) I_out[(size_t)c * K + k] += dl;
    }
  }
  free(drho); free(R1); free(hx); free(gpx); free(bflux); free(fx); free(fy); free(wk);
  return e;
}

int ora_td_solve(const ora_problem *p, const ora_options *o, const ora_material *mt,
                 const double *I0, const double *T0, int n_steps, double *I_out,
                 double *T_out, double *rho, double *Fx, double *Fy, int *inner_iters,
                 double *err_last) {
  const int N = p->nx * p->ny, K = p->K;
  const size_t NK = (size_t)N * K;
  const double V = p->dx * p->dy;
  if (!(mt->c > 0) || !(mt->dt > 0) || !(mt->a >= 0) || mt->sub_iter < 1 || o->synth_form != 0)
    return -1;
  for (int c = 0; c < N; ++c)
    if (!(mt->cv[c] > 0) || !(T0[c] >= 0)) return -1;
  double *In = malloc(sizeof(double) * NK), *Ia = malloc(sizeof(double) * NK),
         *Ib = malloc(sizeof(double) * NK);
  double *Tn = malloc(sizeof(double) * N), *Ta = malloc(sizeof(double) * N),
         *Tb = malloc(sizeof(double) * N), *rn = malloc(sizeof(double) * N),
         *ra = malloc(sizeof(double) * N), *rb = malloc(sizeof(double) * N);
  if (!In || !Ia || !Ib || !Tn || !Ta || !Tb || !rn || !ra || !rb) return -3;
  if (I0) memcpy(Ia, I0, sizeof(double) * NK);
  else memset(Ia, 0, sizeof(double) * NK);
  memcpy(Ta, T0, sizeof(double) * N);
  ora_ctx X = {p, o, {0, 0, NULL, 0, 0.0}, 0, 1.0 / (mt->c * mt->dt)};
  int status = 0;
  for (int n = 0; n < n_steps && status >= 0 && status != 2; ++n) {
    /* time level n: the converged state of the previous step */
    memcpy(In, Ia, sizeof(double) * NK);
    memcpy(Tn, Ta, sizeof(double) * N);
    moments(p, In, rn, NULL, NULL);
    memcpy(ra, rn, sizeof(double) * N);
    int m = 0;
    double err = INFINITY, dmin = INFINITY;
    for (m = 0; m < o->max_iter; ++m) {
      int e = td_iterate(&X, mt, In, rn, Tn, Ia, Ta, Ib, Tb, rb);
      if (e) { status = e; break; }
      double dn, pn, dnT, pnT;
      const double er = err_w(rb, ra, N, V, &dn, &pn);
      const double et = err_w(Tb, Ta, N, V, &dnT, &pnT);
      err = er > et ? er : et;
      double *t = Ia; Ia = Ib; Ib = t;
      t = Ta; Ta = Tb; Tb = t;
      t = ra; ra = rb; rb = t;
      if (!isfinite(err) || dn > 1e3 * fmax(dmin, 1e-9 * pn)) { status = 2; ++m; break; }
      if (dn < dmin) dmin = dn;
      if (err < o->tol) { ++m; break; }
    }
    if (status == 0 && !(err < o->tol)) status = 1;
    if (inner_iters) inner_iters[n] = m;
    if (err_last) err_last[n] = err;
  }
  if (I_out) memcpy(I_out, Ia, sizeof(double) * NK);
  memcpy(T_out, Ta, sizeof(double) * N);
  moments(p, Ia, rho, Fx, Fy);
  if (X.have_S) synth_factor_free(&X.S);
  free(In); free(Ia); free(Ib); free(Tn); free(Ta); free(Tb); free(rn); free(ra); free(rb);
  return status;
}

/* ======================================================================== */
/* Adjoint of the GSIS / SI fixed point (limiter off, no pseudo time).        */
/*                                                                            */
/* With the limiter off one outer iteration is an affine map                  */
/* I' = T(I; p) = G(p) I + c(p) of the intensity, p = (sigma_a, sigma_s, q)    */
/* per cell. For an output J = <g_phi, phi*> + <g_F, F*> of the fixed point   */
/* I* (phi* = sum_k w_k I*_k, F* = sum_k w_k Omega_k I*_k) the adjoint         */
/* lambda solves lambda = G^T lambda + M^T g, and                             */
/* dJ/dp = lambda^T dT(I*; p)/dp. Both are reverse passes through the steps   */
/* of one iteration (residual, increment solve, moments, boundary fluxes,     */
/* HoT, right-hand side, synthetic solve, correction), taken here one step at */
/* a time in reverse order, per cell, face and ordinate. The gradient of the  */
/* adaptive least squares on a Cartesian grid splits into x and y parts (the  */
/* neighbours lie on the axes, so the 2x2 normal matrix is diagonal):         */
/*   G_x = sum_f e_f (U_f - U_c) / sum_f e_f^2 over the x neighbours, with     */
/*   e_f = +-(h/2)(1 + sigma_nb/sigma_c) (alsm) or +-h, the signed distance   */
/*   to the shifted point (Eqs. shifted_j, LSF_mdf).                           */
/* ======================================================================== */

/* Signed shifted distance of neighbour nb across face f of cell c, and its
 * derivatives with respect to sigma_t of c and of nb. */
static double shifted_e(const ora_problem *p, int alsm, int c, int nb, int f,
                        double *de_dc, double *de_dnb) {
  const double h = (f < 2) ? p->dx : p->dy;
  const double sgn = (f == 0 || f == 2) ? 1.0 : -1.0;
  if (!alsm) { *de_dc = 0.0; *de_dnb = 0.0; return sgn * h; }
  const double sc = sig_t(p, c), sn = sig_t(p, nb);
  *de_dnb = sgn * 0.5 * h / sc;
  *de_dc = -sgn * 0.5 * h * sn / (sc * sc);
  return sgn * 0.5 * h * (1.0 + sn / sc);
}

/* Reverse of the gradient of cell (i,j): given the cotangents gbx, gby of
 * (G_x, G_y), add dL/dU into Ub and dL/dsigma_t into stb. */
static void gradient_cell_adj(const ora_problem *p, int alsm, const double *U, int i, int j,
                              double gbx, double gby, double *Ub, double *stb) {
  const int c = j * p->nx + i;
  for (int axis = 0; axis < 2; ++axis) {
    const double gb = axis == 0 ? gbx : gby;
    if (gb == 0.0) continue;
    const int f0 = axis == 0 ? 0 : 2;
    double e[2] = {0, 0}, dec[2] = {0, 0}, den[2] = {0, 0}, du[2] = {0, 0};
    int nbs[2] = {-1, -1};
    double B = 0.0, M = 0.0;
    for (int t = 0; t < 2; ++t) {
      const int f = f0 + t;
      const int nb = neighbour(p, i, j, f);
      nbs[t] = nb;
      if (nb < 0) continue;
      e[t] = shifted_e(p, alsm, c, nb, f, &dec[t], &den[t]);
      du[t] = U ? U[nb] - U[c] : 0.0;   /* only needed for stb */
      B += e[t] * du[t];
      M += e[t] * e[t];
    }
    if (!(M > 0)) continue;
    const double G = B / M;
    for (int t = 0; t < 2; ++t) {
      if (nbs[t] < 0) continue;
      /* dG/dU_nb = e/M, dG/dU_c = -e/M */
      Ub[nbs[t]] += gb * e[t] / M;
      Ub[c] -= gb * e[t] / M;
      if (stb) {
        /* dG/de = (du - 2 e G) / M */
        const double ge = gb * (du[t] - 2.0 * e[t] * G) / M;
        stb[c] += ge * dec[t];
        stb[nbs[t]] += ge * den[t];
      }
    }
  }
}

/* Reverse of rec_face (limiter off): cotangent vb of the value of cell c on
 * face f. Needs the field U for the coefficient part. */
static void rec_face_adj(const ora_problem *p, const ora_options *o, const double *U, int c,
                         int f, double vb, double *Ub, double *stb) {
  Ub[c] += vb;
  if (o->order < 2) return;
  gradient_cell_adj(p, o->alsm, U, c % p->nx, c / p->nx, vb * face_ox(p, f), vb * face_oy(p, f),
                    Ub, stb);
}

/* Everything one iteration computes from I*, kept for the reverse pass. */
typedef struct {
  double *Ih;        /* I^{m+1/2} [N][K] */
  double *dI;        /* increment [N][K] */
  double *phim;      /* phi of I* */
  double *ph, *Fxh, *Fyh;   /* moments of I^{m+1/2} */
  double *bflux;     /* boundary transport fluxes */
  double *gpx, *gpy; /* ALSM gradient of phi_half */
  double *phin;      /* synthetic solution phi' */
} fwd_tape;

static void tape_free(fwd_tape *t) {
  free(t->Ih); free(t->dI); free(t->phim); free(t->ph); free(t->bflux); free(t->gpx);
  free(t->phin);
}

/* Right-hand side of the synthetic equation (central HoT faces). */
static void synth_rhs(const ora_problem *p, const double *ph, const double *hx,
                      const double *hy, const double *bflux, double *b) {
  const int nx = p->nx, ny = p->ny;
  const double V = p->dx * p->dy;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      double s = V * p->q[c];
      for (int f = 0; f < 4; ++f) {
        int nb = neighbour(p, i, j, f);
        double A = face_area(p, f);
        if (nb >= 0)
          s -= A * 0.5 * ((hx[c] + hx[nb]) * NX_[f] + (hy[c] + hy[nb]) * NY_[f]);
        else
          s -= A * (bflux[bface(p, i, j, f)] - kappa_face(p, c, f) * ph[c]);
      }
      b[c] = s;
    }
}

static int tape_build(const ora_problem *p, const ora_options *o, const synth_factor *S,
                      const double *I, fwd_tape *t) {
  const int nx = p->nx, ny = p->ny, N = nx * ny, K = p->K;
  const size_t NK = (size_t)N * K;
  memset(t, 0, sizeof *t);
  double *r = malloc(sizeof(double) * NK);
  t->Ih = malloc(sizeof(double) * NK);
  t->dI = malloc(sizeof(double) * NK);
  t->phim = malloc(sizeof(double) * N);
  t->ph = malloc(sizeof(double) * N * 3);
  t->Fxh = t->ph + N; t->Fyh = t->ph + 2 * N;
  t->bflux = malloc(sizeof(double) * 2 * (nx + ny));
  t->gpx = malloc(sizeof(double) * N * 2); t->gpy = t->gpx + N;
  t->phin = malloc(sizeof(double) * N);
  ora_residual(p, o, I, r);
  ora_sweep(p, o, r, t->dI);
  free(r);
  for (size_t q = 0; q < NK; ++q) t->Ih[q] = I[q] + t->dI[q];
  moments(p, I, t->phim, NULL, NULL);
  moments(p, t->Ih, t->ph, t->Fxh, t->Fyh);
  if (o->method == 0) return 0;
  transport_face_fluxes(p, o, t->Ih, t->bflux, NULL, NULL);
  ora_gradient(p, o->alsm, t->ph, t->gpx, t->gpy);
  double *hx = malloc(sizeof(double) * N * 2), *hy = hx + N, *b = malloc(sizeof(double) * N);
  for (int c = 0; c < N; ++c) {
    hx[c] = t->Fxh[c] + t->gpx[c] / (3.0 * sig_t(p, c));
    hy[c] = t->Fyh[c] + t->gpy[c] / (3.0 * sig_t(p, c));
  }
  synth_rhs(p, t->ph, hx, hy, t->bflux, b);
  int e = synth_solve_with(p, S, b, t->phin);
  free(hx); free(b);
  return e;
}

/* Parameter cotangents accumulated by the gradient pass. */
typedef struct { double *st, *ss, *sa, *q; } par_bar;

/* out = G^T lam (one reverse pass). With tape and pb non-NULL the same pass
 * also accumulates lam^T dT/dp into pb; s_out (optional) receives the
 * unweighted ordinate sum s = sum_k lam_k / (4 pi). */
static int adjoint_pass(const ora_problem *p, const ora_options *o, const synth_factor *S,
                        const double *I, const double *lam, double *out, const fwd_tape *tp,
                        par_bar *pb, double *s_out) {
  const int nx = p->nx, ny = p->ny, N = nx * ny, K = p->K;
  const size_t NK = (size_t)N * K;
  const double V = p->dx * p->dy;
  const int nbf = 2 * (nx + ny);
  double *Ihb = malloc(sizeof(double) * NK);      /* cotangent of I^{m+1/2} */
  double *s = calloc(N, sizeof(double));
  double *phb = calloc(N, sizeof(double));        /* of phi_half */
  double *Fxb = calloc(N, sizeof(double)), *Fyb = calloc(N, sizeof(double));
  double *bfb = calloc(nbf, sizeof(double));      /* of the boundary fluxes */
  double *bb = calloc(N, sizeof(double));         /* of b (= D1^-1 s) */
  memcpy(Ihb, lam, sizeof(double) * NK);
  for (int c = 0; c < N; ++c) {
    double t = 0;
    for (int k = 0; k < K; ++k) t += lam[(size_t)c * K + k];
    s[c] = t / FOUR_PI;
  }
  if (s_out) memcpy(s_out, s, sizeof(double) * N);
  int e = 0;
  if (o->method == 1) {
    /* correction I' = I_half + (phi' - phi_half)/(4 pi):
     * cotangent of phi' is s, of phi_half -s */
    for (int c = 0; c < N; ++c) phb[c] = -s[c];
    /* synthetic solve phi' = D1^-1 b: bb = D1^-1 s (D1 symmetric) */
    e = synth_solve_with(p, S, s, bb);
    if (pb && tp) {
      /* D1 = V sigma_a + sum_int A Gamma (e_c - e_nb)(e_c - e_nb)^T
       *      + sum_bnd A kappa e_c e_c^T; its cotangent is -bb phi'^T */
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const int c = j * nx + i;
          pb->sa[c] -= V * bb[c] * tp->phin[c];
          pb->q[c] += V * bb[c];                              /* b = V q + ... */
          for (int f = 0; f < 4; ++f) {
            const int nb = neighbour(p, i, j, f);
            const double A = face_area(p, f);
            const double h = (f < 2) ? p->dx : p->dy;
            if (nb >= 0) {
              if (nb < c) continue;                           /* each face once */
              const double gbar = -A * (bb[c] - bb[nb]) * (tp->phin[c] - tp->phin[nb]);
              /* Gamma = 2 / (3 (sigma_c + sigma_nb) h) on the uniform grid */
              const double sm = sig_t(p, c) + sig_t(p, nb);
              const double dG = -2.0 / (3.0 * sm * sm * h);
              pb->st[c] += gbar * dG;
              pb->st[nb] += gbar * dG;
            } else {
              /* kappa = (o.n)/(3 sigma |o|^2) + 1/4: in b (+A kappa phi_half)
               * and in D1 (+A kappa on the diagonal) */
              const double kb = A * bb[c] * (tp->ph[c] - tp->phin[c]);
              const double ox = face_ox(p, f), oy = face_oy(p, f);
              const double on = ox * NX_[f] + oy * NY_[f];
              const double st = sig_t(p, c);
              pb->st[c] += kb * (-on / (3.0 * st * st * (ox * ox + oy * oy)));
            }
          }
        }
    }
    /* b = V q - sum_int A 1/2 (HoT_c + HoT_nb).n - sum_bnd A (bflux - kappa phi_half) */
    double *hxb = calloc(N, sizeof(double)), *hyb = calloc(N, sizeof(double));
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = j * nx + i;
        for (int f = 0; f < 4; ++f) {
          const int nb = neighbour(p, i, j, f);
          const double A = face_area(p, f);
          if (nb >= 0) {
            hxb[c] -= bb[c] * A * 0.5 * NX_[f];
            hxb[nb] -= bb[c] * A * 0.5 * NX_[f];
            hyb[c] -= bb[c] * A * 0.5 * NY_[f];
            hyb[nb] -= bb[c] * A * 0.5 * NY_[f];
          } else {
            bfb[bface(p, i, j, f)] -= bb[c] * A;
            phb[c] += bb[c] * A * kappa_face(p, c, f);
          }
        }
      }
    /* HoT = F_half + grad(phi_half) / (3 sigma_t) */
    for (int c = 0; c < N; ++c) { Fxb[c] = hxb[c]; Fyb[c] = hyb[c]; }
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = j * nx + i;
        const double st = sig_t(p, c);
        gradient_cell_adj(p, o->alsm, tp ? tp->ph : NULL, i, j, hxb[c] / (3.0 * st),
                          hyb[c] / (3.0 * st), phb, pb ? pb->st : NULL);
        if (pb && tp)
          pb->st[c] += -(hxb[c] * tp->gpx[c] + hyb[c] * tp->gpy[c]) / (3.0 * st * st);
      }
    free(hxb); free(hyb);
  }
  /* moments of I_half */
  for (int c = 0; c < N; ++c)
    for (int k = 0; k < K; ++k)
      Ihb[(size_t)c * K + k] += p->w[k] * (phb[c] + p->mu[k] * Fxb[c] + p->eta[k] * Fyb[c]);
  /* boundary fluxes bflux_f = sum_k w_k (Omega_k.n_f) I_f,k(I_half):
   * outgoing faces carry the reconstructed value of the boundary cell */
  if (o->method == 1) {
    double *U = malloc(sizeof(double) * N), *Ub = malloc(sizeof(double) * N);
    for (int k = 0; k < K; ++k) {
      for (int c = 0; c < N; ++c) { U[c] = tp ? tp->Ih[(size_t)c * K + k] : 0.0; Ub[c] = 0.0; }
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
          for (int f = 0; f < 4; ++f) {
            if (neighbour(p, i, j, f) >= 0) continue;
            const double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
            if (on < 0) continue;   /* incoming: prescribed */
            const double vb = bfb[bface(p, i, j, f)] * p->w[k] * on;
            rec_face_adj(p, o, U, j * nx + i, f, vb, Ub, pb ? pb->st : NULL);
          }
      for (int c = 0; c < N; ++c) Ihb[(size_t)c * K + k] += Ub[c];
    }
    free(U); free(Ub);
  }
  /* I_half = I + dI: both get Ihb. dI = H^-1 r: rb = H^-T Ihb, visiting
   * cells downstream first (the reverse of the increment solve's order). */
  double *rb = malloc(sizeof(double) * NK);
  for (int k = 0; k < K; ++k) {
    const int i0 = p->mu[k] >= 0 ? nx - 1 : 0, di = p->mu[k] >= 0 ? -1 : 1;
    const int j0 = p->eta[k] >= 0 ? ny - 1 : 0, dj = p->eta[k] >= 0 ? -1 : 1;
    for (int jj = 0, j = j0; jj < ny; ++jj, j += dj)
      for (int ii = 0, i = i0; ii < nx; ++ii, i += di) {
        const int c = j * nx + i;
        double d = sig_t(p, c) + ora_pseudo_shift(p, o, c), rhs = Ihb[(size_t)c * K + k];
        for (int f = 0; f < 4; ++f) {
          double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
          if (on > 0) {
            d += on * area_over_vol(p, f);
            int nb = neighbour(p, i, j, f);
            if (nb >= 0) rhs += on * area_over_vol(p, f) * rb[(size_t)nb * K + k];
          }
        }
        rb[(size_t)c * K + k] = rhs / d;
      }
  }
  /* diagonal of H (sigma_t): cotangent -rb dI */
  if (pb && tp)
    for (int c = 0; c < N; ++c)
      for (int k = 0; k < K; ++k)
        pb->st[c] -= rb[(size_t)c * K + k] * tp->dI[(size_t)c * K + k];
  /* r = (sigma_s phi + q)/(4 pi) - sigma_t I - (1/V) sum_f (Omega.n) A I_f(I) */
  memcpy(out, Ihb, sizeof(double) * NK);
  double *Sb = calloc(N, sizeof(double));
  for (int c = 0; c < N; ++c) {
    double t = 0;
    for (int k = 0; k < K; ++k) t += rb[(size_t)c * K + k];
    Sb[c] = t;
  }
  {
    double *U = malloc(sizeof(double) * N), *Ub = malloc(sizeof(double) * N);
    for (int k = 0; k < K; ++k) {
      for (int c = 0; c < N; ++c) { U[c] = I ? I[(size_t)c * K + k] : 0.0; Ub[c] = 0.0; }
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const int c = j * nx + i;
          const double r = rb[(size_t)c * K + k];
          Ub[c] -= sig_t(p, c) * r;
          if (pb && I) pb->st[c] -= r * U[c];
          for (int f = 0; f < 4; ++f) {
            const double on = p->mu[k] * NX_[f] + p->eta[k] * NY_[f];
            const double vb = -on * area_over_vol(p, f) * r;   /* cotangent of I_f */
            const int nb = neighbour(p, i, j, f);
            if (on >= 0) rec_face_adj(p, o, U, c, f, vb, Ub, pb ? pb->st : NULL);
            else if (nb >= 0) rec_face_adj(p, o, U, nb, OPP_[f], vb, Ub, pb ? pb->st : NULL);
          }
        }
      for (int c = 0; c < N; ++c)
        out[(size_t)c * K + k] += Ub[c] + p->w[k] * p->sig_s[c] * Sb[c] / FOUR_PI;
    }
    free(U); free(Ub);
  }
  if (pb && tp)
    for (int c = 0; c < N; ++c) {
      pb->ss[c] += tp->phim[c] * Sb[c] / FOUR_PI;
      pb->q[c] += Sb[c] / FOUR_PI;
    }
  free(Ihb); free(s); free(phb); free(Fxb); free(Fyb); free(bfb); free(bb); free(rb); free(Sb);
  return e;
}

int ora_adjoint(const ora_problem *p, const ora_options *o, const double *I_star,
                const double *g_phi, const double *g_Fx, const double *g_Fy, double tol,
                int max_iter, double *g_sa, double *g_ss, double *g_q, double *lam_out,
                int *n_iter, double *err_hist) {
  if (o->limiter || o->hot_face != 0 || o->cfl_p != 0 || o->beta != 0 || o->synth_form != 0)
    return -4;
  const int N = p->nx * p->ny, K = p->K;
  const size_t NK = (size_t)N * K;
  const double V = p->dx * p->dy;
  synth_factor S = {0, 0, NULL, 0};
  int e = 0;
  if (o->method == 1 && (e = synth_factor_build(p, 0.0, &S))) return e;
  fwd_tape tp;
  if ((e = tape_build(p, o, &S, I_star, &tp))) { tape_free(&tp); synth_factor_free(&S); return e; }
  /* source M^T g: w_k (g_phi + mu_k g_Fx + eta_k g_Fy) */
  double *src = malloc(sizeof(double) * NK), *la = malloc(sizeof(double) * NK),
         *lb = malloc(sizeof(double) * NK);
  for (int c = 0; c < N; ++c)
    for (int k = 0; k < K; ++k)
      src[(size_t)c * K + k] = p->w[k] * ((g_phi ? g_phi[c] : 0.0) +
                                          p->mu[k] * (g_Fx ? g_Fx[c] : 0.0) +
                                          p->eta[k] * (g_Fy ? g_Fy[c] : 0.0));
  memcpy(la, src, sizeof(double) * NK);
  double *s_old = malloc(sizeof(double) * N), *s_new = malloc(sizeof(double) * N);
  int m = 0, status = 1;
  for (int c = 0; c < N; ++c) {
    double t = 0;
    for (int k = 0; k < K; ++k) t += la[(size_t)c * K + k];
    s_old[c] = t / FOUR_PI;
  }
  /* lambda^{n+1} = G^T lambda^n + M^T g until the ordinate sum settles */
  for (m = 0; m < max_iter; ++m) {
    if ((e = adjoint_pass(p, o, &S, NULL, la, lb, NULL, NULL, NULL))) { status = e; break; }
    for (size_t t = 0; t < NK; ++t) lb[t] += src[t];
    for (int c = 0; c < N; ++c) {
      double t = 0;
      for (int k = 0; k < K; ++k) t += lb[(size_t)c * K + k];
      s_new[c] = t / FOUR_PI;
    }
    double dn_, pn_;
    const double err = err_w(s_new, s_old, N, V, &dn_, &pn_);
    if (err_hist) err_hist[m] = err;
    double *t = la; la = lb; lb = t;
    memcpy(s_old, s_new, sizeof(double) * N);
    if (!isfinite(err)) { status = -2; ++m; break; }
    if (err < tol) { status = 0; ++m; break; }
  }
  if (n_iter) *n_iter = m;
  /* gradient: lambda^T dT(I*)/dp in one more reverse pass with the tape */
  par_bar pb;
  pb.st = calloc(N, sizeof(double)); pb.ss = calloc(N, sizeof(double));
  pb.sa = calloc(N, sizeof(double)); pb.q = calloc(N, sizeof(double));
  if (status >= 0) {
    e = adjoint_pass(p, o, &S, I_star, la, lb, &tp, &pb, NULL);
    if (e) status = e;
  }
  for (int c = 0; c < N; ++c) {
    /* sigma_t = sigma_a + sigma_s */
    if (g_sa) g_sa[c] = pb.sa[c] + pb.st[c];
    if (g_ss) g_ss[c] = pb.ss[c] + pb.st[c];
    if (g_q) g_q[c] = pb.q[c];
  }
  if (lam_out) memcpy(lam_out, la, sizeof(double) * NK);
  free(pb.st); free(pb.ss); free(pb.sa); free(pb.q);
  free(src); free(la); free(lb); free(s_old); free(s_new);
  tape_free(&tp);
  synth_factor_free(&S);
  return status;
}
