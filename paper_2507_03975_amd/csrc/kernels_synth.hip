// kernels_synth.hip -- macroscopic (synthetic) step of GSIS on gfx950.
//
//  hot_rhs : HoT_c = F_c + grad(phi)_c / (3 sigma_t) with the adaptive
//            least-squares gradient (Eqs. GSIS_HoT, LSF_mdf); right-hand side
//            b_c = V q - sum_int A 1/2 (HoT_c + HoT_nb).n
//                  - sum_bnd A (F_T.n - kappa phi_half)        (Eqs. MSE_d, Fij_d,
//                                                  macro_bc_delta_flux)
//  solve   : D1 phi' = b, D1 = V sigma_a + sum_int A Gamma (.) + sum_bnd A kappa
//            (Eqs. Gamma_ij_def, MSE_d_mtx1, elem_mtx_M, Gamma_ij_com2), by
//            CG preconditioned with a geometric multigrid V-cycle
//            (2x2 aggregation, Galerkin coarse operators, red-black
//            Gauss-Seidel smoothing, dense inverse on the coarsest level).
//  update  : delta = phi' - phi_half (Eq. GSIS_update, applied lazily by the
//            transport kernels), Err (Eq. Err_W), next source.
// All reductions are two-stage with a fixed order, so results repeat bit for
// bit.
#include "gsis_internal.h"

#include <algorithm>

namespace gsis {
namespace {

constexpr int kRedBlock = 256;

__device__ inline double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- HoT / RHS
__global__ void k_hot(int nx, int ny, const double *phih, const double *Fx,
                      const double *Fy, const double *sig_t, const double *cE,
                      const double *cW, const double *cN, const double *cS,
                      double *hx, double *hy, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const int i = c % nx, j = c / nx;
  const double u = phih[c];
  const double ue = i + 1 < nx ? phih[c + 1] : u, uw = i > 0 ? phih[c - 1] : u;
  const double un = j + 1 < ny ? phih[c + nx] : u, us = j > 0 ? phih[c - nx] : u;
  const double gx = cE[c] * (ue - u) - cW[c] * (uw - u);
  const double gy = cN[c] * (un - u) - cS[c] * (us - u);
  hx[c] = Fx[c] + gx / (3.0 * sig_t[c]);
  hy[c] = Fy[c] + gy / (3.0 * sig_t[c]);
}

__global__ void k_rhs(int nx, int ny, double dx, double dy, const double *q,
                      const double *hx, const double *hy, const double *phih,
                      const double *bflux, const double *kappa, double *b,
                      const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const int i = c % nx, j = c / nx;
  double s = dx * dy * q[c];
  // east / west (area dy), north / south (area dx)
  if (i + 1 < nx) s -= dy * (0.5 * (hx[c] + hx[c + 1]));
  else s -= dy * (bflux[ny + j] - kappa[ny + j] * phih[c]);
  if (i > 0) s += dy * (0.5 * (hx[c] + hx[c - 1]));
  else s -= dy * (bflux[j] - kappa[j] * phih[c]);
  if (j + 1 < ny) s -= dx * (0.5 * (hy[c] + hy[c + nx]));
  else s -= dx * (bflux[2 * ny + nx + i] - kappa[2 * ny + nx + i] * phih[c]);
  if (j > 0) s += dx * (0.5 * (hy[c] + hy[c - nx]));
  else s -= dx * (bflux[2 * ny + i] - kappa[2 * ny + i] * phih[c]);
  b[c] = s;
}

// ------------------------------------------------------- 5-point operator
__device__ inline double apply5(int nx, int ny, const double *dg, const double *ax,
                                const double *ay, const double *x, int c) {
  const int i = c % nx, j = c / nx;
  double s = dg[c] * x[c];
  if (i + 1 < nx) s -= ax[c] * x[c + 1];
  if (i > 0) s -= ax[c - 1] * x[c - 1];
  if (j + 1 < ny) s -= ay[c] * x[c + nx];
  if (j > 0) s -= ay[c - nx] * x[c - nx];
  return s;
}

// y = A x, optional partial of dot(x, y)
__global__ void k_spmv_dot(int nx, int ny, const double *dg, const double *ax,
                           const double *ay, const double *x, double *y, double *part,
                           const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (c < nx * ny) {
    double yc = apply5(nx, ny, dg, ax, ay, x, c);
    y[c] = yc;
    v = x[c] * yc;
  }
  double t = block_sum(v, sh);
  if (part && threadIdx.x == 0) part[blockIdx.x] = t;
}

// r = b - A x ; partials of r.r and b.b
__global__ void k_residual5(int nx, int ny, const double *dg, const double *ax,
                            const double *ay, const double *x, const double *b, double *r,
                            double *part_rr, double *part_bb, const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double rr = 0.0, bb = 0.0;
  if (c < nx * ny) {
    double rc = b[c] - apply5(nx, ny, dg, ax, ay, x, c);
    r[c] = rc;
    rr = rc * rc;
    bb = b[c] * b[c];
  }
  double t = block_sum(rr, sh);
  if (part_rr && threadIdx.x == 0) part_rr[blockIdx.x] = t;
  if (part_bb) {
    t = block_sum(bb, sh);
    if (threadIdx.x == 0) part_bb[blockIdx.x] = t;
  }
}

// partial of dot(x, y)
__global__ void k_dot(int n, const double *x, const double *y, double *part,
                      const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double v = c < n ? x[c] * y[c] : 0.0;
  double t = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Scalar slots
enum { S_RZ = 0, S_PAP = 1, S_RR = 2, S_BB = 3, S_ALPHA = 4, S_BETA = 5, S_TMP = 6 };

// Sum npart partials into scal[slot]; op: 0 store, 1 alpha = RZ/PAP,
// 2 beta = new/RZ and RZ = new.
__global__ void k_finish(const double *part, int npart, double *scal, int slot, int op,
                         const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  double v = 0.0;
  for (int t = threadIdx.x; t < npart; t += blockDim.x) v += part[t];
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) {
    if (op == 0) scal[slot] = s;
    else if (op == 1) { scal[S_PAP] = s; scal[S_ALPHA] = scal[S_RZ] / s; }
    else { scal[S_BETA] = s / scal[S_RZ]; scal[S_RZ] = s; }
  }
}

// x += alpha p ; r -= alpha Ap ; partial of r.r
__global__ void k_cg_update(int n, double *x, double *r, const double *p, const double *Ap,
                            const double *scal, double *part, const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (c < n) {
    const double al = scal[S_ALPHA];
    x[c] += al * p[c];
    const double rc = r[c] - al * Ap[c];
    r[c] = rc;
    v = rc * rc;
  }
  double t = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// p = z + beta p (beta_mode 0: p = z)
__global__ void k_cg_p(int n, const double *z, double *p, const double *scal, int first,
                       const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  p[c] = first ? z[c] : z[c] + scal[S_BETA] * p[c];
}

// ------------------------------------------------------------ multigrid
// One red (color 0) or black (1) Gauss-Seidel half sweep of A x = b.
__global__ void k_rbgs(int nx, int ny, const double *dg, const double *ax, const double *ay,
                       double *x, const double *b, int color, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const int i = c % nx, j = c / nx;
  if (((i + j) & 1) != color) return;
  double s = b[c];
  if (i + 1 < nx) s += ax[c] * x[c + 1];
  if (i > 0) s += ax[c - 1] * x[c - 1];
  if (j + 1 < ny) s += ay[c] * x[c + nx];
  if (j > 0) s += ay[c - nx] * x[c - nx];
  x[c] = s / dg[c];
}

// r = b - A x on the fine level, then coarse b = sum over the fx x fy
// children of each aggregate.
__global__ void k_restrict(int nx, int ny, const double *dg, const double *ax,
                           const double *ay, const double *x, const double *b, int fx,
                           int fy, int cnx, int cny, double *cb, const int32_t *state) {
  if (state[1] != 0) return;
  const int C = blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= cnx * cny) return;
  const int I = C % cnx, J = C / cnx;
  double s = 0.0;
  for (int dj = 0; dj < fy; ++dj)
    for (int di = 0; di < fx; ++di) {
      const int i = fx * I + di, j = fy * J + dj;
      if (i < nx && j < ny) {
        const int c = j * nx + i;
        s += b[c] - apply5(nx, ny, dg, ax, ay, x, c);
      }
    }
  cb[C] = s;
}

// x_fine += x_coarse of the parent aggregate
__global__ void k_prolong(int nx, int ny, double *x, int fx, int fy, int cnx,
                          const double *cx, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  const int i = c % nx, j = c / nx;
  x[c] += cx[(j / fy) * cnx + (i / fx)];
}

// x = Ainv b (dense, coarsest level); one block per row
__global__ void k_dense_solve(int n, const double *Ainv, const double *b, double *x,
                              const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int row = blockIdx.x;
  double v = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) v += Ainv[(size_t)row * n + t] * b[t];
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) x[row] = s;
}

__global__ void k_zero(int n, double *x, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) x[c] = 0.0;
}

__global__ void k_copy(int n, const double *a, double *b, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) b[c] = a[c];
}

inline int nblk(int n) { return (n + kRedBlock - 1) / kRedBlock; }

// V-cycle on level l: x_l ~= A_l^{-1} b_l (x_l is overwritten).
void vcycle(const PlanDev &P, int l, const double *b, double *x, hipStream_t s) {
  const MGLevel &L = P.mg[l];
  const int n = L.nx * L.ny;
  if (l + 1 == (int)P.mg.size()) {
    hipLaunchKernelGGL(k_dense_solve, dim3(n), dim3(kRedBlock), 0, s, n, P.coarse_inv, b, x,
                       P.state);
    return;
  }
  const MGLevel &C = P.mg[l + 1];
  hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(kRedBlock), 0, s, n, x, P.state);
  for (int color = 0; color < 2; ++color)
    hipLaunchKernelGGL(k_rbgs, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, x, b, color, P.state);
  hipLaunchKernelGGL(k_restrict, dim3(nblk(C.nx * C.ny)), dim3(kRedBlock), 0, s, L.nx, L.ny,
                     L.diag, L.ax, L.ay, x, b, L.fx, L.fy, C.nx, C.ny, C.b, P.state);
  vcycle(P, l + 1, C.b, C.x, s);
  hipLaunchKernelGGL(k_prolong, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, x, L.fx, L.fy,
                     C.nx, C.x, P.state);
  for (int color = 1; color >= 0; --color)
    hipLaunchKernelGGL(k_rbgs, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, x, b, color, P.state);
}

// ------------------------------------------------------------- update / Err
// delta = phi' - phi_half (GSIS) or 0 (SI); Err partials; phi = phi_new.
__global__ void k_update(int n, int method, double V, const double *phinew,
                         const double *phih, double *phi, double *delta, double *part,
                         const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (c < n) {
    const double pn = method ? phinew[c] : phih[c];
    const double d = pn - phi[c];
    num = V * d * d;
    den = V * pn * pn;
    delta[c] = method ? pn - phih[c] : 0.0;
    phi[c] = pn;
  }
  double a = block_sum(num, sh);
  double b = block_sum(den, sh);
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = b; }
}

// Err = sqrt(num/den) -> history, counters, done flag.
__global__ void k_err_finish(const double *part, int npart, double tol, int max_iter,
                             double *hist, double *last_err, int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < npart; t += blockDim.x) { a += part[2 * t]; b += part[2 * t + 1]; }
  double num = block_sum(a, sh);
  double den = block_sum(b, sh);
  if (threadIdx.x == 0) {
    double err = den > 0.0 ? sqrt(num / den) : (num == 0.0 ? 0.0 : INFINITY);
    const int m = state[0];
    hist[m] = err;
    *last_err = err;
    state[0] = m + 1;
    state[2] = 1 - state[2];   // I^{m+1} now lives in the other buffer
    if (!isfinite(err)) state[1] = -1;
    else if (err < tol) state[1] = 1;
    else if (m + 1 >= max_iter) state[1] = 2;
  }
}

// src = (sigma_s phi + q) / (4 pi); the mirrored per-quadrant copies of
// (src, delta/(4 pi)) read by the fused sweep.
__global__ void k_source(int nx, int ny, const double *sig_s, const double *q,
                         const double *phi, const double *delta, double *src, double *dynq,
                         const int32_t *state) {
  if (state[1] != 0) return;
  const int n = nx * ny;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double sc = (sig_s[c] * phi[c] + q[c]) / kFourPi;
  const double dq = delta[c] / kFourPi;
  src[c] = sc;
  const int i = c % nx, j = c / nx;
  for (int qd = 0; qd < 4; ++qd) {
    const int xl = (qd & 1) ? nx - 1 - i : i, yl = (qd & 2) ? ny - 1 - j : j;
    const size_t o = (size_t)qd * 2 * n + dg_idx(xl, yl, nx, ny);
    dynq[o] = sc;          // plane 0 of quadrant qd
    dynq[o + n] = dq;      // plane 1
  }
}

// Final F with the pending correction: F = F_half + delta/(4 pi) sum_k w Omega_k
__global__ void k_final_flux(int n, const double *Fx, const double *Fy, const double *delta,
                             double swmu, double sweta, double *ox, double *oy) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double d = delta[c] / kFourPi;
  ox[c] = Fx[c] + d * swmu;
  oy[c] = Fy[c] + d * sweta;
}

}  // namespace

void launch_source(const PlanDev &P, hipStream_t s) {
  hipLaunchKernelGGL(k_source, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, P.nx, P.ny, P.sig_s, P.q,
                     P.phi, P.delta, P.src, P.dynq, P.state);
}

void launch_hot_rhs(const PlanDev &P, hipStream_t s) {
  hipLaunchKernelGGL(k_hot, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, P.nx, P.ny, P.phih, P.Fx,
                     P.Fy, P.sig_t, P.cE, P.cW, P.cN, P.cS, P.hx, P.hy, P.state);
  hipLaunchKernelGGL(k_rhs, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, P.nx, P.ny, P.dx, P.dy,
                     P.q, P.hx, P.hy, P.phih, P.bflux, P.kappa, P.rhs, P.state);
}

void launch_d1_apply(const PlanDev &P, const double *x, double *y, hipStream_t s) {
  const MGLevel &L = P.mg[0];
  hipLaunchKernelGGL(k_spmv_dot, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag,
                     L.ax, L.ay, x, y, (double *)nullptr, P.state);
}

// Preconditioned CG on D1 phi' = rhs, warm-started from phi (the previous
// synthetic solution). The solution lands in P.mg[0].x. host_scal is pinned
// host memory (>= 4 doubles) used to read the residual norms.
void launch_synth_solve(PlanDev &P, hipStream_t s, double *host_scal) {
  const MGLevel &L = P.mg[0];
  const int n = P.N, nb = nblk(n);
  double *x = L.x;
  hipLaunchKernelGGL(k_copy, dim3(nb), dim3(kRedBlock), 0, s, n, P.phi, x, P.state);
  hipLaunchKernelGGL(k_residual5, dim3(nb), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                     L.ay, x, P.rhs, P.cg_r, P.red, P.red + nb, P.state);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_RR, 0,
                     P.state);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red + nb, nb, P.scal,
                     (int)S_BB, 0, P.state);
  // Stop when ||r|| <= synth_rtol ||r0|| (r0: residual of the warm start) or
  // ||r|| <= 1e-14 ||b|| (rounding floor). Relative to r0, the solve error
  // stays a fixed fraction of this iteration's update, so Err cannot stall
  // at the solver tolerance or read zero because the solve did nothing.
  double rr0 = -1.0;
  for (int it = 0; it <= P.synth_max_iter; ++it) {
    hipMemcpyAsync(host_scal, P.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(host_scal + 4, P.state + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    if (((int32_t *)(host_scal + 4))[0] != 0) return;  // already done
    const double rr = host_scal[S_RR], bb = host_scal[S_BB];
    if (rr0 < 0) rr0 = rr;
    const double stop = std::max(P.synth_rtol * P.synth_rtol * rr0, 1e-28 * bb);
    if (!(rr > stop) || it == P.synth_max_iter) break;
    // z = M^{-1} r
    vcycle(P, 0, P.cg_r, P.cg_z, s);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kRedBlock), 0, s, n, P.cg_r, P.cg_z, P.red,
                       P.state);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_RZ,
                       it == 0 ? 0 : 2, P.state);
    hipLaunchKernelGGL(k_cg_p, dim3(nb), dim3(kRedBlock), 0, s, n, P.cg_z, P.cg_p, P.scal,
                       it == 0 ? 1 : 0, P.state);
    hipLaunchKernelGGL(k_spmv_dot, dim3(nb), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, P.cg_p, P.cg_Ap, P.red, P.state);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_PAP,
                       1, P.state);
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kRedBlock), 0, s, n, x, P.cg_r, P.cg_p,
                       P.cg_Ap, P.scal, P.red, P.state);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_RR,
                       0, P.state);
  }
}

void launch_update(const PlanDev &P, hipStream_t s) {
  const int nb = nblk(P.N);
  const double *phinew = P.mg[0].x;
  hipLaunchKernelGGL(k_update, dim3(nb), dim3(kRedBlock), 0, s, P.N, P.method, P.V, phinew,
                     P.phih, P.phi, P.delta, P.err_parts, P.state);
  hipLaunchKernelGGL(k_err_finish, dim3(1), dim3(kRedBlock), 0, s, P.err_parts, nb, P.tol,
                     P.max_iter, P.err_hist, P.last_err, P.state);
  launch_source(P, s);
}

void launch_apply_delta_final(const PlanDev &P, hipStream_t s, double swmu, double sweta,
                              double *Fx_out, double *Fy_out) {
  hipLaunchKernelGGL(k_final_flux, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, P.N, P.Fx, P.Fy,
                     P.delta, swmu, sweta, Fx_out, Fy_out);
}

}  // namespace gsis
