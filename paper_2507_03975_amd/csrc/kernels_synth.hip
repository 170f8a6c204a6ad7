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

// (i, j) of cell c on a grid nx wide without an integer division: the
// quotient from the hardware reciprocal is off by at most one for c < 2^28
// and is corrected.
__device__ inline void cell_ij(int c, int nx, int &i, int &j) {
  int q = (int)((double)c * __builtin_amdgcn_rcp((double)nx));
  int r = c - q * nx;
  if (r < 0) { --q; r += nx; } else if (r >= nx) { ++q; r -= nx; }
  i = r; j = q;
}

// ---------------------------------------------------------------- HoT / RHS
__global__ void k_hot(int nx, int ny, const double *phih, const double *Fx,
                      const double *Fy, const double *sig_t, const double *cE,
                      const double *cW, const double *cN, const double *cS,
                      double *hx, double *hy, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  int i, j;
  cell_ij(c, nx, i, j);
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
  int i, j;
  cell_ij(c, nx, i, j);
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
  int i, j;
  cell_ij(c, nx, i, j);
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

// Scalar slots
enum { S_RZ = 0, S_PAP = 1, S_RR = 2, S_BB = 3, S_ALPHA = 4, S_BETA = 5, S_STOP = 6 };

// CG kernels run unless the outer iteration is done (state[1]) or this
// synthetic solve has converged (state[3]).
__device__ inline bool cg_off(const int32_t *st) { return st[1] != 0 || st[3] != 0; }

// Sum npart partials, then: op 0 scal[slot] = s; 1 alpha = RZ / (PAP = s);
// 2 beta = s / RZ, RZ = s; 3 RR = s, converged if RR <= STOP;
// 4 RR = s, STOP = max(rtol^2 RR, 1e-28 BB), converged if RR <= STOP.
__global__ void k_finish(const double *part, int npart, double *scal, int slot, int op,
                         double rtol, int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (cg_off(state)) return;
  double v = 0.0;
  for (int t = threadIdx.x; t < npart; t += blockDim.x) v += part[t];
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) {
    if (op == 0) scal[slot] = s;
    else if (op == 1) { scal[S_PAP] = s; scal[S_ALPHA] = scal[S_RZ] / s; }
    else if (op == 2) { scal[S_BETA] = s / scal[S_RZ]; scal[S_RZ] = s; }
    else if (op == 3) { scal[S_RR] = s; if (!(s > scal[S_STOP])) state[3] = 1; }
    else {
      scal[S_RR] = s;
      const double stop = fmax(rtol * rtol * s, 1e-28 * scal[S_BB]);
      scal[S_STOP] = stop;
      if (!(s > stop)) state[3] = 1;
    }
  }
}

// Start of a synthetic solve: warm start x = phi, clear the converged flag.
__global__ void k_cg_begin(int n, const double *phi, double *x, int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) x[c] = phi[c];
  if (c == 0) state[3] = 0;
}

// r = b - A x ; partials of r.r and b.b
__global__ void k_cg_residual(int nx, int ny, const double *dg, const double *ax,
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
  if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
  t = block_sum(bb, sh);
  if (threadIdx.x == 0) part_bb[blockIdx.x] = t;
}

// p_new = z + beta p_old (= z on the first iteration), Ap = A p_new and a
// partial of p_new . Ap. Neighbour values of p_new are formed from z and
// p_old, so one kernel does both.
__global__ void k_cg_pAp(int nx, int ny, const double *dg, const double *ax, const double *ay,
                         const double *z, const double *pold, double *pnew, double *Ap,
                         const double *scal, int first, double *part, const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (cg_off(state)) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const double be = first ? 0.0 : scal[S_BETA];
  auto P = [&](int k) { return first ? z[k] : z[k] + be * pold[k]; };
  double v = 0.0;
  if (c < nx * ny) {
    int i, j;
  cell_ij(c, nx, i, j);
    const double pc = P(c);
    double y = dg[c] * pc;
    if (i + 1 < nx) y -= ax[c] * P(c + 1);
    if (i > 0) y -= ax[c - 1] * P(c - 1);
    if (j + 1 < ny) y -= ay[c] * P(c + nx);
    if (j > 0) y -= ay[c - nx] * P(c - nx);
    pnew[c] = pc;
    Ap[c] = y;
    v = pc * y;
  }
  double t = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += alpha p ; r -= alpha Ap ; partial of r.r
__global__ void k_cg_update(int n, double *x, double *r, const double *p, const double *Ap,
                            const double *scal, double *part, const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (cg_off(state)) return;
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

// ------------------------------------------------------------ multigrid
// Red-black Gauss-Seidel with colour (i + j) & 1 (0 red, 1 black).
//   red:   x_r = (b + sum a x_nb) / d; with zero_init the neighbours are 0
//          (first half sweep from x = 0). With part != nullptr also a partial
//          of sum_c rdot_c x_c over all cells (the preconditioned residual
//          product r.z; black cells are final at this point).
//   black: x_b = (b + sum a (x_nb + omega e_parent(nb))) / d, where e is the
//          coarse-grid correction (nullptr: none). The red cells' own
//          corrected values are never needed: the red half sweep that
//          follows overwrites them.
__global__ void k_mg_red(int nx, int ny, const double *dg, const double *ax, const double *ay,
                         double *x, const double *b, int zero_init, const double *rdot,
                         double *part, const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (cg_off(state)) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (c < nx * ny) {
    int i, j;
  cell_ij(c, nx, i, j);
    double xc;
    if (((i + j) & 1) == 0) {
      double s = b[c];
      if (!zero_init) {
        if (i + 1 < nx) s += ax[c] * x[c + 1];
        if (i > 0) s += ax[c - 1] * x[c - 1];
        if (j + 1 < ny) s += ay[c] * x[c + nx];
        if (j > 0) s += ay[c - nx] * x[c - nx];
      }
      xc = s / dg[c];
      x[c] = xc;
    } else {
      xc = part ? x[c] : 0.0;
    }
    if (part) v = rdot[c] * xc;
  }
  if (part) {
    double t = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

__global__ void k_mg_black(int nx, int ny, const double *dg, const double *ax, const double *ay,
                           double *x, const double *b, const double *e, int fx, int fy, int cnx,
                           double omega, const int32_t *state) {
  if (cg_off(state)) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nx * ny) return;
  int i, j;
  cell_ij(c, nx, i, j);
  if (((i + j) & 1) != 1) return;
  auto X = [&](int ii, int jj) {
    double v = x[jj * nx + ii];
    if (e) v += omega * e[(jj >> (fy >> 1)) * cnx + (ii >> (fx >> 1))];
    return v;
  };
  double s = b[c];
  if (i + 1 < nx) s += ax[c] * X(i + 1, j);
  if (i > 0) s += ax[c - 1] * X(i - 1, j);
  if (j + 1 < ny) s += ay[c] * X(i, j + 1);
  if (j > 0) s += ay[c - nx] * X(i, j - 1);
  x[c] = s / dg[c];
}

// r = b - A x on the fine level, then coarse b = sum over the fx x fy
// children of each aggregate.
__global__ void k_mg_restrict(int nx, int ny, const double *dg, const double *ax,
                              const double *ay, const double *x, const double *b, int fx,
                              int fy, int cnx, int cny, double *cb, const int32_t *state) {
  if (cg_off(state)) return;
  const int C = blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= cnx * cny) return;
  int I, J;
  cell_ij(C, cnx, I, J);
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

// The coarse end of the V-cycle (every level with at most kCoarseWG cells,
// down to the dense solve) in one workgroup of 1024 threads, so the half
// sweeps are separated by workgroup barriers instead of kernel launches.
// The top coarse level keeps its operator in registers (at most 4 cells per
// thread), the lower levels in LDS; all vectors live in LDS.
constexpr int kCoarseWG = 4096;
constexpr int kMaxCoarseLevels = 10;
struct CoarseLevels {
  int nlev;
  int nx[kMaxCoarseLevels], ny[kMaxCoarseLevels], fx[kMaxCoarseLevels], fy[kMaxCoarseLevels];
  const double *dg[kMaxCoarseLevels], *ax[kMaxCoarseLevels], *ay[kMaxCoarseLevels];
  int xoff[kMaxCoarseLevels];   // LDS offset of x_l (b_l follows, n_l later)
  int aoff[kMaxCoarseLevels];   // LDS offset of (dg, ax, ay) of level l >= 1
};

__global__ void __launch_bounds__(1024) k_mg_coarse(CoarseLevels L, const double *bin,
                                                    double *xout, const double *Ainv,
                                                    double omega, double *part,
                                                    const int32_t *state) {
  extern __shared__ double sm[];
  __shared__ double red[1024];
  if (cg_off(state)) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int last = L.nlev - 1;
  const int n0 = L.nx[0] * L.ny[0];
  auto X = [&](int l) { return sm + L.xoff[l]; };
  auto B = [&](int l) { return sm + L.xoff[l] + L.nx[l] * L.ny[l]; };
  // level-0 operator in registers: cells tid + k * nt, k < 4
  double rd[4], re[4], rw[4], rn[4], rs[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = tid + k * nt;
    rd[k] = 1.0; re[k] = rw[k] = rn[k] = rs[k] = 0.0;
    if (c < n0) {
      const int nx = L.nx[0];
      int i, j;
      cell_ij(c, nx, i, j);
      rd[k] = L.dg[0][c];
      if (i + 1 < nx) re[k] = L.ax[0][c];
      if (i > 0) rw[k] = L.ax[0][c - 1];
      if (j + 1 < L.ny[0]) rn[k] = L.ay[0][c];
      if (j > 0) rs[k] = L.ay[0][c - nx];
    }
    if (c < n0) B(0)[c] = bin[c];
  }
  // the coarsest level's dense inverse (n <= 64) in registers
  const int nd = L.nx[last] * L.ny[last];
  double ainv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int row = tid >> 4, col = (tid & 15) + 16 * k;
    ainv[k] = (row < nd && col < nd) ? Ainv[(size_t)row * nd + col] : 0.0;
  }
  // lower levels' operators into LDS
  for (int l = 1; l < L.nlev; ++l) {
    const int n = L.nx[l] * L.ny[l];
    double *a = sm + L.aoff[l];
    for (int c = tid; c < n; c += nt) {
      a[c] = L.dg[l][c]; a[n + c] = L.ax[l][c]; a[2 * n + c] = L.ay[l][c];
    }
  }
  __syncthreads();
  // one red (0) or black (1) half sweep of level l; e: coarse correction of
  // the neighbours (scaled by omega), zero: neighbours are zero
  auto half = [&](int l, int color, bool zero, const double *e) {
    const int nx = L.nx[l], ny = L.ny[l], n = nx * ny;
    double *x = X(l);
    const double *b = B(l);
    const int cnx = e ? L.nx[l + 1] : 1, fx = L.fx[l], fy = L.fy[l];
    auto V = [&](int ii, int jj) {
      double v = x[jj * nx + ii];
      if (e) v += omega * e[(jj >> (fy >> 1)) * cnx + (ii >> (fx >> 1))];
      return v;
    };
    if (l == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = tid + k * nt;
        if (c < n) {
          int i, j;
  cell_ij(c, nx, i, j);
          if (((i + j) & 1) == color) {
            double s = b[c];
            if (!zero) {
              if (i + 1 < nx) s += re[k] * V(i + 1, j);
              if (i > 0) s += rw[k] * V(i - 1, j);
              if (j + 1 < ny) s += rn[k] * V(i, j + 1);
              if (j > 0) s += rs[k] * V(i, j - 1);
            }
            x[c] = s / rd[k];
          }
        }
      }
    } else {
      const double *dg = sm + L.aoff[l], *ax = dg + n, *ay = dg + 2 * n;
      for (int c = tid; c < n; c += nt) {
        int i, j;
  cell_ij(c, nx, i, j);
        if (((i + j) & 1) != color) continue;
        double s = b[c];
        if (!zero) {
          if (i + 1 < nx) s += ax[c] * V(i + 1, j);
          if (i > 0) s += ax[c - 1] * V(i - 1, j);
          if (j + 1 < ny) s += ay[c] * V(i, j + 1);
          if (j > 0) s += ay[c - nx] * V(i, j - 1);
        }
        x[c] = s / dg[c];
      }
    }
    __syncthreads();
  };
  // residual of level l at cell c (operator from registers or LDS)
  auto resid = [&](int l, int c) {
    const int nx = L.nx[l], ny = L.ny[l], n = nx * ny;
    int i, j;
    cell_ij(c, nx, i, j);
    const double *x = X(l);
    double d, e_, w_, n_, s_;
    if (l == 0) {
      const int k = (c - tid) / nt;   // only called with c = tid + k * nt
      d = rd[k]; e_ = re[k]; w_ = rw[k]; n_ = rn[k]; s_ = rs[k];
    } else {
      const double *dg = sm + L.aoff[l], *ax = dg + n, *ay = dg + 2 * n;
      d = dg[c];
      e_ = i + 1 < nx ? ax[c] : 0.0; w_ = i > 0 ? ax[c - 1] : 0.0;
      n_ = j + 1 < ny ? ay[c] : 0.0; s_ = j > 0 ? ay[c - nx] : 0.0;
    }
    double y = d * x[c];
    if (i + 1 < nx) y -= e_ * x[c + 1];
    if (i > 0) y -= w_ * x[c - 1];
    if (j + 1 < ny) y -= n_ * x[c + nx];
    if (j > 0) y -= s_ * x[c - nx];
    return B(l)[c] - y;
  };
  // down: pre-smooth, residual, restriction (the residual goes to LDS
  // scratch first: level l's b is reused for it once x is final)
  for (int l = 0; l < last; ++l) {
    half(l, 0, true, nullptr);
    half(l, 1, false, nullptr);
    // residuals (at most 4 cells per thread) into b_l
    const int n = L.nx[l] * L.ny[l];
    double rr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = tid + k * nt;
      rr[k] = c < n ? resid(l, c) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = tid + k * nt;
      if (c < n) B(l)[c] = rr[k];
    }
    __syncthreads();
    const int nx = L.nx[l], ny = L.ny[l], cnx = L.nx[l + 1], cny = L.ny[l + 1];
    for (int C = tid; C < cnx * cny; C += nt) {
      int I, J;
  cell_ij(C, cnx, I, J);
      double s = 0.0;
      for (int dj = 0; dj < L.fy[l]; ++dj)
        for (int di = 0; di < L.fx[l]; ++di) {
          const int i = L.fx[l] * I + di, j = L.fy[l] * J + dj;
          if (i < nx && j < ny) s += B(l)[j * nx + i];
        }
      B(l + 1)[C] = s;
    }
    __syncthreads();
  }
  // dense solve on the coarsest level (n <= 64): 16 threads per row, the
  // inverse preloaded in registers
  {
    const double *b = B(last);
    const int row = tid >> 4, col0 = tid & 15;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int col = col0 + 16 * k;
      if (row < nd && col < nd) v += ainv[k] * b[col];
    }
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    if (col0 == 0 && row < nd) X(last)[row] = v;
    __syncthreads();
  }
  // up: the restriction overwrote b_l with the residual, so the post
  // smoothing needs the original right-hand side back: the top level reloads
  // it from global memory, lower levels restore it from their residual and
  // pre-smoothed x (b = r + A x).
  for (int l = last - 1; l >= 0; --l) {
    if (l == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = tid + k * nt;
        if (c < n0) B(0)[c] = bin[c];
      }
    } else {
      // b = r + A x with the pre-smoothed x (unchanged since the residual)
      const int n = L.nx[l] * L.ny[l], nx = L.nx[l], ny = L.ny[l];
      const double *dg = sm + L.aoff[l], *ax = dg + n, *ay = dg + 2 * n;
      const double *x = X(l);
      double bv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = tid + k * nt;
        bv[k] = 0.0;
        if (c < n) {
          int i, j;
  cell_ij(c, nx, i, j);
          double y = dg[c] * x[c];
          if (i + 1 < nx) y -= ax[c] * x[c + 1];
          if (i > 0) y -= ax[c - 1] * x[c - 1];
          if (j + 1 < ny) y -= ay[c] * x[c + nx];
          if (j > 0) y -= ay[c - nx] * x[c - nx];
          bv[k] = B(l)[c] + y;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = tid + k * nt;
        if (c < n) B(l)[c] = bv[k];
      }
    }
    __syncthreads();
    half(l, 1, false, X(l + 1));
    half(l, 0, false, nullptr);
  }
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = tid + k * nt;
    if (c < n0) {
      xout[c] = X(0)[c];
      if (part) v += bin[c] * X(0)[c];
    }
  }
  if (part) {
    // single block: the r.z partial is the full sum
    red[tid] = v;
    __syncthreads();
    for (int h = nt / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) part[0] = red[0];
  }
}

__global__ void k_copy(int n, const double *a, double *b, const int32_t *state) {
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) b[c] = a[c];
}

inline int nblk(int n) { return (n + kRedBlock - 1) / kRedBlock; }

constexpr double kOmega = 1.7;   // coarse-grid correction scaling (aggregation MG)

size_t coarse_lds_bytes_from(const PlanDev &P, size_t lc) {
  size_t n = 0;
  for (size_t l = lc; l < P.mg.size(); ++l)
    n += (l == lc ? 2 : 5) * (size_t)P.mg[l].nx * P.mg[l].ny;
  return n * sizeof(double);
}

// First level handled by the single-workgroup kernel: at most kCoarseWG cells
// and its vectors plus the lower levels' operators within the LDS budget
// (160 KB per CU, 8 KB of it static in the kernel).
constexpr size_t kCoarseLdsBudget = 148 * 1024;
int coarse_start(const PlanDev &P) {
  int lc = 0;
  while (lc + 1 < (int)P.mg.size() &&
         (P.mg[lc].nx * P.mg[lc].ny > kCoarseWG || coarse_lds_bytes_from(P, lc) > kCoarseLdsBudget))
    ++lc;
  return lc;
}

size_t coarse_lds_bytes(const PlanDev &P) { return coarse_lds_bytes_from(P, coarse_start(P)); }

// z = M^{-1} r (one V(1,1) cycle with scaled coarse corrections), then the
// r.z sum into scal (first: RZ = r.z; otherwise beta = r.z / RZ, RZ = r.z).
void vcycle(const PlanDev &P, const double *r, double *z, bool first, hipStream_t s) {
  const int lc = coarse_start(P);
  const int nlev = (int)P.mg.size();
  // fine levels: pre-smooth and restrict
  for (int l = 0; l < lc; ++l) {
    const MGLevel &L = P.mg[l], &C = P.mg[l + 1];
    const int n = L.nx * L.ny;
    double *x = l == 0 ? z : L.x;
    const double *b = l == 0 ? r : L.b;
    hipLaunchKernelGGL(k_mg_red, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, x, b, 1, (const double *)nullptr, (double *)nullptr, P.state);
    hipLaunchKernelGGL(k_mg_black, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, x, b, (const double *)nullptr, 1, 1, 1, 0.0, P.state);
    hipLaunchKernelGGL(k_mg_restrict, dim3(nblk(C.nx * C.ny)), dim3(kRedBlock), 0, s, L.nx, L.ny,
                       L.diag, L.ax, L.ay, x, b, L.fx, L.fy, C.nx, C.ny, C.b, P.state);
  }
  // coarse levels in one workgroup
  {
    CoarseLevels CL;
    CL.nlev = nlev - lc;
    int off = 0;
    for (int t = 0; t < CL.nlev; ++t) {
      const MGLevel &L = P.mg[lc + t];
      const int n = L.nx * L.ny;
      CL.nx[t] = L.nx; CL.ny[t] = L.ny; CL.fx[t] = L.fx; CL.fy[t] = L.fy;
      CL.dg[t] = L.diag; CL.ax[t] = L.ax; CL.ay[t] = L.ay;
      CL.xoff[t] = off;
      off += 2 * n;
      CL.aoff[t] = t == 0 ? 0 : off;
      if (t > 0) off += 3 * n;
    }
    const double *bin = lc == 0 ? r : P.mg[lc].b;
    double *xout = lc == 0 ? z : P.mg[lc].x;
    hipLaunchKernelGGL(k_mg_coarse, dim3(1), dim3(1024), coarse_lds_bytes(P), s, CL, bin, xout,
                       P.coarse_inv, kOmega, lc == 0 ? P.red : (double *)nullptr, P.state);
  }
  // fine levels: coarse correction folded into the black half sweep, then red
  for (int l = lc - 1; l >= 0; --l) {
    const MGLevel &L = P.mg[l], &C = P.mg[l + 1];
    const int n = L.nx * L.ny;
    double *x = l == 0 ? z : L.x;
    const double *b = l == 0 ? r : L.b;
    hipLaunchKernelGGL(k_mg_black, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, x, b, (const double *)C.x, L.fx, L.fy, C.nx, kOmega, P.state);
    hipLaunchKernelGGL(k_mg_red, dim3(nblk(n)), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                       L.ay, x, b, 0, l == 0 ? r : (const double *)nullptr,
                       l == 0 ? P.red : (double *)nullptr, P.state);
  }
  const int npart = lc == 0 ? 1 : nblk(P.N);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, npart, P.scal, (int)S_RZ,
                     first ? 0 : 2, 0.0, P.state);
}

// ------------------------------------------------------------- update / Err
// delta = phi' - phi_half (GSIS) or 0 (SI); Err partials; phi = phi_new.
// FP32-mixed mode also records base = phi^m + delta (see the transport file).
__global__ void k_update(int n, int method, int fp32, double V, const double *phinew,
                         const double *phih, double *phi, double *delta, double *base,
                         double *part, const int32_t *state) {
  __shared__ double sh[kRedBlock];
  if (state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (c < n) {
    const double pn = method ? phinew[c] : phih[c];
    const double d = pn - phi[c];
    num = V * d * d;
    den = V * pn * pn;
    const double dl = method ? pn - phih[c] : 0.0;
    delta[c] = dl;
    if (fp32) base[c] = phi[c] + dl;
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
// (src, base/(4 pi), phi/(4 pi)) read by the fused sweep.
__global__ void k_source(int nx, int ny, int fp32, const double *sig_s, const double *q,
                         const double *phi, const double *base, double *src, double *dynq,
                         const int32_t *state) {
  if (state[1] != 0) return;
  const int n = nx * ny;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double sc = (sig_s[c] * phi[c] + q[c]) / kFourPi;
  const double dq = base[c] / kFourPi;
  const double pq = phi[c] / kFourPi;
  src[c] = sc;
  int i, j;
  cell_ij(c, nx, i, j);
  for (int qd = 0; qd < 4; ++qd) {
    const int xl = (qd & 1) ? nx - 1 - i : i, yl = (qd & 2) ? ny - 1 - j : j;
    const size_t o = (size_t)qd * 3 * n + dg_idx(xl, yl, nx, ny);
    dynq[o] = sc;          // plane 0 of quadrant qd
    dynq[o + n] = dq;      // plane 1
    if (fp32) dynq[o + 2 * n] = pq;
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
  hipLaunchKernelGGL(k_source, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, P.nx, P.ny,
                     P.precision == GSIS_FP32_MIXED ? 1 : 0, P.sig_s, P.q, P.phi, P.base, P.src,
                     P.dynq, P.state);
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
void prepare_synth(PlanDev &P) {
  const size_t bytes = coarse_lds_bytes(P);
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute((const void *)k_mg_coarse, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

// Preconditioned CG on D1 phi' = rhs, warm-started from phi (the previous
// synthetic solution); the solution lands in P.mg[0].x. The stop test runs
// on the device (state[3]); the host looks at it every second iteration
// after the fourth (host_flag: pinned int32[2]) and otherwise keeps
// enqueueing, since a converged solve turns the remaining kernels into
// no-ops.
void launch_synth_solve(PlanDev &P, hipStream_t s, int32_t *host_flag) {
  const MGLevel &L = P.mg[0];
  const int n = P.N, nb = nblk(n);
  double *x = L.x;
  hipLaunchKernelGGL(k_cg_begin, dim3(nb), dim3(kRedBlock), 0, s, n, P.phi, x, P.state);
  hipLaunchKernelGGL(k_cg_residual, dim3(nb), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax,
                     L.ay, x, P.rhs, P.cg_r, P.red, P.red + nb, P.state);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red + nb, nb, P.scal, (int)S_BB,
                     0, 0.0, P.state);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_RR, 4,
                     P.synth_rtol, P.state);
  vcycle(P, P.cg_r, P.cg_z, true, s);
  double *pbuf[2] = {P.cg_p, P.cg_p2};
  for (int it = 0; it < P.synth_max_iter; ++it) {
    double *pold = pbuf[it & 1], *pnew = pbuf[(it + 1) & 1];
    hipLaunchKernelGGL(k_cg_pAp, dim3(nb), dim3(kRedBlock), 0, s, L.nx, L.ny, L.diag, L.ax, L.ay,
                       P.cg_z, pold, pnew, P.cg_Ap, P.scal, it == 0 ? 1 : 0, P.red, P.state);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_PAP, 1,
                       0.0, P.state);
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(kRedBlock), 0, s, n, x, P.cg_r, pnew, P.cg_Ap,
                       P.scal, P.red, P.state);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, s, P.red, nb, P.scal, (int)S_RR, 3,
                       0.0, P.state);
    if (it + 1 == P.synth_max_iter) break;
    if (it >= 3 && ((it - 3) & 1) == 0) {
      hipMemcpyAsync(host_flag, P.state + 1, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
      hipStreamSynchronize(s);
      if (host_flag[0] != 0 || host_flag[2] != 0) return;
    }
    vcycle(P, P.cg_r, P.cg_z, false, s);
  }
}

void launch_update(const PlanDev &P, hipStream_t s) {
  const int nb = nblk(P.N);
  const double *phinew = P.mg[0].x;
  hipLaunchKernelGGL(k_update, dim3(nb), dim3(kRedBlock), 0, s, P.N, P.method,
                     P.precision == GSIS_FP32_MIXED ? 1 : 0, P.V, phinew, P.phih, P.phi,
                     P.delta, P.base, P.err_parts, P.state);
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
