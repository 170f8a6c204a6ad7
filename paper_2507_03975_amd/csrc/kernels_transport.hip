// kernels_transport.hip -- transport step of one outer iteration on gfx950.
//
//  residual : r = (sigma_s phi^m + q)/(4 pi) - sigma_t I^m
//                 - (1/V) sum_f (Omega.n_f) A_f I_f                (Eq. RTE_d_res)
//             with I_f the second-order upwind face value (Eqs. Ii,k, Iij):
//             adaptive least-squares gradient (Eqs. shifted_j, LSF_mdf) and
//             the Barth-Jespersen limiter.
//  sweep    : exact solve of the first-order-upwind increment system
//             (Eqs. RTE_d_increment, delta_Iij, RTE_d_mtx, elem_mtx), one
//             ordinate per workgroup, lanes = rows, diagonal wavefront.
//  moments  : phi, F of I^{m+1/2} (Eqs. def_rho, def_F).
//  boundary : F_T . n_out on every boundary face (Sec. 4.4).
//
// The pending GSIS correction delta/(4 pi) (Eq. GSIS_update) is added to
// I^m on every read, so the correction never costs a pass over I.
#include "gsis_internal.h"

namespace gsis {
namespace {

constexpr double kInv4Pi = 1.0 / kFourPi;

struct TArgs {
  int nx, ny, N, K, nbf;
  double dx, dy;
  int order, limiter;
  int qoff[5];
  const double *amu, *aeta, *w, *wmu, *weta;
  double *I0, *I1;   // the two intensity buffers; state[2] names the current one
  double *R;
  const double *sig_t, *src, *delta;
  const double *cE, *cW, *cN, *cS;
  const double *bnd;
  double *phih, *Fx, *Fy, *bflux;
  const int32_t *state;
};

TArgs make_args(const PlanDev &P) {
  TArgs a;
  a.nx = P.nx; a.ny = P.ny; a.N = P.N; a.K = P.K; a.nbf = P.nbf;
  a.dx = P.dx; a.dy = P.dy; a.order = P.order; a.limiter = P.limiter;
  for (int t = 0; t < 5; ++t) a.qoff[t] = P.qoff[t];
  a.amu = P.amu; a.aeta = P.aeta; a.w = P.w; a.wmu = P.wmu; a.weta = P.weta;
  a.I0 = P.I[0]; a.I1 = P.I[1]; a.R = P.R;
  a.sig_t = P.sig_t; a.src = P.src; a.delta = P.delta;
  a.cE = P.cE; a.cW = P.cW; a.cN = P.cN; a.cS = P.cS;
  a.bnd = P.bnd; a.phih = P.phih; a.Fx = P.Fx; a.Fy = P.Fy; a.bflux = P.bflux;
  a.state = P.state;
  return a;
}

__device__ inline const double *Iin_of(const TArgs &a) { return a.state[2] ? a.I1 : a.I0; }
__device__ inline double *Iout_of(const TArgs &a) { return a.state[2] ? a.I0 : a.I1; }

__device__ inline int quadrant_of(const TArgs &a, int kk) {
  return (kk >= a.qoff[1]) + (kk >= a.qoff[2]) + (kk >= a.qoff[3]);
}
// quadrant q: bit 0 = mirrored in x (mu < 0), bit 1 = mirrored in y (eta < 0)
__device__ inline int gcell(const TArgs &a, int q, int xl, int yl) {
  int i = (q & 1) ? a.nx - 1 - xl : xl;
  int j = (q & 2) ? a.ny - 1 - yl : yl;
  return j * a.nx + i;
}

// I^m at a local cell of ordinate kk (buffer value plus pending correction)
__device__ inline double Im(const TArgs &a, const double *Ik, int q, int xl, int yl) {
  return Ik[(size_t)yl * a.nx + xl] + a.delta[gcell(a, q, xl, yl)] * kInv4Pi;
}

// Outgoing face values of a local cell (its local east and north faces):
// U + psi * G . (x_f - x_c) with the ALSM gradient and BJ limiter.
template <typename LoadF>
__device__ inline void out_faces(const TArgs &a, int q, int xl, int yl, LoadF ld,
                                 double &Fe, double &Fn) {
  const double u = ld(xl, yl);
  if (a.order < 2) { Fe = u; Fn = u; return; }
  const bool he = xl + 1 < a.nx, hw = xl > 0, hn = yl + 1 < a.ny, hs = yl > 0;
  const double ue = he ? ld(xl + 1, yl) : u;
  const double uw = hw ? ld(xl - 1, yl) : u;
  const double un = hn ? ld(xl, yl + 1) : u;
  const double us = hs ? ld(xl, yl - 1) : u;
  const int c = gcell(a, q, xl, yl);
  // local east/west are global west/east when the quadrant is mirrored in x
  const double ce = (q & 1) ? a.cW[c] : a.cE[c];
  const double cw = (q & 1) ? a.cE[c] : a.cW[c];
  const double cn = (q & 2) ? a.cS[c] : a.cN[c];
  const double cs = (q & 2) ? a.cN[c] : a.cS[c];
  const double gx = ce * (ue - u) - cw * (uw - u);
  const double gy = cn * (un - u) - cs * (us - u);
  const double hx = gx * (0.5 * a.dx), hy = gy * (0.5 * a.dy);
  double psi = 1.0;
  if (a.limiter) {
    // Barth-Jespersen over the four faces: the face offsets are +-hx, +-hy,
    // so min_f min(1, (Uext - u)/delta_f) = min(1, m / M) exactly.
    const double umax = fmax(fmax(fmax(u, ue), fmax(uw, un)), us);
    const double umin = fmin(fmin(fmin(u, ue), fmin(uw, un)), us);
    const double m = fmin(umax - u, u - umin);
    const double M = fmax(fabs(hx), fabs(hy));
    if (M > 0.0) psi = fmin(1.0, m / M);
  }
  Fe = u + psi * hx;
  Fn = u + psi * hy;
}

// incoming boundary value on the local west face of local row yl / local
// south face of local column xl
__device__ inline double inflow_w(const TArgs &a, int q, int yl, int kk) {
  int j = (q & 2) ? a.ny - 1 - yl : yl;
  int f = (q & 1) ? a.ny + j : j;
  return a.bnd[(size_t)f * a.K + kk];
}
__device__ inline double inflow_s(const TArgs &a, int q, int xl, int kk) {
  int i = (q & 1) ? a.nx - 1 - xl : xl;
  int f = (q & 2) ? 2 * a.ny + a.nx + i : 2 * a.ny + i;
  return a.bnd[(size_t)f * a.K + kk];
}

__global__ void k_residual(TArgs a) {
  if (a.state[1] != 0) return;
  const int kk = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.N) return;
  const int xl = t % a.nx, yl = t / a.nx;
  const int q = quadrant_of(a, kk);
  const double *Ik = Iin_of(a) + (size_t)kk * a.N;
  auto ld = [&](int x, int y) { return Im(a, Ik, q, x, y); };
  double Fe, Fn, Few, Fns, dummy;
  out_faces(a, q, xl, yl, ld, Fe, Fn);
  if (xl > 0) out_faces(a, q, xl - 1, yl, ld, Few, dummy);
  else Few = inflow_w(a, q, yl, kk);
  if (yl > 0) out_faces(a, q, xl, yl - 1, ld, dummy, Fns);
  else Fns = inflow_s(a, q, xl, kk);
  const int c = gcell(a, q, xl, yl);
  const double u = ld(xl, yl);
  const double r = a.src[c] - a.sig_t[c] * u - a.amu[kk] * (Fe - Few) - a.aeta[kk] * (Fn - Fns);
  a.R[(size_t)kk * a.N + t] = r;
}

// Exact increment solve for one ordinate per workgroup. Thread t of a pass
// owns local row y0 + t; at step s it handles column s - t, so every step
// advances one anti-diagonal. dI from the row below comes from lane t-1 at
// the previous step (a shuffle; an LDS slot across waves); dI from the west
// is the lane's own previous value.
__global__ void k_sweep(TArgs a) {
  if (a.state[1] != 0) return;
  const int kk = blockIdx.x;
  const int q = quadrant_of(a, kk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rows_per_pass = blockDim.x;
  const double ax = a.amu[kk], ay = a.aeta[kk];
  const double *Ik = Iin_of(a) + (size_t)kk * a.N;
  double *Ok = Iout_of(a) + (size_t)kk * a.N;
  double *Rk = a.R + (size_t)kk * a.N;
  __shared__ double edge[2][16];
  for (int y0 = 0; y0 < a.ny; y0 += rows_per_pass) {
    const int rows = min(rows_per_pass, a.ny - y0);
    const int yl = y0 + tid;
    const bool rowok = tid < rows;
    const bool top = (tid == rows - 1) && (y0 + rows < a.ny);
    double prev = 0.0;
    const int nsteps = a.nx + rows - 1;
    for (int s = 0; s < nsteps; ++s) {
      const int xl = s - tid;
      double below = __shfl_up(prev, 1, 64);
      if (lane == 0) {
        if (wave > 0) below = edge[(s + 1) & 1][wave - 1];
        else below = (y0 > 0 && xl >= 0 && xl < a.nx) ? Rk[(size_t)(y0 - 1) * a.nx + xl] : 0.0;
      }
      if (rowok && xl >= 0 && xl < a.nx) {
        const size_t o = (size_t)yl * a.nx + xl;
        const int c = gcell(a, q, xl, yl);
        const double west = xl > 0 ? prev : 0.0;
        const double s_ = yl > 0 ? below : 0.0;
        const double r = Rk[o];
        const double di = (r + ax * west + ay * s_) / (a.sig_t[c] + ax + ay);
        Ok[o] = Ik[o] + a.delta[c] * kInv4Pi + di;
        if (top) Rk[o] = di;   // hand the top row to the next pass
        prev = di;
      }
      if (lane == 63) edge[s & 1][wave] = prev;
      __syncthreads();
    }
    __syncthreads();
  }
}

// phi, F of I^{m+1/2}: one thread per cell, sum over every ordinate.
__global__ void k_moments(TArgs a) {
  if (a.state[1] != 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.N) return;
  const int i = c % a.nx, j = c / a.nx;
  double s0 = 0, sx = 0, sy = 0;
  for (int q = 0; q < 4; ++q) {
    const int xl = (q & 1) ? a.nx - 1 - i : i;
    const int yl = (q & 2) ? a.ny - 1 - j : j;
    const size_t o = (size_t)yl * a.nx + xl;
    for (int kk = a.qoff[q]; kk < a.qoff[q + 1]; ++kk) {
      const double v = Iout_of(a)[(size_t)kk * a.N + o];
      s0 += a.w[kk] * v;
      sx += a.wmu[kk] * v;
      sy += a.weta[kk] * v;
    }
  }
  a.phih[c] = s0; a.Fx[c] = sx; a.Fy[c] = sy;
}

// F_T . n_out on each boundary face: one workgroup per face, threads over
// ordinates, fixed-order tree sum.
__global__ void k_boundary_flux(TArgs a) {
  if (a.state[1] != 0) return;
  const int f = blockIdx.x;
  int side, pos;
  if (f < a.ny) { side = 0; pos = f; }                       // W
  else if (f < 2 * a.ny) { side = 1; pos = f - a.ny; }        // E
  else if (f < 2 * a.ny + a.nx) { side = 2; pos = f - 2 * a.ny; }   // S
  else { side = 3; pos = f - 2 * a.ny - a.nx; }               // N
  double acc = 0.0;
  for (int kk = threadIdx.x; kk < a.K; kk += blockDim.x) {
    const int q = quadrant_of(a, kk);
    // w * (Omega . n_out)
    const double won = side == 0 ? -a.wmu[kk] : side == 1 ? a.wmu[kk]
                     : side == 2 ? -a.weta[kk] : a.weta[kk];
    double val = 0.0;
    if (won < 0.0) {
      val = a.bnd[(size_t)f * a.K + kk];
    } else if (won > 0.0) {
      // outgoing: this face is the local east (x sides) or north (y sides)
      // face of the boundary cell in the ordinate's mirrored frame
      int i = side == 0 ? 0 : side == 1 ? a.nx - 1 : pos;
      int j = side == 2 ? 0 : side == 3 ? a.ny - 1 : pos;
      int xl = (q & 1) ? a.nx - 1 - i : i;
      int yl = (q & 2) ? a.ny - 1 - j : j;
      const double *Ok = Iout_of(a) + (size_t)kk * a.N;
      auto ld = [&](int x, int y) { return Ok[(size_t)y * a.nx + x]; };
      double Fe, Fn;
      out_faces(a, q, xl, yl, ld, Fe, Fn);
      val = side < 2 ? Fe : Fn;
    }
    acc += won * val;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.bflux[f] = red[0];
}

}  // namespace

void launch_residual(const PlanDev &P, hipStream_t s) {
  TArgs a = make_args(P);
  dim3 g((P.N + 255) / 256, P.K);
  hipLaunchKernelGGL(k_residual, g, dim3(256), 0, s, a);
}

void launch_sweep(const PlanDev &P, hipStream_t s) {
  TArgs a = make_args(P);
  int rows = ((P.ny + 63) / 64) * 64;
  if (rows > 1024) rows = 1024;
  hipLaunchKernelGGL(k_sweep, dim3(P.K), dim3(rows), 0, s, a);
}

void launch_moments(const PlanDev &P, hipStream_t s) {
  TArgs a = make_args(P);
  hipLaunchKernelGGL(k_moments, dim3((P.N + 255) / 256), dim3(256), 0, s, a);
}

void launch_boundary_flux(const PlanDev &P, hipStream_t s) {
  TArgs a = make_args(P);
  hipLaunchKernelGGL(k_boundary_flux, dim3(P.nbf), dim3(256), 0, s, a);
}

}  // namespace gsis
