// kernels_adjoint.hip -- adjoint of the SI / GSIS fixed point on gfx950.
//
// With the limiter off one outer iteration is affine in the intensity,
// I' = T(I; p) = G I + c(p). For outputs J = <g_phi, phi*> + <g_F, F*> of
// the fixed point I*, the adjoint solves lambda = G^T lambda + M^T g
// (M: the moments phi = sum_k w_k I_k, F = sum_k w_k Omega_k I_k) and gives
// dJ/dp = lambda^T dT(I*; p)/dp for p = sigma_a, sigma_s, q per cell.
//
// G^T lambda is the reverse of one iteration, step by step:
//   correction      s = sum_k lambda_k / (4 pi)          (unweighted sum)
//   synthetic solve bb = D1^-1 s                          (D1 symmetric; the
//                                                          plan's CG + multigrid)
//   right-hand side hb (HoT cotangents), bfb (boundary fluxes), and
//                   phb = -s + sum_bnd A kappa bb + grad^T(hb / (3 sigma_t))
//   moments         Ih_bar = lambda + w (phb + mu hbx + eta hby) + the
//                   transposed reconstruction at outflow walls
//   increment solve rb = H^-T Ih_bar: the first-order upwind sweep run
//                   backwards (downstream cells first)
//   residual        G^T lambda = Ih_bar - sigma_t rb - Div2^T rb
//                                + w sigma_s sum_k(rb) / (4 pi)
// all in the plan's internal layout (ordinates by quadrant, each quadrant in
// its mirrored frame, cells in anti-diagonal order). The gradient pass then
// collects the derivatives of every sigma-dependent coefficient: the
// increment-solve diagonal and the sigma_t I term, the shifted least-squares
// distances (through the coefficient cotangents of the three gradients: the
// transport residual on I*, the wall reconstruction on I^{m+1/2}, the HoT on
// phi^{m+1/2}), 1/(3 sigma_t) in the HoT, kappa, Gamma, and sigma_a in D1.
#include "gsis_internal.h"
#include "wave_ops.h"

#include <cstring>

namespace gsis {
namespace {

constexpr int kB = 256;
constexpr double kInv4Pi = 1.0 / kFourPi;

struct AArgs {
  int nx, ny, N, K, nbf, order, alsm, method;
  double dx, dy, V;
  int qoff[5];
  const double *w, *wmu, *weta, *amu, *aeta;                  // internal ordinates
  const double *sig_t, *sig_s, *cE, *cW, *cN, *cS;            // caller's cell order
  const double *cellq;                                        // [4][N][6] mirrored
  const double *sdq;                                          // [4][N] sigma_t + shift, stored order
  const int *dso;                                             // row-0 storage index per diagonal
  const double *Ih;                                           // I^{m+1/2} [K][N]
  const double *delta, *phi, *phih;
  const double *gphi, *gFx, *gFy;                             // cotangents or null
  double *lam, *ihb, *rb;                                     // [K][N]
  double *s, *s_old, *bb, *hxb, *hyb, *phb, *Sb, *bfb;
  double *part;                                               // [4][5][N]
  double *dbar;                                               // [4][N]
  double *stp;                                                // [N]
  double *errp;
  unsigned long long *hand;                                   // split sweep hand-over
  int32_t *hand_err;
};

__device__ inline int quadrant_of(const AArgs &a, int kk) {
  return (kk >= a.qoff[1]) + (kk >= a.qoff[2]) + (kk >= a.qoff[3]);
}
__device__ inline int gcell(const AArgs &a, int q, int xl, int yl) {
  const int i = (q & 1) ? a.nx - 1 - xl : xl;
  const int j = (q & 2) ? a.ny - 1 - yl : yl;
  return j * a.nx + i;
}
__device__ inline void dg_cell(long long t, int nx, int ny, int &x, int &y) {
  int lo = 0, hi = nx + ny - 2;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (dg_off(mid, nx, ny) <= t) lo = mid; else hi = mid - 1;
  }
  y = dg_ylo(lo, nx) + (int)(t - dg_off(lo, nx, ny));
  x = lo - y;
}
__device__ inline void cell_ij(int c, int nx, int &i, int &j) {
  int q = (int)((double)c * __builtin_amdgcn_rcp((double)nx));
  int r = c - q * nx;
  if (r < 0) { --q; r += nx; } else if (r >= nx) { ++q; r -= nx; }
  i = r; j = q;
}
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
// global boundary faces of the local east face of local row y and of the
// local north face of local column x
__device__ inline int face_e(const AArgs &a, int q, int y) {
  const int j = (q & 2) ? a.ny - 1 - y : y;
  return (q & 1) ? j : a.ny + j;
}
__device__ inline int face_n(const AArgs &a, int q, int x) {
  const int i = (q & 1) ? a.nx - 1 - x : x;
  return (q & 2) ? 2 * a.ny + i : 2 * a.ny + a.nx + i;
}

// Per quadrant, one thread per stored cell: unweighted sum of src over the
// quadrant's ordinates into part[q][c] (c in the caller's order).
__global__ void k_a_qsum(AArgs a, const double *src) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (t >= a.N) return;
  int x, y;
  dg_cell(t, a.nx, a.ny, x, y);
  double v = 0.0;
  for (int kk = a.qoff[q]; kk < a.qoff[q + 1]; ++kk) v += src[(size_t)kk * a.N + t];
  a.part[(size_t)q * a.N + gcell(a, q, x, y)] = v;
}

// out = scale * sum_q part[q]; with err, the Err partials of out against
// s_old (which then takes out).
__global__ void k_a_combine(AArgs a, double *out, double scale, int err) {
  __shared__ double sh[kB];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (c < a.N) {
    const double v = scale * (((a.part[c] + a.part[(size_t)a.N + c]) + a.part[2 * (size_t)a.N + c]) +
                              a.part[3 * (size_t)a.N + c]);
    out[c] = v;
    if (err) {
      const double d = v - a.s_old[c];
      num = a.V * d * d;
      den = a.V * v * v;
      a.s_old[c] = v;
    }
  }
  if (err) {
    const double x = block_sum(num, sh), y = block_sum(den, sh);
    if (threadIdx.x == 0) { a.errp[2 * blockIdx.x] = x; a.errp[2 * blockIdx.x + 1] = y; }
  }
}

__global__ void k_a_err(AArgs a, int npart, double *hist, int m) {
  __shared__ double sh[kB];
  double x = 0.0, y = 0.0;
  for (int t = threadIdx.x; t < npart; t += blockDim.x) { x += a.errp[2 * t]; y += a.errp[2 * t + 1]; }
  x = block_sum(x, sh);
  y = block_sum(y, sh);
  if (threadIdx.x == 0) hist[m] = y > 0.0 ? sqrt(x / y) : (x == 0.0 ? 0.0 : INFINITY);
}

// Right-hand side reversed: HoT cotangents (transpose of the central face
// average) and the boundary-flux cotangents -A bb.
__global__ void k_a_hbar(AArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.N) return;
  int i, j;
  cell_ij(c, a.nx, i, j);
  const int nx = a.nx, ny = a.ny;
  const double Ax = a.dy, Ay = a.dx, b = a.bb[c];
  double hx = 0.0, hy = 0.0;
  // b_c -= A (h_c + h_e)/2 on an interior east face, += A (h_c + h_w)/2 on
  // an interior west face: h_c's cotangent gathers both cells of each face
  if (i + 1 < nx) hx -= 0.5 * Ax * (b - a.bb[c + 1]);
  else a.bfb[ny + j] = -Ax * b;
  if (i > 0) hx += 0.5 * Ax * (b - a.bb[c - 1]);
  else a.bfb[j] = -Ax * b;
  if (j + 1 < ny) hy -= 0.5 * Ay * (b - a.bb[c + nx]);
  else a.bfb[2 * ny + nx + i] = -Ay * b;
  if (j > 0) hy += 0.5 * Ay * (b - a.bb[c - nx]);
  else a.bfb[2 * ny + i] = -Ay * b;
  a.hxb[c] = hx;
  a.hyb[c] = hy;
}

// phb = -s + sum_bnd A kappa bb + (grad^T y)_c with y = hb / (3 sigma_t),
// the transposed least-squares gradient G_x,c = cE (U_e - U_c) - cW (U_w - U_c).
__global__ void k_a_phbar(AArgs a, const double *kappa) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= a.N) return;
  int i, j;
  cell_ij(d, a.nx, i, j);
  const int nx = a.nx, ny = a.ny;
  auto yx = [&](int c) { return a.hxb[c] / (3.0 * a.sig_t[c]); };
  auto yy = [&](int c) { return a.hyb[c] / (3.0 * a.sig_t[c]); };
  double v = -a.s[d];
  const double b = a.bb[d];
  if (i + 1 == nx) v += a.dy * kappa[ny + j] * b;
  if (i == 0) v += a.dy * kappa[j] * b;
  if (j + 1 == ny) v += a.dx * kappa[2 * ny + nx + i] * b;
  if (j == 0) v += a.dx * kappa[2 * ny + i] * b;
  v += yx(d) * (a.cW[d] - a.cE[d]) + yy(d) * (a.cS[d] - a.cN[d]);
  if (i > 0) v += yx(d - 1) * a.cE[d - 1];
  if (i + 1 < nx) v -= yx(d + 1) * a.cW[d + 1];
  if (j > 0) v += yy(d - nx) * a.cN[d - nx];
  if (j + 1 < ny) v -= yy(d + nx) * a.cS[d + nx];
  a.phb[d] = v;
}

// Ih_bar = lambda + w (phb + mu hbx + eta hby) + the outflow-wall
// reconstruction transposed (GSIS); lambda alone (SI).
__global__ void __launch_bounds__(kB) k_a_ihalf(AArgs a) {
  // one thread per stored cell of quadrant blockIdx.y, looping over the
  // quadrant's ordinates: the cell's cotangents, boundary terms and record
  // entries are loaded once for all of them
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (t >= a.N) return;
  const bool gsis = a.method == 1;
  double phb = 0.0, hxb = 0.0, hyb = 0.0;
  double be = 0.0, be2 = 0.0, bn = 0.0, bn2 = 0.0, ce = 0.0, ce2 = 0.0, cn = 0.0, cn2 = 0.0;
  bool xe = false, xe2 = false, yn = false, yn2 = false;
  const double hx = 0.5 * a.dx, hy = 0.5 * a.dy;
  const int so = a.order >= 2;
  if (gsis) {
    int x, y;
    dg_cell(t, a.nx, a.ny, x, y);
    const int c = gcell(a, q, x, y);
    phb = a.phb[c]; hxb = a.hxb[c]; hyb = a.hyb[c];
    const double *Cq = a.cellq + (size_t)q * a.N * 6;
    // local east face of the last column: value u_c + hx (cW (u_c - u_w))
    xe = x == a.nx - 1;
    xe2 = so && x == a.nx - 2;
    yn = y == a.ny - 1;
    yn2 = so && y == a.ny - 2;
    if (xe) { be = a.bfb[face_e(a, q, y)]; ce = so && x > 0 ? hx * Cq[6 * t + 1] : 0.0; }
    if (xe2) { be2 = a.bfb[face_e(a, q, y)]; ce2 = Cq[6 * dg_idx(x + 1, y, a.nx, a.ny) + 1]; }
    if (yn) { bn = a.bfb[face_n(a, q, x)]; cn = so && y > 0 ? hy * Cq[6 * t + 3] : 0.0; }
    if (yn2) { bn2 = a.bfb[face_n(a, q, x)]; cn2 = Cq[6 * dg_idx(x, y + 1, a.nx, a.ny) + 3]; }
  }
  typedef const __attribute__((address_space(4))) double cdouble;
  cdouble *W = (cdouble *)a.w, *WM = (cdouble *)a.wmu, *WE = (cdouble *)a.weta;
  auto one = [&](int kk, double v) {
    if (gsis) {
      v += W[kk] * phb + WM[kk] * hxb + WE[kk] * hyb;
      const double wmx = fabs(WM[kk]), wmy = fabs(WE[kk]);
      if (xe) {
        const double vb = be * wmx;
        v += vb * (1.0 + ce);
      }
      if (xe2) v -= be2 * wmx * hx * ce2;
      if (yn) {
        const double vb = bn * wmy;
        v += vb * (1.0 + cn);
      }
      if (yn2) v -= bn2 * wmy * hy * cn2;
    }
    a.ihb[(size_t)kk * a.N + t] = v;
  };
  // eight ordinates' lambda loaded before any ihb is stored
  constexpr int U = 8;
  int kk = a.qoff[q];
  const int ke = a.qoff[q + 1];
  for (; kk + U <= ke; kk += U) {
    double l[U];
#pragma unroll
    for (int u = 0; u < U; ++u) l[u] = a.lam[(size_t)(kk + u) * a.N + t];
#pragma unroll
    for (int u = 0; u < U; ++u) one(kk + u, l[u]);
  }
  for (; kk < ke; ++kk) one(kk, a.lam[(size_t)kk * a.N + t]);
}

// rb = H^-T ihb per ordinate: rb_c = (ihb_c + ax rb_east + ay rb_north) / d_c,
// d_c = sigma_t + ax + ay, downstream cells first. Thread t of a pass owns
// reversed row y' = y0 + t (local row ny-1-y'); at step s it is at reversed
// column s - t, so each step is one anti-diagonal and both dependencies are
// one step old (own lane; lane t-1, or an LDS slot across waves).
__global__ void k_a_sweep(AArgs a) {
  const int kk = blockIdx.x;
  const int q = quadrant_of(a, kk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rows_pp = blockDim.x;
  const int nx = a.nx, ny = a.ny;
  const double ax = a.amu[kk], ay = a.aeta[kk];
  const double *Cq = a.cellq + (size_t)q * a.N * 6;
  const double *src = a.ihb + (size_t)kk * a.N;
  double *out = a.rb + (size_t)kk * a.N;
  __shared__ double edge[2][16];
  for (int y0 = 0; y0 < ny; y0 += rows_pp) {
    const int rows = min(rows_pp, ny - y0);
    const bool rowok = tid < rows;
    const int yr = y0 + tid;                 // reversed row
    const int yl = ny - 1 - yr;              // local row
    double prev = 0.0;
    const int nsteps = nx + rows - 1;
    for (int st = 0; st < nsteps; ++st) {
      const int xr = st - tid;               // reversed column
      double below = __shfl_up(prev, 1, 64);
      if (lane == 0) {
        if (wave > 0) below = edge[(st + 1) & 1][wave - 1];
        else if (y0 > 0 && xr >= 0 && xr < nx)
          below = out[dg_idx(nx - 1 - xr, ny - y0, nx, ny)];
        else below = 0.0;
      }
      if (rowok && xr >= 0 && xr < nx) {
        const int xl = nx - 1 - xr;
        const long long o = dg_idx(xl, yl, nx, ny);
        const double east = xr > 0 ? prev : 0.0;
        const double north = yr > 0 ? below : 0.0;
        const double d = Cq[6 * o + 5] + ax + ay;
        const double v = (src[o] + ax * east + ay * north) / d;
        out[o] = v;
        prev = v;
      }
      if (lane == 63) edge[st & 1][wave] = prev;
      __syncthreads();
    }
    __syncthreads();
  }
}

// The same sweep for grids of at most 1024 rows, shaped like the forward
// recurrence: lane t owns reversed row t, step s is reversed anti-diagonal s
// (local diagonal nx + ny - 2 - s, so a step's storage indices are one table
// entry plus the lane's row), rb_north is lane t-1's previous value (a DPP
// shift), waves run kAL steps apart and meet at a barrier every kAL steps
// (the top lane's values through an LDS ring), and the operands of a step
// (ihb, sigma_t + shift) are loaded kAL steps ahead. Out-of-range indices
// fall outside the buffer resources: their loads read 0, their stores are
// dropped. rb = ihb / d + (ax / d) rb_east + (ay / d) rb_north.
// SPLIT: as the forward recurrence, the reversed rows spread over np
// workgroups (workgroup b is part b / K of ordinate b % K), the last reversed
// row of a part handed to the next through the plan's hand-over buffer.
constexpr int kAL = 8, kAR = 4 * kAL, kAMaxW = 16;
static_assert(kAMaxW * kAL + 2 * kAL <= kDiagPad, "diagonal table padding");
template <bool SPLIT>
__global__ void __launch_bounds__(kAMaxW * 64) k_a_chain(AArgs a, int np) {
  const int part = SPLIT ? blockIdx.x / a.K : 0;
  const int kk = blockIdx.x - part * a.K;
  const int q = quadrant_of(a, kk);
  const int nx = a.nx, ny = a.ny, N = a.N;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double ax = a.amu[kk], ay = a.aeta[kk], axy = ax + ay;
  const __amdgpu_buffer_rsrc_t Sr = buf_rsrc(a.ihb + (size_t)kk * N, (size_t)N * 8);
  const __amdgpu_buffer_rsrc_t Dr = buf_rsrc(a.sdq + (size_t)q * N, (size_t)N * 8);
  const __amdgpu_buffer_rsrc_t Or = buf_rsrc(a.rb + (size_t)kk * N, (size_t)N * 8);
  const __attribute__((address_space(4))) int *DS =
      (const __attribute__((address_space(4))) int *)(a.dso + kDiagPad);
  __shared__ double edge[kAMaxW][kAR];
  const int r0 = part * (int)blockDim.x;    // first reversed row of this part
  const int rows = min((int)blockDim.x, ny - r0);   // one pass per part
  const int nw = (rows + 63) >> 6;
  const bool rowok = tid < rows;
  const int yl = ny - 1 - (r0 + tid);       // local row of reversed row r0 + tid
  const int xo = rowok ? tid : (1 << 30);   // reversed column = s - xo
  unsigned long long *Hr = nullptr;
  __amdgpu_buffer_rsrc_t Hw = buf_rsrc(nullptr, 0);
  if (SPLIT) {
    unsigned long long *H = a.hand + (size_t)kk * (np - 1) * nx;
    if (part > 0) Hr = H + (size_t)(part - 1) * nx;
    if (part + 1 < np) Hw = buf_rsrc(H + (size_t)part * nx, (size_t)nx * 8);
  }
  unsigned long long hv = 0;
  bool gave_up = false;
  const bool last_lane = SPLIT && tid == rows - 1;
  const int D = nx + ny - 2;
  const int nsteps = nx + rows - 1;
  const int tend = ((nsteps + (nw - 1) * kAL + kAL - 1) / kAL) * kAL;
  const int s0 = -wave * kAL;               // this wave's step at time 0
  double rb_s[kAL] = {}, rb_d[kAL] = {};
  unsigned rb_i[kAL] = {};
  auto load = [&](int t, int so) {          // row-0 storage index so of the step's diagonal
    const unsigned i = (unsigned)(so + yl);
    rb_i[t] = i;
    rb_s[t] = buf_ld64(Sr, i * 8u);
    rb_d[t] = buf_ld64(Dr, i * 8u);
  };
  double vp = 0.0;
  for (int tb = -kAL; tb < tend; tb += kAL) {
    const int sb = tb + s0;
    double bl[kAL];
    if (wave > 0) {
#pragma unroll
      for (int t2 = 0; t2 < kAL; ++t2) bl[t2] = edge[wave - 1][(sb - 1 + t2) & (kAR - 1)];
    } else if (SPLIT && part > 0) {
      hand_take<kAL>(Hr, nx, sb, hv, gave_up, a.hand_err, bl);
    } else {
#pragma unroll
      for (int t2 = 0; t2 < kAL; ++t2) bl[t2] = 0.0;
    }
    int so[kAL];
#pragma unroll
    for (int t2 = 0; t2 < kAL; ++t2) so[t2] = DS[D - (r0 + sb + kAL + t2)];
    double vv[kAL];
#pragma unroll
    for (int t2 = 0; t2 < kAL; ++t2) {
      const int s = sb + t2;
      const int xr = s - xo;
      const bool act = (unsigned)xr < (unsigned)nx;
      const double vN = shr1_fill(vp, bl[t2]);
      const double inv = rcp64(rb_d[t2] + axy);
      const double vn = fma(ax * inv, vp, fma(ay * inv, vN, rb_s[t2] * inv));
      const double v = act ? vn : vp;
      buf_store(v, Or, act ? rb_i[t2] * 8u : kNoCell);
      if (SPLIT && wave == nw - 1 && part + 1 < np)
        hand_put(Hw, v, last_lane && act ? (unsigned)xr * 8u : kNoCell);
      vp = v;
      vv[t2] = v;
      load(t2, so[t2]);
    }
    if (lane == 63) {
#pragma unroll
      for (int t2 = 0; t2 < kAL; ++t2) edge[wave][(sb + t2) & (kAR - 1)] = vv[t2];
    }
    __syncthreads();
  }
}

// lambda' = ihb - sigma_t rb - Div2^T rb + w sigma_s Sb / (4 pi) + M^T g.
// In the ordinate's frame r_c = ... - ax (E_c - E_w) - ay (N_c - N_s) with
// E_c = u_c + hx (cE (u_e - u_c) - cW (u_w - u_c)) the east face value; so
// Ebar_c = -ax (rb_c - rb_e) and ubar_d collects Ebar of d, d-1, d+1.
__global__ void __launch_bounds__(kB) k_a_out(AArgs a) {
  // one thread per stored cell of quadrant blockIdx.y, looping over the
  // quadrant's ordinates: the cell's record entries, neighbour positions and
  // cotangents are loaded once for all of them
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (t >= a.N) return;
  const int nx = a.nx, ny = a.ny;
  int x, y;
  dg_cell(t, nx, ny, x, y);
  const int c = gcell(a, q, x, y);
  const double *Cq = a.cellq + (size_t)q * a.N * 6;
  const double hx = 0.5 * a.dx, hy = 0.5 * a.dy;
  auto I = [&](int xx, int yy) { return dg_idx(xx, yy, nx, ny); };
  const bool hE = x + 1 < nx, hE2 = x + 2 < nx, hW = x > 0;
  const bool hN = y + 1 < ny, hN2 = y + 2 < ny, hS = y > 0;
  const long long tE = hE ? I(x + 1, y) : t, tE2 = hE2 ? I(x + 2, y) : t, tW = hW ? I(x - 1, y) : t;
  const long long tN = hN ? I(x, y + 1) : t, tN2 = hN2 ? I(x, y + 2) : t, tS = hS ? I(x, y - 1) : t;
  const bool so = a.order >= 2;
  const double c0 = Cq[6 * t + 0], c1 = Cq[6 * t + 1], c2 = Cq[6 * t + 2], c3 = Cq[6 * t + 3];
  const double c4 = Cq[6 * t + 4];
  const double cW0 = Cq[6 * tW + 0], cE1 = Cq[6 * tE + 1], cS2 = Cq[6 * tS + 2], cN3 = Cq[6 * tN + 3];
  const double sgs = a.sig_s[c], sbc = a.Sb[c];
  const double gp = a.gphi ? a.gphi[c] : 0.0, gx = a.gFx ? a.gFx[c] : 0.0;
  const double gy = a.gFy ? a.gFy[c] : 0.0;
  // ordinate weights through the constant address space (scalar loads)
  typedef const __attribute__((address_space(4))) double cdouble;
  cdouble *W = (cdouble *)a.w, *WM = (cdouble *)a.wmu, *WE = (cdouble *)a.weta;
  cdouble *AM = (cdouble *)a.amu, *AE = (cdouble *)a.aeta;
  // ordinate kk from its loaded values (rb at the cell and its neighbours,
  // ihb at the cell)
  auto one = [&](int kk, double r0, double rE, double rE2, double rW, double rN, double rN2,
                 double rS, double ih) {
    const double ax = AM[kk], ay = AE[kk];
    double v = ih - c4 * r0;
    double ub = 0.0;
    {
      // Ebar at columns x, x - 1, x + 1 of row y; Nbar likewise
      const double e0 = -ax * (hE ? r0 - rE : r0);
      if (so) {
        ub += e0 * (1.0 - hx * c0 + hx * c1);
        if (hW) ub += (-ax * (rW - r0)) * hx * cW0;
        if (hE) ub -= (-ax * (hE2 ? rE - rE2 : rE)) * hx * cE1;
      } else {
        ub += e0;
      }
      const double n0 = -ay * (hN ? r0 - rN : r0);
      if (so) {
        ub += n0 * (1.0 - hy * c2 + hy * c3);
        if (hS) ub += (-ay * (rS - r0)) * hy * cS2;
        if (hN) ub -= (-ay * (hN2 ? rN - rN2 : rN)) * hy * cN3;
      } else {
        ub += n0;
      }
    }
    v += ub;
    v += W[kk] * sgs * sbc * kInv4Pi;
    double g = 0.0;
    if (a.gphi) g += W[kk] * gp;
    if (a.gFx) g += WM[kk] * gx;
    if (a.gFy) g += WE[kk] * gy;
    a.lam[(size_t)kk * a.N + t] = v + g;
  };
  // four ordinates at a time: every load before any store (the arrays do
  // not overlap, which the compiler cannot see)
  constexpr int U = 4;
  int kk = a.qoff[q];
  const int ke = a.qoff[q + 1];
  for (; kk + U <= ke; kk += U) {
    double r0[U], rE[U], rE2[U], rW[U], rN[U], rN2[U], rS[U], ih[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double *R = a.rb + (size_t)(kk + u) * a.N;
      r0[u] = R[t]; rE[u] = R[tE]; rE2[u] = R[tE2]; rW[u] = R[tW];
      rN[u] = R[tN]; rN2[u] = R[tN2]; rS[u] = R[tS];
      ih[u] = a.ihb[(size_t)(kk + u) * a.N + t];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) one(kk + u, r0[u], rE[u], rE2[u], rW[u], rN[u], rN2[u], rS[u], ih[u]);
  }
  for (; kk < ke; ++kk) {
    const double *R = a.rb + (size_t)kk * a.N;
    one(kk, R[t], R[tE], R[tE2], R[tW], R[tN], R[tN2], R[tS], a.ihb[(size_t)kk * a.N + t]);
  }
}

// Gradient pass, per quadrant and stored cell, summed over the quadrant's
// ordinates: cotangents of the least-squares coefficients (in the caller's
// orientation) from the residual on I* and the wall reconstruction on
// I^{m+1/2}, and -sum_k rb I^{m+1/2} for sigma_t (the sigma_t I term of the
// residual plus the increment-solve diagonal: I* + dI* = I^{m+1/2}).
__global__ void k_a_coef_q(AArgs a) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (t >= a.N) return;
  const int nx = a.nx, ny = a.ny;
  int x, y;
  dg_cell(t, nx, ny, x, y);
  const int c = gcell(a, q, x, y);
  const double *Cq = a.cellq + (size_t)q * a.N * 6;
  (void)Cq;
  const double hx = 0.5 * a.dx, hy = 0.5 * a.dy;
  auto I = [&](int xx, int yy) { return dg_idx(xx, yy, nx, ny); };
  auto dq = [&](int xx, int yy) { return a.delta[gcell(a, q, xx, yy)] * kInv4Pi; };
  const bool he = x + 1 < nx, hw = x > 0, hn = y + 1 < ny, hs = y > 0;
  const long long te = he ? I(x + 1, y) : t, tw = hw ? I(x - 1, y) : t;
  const long long tn = hn ? I(x, y + 1) : t, ts = hs ? I(x, y - 1) : t;
  const double dc = dq(x, y), de = he ? dq(x + 1, y) : 0.0, dw = hw ? dq(x - 1, y) : 0.0;
  const double dn = hn ? dq(x, y + 1) : 0.0, ds = hs ? dq(x, y - 1) : 0.0;
  const bool so = a.order >= 2;
  double cEl = 0, cWl = 0, cNl = 0, cSl = 0, st = 0;
  for (int kk = a.qoff[q]; kk < a.qoff[q + 1]; ++kk) {
    const double *R = a.rb + (size_t)kk * a.N;
    const double *H = a.Ih + (size_t)kk * a.N;
    const double ax = a.amu[kk], ay = a.aeta[kk];
    const double rc = R[t], hc = H[t];
    st -= rc * hc;
    if (!so) continue;
    // residual on I* = I_half + delta/(4 pi)
    const double uc = hc + dc;
    const double gbx = -ax * (he ? rc - R[te] : rc) * hx;
    const double gby = -ay * (hn ? rc - R[tn] : rc) * hy;
    if (he) cEl += gbx * ((H[te] + de) - uc);
    if (hw) cWl -= gbx * ((H[tw] + dw) - uc);
    if (hn) cNl += gby * ((H[tn] + dn) - uc);
    if (hs) cSl -= gby * ((H[ts] + ds) - uc);
    if (a.method == 1) {
      // outflow walls, reconstruction of I_half (no east / north neighbour)
      if (!he && hw) cWl -= a.bfb[face_e(a, q, y)] * fabs(a.wmu[kk]) * hx * (H[tw] - hc);
      if (!hn && hs) cSl -= a.bfb[face_n(a, q, x)] * fabs(a.weta[kk]) * hy * (H[ts] - hc);
    }
  }
  // local east/west are global west/east when the quadrant is mirrored in x
  double *P = a.part + (size_t)q * 5 * a.N;
  P[c] = (q & 1) ? cWl : cEl;
  P[(size_t)a.N + c] = (q & 1) ? cEl : cWl;
  P[2 * (size_t)a.N + c] = (q & 2) ? cSl : cNl;
  P[3 * (size_t)a.N + c] = (q & 2) ? cNl : cSl;
  P[4 * (size_t)a.N + c] = st;
}

// Per cell: coefficient cotangents (all quadrants + the HoT gradient), their
// distance cotangents dbar (cE = dE / (dE^2 + dW^2), cW = dW / (...)), and
// every sigma_t term that involves this cell alone.
__global__ void k_a_grad1(AArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.N) return;
  int i, j;
  cell_ij(c, a.nx, i, j);
  const int nx = a.nx, ny = a.ny, N = a.N;
  double cb[5];
  for (int t = 0; t < 5; ++t) {
    double v = 0.0;
    for (int q = 0; q < 4; ++q) v += a.part[((size_t)q * 5 + t) * N + c];
    cb[t] = v;
  }
  const double sc = a.sig_t[c];
  double st = cb[4];
  const bool he = i + 1 < nx, hw = i > 0, hn = j + 1 < ny, hs = j > 0;
  if (a.method == 1) {
    const double *ph = a.phih;
    const double yx = a.hxb[c] / (3.0 * sc), yy = a.hyb[c] / (3.0 * sc);
    const double u = ph[c];
    if (he) cb[0] += yx * (ph[c + 1] - u);
    if (hw) cb[1] -= yx * (ph[c - 1] - u);
    if (hn) cb[2] += yy * (ph[c + nx] - u);
    if (hs) cb[3] -= yy * (ph[c - nx] - u);
    // HoT = F + grad(phi_half) / (3 sigma_t)
    const double gx = a.cE[c] * ((he ? ph[c + 1] : u) - u) - a.cW[c] * ((hw ? ph[c - 1] : u) - u);
    const double gy = a.cN[c] * ((hn ? ph[c + nx] : u) - u) - a.cS[c] * ((hs ? ph[c - nx] : u) - u);
    st -= (a.hxb[c] * gx + a.hyb[c] * gy) / (3.0 * sc * sc);
    // kappa = 2 / (3 sigma_t h) + 1/4 in b (+A kappa phi_half) and D1 (+A kappa)
    const double b = a.bb[c], pd = a.phih[c] - a.phi[c];
    if (!he) st += a.dy * b * pd * (-2.0 / (3.0 * sc * sc * a.dx));
    if (!hw) st += a.dy * b * pd * (-2.0 / (3.0 * sc * sc * a.dx));
    if (!hn) st += a.dx * b * pd * (-2.0 / (3.0 * sc * sc * a.dy));
    if (!hs) st += a.dx * b * pd * (-2.0 / (3.0 * sc * sc * a.dy));
    // Gamma = 2 / (3 (sigma_c + sigma_nb) h): cotangent -A (bb_c - bb_nb)(phi_c - phi_nb)
    auto gam = [&](int nb, double A, double h) {
      const double sm = sc + a.sig_t[nb];
      const double gb = -A * (b - a.bb[nb]) * (a.phi[c] - a.phi[nb]);
      return gb * (-2.0 / (3.0 * sm * sm * h));
    };
    if (he) st += gam(c + 1, a.dy, a.dx);
    if (hw) st += gam(c - 1, a.dy, a.dx);
    if (hn) st += gam(c + nx, a.dx, a.dy);
    if (hs) st += gam(c - nx, a.dx, a.dy);
  }
  // distances to the shifted points and their cotangents
  double db[4] = {0, 0, 0, 0};
  if (a.alsm) {
    for (int axis = 0; axis < 2; ++axis) {
      const double h = axis == 0 ? a.dx : a.dy;
      const bool hp = axis == 0 ? he : hn, hm = axis == 0 ? hw : hs;
      const int np = axis == 0 ? c + 1 : c + nx, nm = axis == 0 ? c - 1 : c - nx;
      const double dp = hp ? 0.5 * h * (1.0 + a.sig_t[np] / sc) : 0.0;
      const double dm = hm ? 0.5 * h * (1.0 + a.sig_t[nm] / sc) : 0.0;
      const double M = dp * dp + dm * dm;
      if (!(M > 0)) continue;
      const double cbp = cb[2 * axis], cbm = cb[2 * axis + 1];
      const double M2 = M * M;
      const double dbp = cbp * (dm * dm - dp * dp) / M2 + cbm * (-2.0 * dp * dm) / M2;
      const double dbm = cbm * (dp * dp - dm * dm) / M2 + cbp * (-2.0 * dp * dm) / M2;
      db[2 * axis] = hp ? dbp : 0.0;
      db[2 * axis + 1] = hm ? dbm : 0.0;
      // d = h/2 (1 + sigma_nb / sigma_c): own part
      if (hp) st += dbp * (-0.5 * h * a.sig_t[np] / (sc * sc));
      if (hm) st += dbm * (-0.5 * h * a.sig_t[nm] / (sc * sc));
    }
  }
  for (int t = 0; t < 4; ++t) a.dbar[(size_t)t * N + c] = db[t];
  a.stp[c] = st;
}

// sigma_t gradient: own part plus the neighbours' distances that point at
// this cell (d = h/2 (1 + sigma_d / sigma_nb)); then sigma_a, sigma_s, q.
__global__ void k_a_grad2(AArgs a, double *g_sa, double *g_ss, double *g_q) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.N) return;
  int i, j;
  cell_ij(c, a.nx, i, j);
  const int nx = a.nx, ny = a.ny, N = a.N;
  double st = a.stp[c];
  if (a.alsm) {
    // neighbour east of c sees c as its west point, and so on
    if (i + 1 < nx) st += a.dbar[(size_t)1 * N + c + 1] * 0.5 * a.dx / a.sig_t[c + 1];
    if (i > 0) st += a.dbar[(size_t)0 * N + c - 1] * 0.5 * a.dx / a.sig_t[c - 1];
    if (j + 1 < ny) st += a.dbar[(size_t)3 * N + c + nx] * 0.5 * a.dy / a.sig_t[c + nx];
    if (j > 0) st += a.dbar[(size_t)2 * N + c - nx] * 0.5 * a.dy / a.sig_t[c - nx];
  }
  const double Sb = a.Sb[c];
  double sa = 0.0, gq = Sb * kInv4Pi;
  const double ss = a.phi[c] * Sb * kInv4Pi;
  if (a.method == 1) {
    sa -= a.V * a.bb[c] * a.phi[c];
    gq += a.V * a.bb[c];
  }
  if (g_sa) g_sa[c] = sa + st;
  if (g_ss) g_ss[c] = ss + st;
  if (g_q) g_q[c] = gq;
}

inline int nb_(int n) { return (n + kB - 1) / kB; }

}  // namespace

size_t adjoint_args_bytes() { return sizeof(AArgs); }

// Host entry points take the AArgs image built by the plan (see capi.cpp).
void adj_fill_args(const PlanDev &P, const AdjointBuffers &B, const double *gphi,
                   const double *gFx, const double *gFy, void *dst) {
  AArgs a;
  memset(&a, 0, sizeof a);
  a.nx = P.nx; a.ny = P.ny; a.N = P.N; a.K = P.K; a.nbf = P.nbf;
  a.order = P.order; a.alsm = P.alsm; a.method = P.method;
  a.dx = P.dx; a.dy = P.dy; a.V = P.V;
  for (int t = 0; t < 5; ++t) a.qoff[t] = P.qoff[t];
  a.w = P.w; a.wmu = P.wmu; a.weta = P.weta; a.amu = P.amu; a.aeta = P.aeta;
  a.sig_t = P.sig_t; a.sig_s = P.sig_s;
  a.cE = P.cE; a.cW = P.cW; a.cN = P.cN; a.cS = P.cS;
  a.cellq = P.cellq;
  a.sdq = P.sdq;
  a.dso = P.dso;
  a.delta = P.delta; a.phi = P.phi; a.phih = P.phih;
  a.gphi = gphi; a.gFx = gFx; a.gFy = gFy;
  a.lam = B.lam; a.ihb = B.ihb; a.rb = B.rb;
  a.s = B.s; a.s_old = B.s_old; a.bb = B.bb; a.hxb = B.hxb; a.hyb = B.hyb; a.phb = B.phb;
  a.Sb = B.Sb; a.bfb = B.bfb; a.part = B.part; a.dbar = B.dbar; a.stp = B.stp; a.errp = B.errp;
  a.hand = P.hand;
  a.hand_err = P.state + 4;
  memcpy(dst, &a, sizeof a);
}

// lambda <- G^T lambda + M^T g (ihalf_src: the stored I^{m+1/2} buffer).
// With hist, Err of s against the previous s goes to hist[m].
void adj_launch_pass(const PlanDev &P, const AdjointBuffers &B, const void *args,
                     const double *ihalf, const SynthSet &S, double *hist, int m,
                     int32_t *host_flag, hipStream_t s) {
  AArgs a = *reinterpret_cast<const AArgs *>(args);
  a.Ih = ihalf;
  const int N = P.N, nb = nb_(N);
  hipLaunchKernelGGL(k_a_qsum, dim3(nb, 4), dim3(kB), 0, s, a, (const double *)a.lam);
  hipLaunchKernelGGL(k_a_combine, dim3(nb), dim3(kB), 0, s, a, a.s, kInv4Pi, hist ? 1 : 0);
  if (hist) hipLaunchKernelGGL(k_a_err, dim3(1), dim3(kB), 0, s, a, nb, hist, m);
  if (P.method == GSIS_GSIS) {
    launch_synth_solve(S, s, host_flag, 0);
    hipLaunchKernelGGL(k_a_hbar, dim3(nb), dim3(kB), 0, s, a);
    hipLaunchKernelGGL(k_a_phbar, dim3(nb), dim3(kB), 0, s, a, (const double *)P.kappa);
  }
  hipLaunchKernelGGL(k_a_ihalf, dim3(nb, 4), dim3(kB), 0, s, a);
  int rows = ((P.ny + 63) / 64) * 64;
  if (rows > 1024) rows = 1024;
  if (P.chain_parts > 1)
    hipLaunchKernelGGL(k_a_chain<true>, dim3(P.chain_parts * P.K), dim3(P.chain_rows), 0, s, a,
                       P.chain_parts);
  else if (P.ny <= kAMaxW * 64)
    hipLaunchKernelGGL(k_a_chain<false>, dim3(P.K), dim3(rows), 0, s, a, 1);
  else hipLaunchKernelGGL(k_a_sweep, dim3(P.K), dim3(rows), 0, s, a);
  hipLaunchKernelGGL(k_a_qsum, dim3(nb, 4), dim3(kB), 0, s, a, (const double *)a.rb);
  hipLaunchKernelGGL(k_a_combine, dim3(nb), dim3(kB), 0, s, a, a.Sb, 1.0, 0);
  hipLaunchKernelGGL(k_a_out, dim3(nb, 4), dim3(kB), 0, s, a);
  (void)B;
}

// dJ/dp from the quantities the last pass left (bb, hb, phb, bfb, rb, Sb).
void adj_launch_gradient(const PlanDev &P, const void *args, const double *ihalf,
                         double *g_sa, double *g_ss, double *g_q, hipStream_t s) {
  AArgs a = *reinterpret_cast<const AArgs *>(args);
  a.Ih = ihalf;
  const int N = P.N, nb = nb_(N);
  hipLaunchKernelGGL(k_a_coef_q, dim3(nb, 4), dim3(kB), 0, s, a);
  hipLaunchKernelGGL(k_a_grad1, dim3(nb), dim3(kB), 0, s, a);
  hipLaunchKernelGGL(k_a_grad2, dim3(nb), dim3(kB), 0, s, a, g_sa, g_ss, g_q);
}

}  // namespace gsis
