// kernels_synth.hip -- macroscopic (synthetic) step of GSIS on gfx950.
//
//  hot     : HoT_c = F_c + grad(phi)_c / (3 sigma_t) with the adaptive
//            least-squares gradient (Eqs. GSIS_HoT, LSF_mdf); right-hand side
//            b_c = V q - sum_int A 1/2 (HoT_c + HoT_nb).n
//                  - sum_bnd A (F_T.n - kappa phi_half)        (Eqs. MSE_d, Fij_d,
//                                                  macro_bc_delta_flux),
//            formed by the kernel that starts the CG
//  solve   : D1 phi' = b, D1 = V sigma_a + sum_int A Gamma (.) + sum_bnd A kappa
//            (Eqs. Gamma_ij_def, MSE_d_mtx1, elem_mtx_M, Gamma_ij_com2), by
//            CG (one reduction per iteration, the Chronopoulos-Gear form)
//            preconditioned with a geometric multigrid V-cycle (2x2
//            aggregation, Galerkin coarse operators, red-black Gauss-Seidel
//            smoothing, dense inverse on the coarsest level).
//  update  : delta = phi' - phi_half (Eq. GSIS_update, applied lazily by the
//            transport kernels), Err (Eq. Err_W), next source.
//
// Every kernel takes its problem from a SynthDesc record. A launch covers one
// problem (block table NULL) or many: the table maps each block to (problem,
// block of that problem), so the problems of a batch advance together while
// each keeps its own CG scalars, multigrid hierarchy and stop flags.
// All reductions are two-stage with a fixed order, so results repeat bit for
// bit, and a problem gets the same numbers alone or in a batch.
#include "gsis_internal.h"

#include <algorithm>
#include <cstring>

namespace gsis {
namespace {

constexpr int kRedBlock = 256;

// v of the lane given by DPP control C (a permutation within rows of 16)
template <int C>
__device__ inline double dpp_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, C, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), C, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline double read_lane(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Sum over a full wave in a fixed order: quads by the lane permutations
// xor 1 and xor 2 (every lane of a quad ends with the same sum, as addition
// commutes exactly), the four quads of a row by rotations of 4 and 8, then
// the four rows' sums read as scalars and added pairwise.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x124>(v);   // row_ror:4
  v += dpp_d<0x128>(v);   // row_ror:8
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum over the block (every lane of it active, blockDim a multiple of 64):
// wave sums, then the waves' sums in wave order. Every thread gets the same
// value; sh needs one entry per wave.
__device__ inline double block_sum(double v, double *sh) {
  const double w = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
  __syncthreads();
  double r = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
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

// Problem descriptors and block tables are read through the constant
// address space: they do not change while a kernel runs, so their
// (wave-uniform) fields become scalar loads served by the scalar cache
// rather than vector loads, each of which would cost a memory round trip.
typedef __attribute__((address_space(4))) const SynthDesc CDesc;
__device__ inline CDesc &cdesc(const SynthDesc *ds, int p) { return ((CDesc *)ds)[p]; }
// a level's record copied out of a descriptor field by field
__device__ inline LevelDev level(CDesc &D, int l) {
  __attribute__((address_space(4))) const LevelDev &s = D.lev[l];
  LevelDev L;
  L.nx = s.nx; L.ny = s.ny; L.fx = s.fx; L.fy = s.fy;
  L.dg = s.dg; L.ax = s.ax; L.ay = s.ay; L.x = s.x; L.b = s.b; L.xs = s.xs;
  return L;
}

// The block's problem and its block index within that problem.
struct Blk { int p, lb; };
__device__ inline Blk blk(const int2 *bt) {
  if (!bt) return {0, (int)blockIdx.x};
  const __attribute__((address_space(4))) int *q = (const __attribute__((address_space(4))) int *)bt;
  return {q[2 * blockIdx.x], q[2 * blockIdx.x + 1]};
}

// ---------------------------------------------------------------- HoT / RHS
// COMBINE: phi and F of I^{m+1/2} are first summed from the four quadrant
// partials (for the cell and, phi only, its neighbours; quadrants in order,
// plus the FP32-mixed base term), and the cell's values stored.
template <bool COMBINE>
__global__ void k_hot(const SynthDesc *ds, const int2 *bt) {
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1];   // tested after the operands are loaded
  const int nx = D.nx, ny = D.ny, N = D.N;
  const int c = B.lb * kRedBlock + threadIdx.x;
  if (c >= N) return;
  int i, j;
  cell_ij(c, nx, i, j);
  const int ce = i + 1 < nx ? c + 1 : c, cw = i > 0 ? c - 1 : c;
  const int cn = j + 1 < ny ? c + nx : c, cs = j > 0 ? c - nx : c;
  double u, ue, uw, un, us, fx, fy;
  if (COMBINE) {
    const double *P = D.mom_part;
    auto phi_at = [&](int cc) {
      double s0 = 0.0;
      for (int q = 0; q < 4; ++q) s0 += P[(size_t)(3 * q) * N + cc];
      if (D.fp32) s0 += D.phi[cc] / kFourPi * D.sw;
      return s0;
    };
    u = phi_at(c); ue = phi_at(ce); uw = phi_at(cw); un = phi_at(cn); us = phi_at(cs);
    double sx = 0.0, sy = 0.0;
    for (int q = 0; q < 4; ++q) {
      sx += P[(size_t)(3 * q + 1) * N + c];
      sy += P[(size_t)(3 * q + 2) * N + c];
    }
    if (D.fp32) {
      const double sub = D.phi[c] / kFourPi;
      sx += sub * D.swm;
      sy += sub * D.swe;
    }
    fx = sx; fy = sy;
  } else {
    const double *phih = D.phih;
    u = phih[c]; ue = phih[ce]; uw = phih[cw]; un = phih[cn]; us = phih[cs];
    fx = D.Fx[c]; fy = D.Fy[c];
  }
  double hx, hy;
  if (D.hot_face) {
    // transport face fluxes on the cell's east and north faces (sums of the
    // four quadrant partials, in order) minus the compact diffusion flux
    // Gamma_f (phi_c - phi_nb); A Gamma_f is the operator's off-diagonal
    const double *FT = D.ftp;
    double tx = 0.0, ty = 0.0;
    for (int q = 0; q < 4; ++q) {
      tx += FT[(size_t)(2 * q) * N + c];
      ty += FT[(size_t)(2 * q + 1) * N + c];
    }
    const double gE = D.lev[0].ax[c] / D.dy, gN = D.lev[0].ay[c] / D.dx;
    hx = i + 1 < nx ? tx - gE * (u - ue) : 0.0;
    hy = j + 1 < ny ? ty - gN * (u - un) : 0.0;
  } else {
    const double gx = D.cE[c] * (ue - u) - D.cW[c] * (uw - u);
    const double gy = D.cN[c] * (un - u) - D.cS[c] * (us - u);
    hx = fx + gx / (3.0 * D.sig_t[c]);
    hy = fy + gy / (3.0 * D.sig_t[c]);
  }
  if (f1 != 0) return;
  if (COMBINE) {
    D.phih[c] = u;
    D.Fx[c] = fx;
    D.Fy[c] = fy;
  }
  D.hx[c] = hx;
  D.hy[c] = hy;
}

// The time-dependent form's material temperature of sub-iteration sub: T^m,
// then the sub-iterates in two alternating buffers.
__device__ inline double *t_sub(CDesc &D, int sub) {
  return sub == 0 ? D.Tm : ((sub - 1) & 1) ? D.Tsub1 : D.Tsub0;
}

// b_c of cell c = (i, j) from the HoT of the cell and its neighbours (central
// faces), or from the face values h of its faces (transport faces: hx[c] on
// the cell's east face, hy[c] on its north face, normals +x, +y). The
// time-dependent form adds V (rho^n / (c dt) + sigma_a a c T^4) with T the
// temperature Ts of the sub-iteration (D1 carries V / (c dt) on its diagonal):
// then D1 rho' = b is D1 d_rho = R1 of Eqs. MSE_d1, R1_def at rho' = rho + d_rho.
__device__ inline double rhs_at(CDesc &D, int c, int i, int j, const double *Ts) {
  const int nx = D.nx, ny = D.ny;
  const double dx = D.dx, dy = D.dy;
  const double *hx = D.hx, *hy = D.hy, *bflux = D.bflux, *kappa = D.kappa;
  const double ph = D.phih[c];
  const bool tf = D.hot_face != 0;
  double s = dx * dy * D.q[c];
  if (D.td) {
    const double T = Ts[c], T2 = T * T;
    s += dx * dy * (D.rho_n[c] * D.tdiag + D.sig_a[c] * (D.ca * (T2 * T2)));
  }
  // east / west (area dy), north / south (area dx)
  if (i + 1 < nx) s -= dy * (tf ? hx[c] : 0.5 * (hx[c] + hx[c + 1]));
  else s -= dy * (bflux[ny + j] - kappa[ny + j] * ph);
  if (i > 0) s += dy * (tf ? hx[c - 1] : 0.5 * (hx[c] + hx[c - 1]));
  else s -= dy * (bflux[j] - kappa[j] * ph);
  if (j + 1 < ny) s -= dx * (tf ? hy[c] : 0.5 * (hy[c] + hy[c + nx]));
  else s -= dx * (bflux[2 * ny + nx + i] - kappa[2 * ny + nx + i] * ph);
  if (j > 0) s += dx * (tf ? hy[c - nx] : 0.5 * (hy[c] + hy[c - nx]));
  else s -= dx * (bflux[2 * ny + i] - kappa[2 * ny + i] * ph);
  return s;
}

// Scalar slots. r.z of CG iteration k sits in slot rz_slot(k) (two
// alternating slots, so a kernel can read iteration k-1's value while its
// block 0 stores iteration k's).
enum { S_RZ = 0, S_ZW = 1, S_RR = 2, S_BB = 3, S_ALPHA = 4, S_BETA = 5, S_STOP = 6,
       S_NIT = 7, S_RZ1 = 8, S_ALPHA1 = 9, S_VCYCLES = 10 };
__host__ __device__ inline int rz_slot(int k) { return (k & 1) ? S_RZ1 : S_RZ; }
__host__ __device__ inline int alpha_slot(int k) { return (k & 1) ? S_ALPHA1 : S_ALPHA; }

// r of V-cycle v (v = 0 after the warm start, v = it + 1 after CG iteration
// it): the buffers alternate, so a kernel that forms r_{v} for its tile and
// halo never overwrites the r_{v-1} that neighbouring tiles still read.
__device__ inline double *cg_rv(CDesc &D, int v) { return (v & 1) ? D.cg_r2 : D.cg_r; }

// CG kernels run unless the outer iteration is done (state[1]) or this
// synthetic solve has converged (state[3]).
__device__ inline bool cg_off(const int32_t *st) { return st[1] != 0 || st[3] != 0; }

inline int nblk(int n) { return (n + kRedBlock - 1) / kRedBlock; }
__host__ __device__ inline int nblk_d(int n) { return (n + kRedBlock - 1) / kRedBlock; }

// Block partials of a problem's reductions, in separate regions of its red
// array (nb = level-0 blocks of 256 cells): [0, nb) r.r, [nb, 2 nb) b.b,
// then three regions of ntp = max(nb, level-0 tiles) slots: r.z (one per
// level-0 tile, or per block of cells when the whole V-cycle ran in one
// workgroup), r.r once more, one per level-0 tile, from the tile kernel
// that makes the CG update, and z.Az (like r.z). A reduction is finished by the
// kernel that needs its value: every block of it sums the partials in the
// same fixed order, so all blocks hold the same number and results repeat
// bit for bit; block 0 stores it for later kernels. This saves a launch
// per reduction (folding the finish into the producing kernel instead would
// need a device-scope release per block, which on a GPU whose XCDs each
// have their own L2 writes back the L2 every time).
__device__ inline double *red_rr(CDesc &D) { return D.red; }
__device__ inline double *red_bb(CDesc &D) { return D.red + nblk_d(D.N); }
__device__ inline double *red_rz(CDesc &D) { return D.red + 2 * nblk_d(D.N); }
__device__ inline double *red_rrt(CDesc &D) { return D.red + 2 * nblk_d(D.N) + D.ntp; }
__device__ inline double *red_zw(CDesc &D) { return D.red + 2 * nblk_d(D.N) + 2 * D.ntp; }
__device__ inline int n_rz(CDesc &D) { return D.lc == 0 ? nblk_d(D.N) : D.ntile0; }

// The thread's first partial, loaded early (before a kernel waits for its
// flags), and the sum of all n partials: thread t adds p[t], p[t + blockDim],
// ... in that order, then block_sum.
__device__ inline double first_partial(const double *p, int n) {
  return (int)threadIdx.x < n ? p[threadIdx.x] : 0.0;
}
__device__ inline double sum_partials(const double *p, int n, double *sh, double first) {
  double v = 0.0;
  v += first;
  // sixteen loads in flight at a time, added in order (terms past n add 0)
  constexpr int U = 16;
  for (int t0 = threadIdx.x + blockDim.x; t0 < n; t0 += U * (int)blockDim.x) {
    double w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      w[u] = t < n ? p[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v += w[u];
  }
  return block_sum(v, sh);
}

// r.r of the iterate just updated (partials per level-0 tile when the tile
// kernel made the update, else per block of cells): iteration count and
// convergence test against STOP; first (after the warm start): also b.b,
// the count reset and STOP = max(rtol^2 r0.r0, 1e-28 b.b). Every thread of
// the block returns the same decision; thread 0 stores the scalars and the
// flag. Its operands can be loaded early (rr_prefetch), before the caller
// waits for its flags.
struct RRPre {
  double rr, bb, stop;
};
__device__ inline RRPre rr_prefetch(CDesc &D, bool first, bool tiles) {
  const int nb = nblk_d(D.N);
  RRPre q;
  q.rr = tiles ? first_partial(red_rrt(D), D.ntile0) : first_partial(red_rr(D), nb);
  q.bb = first ? first_partial(red_bb(D), nb) : 0.0;
  q.stop = D.scal[S_STOP];
  return q;
}
__device__ inline bool finish_rr(CDesc &D, bool first, bool tiles, double *sh, const RRPre &q) {
  const int nb = nblk_d(D.N);
  const double rr = tiles ? sum_partials(red_rrt(D), D.ntile0, sh, q.rr)
                          : sum_partials(red_rr(D), nb, sh, q.rr);
  double stop;
  double bb = 0.0;
  if (first) {
    bb = sum_partials(red_bb(D), nb, sh, q.bb);
    stop = fmax(D.rtol * D.rtol * rr, 1e-28 * bb);
  } else {
    stop = q.stop;
  }
  const bool conv = !(rr > stop);
  if (threadIdx.x == 0) {
    double *scal = D.scal;
    scal[S_RR] = rr;
    if (first) {
      scal[S_BB] = bb;
      scal[S_STOP] = stop;
    }
    const double nit = first ? 0.0 : scal[S_NIT] + 1.0;
    scal[S_NIT] = nit;
    // converged: 1 + the CG iterations it took (the host's next check point)
    if (conv) D.state[3] = 1 + (int32_t)nit;
  }
  return conv;
}

// The r.r test of the last CG iteration when the iteration cap ends the
// solve (one workgroup per problem).
__global__ void k_finish_rr(const SynthDesc *ds) {
  __shared__ double sh[kRedBlock];
  CDesc &D = cdesc(ds, blockIdx.x);
  const RRPre q = rr_prefetch(D, false, false);
  if (cg_off(D.state)) return;
  (void)finish_rr(D, false, false, sh, q);
}

// The r.r test of CG iteration v - 1 (v > 0) on its level-0 tile partials,
// for a problem whose V-cycle starts with a tile level: the test the level-1
// kernel of V-cycle v would make, run on its own when the host is about to
// look at the flags (that V-cycle's later kernels, which the test would
// usually turn into no-ops, are then launched only if it fails).
__global__ void k_rr_test(const SynthDesc *ds) {
  __shared__ double sh[kRedBlock];
  CDesc &D = cdesc(ds, blockIdx.x);
  const RRPre q = rr_prefetch(D, false, true);
  if (cg_off(D.state)) return;
  (void)finish_rr(D, false, true, sh, q);
}

// Start of a synthetic solve: warm start x = phi, clear the converged flag;
// r = b - A x; partials of r.r and b.b.
// RHS: the right-hand side b is formed here from the HoT (and stored)
// rather than read.
// MODE 0: b given in rhs (the adjoint), warm start phi; 1: b from the HoT
// (rhs_at), warm start phi; 3: as 1 with the level-0 iterate as warm start
// (the time-dependent form's later sub-iterations); 2: the face-averaged
// balance (Eq. Fij_d) by a
// defect-correction sub-iteration: b = rhs_at + corr(x) with x the level-0
// iterate, which is also the warm start, and corr_c = sum over interior
// faces of a_f (x_c - x_nb) + A_f (w_c + w_nb) . n_f / 2, a_f = A_f Gamma_f
// the operator's off-diagonals and w = grad(x) / (3 sigma_t) from
// k_wide_grad: then D1 x' = b is D1 (x' - x) = R1(x).
template <int MODE>
__global__ void k_cg_begin(const SynthDesc *ds, const int2 *bt, int sub) {
  __shared__ double sh[kRedBlock];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1];   // tested after the operands are loaded
  const int c = B.lb * kRedBlock + threadIdx.x;
  const LevelDev L = level(D, 0);
  const bool in = c < D.N;
  const int cc = in ? c : 0;
  int i, j;
  cell_ij(cc, L.nx, i, j);
  const bool hE = i + 1 < L.nx, hW = i > 0, hN = j + 1 < L.ny, hS = j > 0;
  // warm start x for the cell and its neighbours (this kernel writes x)
  const double *X = MODE >= 2 ? L.x : D.phi;
  const double xc = X[cc], xe = X[hE ? cc + 1 : cc], xw = X[hW ? cc - 1 : cc];
  const double xn = X[hN ? cc + L.nx : cc], xs = X[hS ? cc - L.nx : cc];
  const double dg = L.dg[cc], aE = L.ax[cc], aW = L.ax[hW ? cc - 1 : cc];
  const double aN = L.ay[cc], aS = L.ay[hS ? cc - L.nx : cc];
  double b = MODE != 0 ? rhs_at(D, cc, i, j, D.td ? t_sub(D, sub) : nullptr) : D.rhs[cc];
  if (MODE == 2) {
    const double *WX = D.wx, *WY = D.wy;
    const double wxc = WX[cc], wyc = WY[cc];
    const double hdy = 0.5 * D.dy, hdx = 0.5 * D.dx;
    double corr = 0.0;
    if (hE) corr += aE * (xc - xe) + hdy * (wxc + WX[cc + 1]);
    if (hW) corr += aW * (xc - xw) - hdy * (wxc + WX[cc - 1]);
    if (hN) corr += aN * (xc - xn) + hdx * (wyc + WY[cc + L.nx]);
    if (hS) corr += aS * (xc - xs) - hdx * (wyc + WY[cc - L.nx]);
    b += corr;
  }
  if (f1 != 0) return;
  double rr = 0.0, bb = 0.0;
  if (in) {
    double y = dg * xc;
    if (hE) y -= aE * xe;
    if (hW) y -= aW * xw;
    if (hN) y -= aN * xn;
    if (hS) y -= aS * xs;
    const double rc = b - y;
    if (MODE != 0) D.rhs[c] = b;
    L.x[c] = xc;
    D.cg_r[c] = rc;
    rr = rc * rc;
    bb = b * b;
  }
  if (B.lb == 0 && threadIdx.x == 0) D.state[3] = 0;
  double t = block_sum(rr, sh);
  if (threadIdx.x == 0) red_rr(D)[B.lb] = t;
  t = block_sum(bb, sh);
  if (threadIdx.x == 0) red_bb(D)[B.lb] = t;
}

// w = grad(x) / (3 sigma_t) of the level-0 iterate (the HoT's gradient
// coefficients), for the face-averaged balance; FIRST: x = phi^{m+1/2},
// also copied into the iterate (the sub-iterations start there).
template <bool FIRST>
__global__ void k_wide_grad(const SynthDesc *ds, const int2 *bt) {
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1];   // tested after the operands are loaded
  const int nx = D.nx, ny = D.ny;
  const int c = B.lb * kRedBlock + threadIdx.x;
  if (c >= D.N) return;
  int i, j;
  cell_ij(c, nx, i, j);
  const LevelDev L = level(D, 0);
  const double *X = FIRST ? D.phih : L.x;
  const double u = X[c];
  const double ue = i + 1 < nx ? X[c + 1] : u, uw = i > 0 ? X[c - 1] : u;
  const double un = j + 1 < ny ? X[c + nx] : u, us = j > 0 ? X[c - nx] : u;
  const double gx = D.cE[c] * (ue - u) - D.cW[c] * (uw - u);
  const double gy = D.cN[c] * (un - u) - D.cS[c] * (us - u);
  const double s3 = 3.0 * D.sig_t[c];
  if (f1 != 0) return;
  D.wx[c] = gx / s3;
  D.wy[c] = gy / s3;
  if (FIRST) L.x[c] = u;
}

// CG in the form of Chronopoulos and Gear: the V-cycle of iteration it
// gives z = M r and, on its finest level, w = A z with partials of
// gamma = r.z and delta = z.w in one pass, so an iteration needs a single
// global reduction. Then
//   beta = gamma / gamma_prev (0 on the first iteration),
//   alpha = gamma / (delta - beta gamma / alpha_prev) (gamma / delta first),
//   p = z + beta p, s = w + beta s (= A p), x += alpha p, r -= alpha s,
// which is preconditioned CG with A p carried by a recurrence instead of a
// product. s alternates between two buffers with the parity of it.
struct CGCoef {
  double be, al;
};
__device__ inline CGCoef cg_coef(bool first, double ga, double de, double ga_prev,
                                 double al_prev) {
  if (first) return {0.0, ga / de};
  const double be = ga / ga_prev;
  return {be, ga / (de - be * ga / al_prev)};
}
__device__ inline double *cg_s(CDesc &D, int it) { return (it & 1) ? D.cg_s1 : D.cg_s0; }
// the update's scalar operands, loaded before the caller waits for its flags
// (coef_sep: the coefficients themselves, from k_cg_coef)
struct UpdPre {
  double rz0, zw0, ga_prev, al_prev;
};
__device__ inline UpdPre upd_prefetch(CDesc &D, int it) {
  UpdPre q;
  if (D.coef_sep) {
    q.rz0 = it > 0 ? D.scal[S_BETA] : 0.0;
    q.zw0 = D.scal[alpha_slot(it)];
    q.ga_prev = q.al_prev = 0.0;
    return q;
  }
  q.rz0 = first_partial(red_rz(D), n_rz(D));
  q.zw0 = first_partial(red_zw(D), n_rz(D));
  q.ga_prev = it > 0 ? D.scal[rz_slot(it - 1)] : 1.0;
  q.al_prev = it > 0 ? D.scal[alpha_slot(it - 1)] : 1.0;
  return q;
}
// every block forms the coefficients from the same partials in the same
// order; block 0 stores gamma, delta, alpha and beta. With many partials
// (coef_sep) one workgroup does this in k_cg_coef instead, in the same
// order, and the blocks take the stored beta and alpha.
__device__ inline CGCoef upd_coef(CDesc &D, const Blk &B, int it, const UpdPre &q, double *sh) {
  if (D.coef_sep) return {q.rz0, q.zw0};
  const double ga = sum_partials(red_rz(D), n_rz(D), sh, q.rz0);
  const double de = sum_partials(red_zw(D), n_rz(D), sh, q.zw0);
  const CGCoef k = cg_coef(it == 0, ga, de, q.ga_prev, q.al_prev);
  if (B.lb == 0 && threadIdx.x == 0) {
    D.scal[rz_slot(it)] = ga;
    D.scal[alpha_slot(it)] = k.al;
    D.scal[S_BETA] = k.be;
    D.scal[S_ZW] = de;
  }
  return k;
}

// CG coefficients of iteration it for the problems whose level-0 tiles are
// many (coef_sep): one workgroup per problem sums the r.z and z.w partials
// (the order of upd_coef) and stores gamma, delta, alpha and beta, so each
// block of the update reads two scalars instead of every partial. Launched
// after V-cycle it.
constexpr int kCoefSepTiles = 2048;
__global__ void __launch_bounds__(kRedBlock) k_cg_coef(const SynthDesc *ds, int it) {
  __shared__ double sh[kRedBlock];
  CDesc &D = cdesc(ds, blockIdx.x);
  if (!D.coef_sep) return;
  UpdPre q;
  q.rz0 = first_partial(red_rz(D), n_rz(D));
  q.zw0 = first_partial(red_zw(D), n_rz(D));
  q.ga_prev = it > 0 ? D.scal[rz_slot(it - 1)] : 1.0;
  q.al_prev = it > 0 ? D.scal[alpha_slot(it - 1)] : 1.0;
  if (cg_off(D.state)) return;
  const double ga = sum_partials(red_rz(D), n_rz(D), sh, q.rz0);
  const double de = sum_partials(red_zw(D), n_rz(D), sh, q.zw0);
  const CGCoef k = cg_coef(it == 0, ga, de, q.ga_prev, q.al_prev);
  if (threadIdx.x == 0) {
    D.scal[rz_slot(it)] = ga;
    D.scal[alpha_slot(it)] = k.al;
    D.scal[S_BETA] = k.be;
    D.scal[S_ZW] = de;
  }
}

// CG iteration it on every cell of a problem, with the partial of r.r.
// With all = 0 only problems whose whole V-cycle runs in the one-workgroup
// kernel take part: for the others the level-0 tile kernel of the next
// V-cycle makes the update (cg_update_tile).
__global__ void k_cg_update(const SynthDesc *ds, const int2 *bt, int it, int all) {
  __shared__ double sh[kRedBlock];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  if (!all && D.lc > 0) return;
  const int32_t f1 = D.state[1], f3 = D.state[3];
  const int c = B.lb * kRedBlock + threadIdx.x;
  double *x = D.lev[0].x;
  const bool in = c < D.N;
  const int cc = in ? c : 0;
  const double zc = D.cg_z[cc], wc = D.cg_w[cc], xc = x[cc], rc0 = cg_rv(D, it)[cc];
  const double pc0 = it > 0 ? D.cg_p[cc] : 0.0, sc0 = it > 0 ? cg_s(D, it - 1)[cc] : 0.0;
  const UpdPre q = upd_prefetch(D, it);
  if (f1 != 0 || f3 != 0) return;
  const CGCoef k = upd_coef(D, B, it, q, sh);
  double v = 0.0;
  if (in) {
    const double pc = it > 0 ? fma(k.be, pc0, zc) : zc;
    const double sc = it > 0 ? fma(k.be, sc0, wc) : wc;
    D.cg_p[c] = pc;
    cg_s(D, it)[c] = sc;
    x[c] = fma(k.al, pc, xc);
    const double rc = fma(-k.al, sc, rc0);
    cg_rv(D, it + 1)[c] = rc;
    v = rc * rc;
  }
  double t = block_sum(v, sh);
  if (threadIdx.x == 0) red_rr(D)[B.lb] = t;
}

// ------------------------------------------------------------ multigrid
// Level l of a problem: vectors x, b are the CG's z, r on level 0 (r of
// V-cycle v).
__device__ inline double *lev_x(CDesc &D, int l) { return l == 0 ? D.cg_z : D.lev[l].x; }
__device__ inline const double *lev_b(CDesc &D, int l, int v) {
  return l == 0 ? cg_rv(D, v) : D.lev[l].b;
}

// Fine multigrid levels, one tile of kTW x kTH cells per workgroup (one
// thread per cell) with a ring of kHalo cells around it in LDS. Red-black
// Gauss-Seidel uses the colour (i + j) & 1 of the level (0 red, 1 black).
//
//  down: one V(1,1) pre-smoothing from x = 0 -- red x = b / d, then black
//        x = (b + sum a x_nb) / d -- then r = b - A x and the coarse
//        b = sum of r over each aggregate's fx x fy children. Starting from
//        zero makes every value a function of b, d and the couplings within
//        two cells, so the tile and its ring are computed without waiting
//        for other workgroups. The pre-smoothed x of the tile goes to the
//        level's spare vector xs, not to x. On level 0 after a CG step it
//        also makes that step's update (cg_update_tile): b = r_new =
//        r_old - alpha (w + beta s_old) is formed on the whole region from
//        r_old, w and s_old, which earlier kernels left complete.
//  up:   black x = (b + sum a (xs_nb + omega e_parent(nb))) / d with the
//        coarse correction e, then red x = (b + sum a x_nb) / d; the black
//        ring is recomputed so the red cells of the tile see final
//        neighbours. Level 0 has its own kernel (k_mg_up0). It
//        reads the pre-smoothed xs of the ring and writes the final x into a
//        different array, so tiles running later never see a neighbour's
//        final values in place of its pre-smoothed ones.
// Cells outside the level hold d = 1, b = 0 and no couplings.
constexpr int kTW = 32, kTH = 8, kHalo = 2;
constexpr int kRW = kTW + 2 * kHalo, kRH = kTH + 2 * kHalo, kRN = kRW * kRH;
static_assert(kTW * kTH == kRedBlock, "one thread per tile cell");

struct Tile {
  int nx, ny, i0, j0;
};
__device__ inline Tile tile_of(const LevelDev &L, int lb) {
  const int tx = (L.nx + kTW - 1) / kTW;
  int ti, tj;
  cell_ij(lb, tx, ti, tj);
  return {L.nx, L.ny, ti * kTW - kHalo, tj * kTH - kHalo};
}

// b, d and the east / north couplings of the region into LDS (blockDim =
// kRedBlock); AP: also ap (and ap2 unless NULL) of the region into sap
// (sap2); XC: also the pre-smoothed
// x plus the scaled coarse correction, xs + omega e(parent), into sxc. Every
// load of the thread is issued (at a clamped, valid index) before any is
// waited for, so the region costs one memory round trip.
constexpr int kRegionPer = (kRN + kRedBlock - 1) / kRedBlock;
template <bool AP, bool XC>
__device__ inline void load_region_t(const LevelDev &L, const double *b, const Tile &T,
                                     double *sb, double *sd, double *sax, double *say,
                                     const double *ap, double *sap, const double *xs,
                                     const double *e, int enx, int sx_, int sy_, double omega,
                                     double *sxc, const double *ap2 = nullptr,
                                     double *sap2 = nullptr) {
  double vb[kRegionPer], vd[kRegionPer], vx[kRegionPer], vy[kRegionPer];
  double va[kRegionPer], va2[kRegionPer], vs[kRegionPer], ve[kRegionPer];
  bool in[kRegionPer], hx[kRegionPer], hy[kRegionPer];
#pragma unroll
  for (int k = 0; k < kRegionPer; ++k) {
    const int r = threadIdx.x + k * kRedBlock;
    int ri, rj;
    cell_ij(r, kRW, ri, rj);
    const int gi = T.i0 + ri, gj = T.j0 + rj;
    in[k] = r < kRN && gi >= 0 && gi < T.nx && gj >= 0 && gj < T.ny;
    hx[k] = gi + 1 < T.nx;
    hy[k] = gj + 1 < T.ny;
    const int g = in[k] ? gj * T.nx + gi : 0;
    vb[k] = b[g]; vd[k] = L.dg[g]; vx[k] = L.ax[g]; vy[k] = L.ay[g];
    if (AP) va[k] = ap[g];
    if (AP) va2[k] = ap2 ? ap2[g] : 0.0;
    if (XC) {
      vs[k] = xs[g];
      ve[k] = e[in[k] ? (gj >> sy_) * enx + (gi >> sx_) : 0];
    }
  }
#pragma unroll
  for (int k = 0; k < kRegionPer; ++k) {
    const int r = threadIdx.x + k * kRedBlock;
    if (r >= kRN) continue;
    sb[r] = in[k] ? vb[k] : 0.0;
    sd[r] = in[k] ? vd[k] : 1.0;
    sax[r] = in[k] && hx[k] ? vx[k] : 0.0;
    say[r] = in[k] && hy[k] ? vy[k] : 0.0;
    if (AP) sap[r] = in[k] ? va[k] : 0.0;
    if (AP && sap2) sap2[r] = in[k] ? va2[k] : 0.0;
    if (XC) {
      double t = 0.0;
      if (in[k]) {
        t = vs[k];
        t += omega * ve[k];
      }
      sxc[r] = t;
    }
  }
}
__device__ inline void load_region(const LevelDev &L, const double *b, const Tile &T, double *sb,
                                   double *sd, double *sax, double *say) {
  load_region_t<false, false>(L, b, T, sb, sd, sax, say, nullptr, nullptr, nullptr, nullptr, 0,
                              0, 0, 0.0, nullptr);
}

// The CG update of iteration it = v - 1 folded into the level-0 tile kernel
// of V-cycle v: beta and alpha from the r.z and z.w partials (every block
// sums them in the same order), then on the region held in LDS s = w + beta
// s_old (sw holds w, ss s_old; afterwards ss holds s) and r_v = r_{v-1} -
// alpha s (sb holds r_{v-1}, afterwards r_v); for the tile's own cells p =
// z + beta p, x += alpha p, s and r_v to global and a partial of r_v . r_v.
// zc, pc0, xc: the cell's z, p and x; q: the update's scalars, all loaded
// early.
__device__ inline void cg_update_tile(CDesc &D, const Blk &B, const Tile &T, int v, double *sb,
                                      const double *sw, double *ss, double zc, double pc0,
                                      double xc, const UpdPre &q, double *sh) {
  const int it = v - 1;
  const CGCoef k = upd_coef(D, B, it, q, sh);
  for (int r = threadIdx.x; r < kRN; r += blockDim.x) {
    const double sv = it > 0 ? fma(k.be, ss[r], sw[r]) : sw[r];
    ss[r] = sv;
    sb[r] = fma(-k.al, sv, sb[r]);
  }
  __syncthreads();
  const int ti = threadIdx.x % kTW, tj = threadIdx.x / kTW;
  const int r = (tj + kHalo) * kRW + ti + kHalo;
  const int gi = T.i0 + kHalo + ti, gj = T.j0 + kHalo + tj;
  double rr = 0.0;
  if (gi < T.nx && gj < T.ny) {
    const int g = gj * T.nx + gi;
    const double pc = it > 0 ? fma(k.be, pc0, zc) : zc;
    const double rc = sb[r];
    D.cg_p[g] = pc;
    cg_s(D, it)[g] = ss[r];
    D.lev[0].x[g] = fma(k.al, pc, xc);
    cg_rv(D, v)[g] = rc;
    rr = rc * rc;
  }
  const double t = block_sum(rr, sh);
  if (threadIdx.x == 0) red_rrt(D)[B.lb] = t;
}

__global__ void __launch_bounds__(kRedBlock) k_mg_down(const SynthDesc *ds, const int2 *bt, int l,
                                                       int v, int rr_ext) {
  __shared__ double sb[kRN], sd[kRN], sax[kRN], say[kRN], sx[kRN], ss[kRN], sh[kRedBlock];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1], f3 = D.state[3];   // tested after the region loads
  const LevelDev L = level(D, l), CL = level(D, l + 1);
  const bool upd = l == 0 && v > 0;
  double *xs = L.xs;
  const Tile T = tile_of(L, B.lb);
  double zc = 0.0, pc0 = 0.0, xc = 0.0;
  UpdPre q = {0.0, 0.0, 1.0, 1.0};
  if (upd) {
    const int it = v - 1;
    q = upd_prefetch(D, it);
    // r_{v-1}, w and s_old of the region (w into sx, free until the
    // sweeps), z, p and x of the thread's tile cell
    load_region_t<true, false>(L, cg_rv(D, it), T, sb, sd, sax, say, D.cg_w, sx, nullptr,
                               nullptr, 0, 0, 0, 0.0, nullptr, it > 0 ? cg_s(D, it - 1) : nullptr,
                               ss);
    const int gi = T.i0 + kHalo + (int)threadIdx.x % kTW, gj = T.j0 + kHalo + (int)threadIdx.x / kTW;
    if (gi < T.nx && gj < T.ny) {
      const int g = gj * T.nx + gi;
      zc = D.cg_z[g];
      if (it > 0) pc0 = D.cg_p[g];
      xc = D.lev[0].x[g];
    }
  } else {
    load_region(L, lev_b(D, l, v), T, sb, sd, sax, say);
  }
  // the r.r test of the CG step before this V-cycle is made by the next
  // kernel of the cycle (level 1 here, block 0; the other blocks go on: if
  // it converged, their results are not used)
  const bool fin = l == 1 && B.lb == 0 && !rr_ext;   // rr_ext: k_rr_test made it
  RRPre qr = {0.0, 0.0, 0.0};
  if (fin) qr = rr_prefetch(D, v == 0, v > 0);
  if (f1 != 0 || f3 != 0) return;
  if (fin) (void)finish_rr(D, v == 0, v > 0, sh, qr);
  __syncthreads();
  if (upd) cg_update_tile(D, B, T, v, sb, sx, ss, zc, pc0, xc, q, sh);
  // red half sweep from zero on the whole region
  for (int r = threadIdx.x; r < kRN; r += blockDim.x) {
    int ri, rj;
    cell_ij(r, kRW, ri, rj);
    sx[r] = (((T.i0 + ri + T.j0 + rj) & 1) == 0) ? sb[r] / sd[r] : 0.0;
  }
  __syncthreads();
  // black half sweep on the tile and a ring of one
  for (int r = threadIdx.x; r < kRN; r += blockDim.x) {
    int ri, rj;
    cell_ij(r, kRW, ri, rj);
    if (ri < 1 || ri > kRW - 2 || rj < 1 || rj > kRH - 2) continue;
    if (((T.i0 + ri + T.j0 + rj) & 1) != 1) continue;
    double v = sb[r];
    v += sax[r] * sx[r + 1];
    v += sax[r - 1] * sx[r - 1];
    v += say[r] * sx[r + kRW];
    v += say[r - kRW] * sx[r - kRW];
    sx[r] = v / sd[r];
  }
  __syncthreads();
  // residual of the tile cell of this thread; x of the tile to global
  const int ti = threadIdx.x % kTW, tj = threadIdx.x / kTW;
  const int r = (tj + kHalo) * kRW + ti + kHalo;
  const int gi = T.i0 + kHalo + ti, gj = T.j0 + kHalo + tj;
  double y = sd[r] * sx[r];
  y -= sax[r] * sx[r + 1];
  y -= sax[r - 1] * sx[r - 1];
  y -= say[r] * sx[r + kRW];
  y -= say[r - kRW] * sx[r - kRW];
  const double res = sb[r] - y;
  const bool in = gi < T.nx && gj < T.ny;
  if (in) xs[gj * T.nx + gi] = sx[r];
  __syncthreads();
  sb[r] = in ? res : 0.0;   // the tile's residuals (the ring is no longer needed)
  __syncthreads();
  // restriction: coarse cells whose children lie in this tile
  const int fx = L.fx, fy = L.fy, sx_ = fx >> 1, sy_ = fy >> 1;
  const int cw = kTW >> sx_, ch = kTH >> sy_;
  if ((int)threadIdx.x < cw * ch) {
    const int ci = threadIdx.x % cw, cj = threadIdx.x / cw;
    const int CI = ((T.i0 + kHalo) >> sx_) + ci, CJ = ((T.j0 + kHalo) >> sy_) + cj;
    if (CI < CL.nx && CJ < CL.ny) {
      double acc = 0.0;
      for (int dj = 0; dj < fy; ++dj)
        for (int di = 0; di < fx; ++di) {
          const int li = ci * fx + di, lj = cj * fy + dj;
          if (T.i0 + kHalo + li < T.nx && T.j0 + kHalo + lj < T.ny)
            acc += sb[(lj + kHalo) * kRW + li + kHalo];
        }
      CL.b[CJ * CL.nx + CI] = acc;
    }
  }
}

__global__ void __launch_bounds__(kRedBlock) k_mg_up(const SynthDesc *ds, const int2 *bt, int l,
                                                     int vc, double omega) {
  __shared__ double sb[kRN], sd[kRN], sax[kRN], say[kRN], sx[kRN];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1], f3 = D.state[3];   // tested after the region loads
  const LevelDev L = level(D, l), CL = level(D, l + 1);
  const double *b = lev_b(D, l, vc);
  double *x = lev_x(D, l);
  const double *xs = L.xs;
  const double *e = CL.x;
  const Tile T = tile_of(L, B.lb);
  const int sx_ = L.fx >> 1, sy_ = L.fy >> 1;
  // with the pre-smoothed x plus the scaled coarse correction: the black
  // half sweep sees corrected red neighbours
  __shared__ double sxc[kRN];
  load_region_t<false, true>(L, b, T, sb, sd, sax, say, nullptr, nullptr, xs, e, CL.nx, sx_, sy_,
                             omega, sxc);
  if (f1 != 0 || f3 != 0) return;
  __syncthreads();
  // black half sweep on the tile and a ring of one, into sx
  for (int r = threadIdx.x; r < kRN; r += blockDim.x) {
    int ri, rj;
    cell_ij(r, kRW, ri, rj);
    if (ri < 1 || ri > kRW - 2 || rj < 1 || rj > kRH - 2) { sx[r] = 0.0; continue; }
    if (((T.i0 + ri + T.j0 + rj) & 1) != 1) { sx[r] = 0.0; continue; }
    double v = sb[r];
    v += sax[r] * sxc[r + 1];
    v += sax[r - 1] * sxc[r - 1];
    v += say[r] * sxc[r + kRW];
    v += say[r - kRW] * sxc[r - kRW];
    sx[r] = v / sd[r];
  }
  __syncthreads();
  // red half sweep on the tile with the new black neighbours
  const int ti = threadIdx.x % kTW, tj = threadIdx.x / kTW;
  const int r = (tj + kHalo) * kRW + ti + kHalo;
  const int gi = T.i0 + kHalo + ti, gj = T.j0 + kHalo + tj;
  double xv = sx[r];
  if (((gi + gj) & 1) == 0) {
    double v = sb[r];
    v += sax[r] * sx[r + 1];
    v += sax[r - 1] * sx[r - 1];
    v += say[r] * sx[r + kRW];
    v += say[r - kRW] * sx[r - kRW];
    xv = v / sd[r];
  }
  const bool in = gi < T.nx && gj < T.ny;
  if (in) x[gj * T.nx + gi] = xv;
}

// Level 0 going up: as k_mg_up, over a ring of three, so that z is final on
// the tile and a ring of one (black on the tile and a ring of two, red on
// the tile and a ring of one); then w = A z on the tile, z and w to global,
// and partials of r.z and z.w for the CG (b = r).
constexpr int kU0Halo = 3, kU0W = kTW + 2 * kU0Halo, kU0H = kTH + 2 * kU0Halo;
constexpr int kU0N = kU0W * kU0H, kU0Per = (kU0N + kRedBlock - 1) / kRedBlock;
__global__ void __launch_bounds__(kRedBlock) k_mg_up0(const SynthDesc *ds, const int2 *bt, int vc,
                                                      double omega) {
  __shared__ double sb[kU0N], sd[kU0N], sax[kU0N], say[kU0N], sxc[kU0N], sx[kU0N];
  __shared__ double sh[kRedBlock];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1], f3 = D.state[3];   // tested after the region loads
  const LevelDev L = level(D, 0), CL = level(D, 1);
  const double *b = cg_rv(D, vc);
  const int nx = L.nx, ny = L.ny, sx_ = L.fx >> 1, sy_ = L.fy >> 1;
  int ti, tj;
  cell_ij(B.lb, (nx + kTW - 1) / kTW, ti, tj);
  const int i0 = ti * kTW - kU0Halo, j0 = tj * kTH - kU0Halo;
  {
    // every load of the thread first (clamped, valid indices), then LDS
    double vb[kU0Per], vd[kU0Per], vx[kU0Per], vy[kU0Per], vs[kU0Per], ve[kU0Per];
    bool in[kU0Per], hx[kU0Per], hy[kU0Per];
#pragma unroll
    for (int k = 0; k < kU0Per; ++k) {
      const int r = threadIdx.x + k * kRedBlock;
      int ri, rj;
      cell_ij(r, kU0W, ri, rj);
      const int gi = i0 + ri, gj = j0 + rj;
      in[k] = r < kU0N && gi >= 0 && gi < nx && gj >= 0 && gj < ny;
      hx[k] = gi + 1 < nx;
      hy[k] = gj + 1 < ny;
      const int g = in[k] ? gj * nx + gi : 0;
      vb[k] = b[g]; vd[k] = L.dg[g]; vx[k] = L.ax[g]; vy[k] = L.ay[g]; vs[k] = L.xs[g];
      ve[k] = CL.x[in[k] ? (gj >> sy_) * CL.nx + (gi >> sx_) : 0];
    }
#pragma unroll
    for (int k = 0; k < kU0Per; ++k) {
      const int r = threadIdx.x + k * kRedBlock;
      if (r >= kU0N) continue;
      sb[r] = in[k] ? vb[k] : 0.0;
      sd[r] = in[k] ? vd[k] : 1.0;
      sax[r] = in[k] && hx[k] ? vx[k] : 0.0;
      say[r] = in[k] && hy[k] ? vy[k] : 0.0;
      double t = 0.0;
      if (in[k]) {
        t = vs[k];
        t += omega * ve[k];
      }
      sxc[r] = t;
    }
  }
  if (f1 != 0 || f3 != 0) return;
  __syncthreads();
  // black on the region less a ring of one, into sx (other cells 0)
  for (int r = threadIdx.x; r < kU0N; r += blockDim.x) {
    int ri, rj;
    cell_ij(r, kU0W, ri, rj);
    if (ri < 1 || ri > kU0W - 2 || rj < 1 || rj > kU0H - 2 || ((i0 + ri + j0 + rj) & 1) != 1) {
      sx[r] = 0.0;
      continue;
    }
    double v = sb[r];
    v += sax[r] * sxc[r + 1];
    v += sax[r - 1] * sxc[r - 1];
    v += say[r] * sxc[r + kU0W];
    v += say[r - kU0W] * sxc[r - kU0W];
    sx[r] = v / sd[r];
  }
  __syncthreads();
  // red on the region less a ring of two (reads black cells only)
  for (int r = threadIdx.x; r < kU0N; r += blockDim.x) {
    int ri, rj;
    cell_ij(r, kU0W, ri, rj);
    if (ri < 2 || ri > kU0W - 3 || rj < 2 || rj > kU0H - 3 || ((i0 + ri + j0 + rj) & 1) != 0)
      continue;
    double v = sb[r];
    v += sax[r] * sx[r + 1];
    v += sax[r - 1] * sx[r - 1];
    v += say[r] * sx[r + kU0W];
    v += say[r - kU0W] * sx[r - kU0W];
    sx[r] = v / sd[r];
  }
  __syncthreads();
  // the tile cell of this thread: z, w = A z, partials of r.z and z.w
  const int ci = threadIdx.x % kTW, cj = threadIdx.x / kTW;
  const int r = (cj + kU0Halo) * kU0W + ci + kU0Halo;
  const int gi = i0 + kU0Halo + ci, gj = j0 + kU0Halo + cj;
  const bool in = gi < nx && gj < ny;
  const double zv = sx[r];
  double wv = sd[r] * zv;
  wv -= sax[r] * sx[r + 1];
  wv -= sax[r - 1] * sx[r - 1];
  wv -= say[r] * sx[r + kU0W];
  wv -= say[r - kU0W] * sx[r - kU0W];
  if (in) {
    const int g = gj * nx + gi;
    D.cg_z[g] = zv;
    D.cg_w[g] = wv;
  }
  const double trz = block_sum(in ? sb[r] * zv : 0.0, sh);
  const double tzw = block_sum(in ? zv * wv : 0.0, sh);
  if (threadIdx.x == 0) {
    red_rz(D)[B.lb] = trz;
    red_zw(D)[B.lb] = tzw;
  }
}

// The coarse end of the V-cycle (every level from the first with at most
// kCoarseWG cells down to the dense solve) in one workgroup of 1024 threads
// per problem, so the half sweeps are separated by workgroup barriers
// instead of kernel launches.
//  * Each half sweep runs over the cells of one colour only: thread t takes
//    the colour's cells number t, t + 1024 (colour_cell), so no lane idles
//    on a cell of the other colour. Diagonals are applied as precomputed
//    reciprocals.
//  * The top coarse level keeps its cells' operator rows and right-hand
//    side in registers (at most 2 cells of each colour per thread); lower
//    levels keep theirs in LDS. Vectors live in LDS.
//  * After the second (black) half sweep from zero the black residuals
//    vanish, so only red cells form a residual for the restriction.
//  * Going up, the black half sweep reads its red neighbours with the
//    scaled coarse correction added (x + omega e, formed where it is read:
//    the corrected values of black cells are never read), then the red half
//    sweep recomputes the red cells, as in the tile kernels.
//  * The restriction of a level's residuals also makes the next level's
//    first (red, from zero) half sweep, and below the top level it forms the
//    red residuals where it reads them, so each level costs two barriers
//    going down and two going up.
constexpr int kCoarseWG = 4096;
constexpr int kCoarseThreads = 1024;

// Cell number e of colour k ((i + j) & 1 == k) of an nx x ny grid, cells of
// a colour numbered row by row. Rows come in pairs holding nx cells of each
// colour. False past the last cell of the colour.
__device__ inline bool colour_cell(int e, int k, int nx, int ny, int &i, int &j) {
  int r, p;
  cell_ij(e, nx, r, p);                     // e = p nx + r
  const int c0 = (nx + 1 - k) >> 1;         // colour-k cells of the even row
  if (r < c0) { j = 2 * p; i = k + 2 * r; }
  else { j = 2 * p + 1; i = (1 - k) + 2 * (r - c0); }
  return j < ny;
}

// One cell of the top coarse level held by a thread.
struct OwnCell {
  int c, cE, cW, cN, cS;       // index; neighbour indices (itself when missing)
  int pE, pW, pN, pS;          // the neighbours' parents on the next level
  bool ok;
  double d, id, aE, aW, aN, aS, b;
};

__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse(const SynthDesc *ds, double omega,
                                                              int vc, int rr_ext) {
  extern __shared__ double sm[];
  __shared__ double red[kCoarseThreads];
  CDesc &D = cdesc(ds, blockIdx.x);
  // a problem whose V-cycle starts here or on level 1 makes the r.r test of
  // the CG step before it here (level 1: the level-0 tile kernel made the
  // update)
  const bool fin = D.lc == 0 || (D.lc == 1 && !rr_ext);   // rr_ext: k_rr_test made it
  RRPre q = {0.0, 0.0, 0.0};
  if (fin) q = rr_prefetch(D, vc == 0, vc > 0 && D.lc == 1);
  if (cg_off(D.state)) return;
  if (fin && finish_rr(D, vc == 0, vc > 0 && D.lc == 1, red, q)) return;
  __attribute__((address_space(4))) const CoarseLevels &L = D.cl;
  const double *bin = D.lc == 0 ? cg_rv(D, vc) : D.lev[D.lc].b;
  double *xout = D.lc == 0 ? D.cg_z : D.lev[D.lc].x;
  const double *Ainv = D.coarse_inv;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int last = L.nlev - 1;
  const int nx0 = L.nx[0], ny0 = L.ny[0];
  auto X = [&](int t) { return sm + L.xoff[t]; };
  auto Bv = [&](int t) { return sm + L.boff[t]; };
  auto Rv = [&](int t) { return sm + L.roff[t]; };
  // ---- top level: own cells (colour k, slot m) with their operator rows
  OwnCell own[2][2];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      OwnCell &o = own[k][m];
      int i = 0, j = 0;
      o.ok = colour_cell(tid + m * nt, k, nx0, ny0, i, j);
      if (!o.ok) { i = 0; j = 0; }
      const int c = j * nx0 + i;
      const bool hE = o.ok && i + 1 < nx0, hW = o.ok && i > 0;
      const bool hN = o.ok && j + 1 < ny0, hS = o.ok && j > 0;
      o.c = c;
      o.cE = hE ? c + 1 : c; o.cW = hW ? c - 1 : c;
      o.cN = hN ? c + nx0 : c; o.cS = hS ? c - nx0 : c;
      if (last > 0) {
        const int sx = L.fx[0] >> 1, sy = L.fy[0] >> 1, cnx = L.nx[1];
        const int iE = hE ? i + 1 : i, iW = hW ? i - 1 : i, jN = hN ? j + 1 : j, jS = hS ? j - 1 : j;
        o.pE = (j >> sy) * cnx + (iE >> sx); o.pW = (j >> sy) * cnx + (iW >> sx);
        o.pN = (jN >> sy) * cnx + (i >> sx); o.pS = (jS >> sy) * cnx + (i >> sx);
      } else {
        o.pE = o.pW = o.pN = o.pS = 0;
      }
      o.d = o.ok ? L.dg[0][c] : 1.0;
      o.aE = hE ? L.ax[0][c] : 0.0; o.aW = hW ? L.ax[0][c - 1] : 0.0;
      o.aN = hN ? L.ay[0][c] : 0.0; o.aS = hS ? L.ay[0][c - nx0] : 0.0;
      o.b = o.ok ? bin[c] : 0.0;
    }
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int m = 0; m < 2; ++m) own[k][m].id = 1.0 / own[k][m].d;
  // the coarsest level's dense inverse (n <= 64) in registers
  const int nd = L.nx[last] * L.ny[last];
  double ainv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = tid >> 4, col = (tid & 15) + 16 * q;
    ainv[q] = (row < nd && col < nd) ? Ainv[(size_t)row * nd + col] : 0.0;
  }
  // lower levels' operators into LDS (reciprocal diagonal, ax, ay, diagonal)
  for (int t = 1; t < L.nlev; ++t) {
    const int n = L.nx[t] * L.ny[t];
    double *a = sm + L.aoff[t];
    for (int c = tid; c < n; c += nt) {
      const double d = L.dg[t][c];
      a[c] = 1.0 / d; a[n + c] = L.ax[t][c]; a[2 * n + c] = L.ay[t][c]; a[3 * n + c] = d;
    }
  }
  // ---- top-level pieces
  double *x0 = X(0), *r0 = Rv(0);
  auto top_half = [&](int k, bool zero) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const OwnCell &o = own[k][m];
      if (!o.ok) continue;
      double s = o.b;
      if (!zero) {
        s = fma(o.aE, x0[o.cE], s);
        s = fma(o.aW, x0[o.cW], s);
        s = fma(o.aN, x0[o.cN], s);
        s = fma(o.aS, x0[o.cS], s);
      }
      x0[o.c] = s * o.id;
    }
  };
  // level t >= 1: half sweep of colour k over the colour's cells
  auto low_half = [&](int t, int k, bool zero) {
    const int nx = L.nx[t], ny = L.ny[t], n = nx * ny;
    double *x = X(t);
    const double *b = Bv(t), *id = sm + L.aoff[t], *ax = id + n, *ay = id + 2 * n;
    for (int e = tid; 2 * e < n + 1; e += nt) {
      int i, j;
      if (!colour_cell(e, k, nx, ny, i, j)) break;
      const int c = j * nx + i;
      double s = b[c];
      if (!zero) {
        if (i + 1 < nx) s = fma(ax[c], x[c + 1], s);
        if (i > 0) s = fma(ax[c - 1], x[c - 1], s);
        if (j + 1 < ny) s = fma(ay[c], x[c + nx], s);
        if (j > 0) s = fma(ay[c - nx], x[c - nx], s);
      }
      x[c] = s * id[c];
    }
  };
  // black half sweep of the top level with the coarse correction of its red
  // neighbours formed where they are read
  auto top_black_corr = [&]() {
    const double *e = X(1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const OwnCell &o = own[1][m];
      if (!o.ok) continue;
      double s = o.b;
      s = fma(o.aE, fma(omega, e[o.pE], x0[o.cE]), s);
      s = fma(o.aW, fma(omega, e[o.pW], x0[o.cW]), s);
      s = fma(o.aN, fma(omega, e[o.pN], x0[o.cN]), s);
      s = fma(o.aS, fma(omega, e[o.pS], x0[o.cS]), s);
      x0[o.c] = s * o.id;
    }
  };
  // the same on level t >= 1
  auto low_black_corr = [&](int t) {
    const int nx = L.nx[t], ny = L.ny[t], n = nx * ny, sx = L.fx[t] >> 1, sy = L.fy[t] >> 1;
    const int cnx = L.nx[t + 1];
    double *x = X(t);
    const double *e = X(t + 1);
    const double *b = Bv(t), *id = sm + L.aoff[t], *ax = id + n, *ay = id + 2 * n;
    auto xc = [&](int i, int j) {
      return fma(omega, e[(j >> sy) * cnx + (i >> sx)], x[j * nx + i]);
    };
    for (int q = tid; 2 * q < n + 1; q += nt) {
      int i, j;
      if (!colour_cell(q, 1, nx, ny, i, j)) break;
      const int c = j * nx + i;
      double s = b[c];
      if (i + 1 < nx) s = fma(ax[c], xc(i + 1, j), s);
      if (i > 0) s = fma(ax[c - 1], xc(i - 1, j), s);
      if (j + 1 < ny) s = fma(ay[c], xc(i, j + 1), s);
      if (j > 0) s = fma(ay[c - nx], xc(i, j - 1), s);
      x[c] = s * id[c];
    }
  };
  // restriction of level t's residuals into b_{t+1} (level 0: the owners'
  // residuals in r_0; below: the red residuals b - A x formed here, black
  // ones being zero), and on a level t + 1 above the coarsest its red half
  // sweep from zero, x = b / d
  auto restrict_red = [&](int t) {
    const int nx = L.nx[t], ny = L.ny[t], n = nx * ny, fx = L.fx[t], fy = L.fy[t];
    const int cnx = L.nx[t + 1], cn = cnx * L.ny[t + 1];
    const double *x = X(t), *b = Bv(t), *id = sm + L.aoff[t], *ax = id + n, *ay = id + 2 * n;
    const double *dg = id + 3 * n, *r = Rv(t);
    double *cb = Bv(t + 1), *cx = X(t + 1);
    const double *cid = sm + L.aoff[t + 1];
    const bool red_next = t + 1 < last;
    for (int C = tid; C < cn; C += nt) {
      int I, J;
      cell_ij(C, cnx, I, J);
      double v = 0.0;
      for (int dj = 0; dj < fy; ++dj)
        for (int di = 0; di < fx; ++di) {
          const int i = fx * I + di, j = fy * J + dj;
          if (i >= nx || j >= ny) continue;
          const int c = j * nx + i;
          double rv = 0.0;
          if (t == 0) {
            rv = r[c];
          } else if (((i + j) & 1) == 0) {
            double q = b[c];
            if (i + 1 < nx) q = fma(ax[c], x[c + 1], q);
            if (i > 0) q = fma(ax[c - 1], x[c - 1], q);
            if (j + 1 < ny) q = fma(ay[c], x[c + nx], q);
            if (j > 0) q = fma(ay[c - nx], x[c - nx], q);
            rv = fma(-dg[c], x[c], q);
          }
          v += rv;
        }
      cb[C] = v;
      if (red_next && ((I + J) & 1) == 0) cx[C] = v * cid[C];
    }
  };
  __syncthreads();
  if (last == 0) {
    // the top level is the coarsest: dense solve only
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int m = 0; m < 2; ++m)
        if (own[k][m].ok) r0[own[k][m].c] = own[k][m].b;
    __syncthreads();
  } else {
    // ---- down: top level, red from zero, black, red residuals, restrict
    top_half(0, true);
    __syncthreads();
    top_half(1, false);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const OwnCell &o = own[0][m];
      if (o.ok) {
        double s = o.b;
        s = fma(o.aE, x0[o.cE], s);
        s = fma(o.aW, x0[o.cW], s);
        s = fma(o.aN, x0[o.cN], s);
        s = fma(o.aS, x0[o.cS], s);
        r0[o.c] = fma(-o.d, x0[o.c], s);
      }
      if (own[1][m].ok) r0[own[1][m].c] = 0.0;
    }
    __syncthreads();
    restrict_red(0);
    __syncthreads();
    // lower levels: black, then the restriction (with the next level's red)
    for (int t = 1; t < last; ++t) {
      low_half(t, 1, false);
      __syncthreads();
      restrict_red(t);
      __syncthreads();
    }
  }
  // ---- dense solve on the coarsest level: 16 threads per row
  {
    const double *b = last == 0 ? r0 : Bv(last);
    const int row = tid >> 4, col0 = tid & 15;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = col0 + 16 * q;
      if (row < nd && col < nd) v += ainv[q] * b[col];
    }
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    if (col0 == 0 && row < nd) X(last)[row] = v;
    __syncthreads();
  }
  // ---- up: lower levels, then the top level
  if (last > 0) {
    for (int t = last - 1; t >= 1; --t) {
      low_black_corr(t);
      __syncthreads();
      low_half(t, 0, false);
      __syncthreads();
    }
    top_black_corr();
    __syncthreads();
    top_half(0, false);
    __syncthreads();
  }
  // ---- out: x of the top level (when the top level is level 0, k_cg_zw
  // then forms w = A z and the CG's partials)
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const OwnCell &o = own[k][m];
      if (o.ok) xout[o.c] = x0[o.c];
    }
}

// For a problem whose whole V-cycle ran in the one-workgroup kernel: w = A z
// and partials of r.z and z.w per block of cells (r of V-cycle vc).
__global__ void k_cg_zw(const SynthDesc *ds, const int2 *bt, int vc) {
  __shared__ double sh[kRedBlock];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  if (D.lc > 0) return;
  const int32_t f1 = D.state[1], f3 = D.state[3];
  const LevelDev L = level(D, 0);
  const int nx = L.nx, ny = L.ny;
  const int c = B.lb * kRedBlock + threadIdx.x;
  const bool in = c < D.N;
  int i = 0, j = 0;
  if (in) cell_ij(c, nx, i, j);
  const bool hE = in && i + 1 < nx, hW = in && i > 0, hN = in && j + 1 < ny, hS = in && j > 0;
  const int cc = in ? c : 0;
  const double *z = D.cg_z;
  const double zc = z[cc], ze = z[hE ? c + 1 : cc], zw = z[hW ? c - 1 : cc];
  const double zn = z[hN ? c + nx : cc], zs = z[hS ? c - nx : cc];
  const double dg = L.dg[cc], aE = L.ax[cc], aW = L.ax[hW ? c - 1 : cc];
  const double aN = L.ay[cc], aS = L.ay[hS ? c - nx : cc];
  const double rc = cg_rv(D, vc)[cc];
  if (f1 != 0 || f3 != 0) return;
  double wv = dg * zc;
  if (hE) wv -= aE * ze;
  if (hW) wv -= aW * zw;
  if (hN) wv -= aN * zn;
  if (hS) wv -= aS * zs;
  if (in) D.cg_w[c] = wv;
  const double trz = block_sum(in ? rc * zc : 0.0, sh);
  const double tzw = block_sum(in ? zc * wv : 0.0, sh);
  if (threadIdx.x == 0) {
    red_rz(D)[B.lb] = trz;
    red_zw(D)[B.lb] = tzw;
  }
}


constexpr double kOmega = 1.7;   // coarse-grid correction scaling (aggregation MG)

// ------------------------------------------------------------- update / Err
// delta = phi' - phi_half (GSIS) or 0 (SI); Err partials; phi = phi_new.
// FP32-mixed mode also records base = phi^m + delta (see the transport file).
// cond: launched ahead of the host's look at the synthetic solve's flags;
// runs only if that solve has converged (state[3]), else returns
__global__ void k_update(const SynthDesc *ds, const int2 *bt, int cond) {
  __shared__ double sh[kRedBlock];
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1] | (cond && D.state[3] == 0);   // tested after the operand loads
  const int c = B.lb * kRedBlock + threadIdx.x;
  const bool in = c < D.N;
  const int cc = in ? c : 0;
  const double pn = D.method ? D.lev[0].x[cc] : D.phih[cc];
  const double ph = D.phih[cc], po = D.phi[cc];
  // time-dependent form: T^{m+1} = T(sub_iter), against T^m for Err(T)
  const double tn = D.td ? t_sub(D, D.sub_iter)[cc] : 0.0, to = D.td ? D.Tm[cc] : 0.0;
  if (f1 != 0) return;
  double num = 0.0, den = 0.0, numT = 0.0, denT = 0.0;
  if (in) {
    const double d = pn - po;
    num = D.V * d * d;
    den = D.V * pn * pn;
    const double dl = D.method ? pn - ph : 0.0;
    D.delta[c] = dl;
    if (D.fp32) D.base[c] = po + dl;
    D.phi[c] = pn;
    if (D.td) {
      numT = D.V * (tn - to) * (tn - to);
      denT = D.V * tn * tn;
      D.Tm[c] = tn;
    }
  }
  double a = block_sum(num, sh);
  double b = block_sum(den, sh);
  if (threadIdx.x == 0) { D.err_parts[2 * B.lb] = a; D.err_parts[2 * B.lb + 1] = b; }
  if (D.td) {
    a = block_sum(numT, sh);
    b = block_sum(denT, sh);
    if (threadIdx.x == 0) { D.err_parts_T[2 * B.lb] = a; D.err_parts_T[2 * B.lb + 1] = b; }
  }
}

// Time-dependent form: one step of the material equation per cell (Eqs.
// MSE_d2, R2_def, MSE_d_mtx2, elem_mtx_M),
//   T(sub + 1) = T(sub) + R2 / D2,
//   R2 = -cv (T(sub) - T^n) / dt + sigma_a (rho(sub) - a c T(sub)^4),
//   D2 = cv / dt + 4 a c T(sub)^3 sigma_a,
// with rho(sub) = rho^{m+1/2} for sub 0 and for source iteration, else the
// synthetic solution of sub-iteration sub - 1 (the level-0 iterate).
__global__ void k_material(const SynthDesc *ds, const int2 *bt, int sub) {
  const Blk B = blk(bt);
  CDesc &D = cdesc(ds, B.p);
  const int32_t f1 = D.state[1];
  const int c = B.lb * kRedBlock + threadIdx.x;
  if (c >= D.N) return;
  const double *Ts = t_sub(D, sub);
  double *To = ((sub & 1) ? D.Tsub1 : D.Tsub0);
  const double rho = (sub == 0 || !D.method) ? D.phih[c] : D.lev[0].x[c];
  const double T = Ts[c], T2 = T * T, sa = D.sig_a[c], cv = D.cv[c], dt = D.dt;
  const double R2 = -cv * (T - D.Tn[c]) / dt + sa * (rho - D.ca * (T2 * T2));
  const double D2 = cv / dt + 4.0 * D.ca * (T2 * T) * sa;
  if (f1 != 0) return;
  To[c] = T + R2 / D2;
}

// p[e t], p[e (t + blockDim)], ... (t = threadIdx.x; n terms in all) added
// in that order; sixteen loads in flight at a time (terms past n add 0, and
// every sum here is of squares)
__device__ inline double strided_sum(const double *p, int n, int e) {
  constexpr int U = 16;
  double s = 0.0;
  for (int t0 = threadIdx.x; t0 < n; t0 += U * (int)blockDim.x) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      v[u] = t < n ? p[(size_t)e * t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  return s;
}

// One workgroup per problem: Err = sqrt(num/den) -> history, counters, done
// flag; the relative transport residual of the iterate this iteration
// started from, sqrt(sum w r^2 / (sum_k w_k sum_c src^2)) (the cell volume
// cancels on a uniform grid), from the residual kernel's per-wave partials
// and the moments kernel's per-block partials of the same iteration.
// Divergence: Err not finite, or the change ||phi^{m+1} - phi^m||_V above
// 1e3 times its smallest value so far (floored at 1e-9 ||phi^{m+1}||_V, far
// above rounding); Err alone cannot show a geometric blow-up, it tends to
// |1 - 1/g| for a growth factor g. last_err[1] keeps that smallest change.
__device__ inline void err_finish(CDesc &D, double *sh) {
  int32_t *state = D.state;
  if (state[1] != 0) return;
  const int npart = nblk_d(D.N);
  // (the residual-norm partials number one per residual wave: tens of
  // thousands on large grids)
  double a = strided_sum(D.err_parts, npart, 2), b = strided_sum(D.err_parts + 1, npart, 2);
  double rr = strided_sum(D.tres_part, D.n_tres, 1), ss = strided_sum(D.src2_part, D.n_src2, 1);
  double aT = 0.0, bT = 0.0;
  if (D.td) {
    aT = strided_sum(D.err_parts_T, npart, 2);
    bT = strided_sum(D.err_parts_T + 1, npart, 2);
  }
  const double dmin = D.last_err[1];
  double num = block_sum(a, sh);
  double den = block_sum(b, sh);
  rr = block_sum(rr, sh);
  ss = block_sum(ss, sh) * D.sw;
  if (D.td) {
    aT = block_sum(aT, sh);
    bT = block_sum(bT, sh);
  }
  if (threadIdx.x == 0) {
    double err = den > 0.0 ? sqrt(num / den) : (num == 0.0 ? 0.0 : INFINITY);
    if (D.td) {    // max(Err(rho), Err(T)), the criterion after Eq. Err_W
      const double eT = bT > 0.0 ? sqrt(aT / bT) : (aT == 0.0 ? 0.0 : INFINITY);
      err = eT > err ? eT : err;
    }
    const double tres = ss > 0.0 ? sqrt(rr / ss) : (rr == 0.0 ? 0.0 : INFINITY);
    const int m = state[0];
    D.err_hist[m] = err;
    D.tres_hist[m] = tres;
    // V-cycles of this iteration's (last) synthetic solve: the first after
    // the warm start, one per CG iteration
    if (D.method) D.scal[S_VCYCLES] += D.scal[S_NIT] + 1.0;
    const double dn = sqrt(num), pn = sqrt(den);
    D.last_err[0] = err;
    if (dn < dmin) D.last_err[1] = dn;
    state[0] = m + 1;
    state[2] = 1 - state[2];   // I^{m+1} now lives in the other buffer
    if (!isfinite(err) || dn > 1e3 * fmax(dmin, 1e-9 * pn)) state[1] = -1;
    else if (err < D.tol) state[1] = 1;
    else if (m + 1 >= D.max_iter) state[1] = 2;
  }
}

// src = (sigma_s phi + q) / (4 pi); the mirrored per-quadrant copies of
// (src, base/(4 pi), phi/(4 pi)) read by the transport kernels, stored in
// each quadrant's anti-diagonal order. One workgroup per 16 x 16 tile: the
// values go through LDS, then for every quadrant thread t writes the tile's
// t-th cell in that quadrant's anti-diagonal order, so the cells of a
// diagonal run over consecutive lanes and consecutive addresses.
constexpr int kSrcT = 16;
static_assert(kSrcT * kSrcT == kRedBlock, "one thread per tile cell");
__device__ inline void source_tile(CDesc &D, const Blk &B, double *s_sc, double *s_dq,
                                   double *s_pq) {
  const int32_t f1 = D.state[1];   // tested after the operands are loaded
  const int nx = D.nx, ny = D.ny, n = D.N;
  int ti, tj;
  cell_ij(B.lb, (nx + kSrcT - 1) / kSrcT, ti, tj);
  const int i0 = ti * kSrcT, j0 = tj * kSrcT;
  const int t = threadIdx.x;
  {
    const int i = i0 + (t & (kSrcT - 1)), j = j0 + t / kSrcT;
    const bool in = i < nx && j < ny;
    const int c = in ? j * nx + i : 0;
    double sc = (D.sig_s[c] * D.phi[c] + D.q[c]) / kFourPi;
    if (D.td) {                  // emission sigma_a a c (T^m)^4 / (4 pi)
      const double T = D.Tm[c], T2 = T * T;
      sc = (D.sig_s[c] * D.phi[c] + D.sig_a[c] * (D.ca * (T2 * T2)) + D.q[c]) / kFourPi;
    }
    const double dq = D.base[c] / kFourPi;
    const double pq = D.phi[c] / kFourPi;
    if (f1 != 0) return;
    if (in) D.src[c] = sc;
    s_sc[t] = sc; s_dq[t] = dq; s_pq[t] = pq;
  }
  __syncthreads();
  // cell t of a kSrcT x kSrcT square in anti-diagonal order (diagonal e = u +
  // w, then w): (u, w) in the square's own frame
  int e = 0, before = 0;
  for (;; ++e) {
    const int len = e < kSrcT ? e + 1 : 2 * kSrcT - 1 - e;
    if (t < before + len) break;
    before += len;
  }
  const int w = (e < kSrcT ? 0 : e - kSrcT + 1) + (t - before), u = e - w;
  for (int qd = 0; qd < 4; ++qd) {
    // the square in quadrant qd's mirrored frame: u runs against x when x
    // is mirrored, w against y when y is
    const int i = (qd & 1) ? i0 + kSrcT - 1 - u : i0 + u;
    const int j = (qd & 2) ? j0 + kSrcT - 1 - w : j0 + w;
    if (i >= nx || j >= ny) continue;
    const int xl = (qd & 1) ? nx - 1 - i : i, yl = (qd & 2) ? ny - 1 - j : j;
    const size_t o = (size_t)qd * 3 * n + dg_idx(xl, yl, nx, ny);
    const int l = (j - j0) * kSrcT + (i - i0);
    D.dynq[o] = s_sc[l];          // plane 0 of quadrant qd
    D.dynq[o + n] = s_dq[l];      // plane 1
    if (D.fp32) D.dynq[o + 2 * n] = s_pq[l];
  }
}

__global__ void __launch_bounds__(kRedBlock) k_source(const SynthDesc *ds, const int2 *bt) {
  __shared__ double s_sc[kRedBlock], s_dq[kRedBlock], s_pq[kRedBlock];
  const Blk B = blk(bt);
  source_tile(cdesc(ds, B.p), B, s_sc, s_dq, s_pq);
}

// End of an outer iteration: blocks [0, n) finish Err of problem blockIdx.x,
// blocks from n8 (n rounded up to a multiple of 8) make source tiles (table
// bt, or one problem's tiles). The two do not depend on each other; the
// source is written also on the iteration that ends the solve. One problem:
// its ntile tiles (row-major) fall into 8 runs of ts, one per XCD (block
// n8 + b runs on XCD b % 8 and takes tile (b % 8) ts + b / 8), so the
// partly written cache lines at the ends of a tile's diagonal runs mostly
// meet the neighbouring tile's part in the same L2.
__global__ void __launch_bounds__(kRedBlock) k_err_source(const SynthDesc *ds, const int2 *bt,
                                                          int n, int n8, int ntile, int ts,
                                                          int cond) {
  __shared__ double s_sc[kRedBlock], s_dq[kRedBlock], s_pq[kRedBlock];
  if ((int)blockIdx.x < n) {
    CDesc &D = cdesc(ds, blockIdx.x);
    if (cond && D.state[3] == 0) return;   // as k_update
    err_finish(D, s_sc);
    return;
  }
  const int idx = blockIdx.x - n8;
  if (idx < 0) return;
  Blk B;
  if (bt) {
    const __attribute__((address_space(4))) int *q =
        (const __attribute__((address_space(4))) int *)bt;
    B = {q[2 * idx], q[2 * idx + 1]};
  } else {
    const int tile = (idx & 7) * ts + (idx >> 3);
    if (tile >= ntile || (idx >> 3) >= ts) return;
    B = {0, tile};
  }
  CDesc &D = cdesc(ds, B.p);
  if (cond && D.state[3] == 0) return;
  source_tile(D, B, s_sc, s_dq, s_pq);
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

// z = M^{-1} r_v (one V(1,1) cycle with scaled coarse corrections) for
// every problem of the set, with the partials of r.z. V-cycle v > 0 follows
// CG iteration v - 1, whose update its level-0 tile kernel makes. part 1
// launches only that level-0 kernel, part 2 the rest, after k_rr_test has
// made the r.r test (problems that start with a tile level); part 0 all.
void vcycle(const SynthSet &S, int v, hipStream_t s, int part = 0) {
  const SynthDesc *ds = S.desc;
  const int rr_ext = part == 2 ? 1 : 0;
  for (int l = part == 2 ? 1 : 0; l < (part == 1 ? 1 : S.max_lc); ++l)
    hipLaunchKernelGGL(k_mg_down, dim3(S.nb_tile[l]), dim3(kRedBlock), 0, s, ds, S.bt_tile[l], l,
                       v, rr_ext);
  if (part == 1) return;
  hipLaunchKernelGGL(k_mg_coarse, dim3(S.n), dim3(kCoarseThreads), S.coarse_lds, s, ds, kOmega,
                     v, rr_ext);
  for (int l = S.max_lc - 1; l >= 1; --l)
    hipLaunchKernelGGL(k_mg_up, dim3(S.nb_tile[l]), dim3(kRedBlock), 0, s, ds, S.bt_tile[l], l, v,
                       kOmega);
  if (S.max_lc > 0)
    hipLaunchKernelGGL(k_mg_up0, dim3(S.nb_tile[0]), dim3(kRedBlock), 0, s, ds, S.bt_tile[0], v,
                       kOmega);
  if (S.min_lc == 0)
    hipLaunchKernelGGL(k_cg_zw, dim3(S.nb_cell), dim3(kRedBlock), 0, s, ds, S.bt_cell, v);
  if (S.any_coef_sep)
    hipLaunchKernelGGL(k_cg_coef, dim3(S.n), dim3(kRedBlock), 0, s, ds, v);
}

}  // namespace

// ------------------------------------------------------------ host side
size_t coarse_lds_bytes_from(const PlanDev &P, size_t lc) {
  size_t n = 0;
  for (size_t l = lc; l < P.mg.size(); ++l)
    n += (l == lc ? 2 : 7) * (size_t)P.mg[l].nx * P.mg[l].ny;
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

int tiles_of(int nx, int ny) { return ((nx + kTW - 1) / kTW) * ((ny + kTH - 1) / kTH); }
int source_tiles_of(int nx, int ny) {
  return ((nx + kSrcT - 1) / kSrcT) * ((ny + kSrcT - 1) / kSrcT);
}

// The attribute is per kernel, not per plan: it is raised to the largest
// amount any plan may ask for, so that a later plan with a smaller coarse
// cycle never lowers it under an earlier one.
void prepare_synth(size_t coarse_lds) {
  if (coarse_lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void *)k_mg_coarse, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kCoarseLdsBudget);
}

SynthDesc make_synth_desc(const PlanDev &P) {
  SynthDesc D;
  memset(&D, 0, sizeof D);
  D.nx = P.nx; D.ny = P.ny; D.N = P.N;
  D.dx = P.dx; D.dy = P.dy; D.V = P.V;
  D.method = P.method; D.fp32 = P.precision == GSIS_FP32_MIXED ? 1 : 0; D.max_iter = P.max_iter;
  D.tol = P.tol; D.rtol = P.synth_rtol;
  D.sig_t = P.sig_t; D.sig_s = P.sig_s; D.q = P.q;
  D.cE = P.cE; D.cW = P.cW; D.cN = P.cN; D.cS = P.cS; D.kappa = P.kappa;
  D.phih = P.phih; D.Fx = P.Fx; D.Fy = P.Fy; D.bflux = P.bflux;
  D.mom_part = P.mom_part; D.sw = P.sw; D.swm = P.swm; D.swe = P.swe;
  D.hot_face = P.method == GSIS_GSIS ? P.hot_face : 0;
  D.ftp = P.ftp;
  D.sig_a = P.sig_a;
  D.td = P.td; D.sub_iter = P.sub_iter; D.tdiag = P.tdiag; D.ca = P.ca; D.dt = P.dt;
  D.cv = P.cv; D.Tn = P.Tn; D.rho_n = P.rho_n; D.Tm = P.Tm; D.Tsub0 = P.Tsub0;
  D.Tsub1 = P.Tsub1; D.err_parts_T = P.err_parts_T;
  D.hx = P.hx; D.hy = P.hy; D.rhs = P.rhs; D.phi = P.phi; D.delta = P.delta; D.base = P.base;
  D.src = P.src; D.dynq = P.dynq;
  D.cg_r = P.cg_r; D.cg_r2 = P.cg_r2; D.cg_z = P.cg_z; D.cg_p = P.cg_p;
  D.cg_s0 = P.cg_s0; D.cg_s1 = P.cg_s1; D.cg_w = P.cg_w;
  D.wx = P.wide_wx; D.wy = P.wide_wy;
  D.red = P.red; D.scal = P.scal; D.err_parts = P.err_parts; D.err_hist = P.err_hist;
  D.last_err = P.last_err; D.state = P.state;
  D.tres_part = P.tres_part; D.src2_part = P.src2_part; D.tres_hist = P.tres_hist;
  D.n_tres = P.n_tres;
  D.n_src2 = nblk(P.N);
  D.nlev = (int)P.mg.size();
  for (int l = 0; l < D.nlev && l < kMaxLevels; ++l) {
    const MGLevel &L = P.mg[l];
    D.lev[l] = LevelDev{L.nx, L.ny, L.fx, L.fy, L.diag, L.ax, L.ay, L.x, L.b, L.r};
  }
  const int lc = coarse_start(P);
  D.lc = lc;
  D.ntile0 = tiles_of(P.mg[0].nx, P.mg[0].ny);
  D.ntp = std::max(D.ntile0, nblk(P.N));
  D.coef_sep = lc > 0 && D.ntile0 >= kCoefSepTiles ? 1 : 0;
  CoarseLevels &CL = D.cl;
  CL.nlev = D.nlev - lc;
  int off = 0;
  for (int t = 0; t < CL.nlev; ++t) {
    const MGLevel &L = P.mg[lc + t];
    const int n = L.nx * L.ny;
    CL.nx[t] = L.nx; CL.ny[t] = L.ny; CL.fx[t] = L.fx; CL.fy[t] = L.fy;
    CL.dg[t] = L.diag; CL.ax[t] = L.ax; CL.ay[t] = L.ay;
    CL.xoff[t] = off;
    off += n;
    if (t == 0) {
      CL.boff[t] = 0;           // the top level's b stays in registers
    } else {
      CL.boff[t] = off;
      off += n;
    }
    CL.roff[t] = off;
    off += n;
    CL.aoff[t] = t == 0 ? 0 : off;
    if (t > 0) off += 4 * n;
  }
  D.coarse_inv = P.coarse_inv;
  return D;
}

void launch_source(const SynthSet &S, hipStream_t s) {
  hipLaunchKernelGGL(k_source, dim3(S.nb_src), dim3(kRedBlock), 0, s, S.desc, S.bt_src);
}

void launch_wide_grad(const SynthSet &S, hipStream_t s, bool first) {
  if (first)
    hipLaunchKernelGGL(k_wide_grad<true>, dim3(S.nb_cell), dim3(kRedBlock), 0, s, S.desc, S.bt_cell);
  else
    hipLaunchKernelGGL(k_wide_grad<false>, dim3(S.nb_cell), dim3(kRedBlock), 0, s, S.desc, S.bt_cell);
}

void launch_hot(const SynthSet &S, hipStream_t s, bool combine) {
  if (combine)
    hipLaunchKernelGGL(k_hot<true>, dim3(S.nb_cell), dim3(kRedBlock), 0, s, S.desc, S.bt_cell);
  else
    hipLaunchKernelGGL(k_hot<false>, dim3(S.nb_cell), dim3(kRedBlock), 0, s, S.desc, S.bt_cell);
}

// Preconditioned CG (the Chronopoulos-Gear form, see cg_coef) on D1 phi' =
// rhs for every problem of the set, each warm-started from its phi (the
// previous synthetic solution), preconditioned by one V-cycle per
// iteration; solutions land in level 0's x. An iteration is one V-cycle:
// its level-0 down kernel makes the previous iteration's update, its
// level-0 up kernel forms w = A z and the partials of r.z and z.w, and
// every reduction is finished inside the kernel that needs it (see the
// partial regions above). The stop test runs on the device (state[3] per
// problem: 1 + the iterations taken once converged). With host_flag (a
// single problem), the host stops launching once the solve has converged:
// it checks the device flags after the V-cycle that would make the test at
// the iteration count the previous solve took (host_flag[8] keeps that
// count) and after every later one, so a run whose counts stay level waits
// once per solve and launches no V-cycle past convergence. Without it
// (batches, graph capture) exactly synth_max_iter iterations are launched
// and converged problems skip their kernels. spec (an event; single plans,
// plain GSIS): at each check the end of the outer iteration (launch_update,
// made conditional on convergence) is put into the stream before the host
// waits; true is returned when the solve has converged at a check, the
// update then being in the stream.
bool launch_synth_solve(const SynthSet &S, hipStream_t s, int32_t *host_flag, int rhs_mode,
                        int sub, hipEvent_t spec) {
  const SynthDesc *ds = S.desc;
  const dim3 gc(S.nb_cell), bk(kRedBlock);
  if (rhs_mode == 1) hipLaunchKernelGGL(k_cg_begin<1>, gc, bk, 0, s, ds, S.bt_cell, sub);
  else if (rhs_mode == 2) hipLaunchKernelGGL(k_cg_begin<2>, gc, bk, 0, s, ds, S.bt_cell, sub);
  else if (rhs_mode == 3) hipLaunchKernelGGL(k_cg_begin<3>, gc, bk, 0, s, ds, S.bt_cell, sub);
  else hipLaunchKernelGGL(k_cg_begin<0>, gc, bk, 0, s, ds, S.bt_cell, sub);
  vcycle(S, 0, s);
  const int guess = host_flag ? host_flag[8] : 0;
  for (int it = 0; it < S.synth_max_iter; ++it) {
    if (it + 1 == S.synth_max_iter) {
      // no V-cycle follows: the update on its own, then the r.r test
      hipLaunchKernelGGL(k_cg_update, gc, bk, 0, s, ds, S.bt_cell, it, 1);
      hipLaunchKernelGGL(k_finish_rr, dim3(S.n), bk, 0, s, ds);
      break;
    }
    // problems whose V-cycle runs wholly in the one-workgroup kernel have
    // no level-0 tile kernel to make the update
    if (S.min_lc == 0) hipLaunchKernelGGL(k_cg_update, gc, bk, 0, s, ds, S.bt_cell, it, 0);
    const bool due = guess > 0 ? it + 1 >= guess : (it >= 3 && ((it - 3) & 1) == 0);
    const bool check = host_flag && S.state0 && due;
    // at a check of a problem that starts with a tile level, the update and
    // the r.r test go first and the rest of the V-cycle only if it fails
    const bool split = check && S.n == 1 && S.min_lc >= 1;
    if (split) {
      vcycle(S, it + 1, s, 1);   // the update (level 0)
      hipLaunchKernelGGL(k_rr_test, dim3(S.n), bk, 0, s, ds);
    } else {
      vcycle(S, it + 1, s);   // makes the update (level 0) and the r.r test
    }
    if (check) {
      (void)hipMemcpyAsync(host_flag, S.state0 + 1, 3 * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s);
      if (spec) {
        // the end of the outer iteration goes into the stream before the
        // host waits (on the flags' copy alone); it runs only if the solve
        // has converged, so the GPU need not idle while the host wakes
        (void)hipEventRecord(spec, s);
        launch_update(S, s, 1);
        (void)hipEventSynchronize(spec);
      } else {
        (void)hipStreamSynchronize(s);
      }
      if (host_flag[0] != 0) return false;
      if (host_flag[2] != 0) {
        host_flag[8] = max(1, host_flag[2] - 1);
        return spec != nullptr;
      }
      if (split) vcycle(S, it + 1, s, 2);
    }
  }
  return false;
}

void launch_material(const SynthSet &S, hipStream_t s, int sub) {
  hipLaunchKernelGGL(k_material, dim3(S.nb_cell), dim3(kRedBlock), 0, s, S.desc, S.bt_cell, sub);
}

void launch_update(const SynthSet &S, hipStream_t s, int cond) {
  hipLaunchKernelGGL(k_update, dim3(S.nb_cell), dim3(kRedBlock), 0, s, S.desc, S.bt_cell, cond);
  const int n8 = (S.n + 7) / 8 * 8, ts = (S.nb_src + 7) / 8;
  const int nb = S.bt_src ? S.nb_src : 8 * ts;
  hipLaunchKernelGGL(k_err_source, dim3(n8 + nb), dim3(kRedBlock), 0, s, S.desc, S.bt_src, S.n,
                     n8, S.nb_src, ts, cond);
}

void launch_apply_delta_final(const PlanDev &P, hipStream_t s, double swmu, double sweta,
                              double *Fx_out, double *Fy_out) {
  hipLaunchKernelGGL(k_final_flux, dim3(nblk(P.N)), dim3(kRedBlock), 0, s, P.N, P.Fx, P.Fy,
                     P.delta, swmu, sweta, Fx_out, Fy_out);
}

double *synth_iteration_counter(const PlanDev &P) { return P.scal + S_NIT; }
double *synth_vcycle_total(const PlanDev &P) { return P.scal + S_VCYCLES; }

}  // namespace gsis
