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
//
// Storage precision. In FP64 mode the buffers hold I itself and the read adds
// base/(4 pi) with base = delta. In FP32-mixed mode they hold the FP32
// deviation Itilde = I^{m+1/2} - phi^m/(4 pi) (phi^m: the FP64 scalar flux
// the sweep started from), and the read adds base/(4 pi) with
// base = phi^m + delta. Itilde is the anisotropic part plus the last
// change of phi, small where the medium is thick, so its FP32 rounding stays
// far below the cancellation sigma_t I - sigma_s phi/(4 pi). The residual
// (with that cancellation) runs in FP64; the wavefront recurrence, which
// only propagates the residual's increments, and the moment sums of the
// deviations run in FP32, the phi^m/(4 pi) part of the moments in FP64.
#include "gsis_internal.h"
#include "wave_ops.h"

#include <algorithm>
#include <cstring>

namespace gsis {
namespace {

constexpr double kInv4Pi = 1.0 / kFourPi;

struct TArgs {
  int nx, ny, N, K, nbf;
  double dx, dy;
  int order, limiter;
  int qoff[5];
  const double *amu, *aeta, *w, *wmu, *weta;
  void *I0, *I1;     // the two intensity buffers (FP64 or FP32); state[2]
                     // names the current one
  int fp32;          // 1: buffers hold FP32 deviations (see above)
  const double *phi; // phi^m (FP32 mode: the deviation's reference)
  double sw, swm, swe;   // sum_k w_k, w_k mu_k, w_k eta_k
  double *R;
  const double *sig_t, *src, *delta;
  const double *cE, *cW, *cN, *cS;
  const double *bnd;
  double *phih, *Fx, *Fy, *bflux;
  double *mom_part;
  const double *cellq, *dynq;
  double *rowbuf;
  const double *sdq;
  const float *sdq_f;   // FP32-mixed: the same diagonal in FP32 (the FP32 recurrence)
  const float *w_f;     // FP32-mixed: w, w mu, w eta in FP32, [3][K] (the moment sums)
  const int2 *rtiles;
  int n_rtiles;
  const int *dso;    // row-0 storage index per diagonal, at offset kDiagPad
  const int32_t *state;
  unsigned long long *hand;   // row hand-over between the parts of a split
                              // recurrence, [K][parts - 1][nx]
  int32_t *hand_err;          // set when a part gave up waiting for the one below
  double *tres_part;          // [n_rtiles][ordinate pairs] sum of w r^2 per residual wave
  double *src2_part;          // [ceil(N / 256)] sum of src^2 per block of cells
  const double *In;           // time-dependent form: I^n, [K][N] like the intensity
  double tdiag;               // 1/(c dt) (the records' sigma_t already include it)
  int resid_rd;               // diagonals per residual tile (kRDSmall or kRDLarge)
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
  a.mom_part = P.mom_part;
  a.cellq = P.cellq; a.dynq = P.dynq; a.rowbuf = P.rowbuf;
  a.sdq = P.sdq; a.sdq_f = P.sdq_f; a.w_f = P.w_f; a.rtiles = P.rtiles; a.n_rtiles = P.n_rtiles;
  a.dso = P.dso;
  a.fp32 = P.precision == GSIS_FP32_MIXED ? 1 : 0;
  a.phi = P.phi;
  a.sw = P.sw; a.swm = P.swm; a.swe = P.swe;
  a.state = P.state;
  a.hand = P.hand;
  a.hand_err = P.state + 4;
  a.tres_part = P.tres_part;
  a.src2_part = P.src2_part;
  a.In = P.In;
  a.tdiag = P.tdiag;
  a.resid_rd = P.resid_rd;
  return a;
}

template <typename T = double>
__device__ inline const T *Iin_of(const TArgs &a) {
  return (const T *)(a.state[2] ? a.I1 : a.I0);
}
template <typename T = double>
__device__ inline T *Iout_of(const TArgs &a) { return (T *)(a.state[2] ? a.I0 : a.I1); }

__device__ inline int quadrant_of(const TArgs &a, int kk) {
  return (kk >= a.qoff[1]) + (kk >= a.qoff[2]) + (kk >= a.qoff[3]);
}
// The same for a problem's arguments in a batch table, read through the
// constant address space (scalar loads).
typedef __attribute__((address_space(4))) const TArgs CTArgs;
__device__ inline CTArgs &targs_at(const TArgs *t, int p) { return ((CTArgs *)t)[p]; }
template <typename T = double>
__device__ inline const T *Iin_of(CTArgs &a) {
  return (const T *)(a.state[2] ? a.I1 : a.I0);
}
template <typename T = double>
__device__ inline T *Iout_of(CTArgs &a) { return (T *)(a.state[2] ? a.I0 : a.I1); }
__device__ inline int quadrant_of(CTArgs &a, int kk) {
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
  return Ik[dg_idx(xl, yl, a.nx, a.ny)] + a.delta[gcell(a, q, xl, yl)] * kInv4Pi;
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
  a.R[(size_t)kk * a.N + dg_idx(xl, yl, a.nx, a.ny)] = r;
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
        else below = (y0 > 0 && xl >= 0 && xl < a.nx) ? Rk[dg_idx(xl, y0 - 1, a.nx, a.ny)] : 0.0;
      }
      if (rowok && xl >= 0 && xl < a.nx) {
        const size_t o = dg_idx(xl, yl, a.nx, a.ny);
        const int c = gcell(a, q, xl, yl);
        const double west = xl > 0 ? prev : 0.0;
        const double s_ = yl > 0 ? below : 0.0;
        const double r = Rk[o];
        const double sd = a.cellq[((size_t)q * a.N + o) * 6 + 5];
        const double di = (r + ax * west + ay * s_) / (sd + ax + ay);
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


// ---------------------------------------------------------------------------
// Fused transport step: residual (Eq. RTE_d_res) and exact first-order-upwind
// increment solve (Eqs. RTE_d_increment..elem_mtx) in one pass over I.
//
// One workgroup per ordinate covers the whole grid in the ordinate's
// mirrored frame (flow towards +x', +y'). Thread t owns local row y0 + t and
// walks its row; at step s it is at column x = s - t, so a workgroup step
// advances one anti-diagonal and every dependency (west: the lane's own
// previous value; south: lane t-1's previous value) is one step old.
//   * I^m is read once: each lane keeps u(x-1), u(x), u(x+1) of its row in
//     registers; u(x, y-1) and u(x, y+1) are the neighbours' window values
//     (lane shifts; across waves an LDS slot written one step earlier).
//   * face values F_e, F_n of a cell are computed once, by the cell's lane;
//     the west face is the lane's previous F_e, the south face lane t-1's
//     previous F_n.
//   * loads for column x+1 are issued PF steps ahead into a register ring,
//     so memory latency stays off the wavefront's critical path.
// I^{m+1/2} = I^m + dI is written once.
// ---------------------------------------------------------------------------
template <typename T>
struct Slot {
  T ib;                // I^m buffer value at column x+2
  double dq;           // base/(4 pi) at column x+2
  double sub;          // FP32 mode: phi^m/(4 pi) at column x+1
  double src;          // (sigma_s phi + q)/(4 pi) at column x+1
  double2 c0, c1;      // (cE, cW), (cN, cS) at column x+1, mirrored frame
  double2 st;          // sigma_t and the increment-solve diagonal's sigma_t
                       // plus pseudo-time shift, at column x+1
  int i1;              // storage index of column x+1 (clamped)
};

// Walks the anti-diagonals of an nx x ny grid one at a time (scalar state):
// first storage index, first row and length of diagonal d, with d clamped
// into the grid's diagonal range.
struct DiagCursor {
  int nx, ny, d, off, lo, len;
  __device__ void init(int nx_, int ny_, int d0) {
    nx = nx_; ny = ny_;
    const int dc = min(max(d0, 0), nx + ny - 2);
    d = d0;
    off = (int)dg_off(dc, nx, ny);
    lo = dg_ylo(dc, nx);
    len = (int)(dg_off(dc + 1, nx, ny) - off);
  }
  __device__ void advance() {
    ++d;
    if (d >= 1 && d <= nx + ny - 2) {     // move to the next diagonal
      off += len;
      lo = d - nx + 1 > 0 ? d - nx + 1 : 0;
      const int hi = d < ny - 1 ? d : ny - 1;
      len = hi - lo + 1;
    }
  }
  // storage index of row y on the current diagonal, clamped into it
  __device__ int index(int y) const { return off + min(max(y - lo, 0), len - 1); }
};

constexpr int kSouthCap = 2048;   // south-inflow row staged in LDS up to this width

// Workgroups are dealt to the eight XCDs round-robin (workgroup b runs on
// XCD b % 8). Workgroup b takes ordinate start(b % 8) + b / 8, which gives
// every XCD a contiguous run of the (quadrant-sorted) ordinates, so each
// XCD's L2 holds the per-cell records of one or two quadrants instead of
// all four. A bijection of [0, K).
__device__ inline int xcd_ordinate(int b, int K) {
  const int x = b & 7;
  int start = 0;
  for (int xp = 0; xp < x; ++xp) start += (K - xp + 7) >> 3;
  return start + (b >> 3);
}

// The lane is software-pipelined: at step s it solves the increment of
// column x = s - t with the residual it formed at step s-1, and forms the
// residual of column x+1 for step s+1. Only the recurrence
// dI = b + cx dI_west + cy dI_south waits on the neighbour exchange.
// GENERAL = false assumes ny <= blockDim.x (one pass) and nx <= kSouthCap, so
// that no load outside the prefetch ring sits on the step path.
template <int PF, int MAXW, bool GENERAL, typename T>
__device__ __forceinline__ void sweep_ordinate(const TArgs &a, const int kk) {
  constexpr bool kF32 = sizeof(T) == 4;
  const int q = quadrant_of(a, kk);
  const int nx = a.nx, ny = a.ny, N = a.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwav = blockDim.x >> 6;
  const int rows_pp = blockDim.x;
  const double ax = a.amu[kk], ay = a.aeta[kk];
  const double hdx = 0.5 * a.dx, hdy = 0.5 * a.dy;
  const bool second = a.order >= 2, lim = a.limiter != 0;
  const T *Ik = Iin_of<T>(a) + (size_t)kk * N;
  T *Ok = Iout_of<T>(a) + (size_t)kk * N;
  const double *Cq = a.cellq + (size_t)q * N * 6;
  const double2 *C2 = reinterpret_cast<const double2 *>(Cq);
  // planes: src, base/(4 pi), and (FP32 mode) phi^m/(4 pi)
  const double *SRC = a.dynq + (size_t)q * 3 * N;
  const double *DQ = SRC + N;
  const double *SUB = SRC + 2 * N;
  double *RB = a.rowbuf + (size_t)kk * 3 * nx;
  __shared__ double xup[2][MAXW][3];
  __shared__ double xdn[2][MAXW];
  __shared__ double south[kSouthCap];
  // inflow on the local south face of row 0, staged once
  for (int x = tid; x < min(nx, kSouthCap); x += blockDim.x) {
    const int i = (q & 1) ? nx - 1 - x : x;
    const int f = (q & 2) ? 2 * ny + nx + i : 2 * ny + i;
    south[x] = a.bnd[(size_t)f * a.K + kk];
  }
  __syncthreads();

  for (int y0 = 0; y0 < ny; y0 += rows_pp) {
    const int rows = min(rows_pp, ny - y0);
    const int y = y0 + tid;
    const bool rowok = tid < rows;
    const int yc = rowok ? y : y0;               // clamped row for addresses
    const bool hn = y + 1 < ny, hs = y > 0;
    const bool ntop = rowok && tid == rows - 1 && hn;   // north row lies in the next pass
    const bool sfirst = tid == 0 && y0 > 0;             // south row lies in the previous pass
    const bool handoff = rowok && tid == rows - 1 && y0 + rows < ny;
    // inflow on the local west face of this row
    double inW = 0.0;
    if (rowok) {
      const int j = (q & 2) ? ny - 1 - y : y;
      const int f = (q & 1) ? ny + j : j;
      inW = a.bnd[(size_t)f * a.K + kk];
    }
    // Every lane of a step sits on the same diagonal (x = d - y), so the
    // diagonal's offset is scalar state and the lanes address consecutive
    // cells. The cursor runs PF steps ahead, on the diagonal of column x+2
    // of the step being loaded; indices of lanes outside the grid are
    // clamped into the diagonal (never used).
    DiagCursor cur;
    cur.init(nx, ny, y0);                     // column x+1 of step -1
    int inext = cur.index(yc);
    auto load = [&](Slot<T> &sl) {
      const int i1 = inext;                    // column x+1
      cur.advance();
      inext = cur.index(yc);                   // column x+2
      sl.i1 = i1;
      sl.ib = Ik[inext];
      sl.dq = DQ[inext];
      sl.src = SRC[i1];
      sl.c0 = C2[3 * i1];
      sl.c1 = C2[3 * i1 + 1];
      sl.st = C2[3 * i1 + 2];
      if constexpr (kF32) sl.sub = SUB[i1];
    };
    Slot<T> ring[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t) load(ring[t]);
    // u of columns x, x+1, x+2 (the residual column is x+1). Lane 0 forms
    // the residual of column 0 at step -1, so its window starts at u(0, y);
    // the other lanes fill their windows from the ring before they start.
    double uw = 0.0, uc = 0.0, ue;
    {
      const long long i00 = dg_idx(0, yc, nx, ny);
      ue = (double)Ik[i00] + DQ[i00];
    }
    // pipeline registers: residual of column x (b = r / d, cx, cy), face
    // values of the residual column, increment of the chain column
    double b_c = 0.0, cx_c = 0.0, cy_c = 0.0, u_c = 0.0, sub_c = 0.0;
    int i_c = 0;
    double Fe_p = 0.0, Fn_p = 0.0, dI_p = 0.0;
    // steps -1 .. nx+rows-1, padded to a multiple of PF (padding steps have
    // no active lane); at step s the chain column is s - tid and the
    // residual column s - tid + 1
    const int nsteps = ((nx + rows + 1 + PF - 1) / PF) * PF;
    for (int sb = -1; sb < nsteps - 1; sb += PF) {
#pragma unroll
      for (int t = 0; t < PF; ++t) {
        const int s = sb + t;
        const int x = s - tid;                 // chain column
        const int xr = x + 1;                  // residual column
        uw = uc; uc = ue;
        ue = (double)ring[t].ib + ring[t].dq;  // u(x+2)
        // --- exchange with the rows below and above
        double sU = __shfl_up(uw, 1, 64);      // u(xr, y-1)
        double sFn = __shfl_up(Fn_p, 1, 64);   // F_n(xr, y-1)
        double sdI = __shfl_up(dI_p, 1, 64);   // dI(x, y-1)
        double nU = __shfl_down(ue, 1, 64);    // u(xr, y+1)
        if (lane == 0 && wave > 0) {
          sU = xup[(s + 1) & 1][wave - 1][0];
          sFn = xup[(s + 1) & 1][wave - 1][1];
          sdI = xup[(s + 1) & 1][wave - 1][2];
        }
        if (lane == 63 && wave + 1 < nwav) nU = xdn[(s + 1) & 1][wave + 1];
        const bool actc = rowok && x >= 0 && x < nx;      // chain
        const bool actr = rowok && xr >= 0 && xr < nx;    // residual
        if (GENERAL && sfirst) {                  // previous pass's top row
          if (actr) { sU = RB[xr]; sFn = RB[nx + xr]; }
          if (actc) sdI = RB[2 * nx + x];
        }
        if (GENERAL && actr && ntop) {            // next pass's bottom row
          const int o = dg_idx(xr, y + 1, nx, ny);
          nU = (double)Ik[o] + DQ[o];
        }
        // --- increment of the chain column (uses last step's residual)
        double dI = 0.0;
        if (actc) {
          const double dW = x > 0 ? dI_p : 0.0, dS = hs ? sdI : 0.0;
          dI = fma(cx_c, dW, fma(cy_c, dS, b_c));
          if constexpr (kF32) Ok[i_c] = (T)((u_c + dI) - sub_c);
          else Ok[i_c] = u_c + dI;
          if (GENERAL && handoff) RB[2 * nx + x] = dI;
        }
        // --- residual of column xr for the next step
        double Fn = uc;
        if (actr) {
          const double u = uc;
          const double st = ring[t].st.x;
          double Fe = u;
          if (second) {
            const double UE = xr + 1 < nx ? ue : u, UW = xr > 0 ? uw : u;
            const double UN = hn ? nU : u, US = hs ? sU : u;
            const double gx = ring[t].c0.x * (UE - u) - ring[t].c0.y * (UW - u);
            const double gy = ring[t].c1.x * (UN - u) - ring[t].c1.y * (US - u);
            const double hx = gx * hdx, hy = gy * hdy;
            double psi = 1.0;
            if (lim) {
              const double umax = fmax(fmax(fmax(u, UE), fmax(UW, UN)), US);
              const double umin = fmin(fmin(fmin(u, UE), fmin(UW, UN)), US);
              const double m = fmin(umax - u, u - umin);
              const double M = fmax(fabs(hx), fabs(hy));
              if (M > m) psi = m * rcp64(M);
            }
            Fe = fma(psi, hx, u);
            Fn = fma(psi, hy, u);
          }
          double FnS = sFn;
          if (!hs) {
            if (!GENERAL || xr < kSouthCap) {
              FnS = south[xr];
            } else {
              const int i = (q & 1) ? nx - 1 - xr : xr;
              FnS = a.bnd[(size_t)((q & 2) ? 2 * ny + nx + i : 2 * ny + i) * a.K + kk];
            }
          }
          const double FeW = xr > 0 ? Fe_p : inW;
          const double r = ring[t].src - st * u - ax * (Fe - FeW) - ay * (Fn - FnS);
          const double inv = rcp64(ring[t].st.y + ax + ay);
          b_c = r * inv; cx_c = ax * inv; cy_c = ay * inv;
          u_c = u; i_c = ring[t].i1;
          if constexpr (kF32) sub_c = ring[t].sub;
          if (GENERAL && handoff) { RB[xr] = u; RB[nx + xr] = Fn; }
          Fe_p = Fe;
        }
        Fn_p = Fn; dI_p = dI;
        if (lane == 63) {
          xup[s & 1][wave][0] = uc; xup[s & 1][wave][1] = Fn; xup[s & 1][wave][2] = dI;
        }
        if (lane == 0) xdn[s & 1][wave] = (double)ring[(t + 1) % PF].ib + ring[(t + 1) % PF].dq;
        load(ring[t]);                            // refill this slot PF steps ahead
        __builtin_amdgcn_s_waitcnt(0xc07f);     // LDS writes done (lgkmcnt 0 only)
        __builtin_amdgcn_s_barrier();
      }
    }
    __syncthreads();
  }
}

template <int PF, int MAXW, bool GENERAL, typename T>
__global__ void __launch_bounds__(MAXW * 64) k_sweep_fused(TArgs a) {
  if (a.state[1] != 0) return;
  sweep_ordinate<PF, MAXW, GENERAL, T>(a, xcd_ordinate(blockIdx.x, a.K));
}

// Batched sweep: one persistent launch for the ordinates of many problems.
// Each workgroup takes work items (problem, ordinate) from a shared counter,
// in the order of the item table (longest first), and runs the same sweep
// with that problem's arguments; problems that have finished are skipped.
// Every workgroup leaves once the counter passes the table.
template <int PF, int MAXW, typename T>
__global__ void __launch_bounds__(MAXW * 64)
    k_sweep_batch(const TArgs *targs, const int2 *items, int n_items, int *counter) {
  __shared__ int s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const int2 pk = items[it];
    const TArgs &a = targs[pk.x];
    if (a.state[1] == 0) sweep_ordinate<PF, MAXW, true, T>(a, pk.y);
  }
}

// ---------------------------------------------------------------------------
// Split transport step: a residual kernel with no dependence between cells,
// then the first-order-upwind recurrence alone on the wavefront.
//
// With v = I^m + dI the increment solve (Eqs. RTE_d_increment..elem_mtx),
//   dI = b + cx dI_W + cy dI_S,   b = r / d, cx = ax / d, cy = ay / d,
// reads v = bv + cx v_W + cy v_S with bv = u + b - cx u_W - cy u_S
// (u = I^m; the W or S term is absent on an inflow face, where dI = 0). The
// residual kernel forms bv for every cell, all cells in parallel, and writes
// it into the output buffer; the recurrence reads it back in place and leaves
// I^{m+1/2} there. In FP32-mixed mode both work on deviations from
// phi^m/(4 pi): bv = ut + b - cx ut_W - cy ut_S with ut = u - phi^m/(4 pi),
// so the recurrence yields Itilde directly. bv is rounded to the storage type
// once; everything else is FP64.
// ---------------------------------------------------------------------------

// Shifts across the whole 64-lane wave (DPP wave_shr:1 / wave_shl:1): lane i
// gets lane i-1's (i+1's) value; lane 0 (63) keeps its own.

// Second-order values on a cell's local east and north faces, u + psi h with
// the ALSM gradient (Eqs. shifted_j, LSF_mdf) and the Barth-Jespersen
// limiter; a missing neighbour is passed as u.
__device__ __forceinline__ void face_pair(double u, double UE, double UW, double UN, double US,
                                          double2 c0, double2 c1, double hdx, double hdy,
                                          bool second, bool lim, double &Fe, double &Fn) {
  Fe = u;
  Fn = u;
  if (!second) return;
  const double gx = c0.x * (UE - u) - c0.y * (UW - u);
  const double gy = c1.x * (UN - u) - c1.y * (US - u);
  const double hx = gx * hdx, hy = gy * hdy;
  double psi = 1.0;
  if (lim) {
    const double umax = fmax(fmax(fmax(u, UE), fmax(UW, UN)), US);
    const double umin = fmin(fmin(fmin(u, UE), fmin(UW, UN)), US);
    const double m = fmin(umax - u, u - umin);
    const double M = fmax(fabs(hx), fabs(hy));
    const double pl = m * rcp64(M);           // discarded unless M > m
    psi = M > m ? pl : 1.0;
  }
  Fe = fma(psi, hx, u);
  Fn = fma(psi, hy, u);
}


// Residual tiles: a band of 64 rows (one per lane) x RD diagonals, walked a
// diagonal per step after one warm-up step on the diagonal before the tile:
// 31 diagonals, or 47 on grids of 2^26 cell-ordinates and more, where
// fewer, longer tiles re-read fewer halo cells (0.85 -> 0.80 ms at
// 1024x1024x128 FP32-mixed) and there are tiles enough for the chip.
constexpr int kRDSmall = 31, kRDLarge = 47;
constexpr int kRWaves = 4;           // waves per workgroup, one ordinate each
constexpr int kRPF = 4;              // steps of loads in flight


template <typename T>
struct RSlot {
  T ib[2];             // stored values at the lookahead cell (diagonal d+1), per ordinate
  double dq;           // base/(4 pi) there
  double sube;         // FP32 mode: phi^m/(4 pi) there
  double src;          // source at the cell (diagonal d)
  double2 c0, c1, st;  // its coefficient record
  double in[2];        // time-dependent form: I^n at the cell, per ordinate
  unsigned ic;         // its storage index
};

// Ordinates are taken in pairs of one quadrant (the second may be absent
// when the quadrant has an odd count): pair number pi of a problem.
template <class A>
__device__ inline void ordinate_pair(A &a, int pi, int &kA, int &kB) {
  int q = 0, base = 0;
  for (; q < 3; ++q) {
    const int np = (a.qoff[q + 1] - a.qoff[q] + 1) >> 1;
    if (pi < base + np) break;
    base += np;
  }
  kA = a.qoff[q] + 2 * (pi - base);
  kB = kA + 1 < a.qoff[q + 1] ? kA + 1 : -1;
}
template <class A>
__device__ inline int ordinate_pairs(A &a) {
  int n = 0;
  for (int q = 0; q < 4; ++q) n += (a.qoff[q + 1] - a.qoff[q] + 1) >> 1;
  return n;
}

// One wave per (pair of ordinates of one quadrant, tile). Lane l owns row
// y = y0 + l; at step dd its cell is (d0 + dd - y, y), the same cell for
// both ordinates, so the cell's records (coefficients, source, pending
// correction) are loaded once for the two. Each lane keeps u of its row on
// diagonals d-1, d, d+1 per ordinate; u(x, y-1) and u(x, y+1) are the
// neighbour lanes' window values and the south face value is lane l-1's F_n
// of the previous step (DPP shifts). Row y0-1 below lane 0 and row y0+64
// above lane 63 come from a halo pass in which lane j computes diagonal
// d0-2+j (u below), d0-1+j (F_n below) and d0+j (u above) into LDS; each
// step reads its halo values back as LDS broadcasts and feeds them to the
// DPP shifts as lane 0's (lane 63's) fill. Loads use the index dso[d] + y
// through buffer resources: for a lane with no cell it lies on another
// diagonal or out of the buffer (read as 0), and the value is dropped.
// kB < 0: no second ordinate (its loads repeat kA's, its stores are dropped).
// TD: the time-dependent form's residual (Eq. RTE_d_res) also takes
// + I^n / (c dt); the -(1/(c dt)) I^m term rides in the records' sigma_t.
template <typename T, bool TD = false, int RD = kRDSmall, class A>
__device__ __forceinline__ void resid_tile(A &a, const int tile, const int kA, const int kB,
                                           const int wave, const int slot) {
  constexpr int kRD = RD, kRSteps = RD + 1;
  constexpr bool kF32 = sizeof(T) == 4;
  constexpr int PF = kRPF;
  static_assert(kRSteps % PF == 0, "whole turns of the load ring");
  static_assert(kRSteps + PF + 2 <= kDiagPad, "diagonal table padding");
  const int lane = threadIdx.x & 63;
  const int2 tl = a.rtiles[tile];
  const int d0 = tl.x, y0 = tl.y;
  const int nx = a.nx, ny = a.ny, N = a.N;
  const int q = quadrant_of(a, kA);
  const bool hasB = kB >= 0;
  const int kk[2] = {kA, hasB ? kB : kA};
  double ax[2], ay[2], wr[2];
  __amdgpu_buffer_rsrc_t Ib[2], Ob[2], Nb[2];
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    ax[o] = a.amu[kk[o]];
    ay[o] = a.aeta[kk[o]];
    wr[o] = (o == 0 || hasB) ? a.w[kk[o]] : 0.0;   // weight of w r^2 (no double count)
    Ib[o] = buf_rsrc(Iin_of<T>(a) + (size_t)kk[o] * N, (size_t)N * sizeof(T));
    Ob[o] = buf_rsrc(Iout_of<T>(a) + (size_t)kk[o] * N, (o == 0 || hasB) ? (size_t)N * sizeof(T) : 0);
    if constexpr (TD) Nb[o] = buf_rsrc(a.In + (size_t)kk[o] * N, (size_t)N * 8);
  }
  const double hdx = 0.5 * a.dx, hdy = 0.5 * a.dy;
  const bool second = a.order >= 2, lim = a.limiter != 0;
  const __amdgpu_buffer_rsrc_t Cb = buf_rsrc(a.cellq + (size_t)q * N * 6, (size_t)N * 48);
  const double *SRC = a.dynq + (size_t)q * 3 * N;
  const __amdgpu_buffer_rsrc_t Sb = buf_rsrc(SRC, (size_t)N * 8);
  const __amdgpu_buffer_rsrc_t Qb = buf_rsrc(SRC + N, (size_t)N * 8);
  const __amdgpu_buffer_rsrc_t Ub = buf_rsrc(SRC + 2 * N, (size_t)N * 8);
  const __attribute__((address_space(4))) int *DS =
      (const __attribute__((address_space(4))) int *)(a.dso + kDiagPad);
  const int y = y0 + lane;
  const bool rowok = y < ny, hn = y + 1 < ny, hs = y > 0;
  // ---- halo (see above) into LDS: lane j's values at [wave][ordinate][slot][j]
  __shared__ double hal[kRWaves][2][4][kRSteps + 1];
  {
    auto cidx = [&](int x, int yy) {       // storage index, clamped into the grid
      x = min(max(x, 0), nx - 1);
      yy = min(max(yy, 0), ny - 1);
      return (unsigned)(a.dso[kDiagPad + x + yy] + yy);
    };
    const int ys = y0 - 1;
    const int xu = d0 - 2 + lane - ys, xf = d0 - 1 + lane - ys, xn = d0 + lane - (y0 + 64);
    const unsigned iu = cidx(xu, ys), jf = cidx(xf, ys), je = cidx(xf + 1, ys);
    const unsigned jw = cidx(xf - 1, ys), jn = cidx(xf, y0), js = cidx(xf, ys - 1);
    const unsigned iN = cidx(xn, y0 + 64);
    const double2 f0 = buf_ld128(Cb, jf * 48u), f1 = buf_ld128(Cb, jf * 48u + 16u);
    const double su = kF32 ? buf_ld64(Ub, iu * 8u) : 0.0;
    const double qu = buf_ld64(Qb, iu * 8u), qf = buf_ld64(Qb, jf * 8u);
    const double qe = buf_ld64(Qb, je * 8u), qw = buf_ld64(Qb, jw * 8u);
    const double qn = buf_ld64(Qb, jn * 8u), qs = buf_ld64(Qb, js * 8u), qN = buf_ld64(Qb, iN * 8u);
    const int xi = min(d0 + lane, nx - 1);
    const int gi = (q & 1) ? nx - 1 - xi : xi;
    const size_t fs = (size_t)((q & 2) ? 2 * ny + nx + gi : 2 * ny + gi) * a.K;
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const double vu = (double)buf_ldT<T>(Ib[o], iu) + qu, vf = (double)buf_ldT<T>(Ib[o], jf) + qf;
      const double ve = (double)buf_ldT<T>(Ib[o], je) + qe, vw = (double)buf_ldT<T>(Ib[o], jw) + qw;
      const double vn = (double)buf_ldT<T>(Ib[o], jn) + qn, vs = (double)buf_ldT<T>(Ib[o], js) + qs;
      const double vN = (double)buf_ldT<T>(Ib[o], iN) + qN;
      const double vin = a.bnd[fs + kk[o]];
      double Fe, Fn;
      face_pair(vf, xf + 1 < nx ? ve : vf, xf > 0 ? vw : vf, vn, ys > 0 ? vs : vf, f0, f1, hdx,
                hdy, second, lim, Fe, Fn);
      double hu = 0.0, hsb = 0.0, hf = 0.0, hnv = 0.0;
      if (y0 > 0) {
        if (lane <= kRD && xu >= 0 && xu < nx) { hu = vu; hsb = su; }
        if (lane < kRD && xf >= 0 && xf < nx) hf = Fn;
      } else if (lane < kRD && d0 + lane < nx) {
        hf = vin;
      }
      if (y0 + 64 < ny && lane <= kRD && xn >= 0 && xn < nx) hnv = vN;
      if (lane <= kRD) {
        hal[wave][o][0][lane] = hu;
        hal[wave][o][1][lane] = hf;
        hal[wave][o][2][lane] = hnv;
        hal[wave][o][3][lane] = hsb;
      }
    }
  }
  // inflow on the local west face of the lane's row
  double inW[2];
  {
    const int yr = min(y, ny - 1);
    const int j = (q & 2) ? ny - 1 - yr : yr;
    const size_t fw = (size_t)((q & 1) ? ny + j : j) * a.K;
    inW[0] = a.bnd[fw + kk[0]];
    inW[1] = a.bnd[fw + kk[1]];
  }
  // ---- window u(d0-2, y), u(d0-1, y); then the load ring from step -1
  double uc[2], ue[2], subc = 0.0, sube = 0.0;
  {
    const unsigned i0 = (unsigned)(DS[d0 - 2] + y), i1 = (unsigned)(DS[d0 - 1] + y);
    const double q0 = buf_ld64(Qb, i0 * 8u), q1 = buf_ld64(Qb, i1 * 8u);
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      uc[o] = (double)buf_ldT<T>(Ib[o], i0) + q0;
      ue[o] = (double)buf_ldT<T>(Ib[o], i1) + q1;
    }
    if constexpr (kF32) { subc = buf_ld64(Ub, i0 * 8u); sube = buf_ld64(Ub, i1 * 8u); }
  }
  auto load = [&](RSlot<T> &sl, int d) {     // cell on diagonal d, lookahead on d + 1
    const unsigned ic = (unsigned)(DS[d] + y), il = (unsigned)(DS[d + 1] + y);
    sl.ic = ic;
    sl.ib[0] = buf_ldT<T>(Ib[0], il);
    sl.ib[1] = buf_ldT<T>(Ib[1], il);
    sl.dq = buf_ld64(Qb, il * 8u);
    if constexpr (kF32) sl.sube = buf_ld64(Ub, il * 8u);
    sl.src = buf_ld64(Sb, ic * 8u);
    sl.c0 = buf_ld128(Cb, ic * 48u);
    sl.c1 = buf_ld128(Cb, ic * 48u + 16u);
    sl.st = buf_ld128(Cb, ic * 48u + 32u);
    if constexpr (TD) {
      sl.in[0] = buf_ld64(Nb[0], ic * 8u);
      sl.in[1] = buf_ld64(Nb[1], ic * 8u);
    }
  };
  RSlot<T> ring[PF];
#pragma unroll
  for (int t = 0; t < PF; ++t) load(ring[t], d0 - 1 + t);
  double uw[2] = {0.0, 0.0}, Fe_p[2] = {0.0, 0.0}, Fn_p[2] = {0.0, 0.0}, subw = 0.0;
  double rr = 0.0;                            // sum of w r^2 over the lane's cells
  for (int sb = 0; sb < kRSteps; sb += PF) {
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int dd = sb + t - 1;              // diagonal d0 + dd
      RSlot<T> &sl = ring[t];
      if constexpr (kF32) { subw = subc; subc = sube; sube = sl.sube; }
      double sS = 0.0;
      if constexpr (kF32) sS = shr1_fill(subw, hal[wave][0][3][dd + 1]);
      const int x = d0 + dd - y;
      const bool ok = dd >= 0 && rowok && x >= 0 && x < nx;
      const double inv0 = sl.st.y;
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        uw[o] = uc[o]; uc[o] = ue[o]; ue[o] = (double)sl.ib[o] + sl.dq;
        // row below lane 0 / above lane 63 from the halo (LDS broadcasts)
        const double uS = shr1_fill(uw[o], hal[wave][o][0][dd + 1]);
        const double FnS = shr1_fill(Fn_p[o], hal[wave][o][1][dd < 0 ? 0 : dd]);
        const double uN = shl1_fill(ue[o], hal[wave][o][2][dd + 1]);
        const double u = uc[o];
        const double UE = x + 1 < nx ? ue[o] : u, UW = x > 0 ? uw[o] : u;
        const double UN = hn ? uN : u, US = hs ? uS : u;
        double Fe, Fn;
        face_pair(u, UE, UW, UN, US, sl.c0, sl.c1, hdx, hdy, second, lim, Fe, Fn);
        const double FeW = x > 0 ? Fe_p[o] : inW[o];
        double r = sl.src - sl.st.x * u - ax[o] * (Fe - FeW) - ay[o] * (Fn - FnS);
        if constexpr (TD) r += a.tdiag * sl.in[o];
        const double inv = rcp64(inv0 + (ax[o] + ay[o]));   // as in the recurrence
        double t0 = kF32 ? u - subc : u;
        const double tw = fma(-(ax[o] * inv), kF32 ? uw[o] - subw : uw[o], t0);
        t0 = x > 0 ? tw : t0;
        const double ts = fma(-(ay[o] * inv), kF32 ? uS - sS : uS, t0);
        t0 = hs ? ts : t0;
        buf_store((T)(t0 + r * inv), Ob[o], ok ? sl.ic * (unsigned)sizeof(T) : kNoCell);
        rr = ok ? fma(wr[o] * r, r, rr) : rr;
        Fe_p[o] = Fe;
        Fn_p[o] = Fn;
      }
      load(sl, d0 + dd + PF);                 // past the tile: unused
    }
  }
  // the wave's sum (fixed order), one partial per (tile, ordinate pair)
  rr = wave_sum64(rr);
  if (lane == 0) a.tres_part[slot] = rr;
}

template <typename T, bool TD = false, int RD = kRDSmall>
__global__ void __launch_bounds__(kRWaves * 64) k_resid(TArgs a) {
  if (a.state[1] != 0) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  // workgroup b runs on XCD b % 8; each XCD takes a contiguous run of
  // groups of ordinate pairs (quadrant-sorted) and walks the tiles for them
  const int G = (ordinate_pairs(a) + kRWaves - 1) / kRWaves;
  const int xc = blockIdx.x & 7, bi = blockIdx.x >> 3;
  const int gcnt = (G - xc + 7) >> 3;
  if (gcnt <= 0) return;
  const int tile = bi / gcnt;
  if (tile >= a.n_rtiles) return;
  int gstart = 0;
  for (int xp = 0; xp < xc; ++xp) gstart += (G - xp + 7) >> 3;
  const int pi = (gstart + bi % gcnt) * kRWaves + wave;
  if (pi >= ordinate_pairs(a)) return;
  int kA, kB;
  ordinate_pair(a, pi, kA, kB);
  resid_tile<T, TD, RD>(a, tile, kA, kB, wave, tile * ordinate_pairs(a) + pi);
}

// Batched residual: one workgroup per item (problem, tile, group of four
// ordinate pairs) of every problem that has not finished.
template <typename T>
__global__ void __launch_bounds__(kRWaves * 64) k_resid_batch(const TArgs *targs,
                                                             const int4 *items) {
  const __attribute__((address_space(4))) int *it =
      (const __attribute__((address_space(4))) int *)items + 4 * blockIdx.x;
  CTArgs &a = targs_at(targs, it[0]);
  if (a.state[1] != 0) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pi = it[2] * kRWaves + wave;
  if (pi >= ordinate_pairs(a)) return;
  int kA, kB;
  ordinate_pair(a, pi, kA, kB);
  // the problem's own tile length
  if (a.resid_rd == kRDLarge)
    resid_tile<T, false, kRDLarge>(a, it[1], kA, kB, wave, it[1] * ordinate_pairs(a) + pi);
  else
    resid_tile<T, false, kRDSmall>(a, it[1], kA, kB, wave, it[1] * ordinate_pairs(a) + pi);
}

// Recurrence v = bv + cx v_W + cy v_S for one ordinate per workgroup; lane t
// of a pass owns row y0 + t and at step s handles column s - t (every step
// one anti-diagonal). v_W is the lane's previous value, v_S lane t-1's (a DPP
// shift). A lane's value stays 0 until its row starts, and lane 0 of the
// bottom row gets 0 from below, so the inflow faces need no test: their
// terms multiply 0. Across waves the waves run LAG steps apart: wave w does
// step s at time s + w LAG and the workgroup meets at a barrier every LAG
// times, so the top lane's values that wave w+1 needs were written at least
// one barrier earlier; they pass through an LDS ring of 4 LAG steps and are
// read once per LAG steps. With MULTI, rows beyond one pass are handed over
// in rowbuf (alternate halves, so a pass never writes what it reads).
//
// SPLIT spreads the rows of one ordinate over np workgroups (part p takes
// rows [p rows_pp, (p + 1) rows_pp)): a wave's step costs about the same
// whatever else runs, but waves that share a SIMD take turns, so parts of
// about four waves keep one wave per SIMD. The top row of part p reaches
// part p + 1 through hand[(kk (np - 1) + p) nx + x] (hand_take / hand_put).
// Part p + 1 has the higher workgroup index, so it is dispatched after part
// p and a waiting part never holds back the part it waits for; a wait still
// ends after kHandSpin polls, setting hand_err (the results are then not
// valid).
constexpr int kCPF = 8;              // steps of loads in flight
constexpr int kCLag = 8;
constexpr int kCMaxW = 16;           // up to 1024 rows per pass

// Loads use the index dso[d] + y of the lane's row on the step's diagonal
// d: for a lane with no cell it points at another diagonal or out of the
// buffer (the hardware returns 0 there), and the value is never used.
//
// The recurrence runs in the storage type T: FP64, or FP32 in the
// FP32-mixed form, where its values are deviations from phi^m/(4 pi) (small
// where the medium is thick) and its right-hand side already holds the
// residual formed in FP64; the diagonal sigma_t + shift then comes from an
// FP32 copy (sdq_f) and 1/d from the single-precision reciprocal.
__device__ inline float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_t(double x) { return rcp64(x); }

template <typename T, bool MULTI, bool SPLIT = false, class A>
__device__ __forceinline__ void chain_ordinate(A &a, const int kk, const int part = 0,
                                               const int np = 1) {
  constexpr int PF = kCPF, LAG = kCLag, R = 4 * kCLag;
  constexpr bool kF32 = sizeof(T) == 4;
  static_assert((R & (R - 1)) == 0 && LAG == PF, "ring sizes");
  static_assert(!(SPLIT && MULTI), "a split recurrence runs one pass per part");
  static_assert(kCMaxW * kCLag + 2 * kCPF + kCLag <= kDiagPad, "diagonal table padding");
  const int q = quadrant_of(a, kk);
  const int nx = a.nx, ny = a.ny, N = a.N;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave
  const int rows_pp = blockDim.x;
  const T ax = (T)a.amu[kk], ay = (T)a.aeta[kk], axy = (T)(a.amu[kk] + a.aeta[kk]);
  const T *Ok = Iout_of<T>(a) + (size_t)kk * N;
  const __amdgpu_buffer_rsrc_t Ob = buf_rsrc(Ok, (size_t)N * sizeof(T));
  const __amdgpu_buffer_rsrc_t Sb =
      kF32 ? buf_rsrc(a.sdq_f + (size_t)q * N, (size_t)N * 4)
           : buf_rsrc(a.sdq + (size_t)q * N, (size_t)N * 8);
  // read through the constant address space: wave-uniform reads of it are
  // scalar loads and stay out of the vector memory counter
  const __attribute__((address_space(4))) int *DS =
      (const __attribute__((address_space(4))) int *)(a.dso + kDiagPad);
  double *RB = a.rowbuf + (size_t)kk * 3 * nx;
  __shared__ T edge[kCMaxW][R];
  // SPLIT: Hr the part below's top row (read), Hw this part's (written;
  // an empty resource for the top part)
  unsigned long long *Hr = nullptr;
  __amdgpu_buffer_rsrc_t Hw = buf_rsrc(nullptr, 0);
  if constexpr (SPLIT) {
    unsigned long long *H = a.hand + (size_t)kk * (np - 1) * nx;
    if (part > 0) Hr = H + (size_t)(part - 1) * nx;
    if (part + 1 < np) Hw = buf_rsrc(H + (size_t)part * nx, (size_t)nx * 8);
  }
  const int ybeg = SPLIT ? part * rows_pp : 0;
  const int yend = SPLIT ? min(ny, ybeg + rows_pp) : ny;
  for (int y0 = ybeg, pass = 0; y0 < yend; y0 += rows_pp, ++pass) {
    const int rows = min(rows_pp, ny - y0);
    const int nw = (rows + 63) >> 6;
    const int y = y0 + tid;
    const bool rowok = tid < rows;
    const int xo = rowok ? tid : (1 << 30);   // x = s - xo; rows past the grid never act
    const bool handoff = MULTI && rowok && tid == rows - 1 && y0 + rows < ny;
    const __amdgpu_buffer_rsrc_t RBr = buf_rsrc(RB + (pass & 1) * nx, (size_t)nx * 8);
    const __amdgpu_buffer_rsrc_t RBw = buf_rsrc(RB + ((pass + 1) & 1) * nx, (size_t)nx * 8);
    const int nsteps = nx + rows - 1;
    const int tend = ((nsteps + (nw - 1) * LAG + LAG - 1) / LAG) * LAG;
    const int s0 = -wave * LAG;               // this wave's step at time 0
    // The ring is filled by a first block of steps before any lane's row
    // starts (no lane acts there), so every block of the loop, the first
    // included, runs the same code and the loads keep PF steps in flight.
    T rb_b[PF] = {}, rb_sd[PF] = {};
    double rb_v[PF] = {};
    unsigned rb_i[PF] = {};
    auto load = [&](int t, int so, int st) {  // step st, row-0 index so of its diagonal
      const unsigned i = (unsigned)(so + y);
      rb_i[t] = i;
      if constexpr (sizeof(T) == 8) {
        rb_b[t] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(Ob, (int)(i * 8u), 0, 0));
        rb_sd[t] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(Sb, (int)(i * 8u), 0, 0));
      } else {
        rb_b[t] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(Ob, (int)(i * 4u), 0, 0));
        rb_sd[t] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(Sb, (int)(i * 4u), 0, 0));
      }
      if constexpr (MULTI) {
        // v below the first row of a later pass (column = step for lane 0)
        const unsigned c = (unsigned)min(max(st, 0), nx - 1);
        rb_v[t] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(RBr, (int)(c * 8u), 0, 0));
      }
    };
    T vp = 0;
    // SPLIT, wave 0 of a part above the first: lane l < LAG holds the hand-over
    // entry of column (block's first step) + l, loaded one block ahead; 0 for
    // columns outside the grid
    unsigned long long hv = 0;
    bool gave_up = false;                     // a wait timed out: wait no more
    const bool top_lane = SPLIT && tid == rows - 1;   // this part's top row
    // diagonal offsets of a block's loads, one block ahead: lane l holds that
    // of the block's load l, read back as a wave-uniform lane value (a vector
    // load, in order with the ring's, so no scalar-load wait in a block)
    int dsn = DS[y0 - LAG + s0 + PF + (lane & (LAG - 1))];
    // (the first one lands before the loop: still in flight at the loop
    // head, the wait pass would cover it conservatively in every block, with
    // all the ring's loads behind it)
    asm volatile("" : "+v"(dsn));
    for (int tb = -LAG; tb < tend; tb += LAG) {
      const int sb = tb + s0;                 // this wave's first step of the block
      const int dsc = dsn;
      dsn = DS[y0 + sb + LAG + PF + (lane & (LAG - 1))];
      // v below lane 0 for the block's steps: the wave below's top lane
      // (written at least one barrier ago), the part below, the previous
      // pass, or 0
      T bl[LAG];
      if (wave > 0) {
#pragma unroll
        for (int t2 = 0; t2 < LAG; ++t2) bl[t2] = edge[wave - 1][(sb - 1 + t2) & (R - 1)];
      } else if (SPLIT && part > 0) {
        double hb[LAG];
        hand_take<LAG>(Hr, nx, sb, hv, gave_up, a.hand_err, hb);   // lane 0's column is its step
#pragma unroll
        for (int t2 = 0; t2 < LAG; ++t2) bl[t2] = (T)hb[t2];
      } else {
#pragma unroll
        for (int t2 = 0; t2 < LAG; ++t2) bl[t2] = (MULTI && y0 > 0) ? (T)rb_v[t2] : (T)0;
      }
      int so[LAG];                            // diagonals of the loads issued in this block
#pragma unroll
      for (int t2 = 0; t2 < LAG; ++t2) so[t2] = __builtin_amdgcn_readlane(dsc, t2);
      T vv[LAG];
#pragma unroll
      for (int t2 = 0; t2 < LAG; ++t2) {
        const int s = sb + t2;
        const int x = s - xo;
        const bool act = (unsigned)x < (unsigned)nx;
        const T vS = shr1_fill(vp, bl[t2]);
        const T inv = rcp_t(rb_sd[t2] + axy);
        const T vn = fma(ax * inv, vp, fma(ay * inv, vS, rb_b[t2]));
        const T v = act ? vn : vp;
        buf_store(v, Ob, act ? rb_i[t2] * (unsigned)sizeof(T) : kNoCell);
        if constexpr (MULTI) buf_store((double)v, RBw, handoff && act ? (unsigned)x * 8u : kNoCell);
        if constexpr (SPLIT) {
          if (wave == nw - 1 && part + 1 < np)
            hand_put(Hw, (double)v, top_lane && act ? (unsigned)x * 8u : kNoCell);
        }
        vp = v;
        vv[t2] = v;
        load(t2, so[t2], s + PF);
      }
      // the top lane's values of the block, for the wave above
      if (lane == 63) {
#pragma unroll
        for (int t2 = 0; t2 < LAG; ++t2) edge[wave][(sb + t2) & (R - 1)] = vv[t2];
      }
      lds_barrier();
    }
    __syncthreads();   // the pass's row hand-off (rowbuf, global memory)
  }
}

template <typename T, bool MULTI>
__global__ void __launch_bounds__(kCMaxW * 64) k_chain(TArgs a) {
  if (a.state[1] != 0) return;
  chain_ordinate<T, MULTI>(a, xcd_ordinate(blockIdx.x, a.K));
}

// Split recurrence: workgroup b is part b / K of ordinate b % K (the same XCD
// for every part of an ordinate when K is a multiple of 8).
template <typename T>
__global__ void __launch_bounds__(kCMaxW * 64) k_chain_split(TArgs a, int np) {
  if (a.state[1] != 0) return;
  const int part = blockIdx.x / a.K;
  chain_ordinate<T, false, true>(a, xcd_ordinate(blockIdx.x - part * a.K, a.K), part, np);
}

// ---------------------------------------------------------------------------
// Pipelined transport step: the residual and the recurrence in one launch,
// the recurrence's right-hand side passed through LDS instead of HBM.
//
// Workgroup b is part p = b / K (rows [p 64 NB, (p + 1) 64 NB)) of ordinate
// xcd_ordinate(b % K), with 2 NB waves: wave w < NB runs the recurrence of
// band w (rows p 64 NB + 64 w + lane), wave NB + w forms the residual of the
// same band. Lane l of band w sits at row offset t = 64 w + l and at step s
// at column x = s - t, so a step is one anti-diagonal (s plus the part's
// first row), as in the split kernels. Time runs in blocks of LAG steps with
// one barrier per block. In block i the residual wave of band w forms steps
// [LAG (i - w), +LAG) and writes (bv, 1/d) per step and lane into LDS slot
// i & 1; the recurrence wave of band w takes steps [LAG (i - w - 1), +LAG)
// from slot (i - 1) & 1, written one barrier earlier.
//
// Neighbour rows. Inside a band they are the DPP-shifted lanes. The residual
// wave of band w > 0 takes u, F_n (and, FP32-mixed, phi^m/(4 pi)) of the row
// below from band w - 1's top lane through an LDS ring (that wave runs a
// block ahead); band 0 of part 0 has the south inflow there, and band 0 of a
// later part forms the face value of the row below itself (from I^m and the
// records, so it has the same bits as the part below). The row above a band
// runs later, so its u (I^m only) is loaded directly. These per-step values
// are loaded a block ahead into lanes 0..LAG-1 and broadcast with readlane.
// The recurrence waves are the split recurrence's steps: v of the row below
// from band w - 1's top lane (LDS ring), from part p - 1 (hand_take /
// hand_put), or 0 below the grid. Every value is formed by the same
// operations as in the split path, so the two give the same bits.
// ---------------------------------------------------------------------------
constexpr int kPLag = 8;            // steps per block (one barrier per block)
constexpr int kPRing = 4 * kPLag;   // the edge rings, in steps

template <typename T>
struct PPair {
  T bv, inv;           // the recurrence's right-hand side and 1/d
};

template <typename T>
struct PSlot {
  T ib;                // stored value at the lookahead cell (next diagonal)
  double dq;           // base/(4 pi) there
  double sube;         // FP32 mode: phi^m/(4 pi) there
  double src;          // source at the cell
  double2 c0, c1, st;  // its record
  double in;           // time-dependent form: I^n at the cell
};

// Loads of the per-step neighbour values of a residual block (lane j: step
// j of the block): the row above the band and, for band 0, the south inflow
// or the 5-point stencil of the row below the part.
struct PHalo {
  double nI, nq;                 // u of the row above: stored value, base/(4 pi)
  double vin;                    // south inflow (part 0)
  double fI, fq, eI, eq, wI, wq, uI, uq, sI, sq, sub;   // row below: the cell, E, W, N, S
  double2 f0, f1;                // its record
};

// The two roles run loops of their own (the same number of barriers), so
// that neither holds the other's registers. The recurrence waves, which
// have time to spare, also load and form the residual waves' neighbour
// values of the row above the band and of the row below band 0 a block
// ahead and pass them through LDS.
template <typename T, bool TD, int NB, int PF>
__device__ __forceinline__ void pipe_ordinate(const TArgs &a, const int kk, const int part,
                                              const int np) {
  constexpr bool kF32 = sizeof(T) == 4;
  constexpr int LAG = kPLag, R = kPRing;
  static_assert(LAG % PF == 0, "whole turns of the load ring per block");
  static_assert((R & (R - 1)) == 0 && R >= 4 * LAG, "ring sizes");
  static_assert(NB * LAG + 3 * LAG + PF + 2 <= kDiagPad, "diagonal table padding");
  const int q = quadrant_of(a, kk);
  const int nx = a.nx, ny = a.ny, N = a.N;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
  const bool res = wv >= NB;                    // a residual wave
  const int band = res ? wv - NB : wv;
  const int y0 = part * 64 * NB;                // the part's first row
  const int rows = min(64 * NB, ny - y0);
  const int nbw = (rows + 63) >> 6;             // bands with rows
  const int t = band * 64 + lane;               // row offset in the part
  const int y = y0 + t;
  const bool rowok = t < rows;
  const int nsteps = nx + rows - 1;
  const int tend = ((nsteps + (nbw - 1) * LAG + LAG - 1) / LAG) * LAG;
  const __attribute__((address_space(4))) int *DS =
      (const __attribute__((address_space(4))) int *)(a.dso + kDiagPad);
  const double axd = a.amu[kk], ayd = a.aeta[kk];
  const __amdgpu_buffer_rsrc_t Ib =
      buf_rsrc(Iin_of<T>(a) + (size_t)kk * N, (size_t)N * sizeof(T));
  const __amdgpu_buffer_rsrc_t Cb = buf_rsrc(a.cellq + (size_t)q * N * 6, (size_t)N * 48);
  const double *SRC = a.dynq + (size_t)q * 3 * N;
  const __amdgpu_buffer_rsrc_t Qb = buf_rsrc(SRC + N, (size_t)N * 8);
  const __amdgpu_buffer_rsrc_t Ub = buf_rsrc(SRC + 2 * N, (size_t)N * 8);
  const double hdx = 0.5 * a.dx, hdy = 0.5 * a.dy;
  const bool second = a.order >= 2, lim = a.limiter != 0;

  __shared__ PPair<T> pbuf[2][NB][LAG][64];
  __shared__ double pedge[NB][3][R];            // residual waves: u, F_n, sub of the top row
  __shared__ T cedge[NB][R];                    // recurrence waves: v of the top row
  __shared__ double hal[2][NB][4][LAG];         // u, F_n, sub below lane 0, u above lane 63

  if (res) {
    // ---------------------------------------------------------- residual wave
    const __amdgpu_buffer_rsrc_t Sb = buf_rsrc(SRC, (size_t)N * 8);
    __amdgpu_buffer_rsrc_t Nb = buf_rsrc(nullptr, 0);
    if constexpr (TD) Nb = buf_rsrc(a.In + (size_t)kk * N, (size_t)N * 8);
    const bool hn = y + 1 < ny, hs = y > 0;
    const T axy = (T)(axd + ayd);
    const double wk = a.w[kk];
    auto load = [&](PSlot<T> &sl, int s) {      // step s: the cell, and the lookahead cell
      const int D = s + y0;
      const unsigned ic = (unsigned)(DS[D] + y), il = (unsigned)(DS[D + 1] + y);
      sl.ib = buf_ldT<T>(Ib, il);
      sl.dq = buf_ld64(Qb, il * 8u);
      if constexpr (kF32) sl.sube = buf_ld64(Ub, il * 8u);
      sl.src = buf_ld64(Sb, ic * 8u);
      sl.c0 = buf_ld128(Cb, ic * 48u);
      sl.c1 = buf_ld128(Cb, ic * 48u + 16u);
      sl.st = buf_ld128(Cb, ic * 48u + 32u);
      if constexpr (TD) sl.in = buf_ld64(Nb, ic * 8u);
    };
    double inW = 0.0;                           // inflow on the local west face of the row
    {
      const int yr = min(y, ny - 1);
      const int j = (q & 2) ? ny - 1 - yr : yr;
      inW = a.bnd[(size_t)((q & 1) ? ny + j : j) * a.K + kk];
    }
    PSlot<T> ring[PF];
    double uw = 0.0, uc = 0.0, ue = 0.0, subw = 0.0, subc = 0.0, sube = 0.0;
    double Fe_p = 0.0, Fn_p = 0.0, rr = 0.0;
    double fU = 0.0, fFn = 0.0, fS = 0.0, fN = 0.0;   // lane j < LAG: step j's neighbour values
    if (band < nbw) {
      // window u(D - 1), u(D) of the first step's diagonal D, and the load ring
      const int s0 = -LAG * band;
      const unsigned i0 = (unsigned)(DS[s0 + y0 - 1] + y), i1 = (unsigned)(DS[s0 + y0] + y);
      uc = (double)buf_ldT<T>(Ib, i0) + buf_ld64(Qb, i0 * 8u);
      ue = (double)buf_ldT<T>(Ib, i1) + buf_ld64(Qb, i1 * 8u);
      if constexpr (kF32) { subc = buf_ld64(Ub, i0 * 8u); sube = buf_ld64(Ub, i1 * 8u); }
#pragma unroll
      for (int p = 0; p < PF; ++p) load(ring[p], s0 + p);
    }
    // Everything loaded so far (the ring, the window, the west inflow) lands
    // before the loop: with loads of the entry still counted at the loop
    // head, the compiler's wait for the loop-invariant inflow would cover
    // every load of the previous block and leave the ring one step deep.
    __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();                            // the first block's neighbour values
    for (int tb = -LAG, it = 0; tb < tend; tb += LAG, ++it) {
      if (band < nbw) {
        const int sb = tb + LAG - LAG * band;   // this block's first step
        if (lane < LAG) {
          fN = hal[it & 1][band][3][lane];
          if (band > 0) {                       // band - 1's top row, a block ago
            const int e = (sb - 1 + lane) & (R - 1);
            fU = pedge[band - 1][0][e];
            fFn = pedge[band - 1][1][e];
            fS = pedge[band - 1][2][e];
          } else {
            fU = hal[it & 1][band][0][lane];
            fFn = hal[it & 1][band][1][lane];
            fS = hal[it & 1][band][2][lane];
          }
        }
#pragma unroll
        for (int j = 0; j < LAG; ++j) {
          const int s = sb + j;
          PSlot<T> &sl = ring[j % PF];
          if constexpr (kF32) { subw = subc; subc = sube; sube = sl.sube; }
          uw = uc; uc = ue; ue = (double)sl.ib + sl.dq;
          const double uS = shr1_fill(uw, rdlane(fU, j));
          const double FnS = shr1_fill(Fn_p, rdlane(fFn, j));
          const double uN = shl1_fill(ue, rdlane(fN, j));
          double sS = 0.0;
          if constexpr (kF32) sS = shr1_fill(subw, rdlane(fS, j));
          const int x = s - t;
          const bool ok = rowok && x >= 0 && x < nx;
          const double u = uc;
          const double UE = x + 1 < nx ? ue : u, UW = x > 0 ? uw : u;
          const double UN = hn ? uN : u, US = hs ? uS : u;
          double Fe, Fn;
          face_pair(u, UE, UW, UN, US, sl.c0, sl.c1, hdx, hdy, second, lim, Fe, Fn);
          const double FeW = x > 0 ? Fe_p : inW;
          double r = sl.src - sl.st.x * u - axd * (Fe - FeW) - ayd * (Fn - FnS);
          if constexpr (TD) r += a.tdiag * sl.in;
          const double inv = rcp64(sl.st.y + (axd + ayd));   // as in the recurrence
          double t0 = kF32 ? u - subc : u;
          const double tw = fma(-(axd * inv), kF32 ? uw - subw : uw, t0);
          t0 = x > 0 ? tw : t0;
          const double ts = fma(-(ayd * inv), kF32 ? uS - sS : uS, t0);
          t0 = hs ? ts : t0;
          PPair<T> pp;
          pp.bv = (T)(t0 + r * inv);
          if constexpr (kF32) pp.inv = rcp_t((float)sl.st.y + axy);
          else pp.inv = inv;
          pbuf[it & 1][band][j][lane] = pp;
          rr = ok ? fma(wk * r, r, rr) : rr;
          Fe_p = Fe;
          Fn_p = Fn;
          if (lane == 63) {
            pedge[band][0][s & (R - 1)] = uc;
            pedge[band][1][s & (R - 1)] = Fn;
            pedge[band][2][s & (R - 1)] = subc;
          }
          load(sl, s + PF);
        }
      }
      lds_barrier();
    }
    // the wave's sum of w r^2 (fixed order), one partial per (ordinate, part, band)
    rr = wave_sum64(rr);
    if (lane == 0) a.tres_part[((size_t)kk * np + part) * NB + band] = rr;
  } else {
    // -------------------------------------------------------- recurrence wave
    const T ax = (T)axd, ay = (T)ayd;
    const __amdgpu_buffer_rsrc_t Ob =
        buf_rsrc(Iout_of<T>(a) + (size_t)kk * N, (size_t)N * sizeof(T));
    const int yN = y0 + 64 * band + 64;         // the row above the band
    const bool northed = yN < ny;
    const int yh = y0 - 1;                      // the row below the part
    auto ldT = [&](unsigned i, bool m) -> double {
      if constexpr (kF32)
        return (double)__builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(Ib, (int)(m ? i * 4u : kNoCell), 0, 0));
      else
        return buf_ld64(Ib, m ? i * 8u : kNoCell);
    };
    // Indices are formed arithmetically and every wave issues the same loads
    // (those it does not need go to kNoCell and read 0): a load whose address
    // came from another load, or loads on one side of a branch whose results
    // the two sides merge, would make the wave wait for them before its
    // recurrence steps.
    const int nd = nx + ny - 1;
    auto cidx = [&](int xx, int yy) {           // storage index, clamped into the grid
      xx = min(max(xx, 0), nx - 1);
      yy = min(max(yy, 0), ny - 1);
      return (unsigned)(dg_row0(xx + yy, nx, ny) + yy);
    };
    const __amdgpu_buffer_rsrc_t Bb = buf_rsrc(a.bnd, (size_t)a.nbf * a.K * 8);
    const bool mN = lane < LAG && northed;
    const bool mB = lane < LAG && band == 0 && part == 0;
    const bool mS = lane < LAG && band == 0 && part > 0;
    auto halo_load = [&](PHalo &h, int sbn) {   // lane j < LAG: step sbn + j
      const int s = sbn + lane;
      // lane 63's north neighbour, on the next diagonal
      const unsigned iN = (unsigned)(dg_row0(min(max(s + y0 + 1, 0), nd - 1), nx, ny) + yN);
      h.nI = ldT(iN, mN);
      h.nq = buf_ld64(Qb, mN ? iN * 8u : kNoCell);
      // south inflow of lane 0's column (the step)
      const int xi = min(max(s, 0), nx - 1);
      const int gi = (q & 1) ? nx - 1 - xi : xi;
      const unsigned fb = (unsigned)(((q & 2) ? 2 * ny + nx + gi : 2 * ny + gi) * a.K + kk);
      h.vin = buf_ld64(Bb, mB ? fb * 8u : kNoCell);
      // the row below the part around lane 0's column
      const unsigned jf = cidx(s, yh), je = cidx(s + 1, yh), jw = cidx(s - 1, yh);
      const unsigned jn = cidx(s, y0), js = cidx(s, yh - 1);
      h.fI = ldT(jf, mS); h.fq = buf_ld64(Qb, mS ? jf * 8u : kNoCell);
      h.eI = ldT(je, mS); h.eq = buf_ld64(Qb, mS ? je * 8u : kNoCell);
      h.wI = ldT(jw, mS); h.wq = buf_ld64(Qb, mS ? jw * 8u : kNoCell);
      h.uI = ldT(jn, mS); h.uq = buf_ld64(Qb, mS ? jn * 8u : kNoCell);
      h.sI = ldT(js, mS); h.sq = buf_ld64(Qb, mS ? js * 8u : kNoCell);
      h.f0 = buf_ld128(Cb, mS ? jf * 48u : kNoCell);
      h.f1 = buf_ld128(Cb, mS ? jf * 48u + 16u : kNoCell);
      h.sub = kF32 ? buf_ld64(Ub, mS ? jf * 8u : kNoCell) : 0.0;
    };
    auto halo_put = [&](const PHalo &h, int sbn, int slot) {
      const int x = sbn + lane;
      const double u = h.fI + h.fq, ve = h.eI + h.eq, vw = h.wI + h.wq;
      const double vn = h.uI + h.uq, vs = h.sI + h.sq;
      double Fe, Fn;
      face_pair(u, x + 1 < nx ? ve : u, x > 0 ? vw : u, vn, yh > 0 ? vs : u, h.f0, h.f1, hdx, hdy,
                second, lim, Fe, Fn);
      const bool below = band == 0 && part > 0;
      if (lane < LAG) {
        hal[slot][band][0][lane] = below ? u : 0.0;
        hal[slot][band][1][lane] = below ? Fn : h.vin;
        hal[slot][band][2][lane] = below && kF32 ? h.sub : 0.0;
        hal[slot][band][3][lane] = northed ? h.nI + h.nq : 0.0;
      }
    };
    unsigned long long *Hr = nullptr;
    __amdgpu_buffer_rsrc_t Hw = buf_rsrc(nullptr, 0);
    {
      unsigned long long *H = a.hand + (size_t)kk * (np - 1) * nx;
      if (part > 0) Hr = H + (size_t)(part - 1) * nx;
      if (part + 1 < np) Hw = buf_rsrc(H + (size_t)part * nx, (size_t)nx * 8);
    }
    const bool top_lane = t == rows - 1;        // the part's top row
    T vp = 0;
    unsigned long long hv = 0;
    bool gave_up = false;
    PHalo hl;
    if (band < nbw) {                           // the residual wave's first block
      halo_load(hl, -LAG * band);
      halo_put(hl, -LAG * band, 0);
    }
    lds_barrier();
    for (int tb = -LAG, it = 0; tb < tend; tb += LAG, ++it) {
      if (band < nbw) {
        const int sbr = tb + 2 * LAG - LAG * band;   // the residual wave's next block
        halo_load(hl, sbr);
        const int sb = tb - LAG * band;         // this block's first step
        T bl[LAG];                              // v below lane 0
        if (band > 0) {
#pragma unroll
          for (int j = 0; j < LAG; ++j) bl[j] = cedge[band - 1][(sb - 1 + j) & (R - 1)];
        } else if (part > 0) {
          double hb[LAG];
          hand_take<LAG>(Hr, nx, sb, hv, gave_up, a.hand_err, hb);   // lane 0's column is its step
#pragma unroll
          for (int j = 0; j < LAG; ++j) bl[j] = (T)hb[j];
        } else {
#pragma unroll
          for (int j = 0; j < LAG; ++j) bl[j] = (T)0;
        }
        T vv[LAG];
#pragma unroll
        for (int j = 0; j < LAG; ++j) {
          const int s = sb + j;
          const int x = s - t;
          const bool act = rowok && (unsigned)x < (unsigned)nx;
          const PPair<T> pv = pbuf[(it + 1) & 1][band][j][lane];
          const T vS = shr1_fill(vp, bl[j]);
          const T vn = fma(ax * pv.inv, vp, fma(ay * pv.inv, vS, pv.bv));
          const T v = act ? vn : vp;
          buf_store(v, Ob, act ? (unsigned)(DS[y0 + s] + y) * (unsigned)sizeof(T) : kNoCell);
          if (band == nbw - 1 && part + 1 < np)
            hand_put(Hw, (double)v, top_lane && act ? (unsigned)x * 8u : kNoCell);
          vp = v;
          vv[j] = v;
        }
        if (lane == 63) {
#pragma unroll
          for (int j = 0; j < LAG; ++j) cedge[band][(sb + j) & (R - 1)] = vv[j];
        }
        halo_put(hl, sbr, (it + 1) & 1);
      }
      lds_barrier();
    }
  }
}

template <typename T, bool TD, int NB, int PF>
__global__ void __launch_bounds__(2 * NB * 64) k_pipe(TArgs a, int np) {
  if (a.state[1] != 0) return;
  const int part = blockIdx.x / a.K;
  pipe_ordinate<T, TD, NB, PF>(a, xcd_ordinate(blockIdx.x - part * a.K, a.K), part, np);
}

__global__ void k_fill_u64(unsigned long long *p, size_t n, unsigned long long v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Batched recurrence: a persistent launch whose workgroups take work items
// (problem, ordinate) from a shared counter in the order of the item table
// (longest first) and run the recurrence with that problem's arguments, in
// row passes of blockDim rows; problems that have finished are skipped.
// Every workgroup leaves once the counter passes the table.
template <typename T>
__global__ void __launch_bounds__(kCMaxW * 64)
    k_chain_batch(const TArgs *targs, const int2 *items, int n_items, int *counter) {
  __shared__ int s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const int2 pk = items[it];
    CTArgs &a = targs_at(targs, pk.x);
    if (a.state[1] == 0) chain_ordinate<T, true>(a, pk.y);
  }
}

__global__ void k_zero_int(int *p) { *p = 0; }

// phi, F of I^{m+1/2} in two passes: per quadrant and tile, sums over the
// quadrant's ordinates into partials at the caller's cell index (below);
// then the four partials are added in a fixed order. dg_cell: the cell (x,
// y) of stored index t.
__device__ inline void dg_cell(long long t, int nx, int ny, int &x, int &y) {
  int lo = 0, hi = nx + ny - 2;               // find d with off(d) <= t < off(d+1)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (dg_off(mid, nx, ny) <= t) lo = mid; else hi = mid - 1;
  }
  y = dg_ylo(lo, nx) + (int)(t - dg_off(lo, nx, ny));
  x = lo - y;
}

// Sum of src^2 = ((sigma_s phi^m + q)/(4 pi))^2 over the cells of one block
// of 256 (natural cell order), for the relative transport residual; every
// thread of the block takes part, thread 0 stores the block's sum.
__device__ __forceinline__ void src2_block(const TArgs &a, const int blk) {
  __shared__ double red[256];
  const int c = blk * 256 + (int)threadIdx.x;
  const double v = c < a.N ? a.src[c] : 0.0;
  red[threadIdx.x] = v * v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && a.state[1] == 0) a.src2_part[blk] = red[0];
}

// Moment partials of one quadrant over one MT x MT tile of the caller's
// grid (MT = 16 or 32), MT^2 / 256 cells per thread. In the quadrant's
// mirrored frame the tile is a square whose anti-diagonals are contiguous
// runs (up to MT cells) of the stored intensity: the square's cells are
// numbered in anti-diagonal order and thread t takes cells t, t + 256, ...,
// so the loads of a wave run along those runs; the sums go through LDS and
// the partials are stored by rows of the caller's grid. Larger tiles waste
// less of the cache lines at the runs' ends; smaller ones give small grids
// more workgroups. ftp (transport-face HoT): the thread also forms its
// cells' interior face fluxes.
// cell t of a kMT x kMT square in anti-diagonal order (diagonal e = u + w,
// then w): its place (u, w) in the square
template <int kMT>
__device__ inline void square_diag(int t, int &u, int &w) {
  int e = 0, before = 0;
  for (;; ++e) {
    const int len = e < kMT ? e + 1 : 2 * kMT - 1 - e;
    if (t < before + len) break;
    before += len;
  }
  w = (e < kMT ? 0 : e - kMT + 1) + (t - before);
  u = e - w;
}

template <typename T>
__device__ void face_flux_q(const TArgs &a, double *ftp, const long long t, const int q);

template <typename T, int kMT>
__device__ __forceinline__ void moments_tile(const TArgs &a, double *part, double *ftp,
                                             const int tile, const int q) {
  constexpr int kMC = kMT * kMT / 256;
  static_assert(kMC * 256 == kMT * kMT, "whole cells per thread");
  __shared__ double sm[3][kMT * kMT];
  const int f1 = a.state[1];   // tested once the first values are loaded
  const int nx = a.nx, ny = a.ny, N = a.N;
  const int tw = (nx + kMT - 1) / kMT;
  const int i0 = (tile % tw) * kMT, j0 = (tile / tw) * kMT;
  int u[kMC], w[kMC];
  bool in[kMC];
  long long t[kMC];
#pragma unroll
  for (int h = 0; h < kMC; ++h) {
    square_diag<kMT>((int)threadIdx.x + 256 * h, u[h], w[h]);
    // the square in the quadrant's frame: local x runs against x when the
    // quadrant is mirrored in x, local y against y when mirrored in y
    const int xl = (q & 1) ? nx - i0 - kMT + u[h] : i0 + u[h];
    const int yl = (q & 2) ? ny - j0 - kMT + w[h] : j0 + w[h];
    in[h] = xl >= 0 && xl < nx && yl >= 0 && yl < ny;
    t[h] = in[h] ? dg_idx(xl, yl, nx, ny) : 0;
    if (ftp && in[h]) face_flux_q<T>(a, ftp, t[h], q);
  }
  const T *O = Iout_of<T>(a);
  // weights through the constant address space (scalar loads); each cell's
  // ordinates are loaded eight at a time (all the thread's cells at once)
  // before they are summed, in the same order as one at a time
  typedef const __attribute__((address_space(4))) double cdouble;
  cdouble *W = (cdouble *)a.w, *WM = (cdouble *)a.wmu, *WE = (cdouble *)a.weta;
  double s0[kMC], sx[kMC], sy[kMC];
  const int kb = a.qoff[q], ke = a.qoff[q + 1];
  if constexpr (sizeof(T) == 4) {
    // FP32-mixed form: the stored deviations are summed in FP32, each group
    // of eight ordinates as a balanced tree and the groups in order (the
    // rounding of the sum stays near that of the FP32 values themselves);
    // the combine adds the phi^m/(4 pi) part in FP64
    typedef const __attribute__((address_space(4))) float cfloat;
    cfloat *Wf = (cfloat *)a.w_f, *WMf = Wf + a.K, *WEf = Wf + 2 * a.K;
    float f0[kMC] = {}, fx[kMC] = {}, fy[kMC] = {};
    auto tree8 = [](const float (&p)[8]) {
      return ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    };
    int kk = kb;
    for (; kk + 8 <= ke; kk += 8) {
      float v[kMC][8];
#pragma unroll
      for (int h = 0; h < kMC; ++h)
#pragma unroll
        for (int m = 0; m < 8; ++m) v[h][m] = in[h] ? (float)O[(size_t)(kk + m) * N + t[h]] : 0.f;
#pragma unroll
      for (int h = 0; h < kMC; ++h) {
        float p0[8], px[8], py[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          p0[m] = Wf[kk + m] * v[h][m];
          px[m] = WMf[kk + m] * v[h][m];
          py[m] = WEf[kk + m] * v[h][m];
        }
        f0[h] += tree8(p0);
        fx[h] += tree8(px);
        fy[h] += tree8(py);
      }
    }
    for (; kk < ke; ++kk) {
#pragma unroll
      for (int h = 0; h < kMC; ++h) {
        const float v = in[h] ? (float)O[(size_t)kk * N + t[h]] : 0.f;
        f0[h] = fmaf(Wf[kk], v, f0[h]);
        fx[h] = fmaf(WMf[kk], v, fx[h]);
        fy[h] = fmaf(WEf[kk], v, fy[h]);
      }
    }
#pragma unroll
    for (int h = 0; h < kMC; ++h) {
      s0[h] = (double)f0[h]; sx[h] = (double)fx[h]; sy[h] = (double)fy[h];
    }
  } else {
#pragma unroll
    for (int h = 0; h < kMC; ++h) s0[h] = sx[h] = sy[h] = 0.0;
    int kk = kb;
    for (; kk + 8 <= ke; kk += 8) {
      double v[kMC][8];
#pragma unroll
      for (int h = 0; h < kMC; ++h)
#pragma unroll
        for (int m = 0; m < 8; ++m) v[h][m] = in[h] ? (double)O[(size_t)(kk + m) * N + t[h]] : 0.0;
#pragma unroll
      for (int h = 0; h < kMC; ++h)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          s0[h] += W[kk + m] * v[h][m];
          sx[h] += WM[kk + m] * v[h][m];
          sy[h] += WE[kk + m] * v[h][m];
        }
    }
    for (; kk < ke; ++kk) {
#pragma unroll
      for (int h = 0; h < kMC; ++h) {
        const double v = in[h] ? (double)O[(size_t)kk * N + t[h]] : 0.0;
        s0[h] += W[kk] * v;
        sx[h] += WM[kk] * v;
        sy[h] += WE[kk] * v;
      }
    }
  }
  if (f1 != 0) return;   // the whole block
#pragma unroll
  for (int h = 0; h < kMC; ++h) {
    // place in the tile of the caller's grid
    const int l = ((q & 2) ? kMT - 1 - w[h] : w[h]) * kMT + ((q & 1) ? kMT - 1 - u[h] : u[h]);
    sm[0][l] = s0[h];
    sm[1][l] = sx[h];
    sm[2][l] = sy[h];
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < kMC; ++h) {
    const int l = (int)threadIdx.x + 256 * h;
    const int i = i0 + (l & (kMT - 1)), j = j0 + l / kMT;
    if (i < nx && j < ny) {
      const size_t c = (size_t)j * nx + i;
      part[(size_t)(3 * q) * N + c] = sm[0][l];
      part[(size_t)(3 * q + 1) * N + c] = sm[1][l];
      part[(size_t)(3 * q + 2) * N + c] = sm[2][l];
    }
  }
}

// src^2 over the blocks of 256 cells (natural order) that go with moment
// tile `tile`: blocks kMC tile .. kMC tile + kMC - 1, those below nbc (the
// tiles number at least nbc / kMC)
template <int kMT>
__device__ __forceinline__ void src2_tile(const TArgs &a, const int tile) {
  constexpr int kMC = kMT * kMT / 256;
  const int nbc = (a.N + 255) / 256;
#pragma unroll
  for (int h = 0; h < kMC; ++h)
    if (kMC * tile + h < nbc) src2_block(a, kMC * tile + h);
}

// Transport fluxes through the interior faces (GSIS with transport-face HoT,
// Sec. 3.1 in Alcouffe's full form): per quadrant and stored cell, the sums
// over the quadrant's ordinates of w_k mu_k I_e and w_k eta_k I_n, with I_e,
// I_n the cell's second-order values on its local east and north faces (the
// residual's reconstruction, Eqs. Ii,k and Iij, of I^{m+1/2}). In the
// quadrant's frame the flow leaves through those faces, so the cell is their
// upwind cell. Each sum is stored at the face's place in the caller's grid:
// the east (+x) face of cell c, or of c - 1 when the quadrant is mirrored in
// x; the north face of c, or of c - nx when mirrored in y.
template <typename T>
__device__ void face_flux_q(const TArgs &a, double *ftp, const long long t, const int q) {
  const int f1 = a.state[1];
  if (t >= a.N) return;
  const int nx = a.nx, ny = a.ny, N = a.N;
  int x, y;
  dg_cell(t, nx, ny, x, y);
  const int c = gcell(a, q, x, y);
  const bool he = x + 1 < nx, hw = x > 0, hn = y + 1 < ny, hs = y > 0;
  if (!he && !hn) return;                     // both outgoing faces are walls
  const long long iE = he ? dg_idx(x + 1, y, nx, ny) : t, iW = hw ? dg_idx(x - 1, y, nx, ny) : t;
  const long long iN = hn ? dg_idx(x, y + 1, nx, ny) : t, iS = hs ? dg_idx(x, y - 1, nx, ny) : t;
  const double2 *R = reinterpret_cast<const double2 *>(a.cellq + ((size_t)q * N + t) * 6);
  const double2 c0 = R[0], c1 = R[1];
  const double *SUB = a.dynq + ((size_t)q * 3 + 2) * N;
  const double sc = a.fp32 ? SUB[t] : 0.0, se = a.fp32 ? SUB[iE] : 0.0;
  const double sw = a.fp32 ? SUB[iW] : 0.0, sn = a.fp32 ? SUB[iN] : 0.0;
  const double ss = a.fp32 ? SUB[iS] : 0.0;
  const T *O = Iout_of<T>(a);
  const double hdx = 0.5 * a.dx, hdy = 0.5 * a.dy;
  const bool second = a.order >= 2, lim = a.limiter != 0;
  double pe = 0.0, pn = 0.0;
  for (int kk = a.qoff[q]; kk < a.qoff[q + 1]; ++kk) {
    const T *Ok = O + (size_t)kk * N;
    const double u = (double)Ok[t] + sc;
    const double UE = he ? (double)Ok[iE] + se : u, UW = hw ? (double)Ok[iW] + sw : u;
    const double UN = hn ? (double)Ok[iN] + sn : u, US = hs ? (double)Ok[iS] + ss : u;
    double Fe, Fn;
    face_pair(u, UE, UW, UN, US, c0, c1, hdx, hdy, second, lim, Fe, Fn);
    pe += a.wmu[kk] * Fe;
    pn += a.weta[kk] * Fn;
  }
  if (f1 != 0) return;
  if (he) ftp[(size_t)(2 * q) * N + ((q & 1) ? c - 1 : c)] = pe;
  if (hn) ftp[(size_t)(2 * q + 1) * N + ((q & 2) ? c - nx : c)] = pn;
}

// Tiles by XCD: the tiles (row-major) fall into 8 runs of ts = ceil(ntile /
// 8), one per XCD, so tiles whose stored diagonals share cache lines mostly
// meet in one L2. Block b (of a range that starts at a multiple of 8) runs
// on XCD b % 8 and takes tile (b % 8) ts + b / 8, none past the grid.
__device__ inline int xcd_tile(int b, int ts) { return (b & 7) * ts + (b >> 3); }

// Moment partials: block (tile slot, quadrant); the quadrant-0 blocks also
// sum src^2 over the tile's blocks of 256 cells (src2_tile).
template <typename T, int MT>
__global__ void k_moments_q(TArgs a, double *part, int ntile, int ts) {
  const int tile = xcd_tile(blockIdx.x, ts);
  if (tile >= ntile || (blockIdx.x >> 3) >= ts) return;
  if (blockIdx.y == 0) src2_tile<MT>(a, tile);
  moments_tile<T, MT>(a, part, nullptr, tile, blockIdx.y);
}

// Batched launches: bt maps block -> (problem, tile of that problem, or -1:
// none), each problem's tiles in runs by XCD as above; kBatchMT x kBatchMT
// tiles.
constexpr int kBatchMT = 32;
template <typename T>
__global__ void k_moments_q_b(const TArgs *tas, const int2 *bt) {
  const int2 v = bt[blockIdx.x];
  if (v.y < 0) return;
  const TArgs &a = tas[v.x];
  if (blockIdx.y == 0) src2_tile<kBatchMT>(a, v.y);
  moments_tile<T, kBatchMT>(a, a.mom_part, nullptr, v.y, blockIdx.y);
}

__device__ __forceinline__ void moments_combine(const TArgs &a, const double *part, const int c) {
  const int f1 = a.state[1];   // tested after the loads
  if (c >= a.N) return;
  double v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = part[(size_t)k * a.N + c];
  const double ph = a.fp32 ? a.phi[c] : 0.0;
  if (f1 != 0) return;
  double s0 = 0, sx = 0, sy = 0;
  for (int q = 0; q < 4; ++q) {
    s0 += v[3 * q];
    sx += v[3 * q + 1];
    sy += v[3 * q + 2];
  }
  if (a.fp32) {                               // I^{m+1/2} = Itilde + phi^m/(4 pi)
    const double sub = ph / kFourPi;
    s0 += sub * a.sw; sx += sub * a.swm; sy += sub * a.swe;
  }
  a.phih[c] = s0; a.Fx[c] = sx; a.Fy[c] = sy;
}

__global__ void k_moments_combine(TArgs a, const double *part) {
  moments_combine(a, part, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void k_moments_combine_b(const TArgs *tas, const int2 *bt) {
  const int2 v = bt[blockIdx.x];
  const TArgs &a = tas[v.x];
  moments_combine(a, a.mom_part, v.y * blockDim.x + threadIdx.x);
}

// Wall face f: its side (0 W, 1 E, 2 S, 3 N) and position along it, and
// ordinate kk's term w (Omega . n_out) I of F_T . n_out there.
__device__ inline void face_side(const TArgs &a, const int f, int &side, int &pos) {
  if (f < a.ny) { side = 0; pos = f; }                       // W
  else if (f < 2 * a.ny) { side = 1; pos = f - a.ny; }        // E
  else if (f < 2 * a.ny + a.nx) { side = 2; pos = f - 2 * a.ny; }   // S
  else { side = 3; pos = f - 2 * a.ny - a.nx; }               // N
}
__device__ __forceinline__ double face_term(const TArgs &a, const int f, const int side,
                                            const int pos, const int kk) {
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
    const long long base = (long long)kk * a.N;
    const double *SUB = a.dynq + ((size_t)q * 3 + 2) * a.N;
    auto ld = [&](int x, int y) {
      const long long o = dg_idx(x, y, a.nx, a.ny);
      if (a.fp32) return (double)Iout_of<float>(a)[base + o] + SUB[o];
      return Iout_of<double>(a)[base + o];
    };
    double Fe, Fn;
    out_faces(a, q, xl, yl, ld, Fe, Fn);
    val = side < 2 ? Fe : Fn;
  }
  return won * val;
}

// F_T . n_out on wall face f: one wave, lanes over ordinates, a fixed-order
// wave sum
__device__ __forceinline__ void boundary_flux_wave(const TArgs &a, const int f) {
  const int f1 = a.state[1];
  const int lane = threadIdx.x & 63;
  int side, pos;
  face_side(a, f, side, pos);
  double acc = 0.0;
  for (int kk = lane; kk < a.K; kk += 64) acc += face_term(a, f, side, pos, kk);
  acc = wave_sum64(acc);
  if (lane == 0 && f1 == 0) a.bflux[f] = acc;
}

// The boundary faces' F_T . n (blocks [0, nbf)) and the per-quadrant moment
// partials (the other blocks, quadrant-major) in one launch: both only read
// the swept intensity; the four partials are combined by the HoT kernel.
// With ftp (transport-face HoT) the moment blocks also form the quadrant's
// interior face fluxes.
template <typename T, int MT>
__global__ void k_moments_q_bflux(TArgs a, double *part, int nbf8, int ntile, int ts,
                                  double *ftp) {
  // nbf8: blocks of four wall faces (one per wave), rounded up to a
  // multiple of 8
  const int b = (int)blockIdx.x - nbf8;
  if (b < 0) {
    const int f = 4 * (int)blockIdx.x + ((int)threadIdx.x >> 6);
    if (f < a.nbf) boundary_flux_wave(a, f);
    return;
  }
  const int q = b / (8 * ts), r = b - q * 8 * ts;
  const int tile = xcd_tile(r, ts);
  if (tile >= ntile || (r >> 3) >= ts) return;
  if (q == 0) src2_tile<MT>(a, tile);
  moments_tile<T, MT>(a, part, ftp, tile, q);
}

// Batched wall faces: four (problem, face) entries per workgroup, a wave each.
__global__ void k_boundary_flux_b(const TArgs *tas, const int2 *bt, int n) {
  const int e = 4 * (int)blockIdx.x + ((int)threadIdx.x >> 6);
  if (e >= n) return;
  const int2 v = bt[e];
  boundary_flux_wave(tas[v.x], v.y);
}

}  // namespace

template <typename T>
void launch_fused(const TArgs &a, const PlanDev &P, int rows, hipStream_t s) {
  const int w = rows / 64;
  const bool general = P.ny > rows || P.nx > kSouthCap;
  if (general)
    hipLaunchKernelGGL((k_sweep_fused<2, 16, true, T>), dim3(P.K), dim3(rows), 0, s, a);
  else if (w <= 4)
    hipLaunchKernelGGL((k_sweep_fused<6, 4, false, T>), dim3(P.K), dim3(rows), 0, s, a);
  else if (w <= 8)
    hipLaunchKernelGGL((k_sweep_fused<4, 8, false, T>), dim3(P.K), dim3(rows), 0, s, a);
  else
    hipLaunchKernelGGL((k_sweep_fused<2, 16, false, T>), dim3(P.K), dim3(rows), 0, s, a);
}

namespace {
int sweep_rows(const PlanDev &P) {
  const int rows = ((P.ny + 63) / 64) * 64;
  return rows > 1024 ? 1024 : rows;
}
}  // namespace

// sweep_impl 0: residual kernel, then the recurrence in place; 1: plain
// two-kernel reference (FP64 only; FP32 falls back to the fused kernel);
// 2: fused wavefront sweep; 3: pipelined residual + recurrence (2 and 3 put
// nothing in the residual phase).
void launch_residual(const PlanDev &P, hipStream_t s) {
  const TArgs a = make_args(P);
  if (P.sweep_impl == 2 || P.sweep_impl == 3 || (P.sweep_impl == 1 && a.fp32)) return;
  if (P.sweep_impl == 1) {
    hipLaunchKernelGGL(k_residual, dim3((P.N + 255) / 256, P.K), dim3(256), 0, s, a);
    return;
  }
  int pairs = 0;
  for (int q = 0; q < 4; ++q) pairs += (P.qoff[q + 1] - P.qoff[q] + 1) / 2;
  const int G = (pairs + kRWaves - 1) / kRWaves;
  const dim3 g(8 * ((G + 7) / 8) * P.n_rtiles), b(kRWaves * 64);
  if (P.resid_rd == kRDLarge) {
    if (P.td) hipLaunchKernelGGL((k_resid<double, true, kRDLarge>), g, b, 0, s, a);
    else if (a.fp32) hipLaunchKernelGGL((k_resid<float, false, kRDLarge>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_resid<double, false, kRDLarge>), g, b, 0, s, a);
  } else {
    if (P.td) hipLaunchKernelGGL((k_resid<double, true>), g, b, 0, s, a);
    else if (a.fp32) hipLaunchKernelGGL(k_resid<float>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_resid<double>, g, b, 0, s, a);
  }
}

namespace {
// Start of a time step: I^n = stored I + pending correction / (4 pi) for
// every cell-ordinate (blocks over ordinate planes), rho^n = rho^m and T^n =
// T^m per cell, and the step's iteration count, stop flag and smallest change
// cleared (block 0).
__global__ void k_td_begin(TArgs a, double *In, const double *Tm, double *Tn, double *rho_n,
                           int32_t *state, double *last_err) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int kk = blockIdx.y;
  if (kk < a.K) {
    if (t < a.N) {
      const int q = quadrant_of(a, kk);
      const double *DQ = a.dynq + ((size_t)q * 3 + 1) * a.N;
      In[(size_t)kk * a.N + t] = Iin_of<double>(a)[(size_t)kk * a.N + t] + DQ[t];
    }
    return;
  }
  if (t < a.N) {
    Tn[t] = Tm[t];
    rho_n[t] = a.phi[t];
  }
  if (t == 0) {
    state[0] = 0;
    state[1] = 0;
    last_err[1] = INFINITY;
  }
}
}  // namespace

void launch_td_begin(const PlanDev &P, hipStream_t s) {
  const TArgs a = make_args(P);
  hipLaunchKernelGGL(k_td_begin, dim3((P.N + 255) / 256, P.K + 1), dim3(256), 0, s, a, P.In,
                     (const double *)P.Tm, P.Tn, P.rho_n, P.state, P.last_err);
}

namespace {
template <typename T, bool TD>
void launch_pipe_t(const TArgs &a, const PlanDev &P, hipStream_t s) {
  constexpr int PF = 8;
  const dim3 g(P.pipe_parts * P.K);
  if (P.pipe_bands == 1)
    hipLaunchKernelGGL((k_pipe<T, TD, 1, PF>), g, dim3(128), 0, s, a, P.pipe_parts);
  else if (P.pipe_bands == 2)
    hipLaunchKernelGGL((k_pipe<T, TD, 2, PF>), g, dim3(256), 0, s, a, P.pipe_parts);
  else
    hipLaunchKernelGGL((k_pipe<T, TD, 4, PF>), g, dim3(512), 0, s, a, P.pipe_parts);
}
}  // namespace

void launch_sweep(const PlanDev &P, hipStream_t s) {
  const TArgs a = make_args(P);
  const int rows = sweep_rows(P);
  if (P.sweep_impl == 3) {
    if (P.td) launch_pipe_t<double, true>(a, P, s);
    else if (a.fp32) launch_pipe_t<float, false>(a, P, s);
    else launch_pipe_t<double, false>(a, P, s);
    return;
  }
  if (P.sweep_impl == 2 || (P.sweep_impl == 1 && a.fp32)) {
    if (a.fp32) launch_fused<float>(a, P, rows, s);
    else launch_fused<double>(a, P, rows, s);
    return;
  }
  if (P.sweep_impl == 1) {
    hipLaunchKernelGGL(k_sweep, dim3(P.K), dim3(rows), 0, s, a);
    return;
  }
  if (P.chain_parts > 1) {
    const dim3 g(P.chain_parts * P.K), b(P.chain_rows);
    if (a.fp32) hipLaunchKernelGGL(k_chain_split<float>, g, b, 0, s, a, P.chain_parts);
    else hipLaunchKernelGGL(k_chain_split<double>, g, b, 0, s, a, P.chain_parts);
    return;
  }
  if (a.fp32) {
    if (P.ny > rows) hipLaunchKernelGGL((k_chain<float, true>), dim3(P.K), dim3(rows), 0, s, a);
    else hipLaunchKernelGGL((k_chain<float, false>), dim3(P.K), dim3(rows), 0, s, a);
  } else {
    if (P.ny > rows) hipLaunchKernelGGL((k_chain<double, true>), dim3(P.K), dim3(rows), 0, s, a);
    else hipLaunchKernelGGL((k_chain<double, false>), dim3(P.K), dim3(rows), 0, s, a);
  }
}

std::vector<int> diag_row0_table(int nx, int ny) {
  const int nd = nx + ny - 1;
  std::vector<int> t((size_t)nd + 2 * kDiagPad);
  for (int e = 0; e < (int)t.size(); ++e) {
    const int d = e - kDiagPad;
    if (d < 0) t[e] = -(1 << 28);
    else if (d >= nd) t[e] = 1 << 28;
    else t[e] = dg_row0(d, nx, ny);
  }
  return t;
}

int residual_pairs(const PlanDev &P) {
  int pairs = 0;
  for (int q = 0; q < 4; ++q) pairs += (P.qoff[q + 1] - P.qoff[q] + 1) / 2;
  return pairs;
}

int moment_tile_size(int nx, int ny) { return (long long)nx * ny >= (1 << 18) ? 32 : 16; }
int moment_tile_size_batch() { return kBatchMT; }
int moment_tiles_of(int nx, int ny, int mt) {
  return ((nx + mt - 1) / mt) * ((ny + mt - 1) / mt);
}

int residual_tile_diagonals(long long cell_ordinates) {
  return cell_ordinates >= (1LL << 26) ? kRDLarge : kRDSmall;
}

std::vector<int2> residual_tiles(int nx, int ny, int rd) {
  std::vector<int2> t;
  for (int y0 = 0; y0 < ny; y0 += 64) {
    const int y1 = std::min(y0 + 63, ny - 1);
    for (int d0 = y0; d0 <= y1 + nx - 1; d0 += rd) t.push_back(make_int2(d0, y0));
  }
  return t;
}

// ---- batched sweep
size_t targs_bytes() { return sizeof(TArgs); }

void launch_hand_reset(const PlanDev &P, hipStream_t s) {
  const int hp = std::max(P.chain_parts, P.pipe_parts);
  if (hp <= 1) return;
  const size_t n = (size_t)P.K * (hp - 1) * P.nx;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P.hand, n,
                     kHandEmpty);
}
void fill_targs(const PlanDev &P, void *dst) {
  const TArgs a = make_args(P);
  memcpy(dst, &a, sizeof a);
}

namespace {
template <int PF, int MAXW, typename T>
const void *batch_kernel() {
  return reinterpret_cast<const void *>(&k_sweep_batch<PF, MAXW, T>);
}
const void *batch_kernel_for(int cfg, bool fp32) {
  switch (cfg) {
    case 0: return fp32 ? batch_kernel<4, 1, float>() : batch_kernel<4, 1, double>();
    case 1: return fp32 ? batch_kernel<6, 1, float>() : batch_kernel<6, 1, double>();
    case 2: return fp32 ? batch_kernel<4, 2, float>() : batch_kernel<4, 2, double>();
    case 3: return fp32 ? batch_kernel<6, 2, float>() : batch_kernel<6, 2, double>();
    case 4: return fp32 ? batch_kernel<4, 4, float>() : batch_kernel<4, 4, double>();
    case 5: return fp32 ? batch_kernel<2, 8, float>() : batch_kernel<2, 8, double>();
    default: return nullptr;
  }
}
}  // namespace

const BatchSweepConfig kBatchSweepConfigs[kNumBatchSweepConfigs] = {
    {64, 4}, {64, 6}, {128, 4}, {128, 6}, {256, 4}, {512, 2}};

const BatchSweepConfig kBatchChainConfigs[kNumBatchChainConfigs] = {
    {64, kCPF}, {128, kCPF}, {256, kCPF}, {512, kCPF}};
static_assert(kResidWaves == kRWaves, "residual items hold kRWaves ordinates");

int chain_batch_blocks_per_cu(int cfg, bool fp32) {
  int nb = 0;
  const void *k = fp32 ? reinterpret_cast<const void *>(&k_chain_batch<float>)
                       : reinterpret_cast<const void *>(&k_chain_batch<double>);
  if (cfg < 0 || cfg >= kNumBatchChainConfigs ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBatchChainConfigs[cfg].rows, 0) !=
          hipSuccess)
    return 0;
  return nb;
}

void launch_resid_batch(const void *targs, const int4 *items, int n_items, bool fp32,
                        hipStream_t s) {
  const TArgs *ta = reinterpret_cast<const TArgs *>(targs);
  if (fp32) hipLaunchKernelGGL(k_resid_batch<float>, dim3(n_items), dim3(kRWaves * 64), 0, s, ta, items);
  else hipLaunchKernelGGL(k_resid_batch<double>, dim3(n_items), dim3(kRWaves * 64), 0, s, ta, items);
}

void launch_chain_batch(const void *targs, const int2 *items, int n_items, int *counter, int cfg,
                        bool fp32, int grid, hipStream_t s) {
  const TArgs *ta = reinterpret_cast<const TArgs *>(targs);
  const int rows = kBatchChainConfigs[cfg].rows;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, counter);
  if (fp32)
    hipLaunchKernelGGL(k_chain_batch<float>, dim3(grid), dim3(rows), 0, s, ta, items, n_items, counter);
  else
    hipLaunchKernelGGL(k_chain_batch<double>, dim3(grid), dim3(rows), 0, s, ta, items, n_items, counter);
}

int sweep_batch_blocks_per_cu(int cfg, bool fp32) {
  int nb = 0;
  const void *k = batch_kernel_for(cfg, fp32);
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBatchSweepConfigs[cfg].rows, 0) !=
                hipSuccess)
    return 0;
  return nb;
}

void launch_sweep_batch(const void *targs, const int2 *items, int n_items, int *counter, int cfg,
                        bool fp32, int grid, hipStream_t s) {
  const TArgs *ta = reinterpret_cast<const TArgs *>(targs);
  const int rows = kBatchSweepConfigs[cfg].rows;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, counter);
#define GSIS_BATCH_LAUNCH(PF, W)                                                              \
  if (fp32)                                                                                   \
    hipLaunchKernelGGL((k_sweep_batch<PF, W, float>), dim3(grid), dim3(rows), 0, s, ta, items, \
                       n_items, counter);                                                     \
  else                                                                                        \
    hipLaunchKernelGGL((k_sweep_batch<PF, W, double>), dim3(grid), dim3(rows), 0, s, ta,      \
                       items, n_items, counter);
  switch (cfg) {
    case 0: GSIS_BATCH_LAUNCH(4, 1) break;
    case 1: GSIS_BATCH_LAUNCH(6, 1) break;
    case 2: GSIS_BATCH_LAUNCH(4, 2) break;
    case 3: GSIS_BATCH_LAUNCH(6, 2) break;
    case 4: GSIS_BATCH_LAUNCH(4, 4) break;
    default: GSIS_BATCH_LAUNCH(2, 8) break;
  }
#undef GSIS_BATCH_LAUNCH
}

template <typename T, int MT>
void launch_moments_t(const TArgs &a, const PlanDev &P, hipStream_t s, bool bflux) {
  const int ntile = moment_tiles_of(P.nx, P.ny, MT);
  const int ts = (ntile + 7) / 8;   // tiles per XCD
  if (bflux) {   // the combine follows in the HoT kernel
    const int nbf8 = ((P.nbf + 3) / 4 + 7) / 8 * 8;
    hipLaunchKernelGGL((k_moments_q_bflux<T, MT>), dim3(nbf8 + 4 * 8 * ts), dim3(256), 0, s, a,
                       P.mom_part, nbf8, ntile, ts, P.hot_face ? P.ftp : nullptr);
    return;
  }
  hipLaunchKernelGGL((k_moments_q<T, MT>), dim3(8 * ts, 4), dim3(256), 0, s, a, P.mom_part, ntile,
                     ts);
  hipLaunchKernelGGL(k_moments_combine, dim3((P.N + 255) / 256), dim3(256), 0, s, a,
                     (const double *)P.mom_part);
}

void launch_moments(const PlanDev &P, hipStream_t s, bool bflux) {
  const TArgs a = make_args(P);
  const bool big = moment_tile_size(P.nx, P.ny) == 32;
  if (a.fp32) {
    if (big) launch_moments_t<float, 32>(a, P, s, bflux);
    else launch_moments_t<float, 16>(a, P, s, bflux);
  } else {
    if (big) launch_moments_t<double, 32>(a, P, s, bflux);
    else launch_moments_t<double, 16>(a, P, s, bflux);
  }
}

void launch_moments_batch(const void *targs, const int2 *bt_cell, int nb_cell,
                          const int2 *bt_tile, int nb_tile, bool fp32, hipStream_t s) {
  const TArgs *ta = reinterpret_cast<const TArgs *>(targs);
  if (fp32)
    hipLaunchKernelGGL(k_moments_q_b<float>, dim3(nb_tile, 4), dim3(256), 0, s, ta, bt_tile);
  else
    hipLaunchKernelGGL(k_moments_q_b<double>, dim3(nb_tile, 4), dim3(256), 0, s, ta, bt_tile);
  hipLaunchKernelGGL(k_moments_combine_b, dim3(nb_cell), dim3(256), 0, s, ta, bt_cell);
}

void launch_boundary_flux_batch(const void *targs, const int2 *bt_face, int nb_face,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_boundary_flux_b, dim3((nb_face + 3) / 4), dim3(256), 0, s,
                     reinterpret_cast<const TArgs *>(targs), bt_face, nb_face);
}

}  // namespace gsis
