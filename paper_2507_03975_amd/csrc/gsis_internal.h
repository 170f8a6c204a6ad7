// gsis_internal.h -- device state of a plan and the kernel launchers.
//
// Internal layout (chosen for gfx950; independent of the caller's layout):
//  * ordinates are regrouped by quadrant q (sign of mu, sign of eta); inside
//    quadrant q the grid is mirrored so that every quadrant sweeps towards
//    +x', +y' (local coordinates x' = i or nx-1-i, y' = j or ny-1-j);
//  * the angular intensity is ordinate-major, I[kk][dg_idx(x', y')] with kk
//    the internal ordinate index (quadrant-major) and the cells of each
//    ordinate in anti-diagonal order (dg_idx below);
//  * every per-cell array is in the caller's order c = j*nx + i.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>
#include <string>

#include "gsis.h"

namespace gsis {

constexpr double kFourPi = 12.566370614359172953850573533118;

// Anti-diagonal storage order of an nx x ny grid (in a quadrant's mirrored
// frame): cells are stored diagonal by diagonal (d = x + y), rows ascending
// inside a diagonal. A wavefront step touches one diagonal, so the lanes of a
// step read and write contiguous memory.
__host__ __device__ inline long long dg_off(long long d, long long nx, long long ny) {
  const long long A = nx < ny ? nx : ny, B = nx < ny ? ny : nx;
  if (d <= A) return d * (d + 1) / 2;
  long long o = A * (A + 1) / 2;
  if (d <= B) return o + (d - A) * A;
  o += (B - A) * A;
  const long long t = d - B;
  return o + t * (nx + ny - 1 - B) - t * (t - 1) / 2;
}
__host__ __device__ inline int dg_ylo(int d, int nx) { return d - nx + 1 > 0 ? d - nx + 1 : 0; }
__host__ __device__ inline long long dg_idx(int x, int y, int nx, int ny) {
  const int d = x + y;
  return dg_off(d, nx, ny) + (y - dg_ylo(d, nx));
}

// One multigrid level of the synthetic operator D1 (5-point, SPD):
//   (D x)_c = diag_c x_c - ax_c x_{c+1} - ax_{c-1} x_{c-1}
//             - ay_c x_{c+nx} - ay_{c-nx} x_{c-nx}
// where ax_c couples (i,j)-(i+1,j) and ay_c couples (i,j)-(i,j+1).
struct MGLevel {
  int nx = 0, ny = 0;
  int fx = 1, fy = 1;   // aggregate size towards the next coarser level
  double *diag = nullptr, *ax = nullptr, *ay = nullptr;
  double *x = nullptr, *b = nullptr, *r = nullptr;  // work vectors (levels >= 1)
};

struct PlanDev {
  // problem
  int nx = 0, ny = 0, N = 0, K = 0, nbf = 0;
  double dx = 0, dy = 0, V = 0;
  int Kq[4] = {0, 0, 0, 0}, qoff[5] = {0, 0, 0, 0, 0};
  // options
  int method = 1, precision = 0, order = 2, limiter = 1, alsm = 1, hot_face = 0;
  double tol = 1e-6, synth_rtol = 1e-10;
  int max_iter = 1000, synth_max_iter = 50;
  // per internal ordinate
  double *amu = nullptr, *aeta = nullptr;   // |mu|/dx, |eta|/dy
  double *w = nullptr, *wmu = nullptr, *weta = nullptr;  // w, w*mu, w*eta (signed)
  double sw = 0, swm = 0, swe = 0;                        // their sums
  // intensities (two copies; FP64, or FP32 deviations in FP32-mixed mode)
  // and the residual buffer, [K][N] local layout
  void *I[2] = {nullptr, nullptr};
  double *R = nullptr;
  // per quadrant, in that quadrant's mirrored frame: cellq[q][N][6] =
  // (cE, cW, cN, cS, sigma_t, sigma_t + pseudo-time shift) with E/W/N/S
  // local; dynq[q][3][N] = planes src, base/(4 pi) and phi/(4 pi),
  // rewritten after every update
  double *cellq = nullptr, *dynq = nullptr;
  double *rowbuf = nullptr;    // [K][3][nx] hand-off between sweep passes
  int sweep_impl = 0;          // 0 fused wavefront sweep, 1 two-kernel reference
  // per cell
  double *sig_t = nullptr, *sig_a = nullptr, *sig_s = nullptr, *q = nullptr;
  double *cE = nullptr, *cW = nullptr, *cN = nullptr, *cS = nullptr;  // ALSM
  double *src = nullptr;       // (sigma_s phi^m + q)/(4 pi)
  double *phi = nullptr;       // phi^m
  double *phih = nullptr, *Fx = nullptr, *Fy = nullptr;  // moments of I^{m+1/2}
  double *mom_part = nullptr;  // [4][3][N] per-quadrant partial moments
  double *delta = nullptr;     // pending GSIS correction (phi' - phi_half)
  double *base = nullptr;      // what the next read adds (over 4 pi) to the stored
                               // intensity: delta (FP64; same array), or
                               // phi^m + delta (FP32-mixed deviations)
  double *hx = nullptr, *hy = nullptr;   // HoT
  double *rhs = nullptr;
  // boundary
  double *bnd = nullptr;       // [nbf][K] internal ordinate order, incoming values
  double *bflux = nullptr;     // [nbf] F_T . n_out
  double *kappa = nullptr;     // [nbf]
  // synthetic solve
  std::vector<MGLevel> mg;
  double *coarse_inv = nullptr;  // dense inverse of the coarsest operator
  int coarse_n = 0;
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_p2 = nullptr, *cg_Ap = nullptr;
  double *red = nullptr;       // block partial sums
  double *scal = nullptr;      // device scalars (see kernels_synth.hip)
  int red_blocks = 0;
  // iteration state on device
  double *err_hist = nullptr;  // [max_iter]
  double *err_parts = nullptr; // block partials for Err
  int32_t *state = nullptr;    // [0] iterations done, [1] done flag (1 converged,
                               // -1 diverged, 2 max_iter), [2] current I buffer,
                               // [3] synthetic CG converged
  double *last_err = nullptr;
};

// ---- transport kernels (kernels_transport.hip)
void launch_transport(const PlanDev &P, hipStream_t s);   // residual + sweep
void launch_moments(const PlanDev &P, hipStream_t s);
void launch_boundary_flux(const PlanDev &P, hipStream_t s);

// ---- synthetic / update kernels (kernels_synth.hip)
void launch_source(const PlanDev &P, hipStream_t s);          // src from phi
void launch_hot_rhs(const PlanDev &P, hipStream_t s);
void prepare_synth(PlanDev &P);
void launch_synth_solve(PlanDev &P, hipStream_t s, int32_t *host_flag);
void launch_update(const PlanDev &P, hipStream_t s);
void launch_apply_delta_final(const PlanDev &P, hipStream_t s, double swmu, double sweta,
                              double *Fx_out, double *Fy_out);
void launch_d1_apply(const PlanDev &P, const double *x, double *y, hipStream_t s);

}  // namespace gsis
