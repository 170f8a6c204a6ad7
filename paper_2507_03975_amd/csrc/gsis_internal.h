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
// Storage index of row 0 on anti-diagonal d, dg_off(d) - dg_ylo(d), in
// 32-bit arithmetic, for 0 <= d < nx + ny - 1 of a grid of fewer than 2^31
// cells (every product below is at most twice the cell count).
__host__ __device__ inline int dg_row0(int d, int nx, int ny) {
  const int A = nx < ny ? nx : ny, B = nx < ny ? ny : nx;
  int o;
  if (d <= A) {
    o = d * (d + 1) / 2;
  } else if (d <= B) {
    o = A * (A + 1) / 2 + (d - A) * A;
  } else {
    const int t = d - B;
    o = A * (A + 1) / 2 + (B - A) * A + t * (nx + ny - 1 - B) - t * (t - 1) / 2;
  }
  return o - (d - nx + 1 > 0 ? d - nx + 1 : 0);
}

// One multigrid level of the synthetic operator D1 (5-point, SPD):
//   (D x)_c = diag_c x_c - ax_c x_{c+1} - ax_{c-1} x_{c-1}
//             - ay_c x_{c+nx} - ay_{c-nx} x_{c-nx}
// where ax_c couples (i,j)-(i+1,j) and ay_c couples (i,j)-(i,j+1).
struct MGLevel {
  int nx = 0, ny = 0;
  int fx = 1, fy = 1;   // aggregate size towards the next coarser level
  double *diag = nullptr, *ax = nullptr, *ay = nullptr;
  double *x = nullptr, *b = nullptr, *r = nullptr;  // work vectors (x, b: levels >= 1;
                                                    // r: pre-smoothed x, every level)
};

// ---- synthetic step, one problem or many: every kernel of the synthetic
// step reads its problem from a device array of SynthDesc records, and a
// block table (problem, block of that problem) spreads one launch over many
// problems (NULL table: a single problem, block = blockIdx.x).
constexpr int kMaxLevels = 40;
constexpr int kMaxCoarseLevels = 10;
struct CoarseLevels {
  int nlev;
  int nx[kMaxCoarseLevels], ny[kMaxCoarseLevels], fx[kMaxCoarseLevels], fy[kMaxCoarseLevels];
  const double *dg[kMaxCoarseLevels], *ax[kMaxCoarseLevels], *ay[kMaxCoarseLevels];
  // LDS offsets (doubles): level 0 holds x, r; a level t >= 1 holds x, b,
  // r and its operator (1/diag, ax, ay, diag at aoff + 0, n, 2n, 3n)
  int xoff[kMaxCoarseLevels], boff[kMaxCoarseLevels], roff[kMaxCoarseLevels];
  int aoff[kMaxCoarseLevels];
};
struct LevelDev {
  int nx, ny, fx, fy;
  const double *dg, *ax, *ay;
  double *x, *b;                // levels >= 1 (level 0 uses the CG's z and r)
  double *xs;                   // pre-smoothed x of a fine level (tile kernels)
};
struct SynthDesc {
  int nx, ny, N;
  double dx, dy, V;
  int method, fp32, max_iter;
  double tol, rtol;
  const double *sig_t, *sig_s, *sig_a, *q, *cE, *cW, *cN, *cS, *kappa;
  double *phih, *Fx, *Fy;       // moments of I^{m+1/2} (k_hot<true> writes them)
  const double *bflux;
  const double *mom_part;       // [4][3][N] per-quadrant partial moments
  int hot_face;                 // 1: HoT from transport face fluxes (ftp)
  const double *ftp;            // [4][2][N] per-quadrant transport flux through
                                // the east (+x) and north (+y) face of each cell
  double sw, swm, swe;          // sums of w, w mu, w eta (FP32-mixed base terms)
  double *hx, *hy, *rhs, *phi, *delta, *base, *src, *dynq;
  // time-dependent form (td = 1): backward-Euler step with 1/(c dt) = tdiag,
  // emission ca T^4 (ca = a c), material T^m (Tm), time level n (Tn, rho_n),
  // sub-iterates T(s) (s >= 1) in Tsub[(s - 1) & 1], sub_iter per iteration
  int td, sub_iter;
  double tdiag, ca, dt;
  const double *cv, *Tn, *rho_n;
  double *Tm, *Tsub0, *Tsub1, *err_parts_T;
  // CG vectors: r alternates between cg_r and cg_r2 with the V-cycle count,
  // s = A p between cg_s0 and cg_s1 with the iteration; z = M r, w = A z
  double *cg_r, *cg_r2, *cg_z, *cg_p, *cg_s0, *cg_s1, *cg_w;
  double *wx, *wy;              // face-averaged balance: grad(x) / (3 sigma_t)
  double *red, *scal, *err_parts, *err_hist, *last_err;  // last_err[0] last Err, [1] smallest change
  // relative transport residual of the iterate entering each iteration:
  // per-wave sums of w r^2 from the residual kernel and per-block sums of
  // src^2 from the moments kernels, finished with Err
  const double *tres_part, *src2_part;
  int n_tres, n_src2;
  double *tres_hist;
  int32_t *state;
  int nlev, lc;                 // levels; first level of the one-workgroup cycle
  int ntile0;                   // multigrid tiles of level 0
  int ntp;                      // slots of each tile-partial region: max(ntile0, cell blocks)
  int coef_sep;                 // 1: the CG coefficients come from k_cg_coef (many partials)
  LevelDev lev[kMaxLevels];
  CoarseLevels cl;
  const double *coarse_inv;
};
// Host-side description of one launch set (a plan, or a batch of plans).
struct SynthSet {
  int n = 0;                          // problems
  SynthDesc *desc = nullptr;          // device [n]
  int max_lc = 0;                     // deepest first coarse level
  int min_lc = 0;                     // shallowest first coarse level
  size_t coarse_lds = 0;              // dynamic LDS of the coarse kernel
  int synth_max_iter = 50;
  // block tables (nullptr for a single problem) and their block counts
  int2 *bt_cell = nullptr;            // level-0 cells of every problem
  int nb_cell = 0;
  int2 *bt_src = nullptr;             // 16 x 16 cell tiles of every problem (source kernel)
  int nb_src = 0;
  std::vector<int2 *> bt_tile;        // [l]: level-l tiles of problems with lc > l
  std::vector<int> nb_tile;
  int32_t *state0 = nullptr;          // single problem: its state (host checks)
  bool any_coef_sep = false;          // some problem's CG coefficients come from k_cg_coef
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
  unsigned long long *hand = nullptr;  // [K][parts - 1][nx] row hand-over between
                               // the workgroups of one ordinate (split recurrence
                               // or pipelined step; sized for the larger)
  int chain_parts = 1;         // workgroups per ordinate in the recurrence
  int chain_rows = 0;          // rows per part (a multiple of 64, <= 1024)
  int pipe_bands = 0;          // pipelined step: bands of 64 rows per workgroup (1, 2, 4)
  int pipe_parts = 1;          // pipelined step: workgroups per ordinate
  int n_tres = 0;              // partial sums of w r^2 the transport step writes
  double *sdq = nullptr;       // [q][N] sigma_t + pseudo-time shift per stored cell
  float *sdq_f = nullptr;      // FP32-mixed: the same in FP32 (FP32 recurrence)
  float *w_f = nullptr;        // FP32-mixed: w, w mu, w eta in FP32 ([3][K], moment sums)
  int2 *rtiles = nullptr;      // residual-kernel tiles (first diagonal, first row)
  int *dso = nullptr;          // [kDiagPad + nx + ny - 1 + kDiagPad] storage index of
                               // row 0 on each anti-diagonal (dg_off - ylo), padded
  int n_rtiles = 0;
  int resid_rd = 31;           // diagonals per residual tile
  int sweep_impl = 0;          // 0 residual kernel + wavefront recurrence,
                               // 1 two-kernel reference, 2 fused wavefront sweep,
                               // 3 pipelined residual + recurrence
  // per cell
  double *sig_t = nullptr, *sig_a = nullptr, *sig_s = nullptr, *q = nullptr;
  double *cE = nullptr, *cW = nullptr, *cN = nullptr, *cS = nullptr;  // ALSM
  double *src = nullptr;       // (sigma_s phi^m + q)/(4 pi)
  double *phi = nullptr;       // phi^m
  double *phih = nullptr, *Fx = nullptr, *Fy = nullptr;  // moments of I^{m+1/2}
  double *mom_part = nullptr;  // [4][3][N] per-quadrant partial moments
  double *ftp = nullptr;       // transport-face HoT: [4][2][N] per-quadrant
                               // sum_k w_k (Omega_k . n) I_f,k on the east / north
                               // face of each cell (reconstructed upwind values)
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
  double *cg_r = nullptr, *cg_r2 = nullptr, *cg_z = nullptr, *cg_p = nullptr;
  double *cg_s0 = nullptr, *cg_s1 = nullptr, *cg_w = nullptr;
  // synthetic balance: 0 compact Gamma flux; 1 face average of the cells'
  // diffusive fluxes (Eq. Fij_d) by synth_sub defect-correction solves
  int synth_form = 0, synth_sub = 1;
  double *wide_wx = nullptr, *wide_wy = nullptr;
  double *red = nullptr;       // block partial sums
  double *scal = nullptr;      // device scalars (see kernels_synth.hip)
  int red_blocks = 0;
  // iteration state on device
  double *err_hist = nullptr;  // [max_iter]
  double *err_parts = nullptr; // block partials for Err
  double *tres_hist = nullptr; // [max_iter] relative transport residual of I^m
  double *tres_part = nullptr; // [n_rtiles * ordinate pairs] sums of w r^2 per residual wave
  double *src2_part = nullptr; // [ceil(N / 256)] sums of src^2 per block of cells
  // time-dependent form (gsis_td_create): 1/(c dt), a c, dt, sub-iterations
  int td = 0, sub_iter = 1;
  double tdiag = 0, ca = 0, dt = 0;
  double *cv = nullptr, *Tm = nullptr, *Tn = nullptr, *Tsub0 = nullptr, *Tsub1 = nullptr;
  double *rho_n = nullptr, *err_parts_T = nullptr;
  double *In = nullptr;        // [K][N] I^n in the intensity layout (FP64)
  int32_t *state = nullptr;    // [0] iterations done, [1] done flag (1 converged,
                               // -1 diverged, 2 max_iter), [2] current I buffer,
                               // [3] synthetic CG converged, [4] a split
                               // recurrence's hand-over timed out
  double *last_err = nullptr;  // [2]: Err of the last iteration, smallest ||phi^{m+1} - phi^m||_V
  SynthSet S;                  // launch set of this plan alone
  int lc = 0;                  // first level of the one-workgroup cycle
};

// ---- transport kernels (kernels_transport.hip)
// Transport step: residual of every cell-ordinate, then the wavefront
// increment solve (for the fused kernel the residual launch is empty).
void launch_residual(const PlanDev &P, hipStream_t s);
void launch_sweep(const PlanDev &P, hipStream_t s);
// Puts every entry of the split recurrence's hand-over buffer in its empty
// state (plan set-up and reset; the recurrence keeps it so between launches).
void launch_hand_reset(const PlanDev &P, hipStream_t s);
// Tiles of the residual kernel for an nx x ny grid: (first diagonal, first
// row) of each band of rows x run of diagonals that holds a cell.
// Residual-kernel tiles of rd diagonals (residual_tile_diagonals: 31, or 47
// from 2^26 cell-ordinates on)
int residual_tile_diagonals(long long cell_ordinates);
std::vector<int2> residual_tiles(int nx, int ny, int rd);
// Ordinate pairs of one quadrant the residual kernel takes per wave (the
// residual-norm partials are indexed tile * pairs + pair).
int residual_pairs(const PlanDev &P);
// Storage index of row 0 on anti-diagonal d (dg_off(d) - ylo(d)), for d in
// [-kDiagPad, nx + ny - 1 + kDiagPad); outside the grid's diagonals the value
// sends every row out of the intensity buffer.
constexpr int kDiagPad = 256;
std::vector<int> diag_row0_table(int nx, int ny);
// Batched sweep: per-problem kernel arguments (fill_targs into a device
// table of targs_bytes() records), work items (problem, internal ordinate),
// a device counter, and one of the compiled launch configurations.
struct BatchSweepConfig { int rows, pf; };
constexpr int kNumBatchSweepConfigs = 6;
extern const BatchSweepConfig kBatchSweepConfigs[kNumBatchSweepConfigs];
// Split transport step of a batch: residual items (problem, tile, group of
// four ordinates), then a persistent recurrence over (problem, ordinate)
// items with rows per pass from kBatchChainConfigs (prefetch fixed).
constexpr int kNumBatchChainConfigs = 4;
extern const BatchSweepConfig kBatchChainConfigs[kNumBatchChainConfigs];
int chain_batch_blocks_per_cu(int cfg, bool fp32);
constexpr int kResidWaves = 4;     // ordinate pairs (of one quadrant) per residual item
void launch_resid_batch(const void *targs, const int4 *items, int n_items, bool fp32,
                        hipStream_t s);
void launch_chain_batch(const void *targs, const int2 *items, int n_items, int *counter, int cfg,
                        bool fp32, int grid, hipStream_t s);
size_t targs_bytes();
void fill_targs(const PlanDev &P, void *dst);
int sweep_batch_blocks_per_cu(int cfg, bool fp32);
void launch_sweep_batch(const void *targs, const int2 *items, int n_items, int *counter, int cfg,
                        bool fp32, int grid, hipStream_t s);
// moments of a batch: partials over (problem, moment tile or -1) blocks
// (moment_tile_size_batch), then the combine over (problem, 256-cell block)
// blocks; boundary fluxes over (problem, boundary face)
void launch_moments_batch(const void *targs, const int2 *bt_cell, int nb_cell,
                          const int2 *bt_tile, int nb_tile, bool fp32, hipStream_t s);
void launch_boundary_flux_batch(const void *targs, const int2 *bt_face, int nb_face,
                                hipStream_t s);
// phi, F of the swept intensity; with bflux (GSIS) only the per-quadrant
// partials, which launch_hot(.., true) combines, and the boundary faces'
// F_T . n in the same launch
void launch_moments(const PlanDev &P, hipStream_t s, bool bflux);

// ---- synthetic / update kernels (kernels_synth.hip)
// Descriptor of plan P's synthetic step (host copy; P's arrays and levels
// must exist) and the first level of its one-workgroup coarse cycle.
SynthDesc make_synth_desc(const PlanDev &P);
int coarse_start(const PlanDev &P);
size_t coarse_lds_bytes(const PlanDev &P);
int tiles_of(int nx, int ny);   // multigrid tiles covering an nx x ny level
int source_tiles_of(int nx, int ny);   // 16 x 16 tiles of the source kernel
// tiles of the moment kernels: edge mt (16 or 32; moment_tile_size for a
// plan, moment_tile_size_batch for batches)
int moment_tile_size(int nx, int ny);
int moment_tile_size_batch();
int moment_tiles_of(int nx, int ny, int mt);
void prepare_synth(size_t coarse_lds);      // kernel attribute for the LDS size
void launch_source(const SynthSet &S, hipStream_t s);          // src from phi
// HoT of every cell; combine: first phi, F of I^{m+1/2} from the quadrant
// partials (a single plan; batches combine in their own launch)
void launch_hot(const SynthSet &S, hipStream_t s, bool combine);
// grad(x) / (3 sigma_t) of the level-0 iterate for the face-averaged
// balance; first: x = phi^{m+1/2}, copied into the iterate
void launch_wide_grad(const SynthSet &S, hipStream_t s, bool first);
// host_flag: pinned int32[3] for the host's stop checks (single problem);
// NULL never waits and enqueues exactly S.synth_max_iter iterations.
// rhs_mode 1: the first kernel forms the right-hand side from the HoT
// (forward solve), warm start phi; 2: the same plus the face-averaged
// balance's correction at the level-0 iterate, which is the warm start (one
// defect-correction sub-iteration, after launch_wide_grad); 0: it reads the
// descriptor's rhs (adjoint).
// sub: the time-dependent form's sub-iteration (its right-hand side takes
// the emission of T(sub)); rhs_mode 3: as 1 with the level-0 iterate (the
// previous sub-iterate) as warm start.
// spec: see the definition (true: the end of the outer iteration is
// already in the stream)
bool launch_synth_solve(const SynthSet &S, hipStream_t s, int32_t *host_flag, int rhs_mode,
                        int sub = 0, hipEvent_t spec = nullptr);
// Time-dependent form: T(sub + 1) = T(sub) + R2 / D2 (Eqs. MSE_d2, R2_def,
// MSE_d_mtx2, elem_mtx_M) with rho(sub) (rho^{m+1/2} at sub 0 or for source
// iteration, else the last synthetic solution)
void launch_material(const SynthSet &S, hipStream_t s, int sub);
// cond: only for problems whose synthetic solve has converged (state[3])
void launch_update(const SynthSet &S, hipStream_t s, int cond = 0);
// Time-dependent form, start of a time step: I^n = the current iterate (with
// its pending correction), rho^n, T^n; the step's counters and flags cleared
void launch_td_begin(const PlanDev &P, hipStream_t s);
void launch_apply_delta_final(const PlanDev &P, hipStream_t s, double swmu, double sweta,
                              double *Fx_out, double *Fy_out);
// CG iterations of P's last synthetic solve (one device double)
double *synth_iteration_counter(const PlanDev &P);
// V-cycles of all synthetic solves since the last reset (one device double)
double *synth_vcycle_total(const PlanDev &P);

// ---- adjoint (kernels_adjoint.hip)
struct AdjointBuffers {
  double *lam = nullptr, *ihb = nullptr, *rb = nullptr;          // [K][N]
  double *s = nullptr, *s_old = nullptr, *bb = nullptr, *hxb = nullptr, *hyb = nullptr;
  double *phb = nullptr, *Sb = nullptr, *bfb = nullptr;
  double *part = nullptr;      // [4][5][N]
  double *dbar = nullptr;      // [4][N]
  double *stp = nullptr, *errp = nullptr, *hist = nullptr;
  double *gphi = nullptr, *gFx = nullptr, *gFy = nullptr;        // device cotangents
  double *g_sa = nullptr, *g_ss = nullptr, *g_q = nullptr;       // device gradients
  int32_t *state = nullptr;    // synthetic-solve state of the adjoint solves
  SynthSet S;                  // D1 bb = s with the plan's hierarchy
  std::vector<char> args;      // kernel-argument image
  int max_hist = 0;
};
size_t adjoint_args_bytes();
void adj_fill_args(const PlanDev &P, const AdjointBuffers &B, const double *gphi,
                   const double *gFx, const double *gFy, void *dst);
// host_flag: pinned int32[3] for the synthetic solve's stop checks, or NULL
void adj_launch_pass(const PlanDev &P, const AdjointBuffers &B, const void *args,
                     const double *ihalf, const SynthSet &S, double *hist, int m,
                     int32_t *host_flag, hipStream_t s);
void adj_launch_gradient(const PlanDev &P, const void *args, const double *ihalf, double *g_sa,
                         double *g_ss, double *g_q, hipStream_t s);

}  // namespace gsis
