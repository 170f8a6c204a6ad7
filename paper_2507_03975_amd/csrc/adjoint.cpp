// adjoint.cpp -- C-ABI of the adjoint: gradients of outputs of a converged
// plan with respect to sigma_a, sigma_s and q per cell (the reverse pass
// itself is in kernels_adjoint.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/gsis.h"
#include "plan.h"

namespace {

// Adjoint buffers of a plan, allocated on first use and freed with the plan.
gsis_status adjoint_setup(gsis_plan *pl) {
  if (pl->adj) return GSIS_OK;
  PlanDev &P = pl->P;
  AdjointBuffers *B = new AdjointBuffers;
  pl->adj = B;
  const size_t N = P.N, NK = (size_t)P.N * P.K;
  gsis_status st;
  if ((st = dalloc(pl, &B->lam, NK)) || (st = dalloc(pl, &B->ihb, NK)) ||
      (st = dalloc(pl, &B->rb, NK)) || (st = dalloc(pl, &B->s, N)) ||
      (st = dalloc(pl, &B->s_old, N)) || (st = dalloc(pl, &B->bb, N)) ||
      (st = dalloc(pl, &B->hxb, N)) || (st = dalloc(pl, &B->hyb, N)) ||
      (st = dalloc(pl, &B->phb, N)) || (st = dalloc(pl, &B->Sb, N)) ||
      (st = dalloc(pl, &B->bfb, P.nbf)) || (st = dalloc(pl, &B->part, 20 * N)) ||
      (st = dalloc(pl, &B->dbar, 4 * N)) || (st = dalloc(pl, &B->stp, N)) ||
      (st = dalloc(pl, &B->errp, 2 * ((N + 255) / 256) + 2)) ||
      (st = dalloc(pl, &B->gphi, N)) || (st = dalloc(pl, &B->gFx, N)) ||
      (st = dalloc(pl, &B->gFy, N)) || (st = dalloc(pl, &B->g_sa, N)) ||
      (st = dalloc(pl, &B->g_ss, N)) || (st = dalloc(pl, &B->g_q, N)) ||
      (st = dalloc(pl, &B->state, 4)))
    return st;
  HIPCHK(pl->ctx, hipMemset(B->state, 0, 4 * sizeof(int32_t)));
  HIPCHK(pl->ctx, hipMemset(B->bfb, 0, P.nbf * sizeof(double)));
  // the plan's synthetic-solve set with the adjoint's right-hand side s,
  // solution (and warm start) bb and its own state
  SynthDesc D = make_synth_desc(P);
  D.rhs = B->s;
  D.phi = B->bb;
  D.lev[0].x = B->bb;
  D.state = B->state;
  {
    char *d = nullptr;
    if ((st = dalloc(pl, &d, sizeof D))) return st;
    HIPCHK(pl->ctx, hipMemcpy(d, &D, sizeof D, hipMemcpyHostToDevice));
    B->S = P.S;
    B->S.desc = (SynthDesc *)d;
    B->S.state0 = B->state;
  }
  B->args.resize(adjoint_args_bytes());
  adj_fill_args(P, *B, B->gphi, B->gFx, B->gFy, B->args.data());
  return GSIS_OK;
}

gsis_status fetch_cot(gsis_plan *pl, const double *src, double *dst, size_t n) {
  hipStream_t s = pl->stream;
  if (!src) {
    HIPCHK(pl->ctx, hipMemsetAsync(dst, 0, n * sizeof(double), s));
    return GSIS_OK;
  }
  HIPCHK(pl->ctx, hipMemcpyAsync(dst, src, n * sizeof(double),
                                 pl->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 s));
  return GSIS_OK;
}

}  // namespace

void adjoint_release(gsis_plan *pl) {
  delete pl->adj;
  pl->adj = nullptr;
}

extern "C" {

gsis_status gsis_plan_adjoint(gsis_plan *pl, const double *g_phi, const double *g_Fx,
                              const double *g_Fy, double tol, int32_t max_iter,
                              double *g_sigma_a, double *g_sigma_s, double *g_q,
                              gsis_adjoint_info *info) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  PlanDev &P = pl->P;
  if (P.limiter || P.precision != GSIS_FP64 || P.hot_face != GSIS_HOT_CENTRAL || pl->pseudo ||
      P.synth_form != 0)
    return fail(ctx, GSIS_E_UNSUPPORTED,
                "the adjoint needs limiter = 0, FP64, central HoT faces, no pseudo time and "
                "the compact synthetic flux");
  if (max_iter < 1) return fail(ctx, GSIS_E_INVALID_ARG, "max_iter must be >= 1");
  if (!(tol >= 0)) return fail(ctx, GSIS_E_INVALID_ARG, "tol must be >= 0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int32_t n_fwd = 0, conv = 0;
  double le = 0;
  gsis_status st = gsis_plan_status(pl, &n_fwd, &conv, &le);
  if (st) return st;
  if (conv != 1)
    return fail(ctx, GSIS_E_INVALID_ARG, "the plan has not converged (Err < tol) yet");
  if ((st = adjoint_setup(pl))) return st;
  AdjointBuffers &B = *pl->adj;
  hipStream_t s = pl->stream;
  const size_t N = P.N, NK = (size_t)P.N * P.K;
  if (B.max_hist < max_iter + 1) {
    if ((st = dalloc(pl, &B.hist, (size_t)max_iter + 1))) return st;
    B.max_hist = max_iter + 1;
  }
  if ((st = fetch_cot(pl, g_phi, B.gphi, N)) || (st = fetch_cot(pl, g_Fx, B.gFx, N)) ||
      (st = fetch_cot(pl, g_Fy, B.gFy, N)))
    return st;
  // the stored I^{m+1/2} of the last iteration sits in buffer state[2]
  int32_t stv[4];
  HIPCHK(ctx, hipMemcpyAsync(stv, P.state, sizeof stv, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  const double *ihalf = (const double *)P.I[stv[2] ? 1 : 0];
  HIPCHK(ctx, hipMemsetAsync(B.lam, 0, NK * sizeof(double), s));
  HIPCHK(ctx, hipMemsetAsync(B.s_old, 0, N * sizeof(double), s));
  HIPCHK(ctx, hipMemsetAsync(B.bb, 0, N * sizeof(double), s));
  HIPCHK(ctx, hipMemsetAsync(B.state, 0, 4 * sizeof(int32_t), s));
  // lambda^{n+1} = G^T lambda^n + M^T g from lambda = 0; the first pass
  // gives M^T g, Err compares successive ordinate sums
  int m = 0, status = 1;
  double err = INFINITY;
  std::vector<double> h(max_iter + 1);
  const int check = 4;
  while (m < max_iter) {
    const int todo = std::min(check, max_iter - m);
    for (int t = 0; t < todo; ++t, ++m)
      adj_launch_pass(P, B, B.args.data(), ihalf, B.S, B.hist, m, (int32_t *)pl->host_scal + 4, s);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(h.data(), B.hist, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    // Err of pass t compares the sums of lambda^t and lambda^{t-1}; pass 0
    // starts from zero
    bool done = false;
    for (int t = std::max(2, m - todo); t < m; ++t) {
      err = h[t];
      if (!std::isfinite(err)) { status = -1; done = true; break; }
      if (err < tol) { status = 0; m = t + 1; done = true; break; }
    }
    if (done) break;
  }
  if (status == -1) return fail(ctx, GSIS_DIVERGED, "adjoint iteration diverged");
  // gradient: one more pass with lambda* (it recomputes every cotangent the
  // derivatives need), then the per-cell assembly
  adj_launch_pass(P, B, B.args.data(), ihalf, B.S, nullptr, 0, (int32_t *)pl->host_scal + 4, s);
  adj_launch_gradient(P, B.args.data(), ihalf, B.g_sa, B.g_ss, B.g_q, s);
  HIPCHK(ctx, hipGetLastError());
  const hipMemcpyKind k = pl->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (g_sigma_a) HIPCHK(ctx, hipMemcpyAsync(g_sigma_a, B.g_sa, N * sizeof(double), k, s));
  if (g_sigma_s) HIPCHK(ctx, hipMemcpyAsync(g_sigma_s, B.g_ss, N * sizeof(double), k, s));
  if (g_q) HIPCHK(ctx, hipMemcpyAsync(g_q, B.g_q, N * sizeof(double), k, s));
  int32_t hand_err = 0;
  HIPCHK(ctx, hipMemcpyAsync(&hand_err, P.state + 4, sizeof hand_err, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (hand_err != 0)
    return fail(ctx, GSIS_E_DEVICE,
                "the sweep's workgroups of one ordinate stopped waiting for each other; "
                "reset the plan");
  if (info) {
    info->n_iter = m;
    info->final_err = err;
    info->forward_iter = n_fwd;
  }
  return status == 0 ? GSIS_OK : GSIS_NOT_CONVERGED;
}

gsis_status gsis_adjoint(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                         const double *g_phi, const double *g_Fx, const double *g_Fy,
                         double *g_sigma_a, double *g_sigma_s, double *g_q, gsis_result *fwd,
                         gsis_adjoint_info *info) {
  if (!ctx) return fail(nullptr, GSIS_E_INVALID_ARG, "ctx is NULL");
  gsis_plan *pl = nullptr;
  gsis_status st = gsis_plan_create(ctx, p, o, &pl);
  if (st) return st;
  int32_t n = 0, conv = 0;
  double le = 0;
  while (true) {
    const int todo = std::min(8, o->max_iter - n);
    if (todo <= 0) break;
    if ((st = gsis_plan_iterate(pl, todo)) || (st = gsis_plan_status(pl, &n, &conv, &le))) {
      gsis_plan_destroy(pl);
      return st;
    }
    if (conv != 0 || n >= o->max_iter) break;
  }
  if (conv != 1) {
    gsis_plan_destroy(pl);
    return fail(ctx, GSIS_NOT_CONVERGED, "forward solve did not converge in %d iterations", n);
  }
  if (fwd && (st = gsis_plan_read(pl, fwd))) {
    gsis_plan_destroy(pl);
    return st;
  }
  st = gsis_plan_adjoint(pl, g_phi, g_Fx, g_Fy, o->tol, o->max_iter, g_sigma_a, g_sigma_s, g_q,
                         info);
  gsis_plan_destroy(pl);
  return st;
}

}  // extern "C"
