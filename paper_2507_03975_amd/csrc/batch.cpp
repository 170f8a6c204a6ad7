// batch.cpp -- many independent problems of uneven size solved together.
//
// Every problem keeps its own plan (intensities, per-quadrant records,
// boundary data, multigrid hierarchy, CG scalars, state and convergence
// flag). One outer iteration of the batch is:
//   * one persistent sweep launch over the work items (problem, ordinate)
//     of all problems, longest first, with the launch configuration picked
//     by timing every compiled configuration on the batch itself;
//   * moments, boundary fluxes, HoT, right-hand side, each one launch over
//     (problem, block) tables;
//   * the synthetic CG + multigrid solves of all problems in lockstep: each
//     CG or multigrid step is one launch over the problems that have that
//     level, the coarse cycle one workgroup per problem, and every problem
//     keeps its own scalars and stop flag;
//   * correction, Err, next source, again one launch each.
// A problem therefore gets the same numbers as when solved alone, except
// that the CG runs a fixed number of iterations per outer iteration (device
// stop test per problem) instead of the host checking for convergence.
// Problems that have converged turn their kernels into no-ops. The whole
// iteration is captured once in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/gsis.h"
#include "plan.h"

namespace {

__global__ void k_gather_status(int n, const int32_t *const *states, const double *const *errs,
                                int32_t *st_out, double *err_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  for (int t = 0; t < 4; ++t) st_out[4 * p + t] = states[p][t];
  err_out[p] = *errs[p];
}

}  // namespace

struct gsis_batch {
  gsis_ctx *ctx = nullptr;
  int n = 0;
  int method = GSIS_GSIS;
  bool fp32 = false;
  std::vector<gsis_plan *> subs;
  SynthSet S;                      // synthetic step of all problems
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device tables
  void *targs = nullptr;
  int2 *items = nullptr;
  int n_items = 0;
  int *counter = nullptr;
  int2 *bt_face = nullptr;         // (problem, boundary face)
  int nb_face = 0;
  int32_t **state_p = nullptr;
  double **err_p = nullptr;
  int32_t *st_all = nullptr;
  double *err_all = nullptr;
  std::vector<void *> allocs;
  int32_t *host_flag = nullptr;    // pinned
  // tuning
  int cfg = 0, grid = 0, cg_iters = 0;
  double cfg_ms[kNumBatchSweepConfigs] = {};
  int use_graph = 1;
  hipGraphExec_t gexec = nullptr;
};

namespace {

template <typename T>
gsis_status balloc(gsis_batch *b, T **p, size_t n) {
  void *v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess)
    return fail(b->ctx, GSIS_E_OOM, "hipMalloc(%zu bytes): %s", n * sizeof(T),
                hipGetErrorString(e));
  b->allocs.push_back(v);
  *p = (T *)v;
  return GSIS_OK;
}

template <typename T>
gsis_status bupload(gsis_batch *b, T **p, const std::vector<T> &h) {
  gsis_status st = balloc(b, p, h.size());
  if (st) return st;
  if (!h.empty())
    HIPCHK(b->ctx, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return GSIS_OK;
}

// One outer iteration of the batch on b->stream. host_flag NULL: no host
// waits (graph capture).
void enqueue_iteration(gsis_batch *b, bool capture) {
  hipStream_t s = b->stream;
  (void)capture;
  launch_sweep_batch(b->targs, b->items, b->n_items, b->counter, b->cfg, b->fp32, b->grid, s);
  launch_moments_batch(b->targs, b->S.bt_cell, b->S.nb_cell, b->fp32, s);
  if (b->method == GSIS_GSIS) {
    launch_boundary_flux_batch(b->targs, b->bt_face, b->nb_face, s);
    launch_hot_rhs(b->S, s);
    launch_synth_solve(b->S, s, nullptr);
  }
  launch_update(b->S, s);
}

gsis_status reset_all(gsis_batch *b) {
  gsis_status st;
  for (gsis_plan *pl : b->subs)
    if ((st = gsis_plan_reset(pl))) return st;
  return GSIS_OK;
}

void destroy(gsis_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (gsis_plan *pl : b->subs) gsis_plan_destroy(pl);
  for (void *v : b->allocs) (void)hipFree(v);
  if (b->host_flag) (void)hipHostFree(b->host_flag);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // namespace

extern "C" {

gsis_status gsis_batch_create(gsis_ctx *ctx, int32_t n, const gsis_problem *p,
                              const gsis_options *o, gsis_batch **out) {
  if (!ctx) return fail(nullptr, GSIS_E_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(ctx, GSIS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(ctx, GSIS_E_INVALID_ARG, "n must be >= 1 (got %d)", n);
  if (!p || !o) return fail(ctx, GSIS_E_INVALID_ARG, "problems or options is NULL");
  if (o->I0) return fail(ctx, GSIS_E_INVALID_ARG, "options.I0 must be NULL for a batch");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  gsis_batch *b = new gsis_batch;
  b->ctx = ctx;
  b->n = n;
  b->method = o->method;
  b->fp32 = o->precision == GSIS_FP32_MIXED;
  b->use_graph = o->graph ? 1 : 0;
  auto bail = [&](gsis_status s) {
    // keep the message: destroy() may run HIP calls but sets no error
    destroy(b);
    return s;
  };
  if (o->stream) {
    b->stream = (hipStream_t)o->stream;
  } else {
    hipError_t e = hipStreamCreate(&b->stream);
    if (e != hipSuccess)
      return bail(fail(ctx, GSIS_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
    b->own_stream = true;
  }
  gsis_status st;
  // -- one plan per problem, all on the batch stream
  gsis_options so = *o;
  so.stream = b->stream;
  so.profile = 0;
  for (int i = 0; i < n; ++i) {
    gsis_plan *pl = nullptr;
    if ((st = gsis_plan_create(ctx, &p[i], &so, &pl))) {
      std::string msg = ctx->err;
      destroy(b);
      return fail(ctx, st, "problem %d: %s", i, msg.c_str());
    }
    b->subs.push_back(pl);
  }
  // -- per-problem kernel arguments and the sweep work items, longest first
  const size_t tb = targs_bytes();
  std::vector<char> th(tb * n);
  std::vector<std::pair<double, int2>> it;
  for (int i = 0; i < n; ++i) {
    const PlanDev &P = b->subs[i]->P;
    fill_targs(P, th.data() + tb * i);
    const double cost = (double)P.ny * (P.nx + std::min(P.ny, 128));
    for (int kk = 0; kk < P.K; ++kk) it.push_back({cost, make_int2(i, kk)});
  }
  std::stable_sort(it.begin(), it.end(),
                   [](const std::pair<double, int2> &a, const std::pair<double, int2> &c) {
                     return a.first > c.first;
                   });
  std::vector<int2> items(it.size());
  for (size_t t = 0; t < it.size(); ++t) items[t] = it[t].second;
  b->n_items = (int)items.size();
  {
    char *d = nullptr;
    if ((st = balloc(b, &d, th.size()))) return bail(st);
    HIPCHK(ctx, hipMemcpy(d, th.data(), th.size(), hipMemcpyHostToDevice));
    b->targs = d;
  }
  if ((st = bupload(b, &b->items, items)) || (st = balloc(b, &b->counter, 1))) return bail(st);
  // -- status gather tables
  {
    std::vector<int32_t *> sp(n);
    std::vector<double *> ep(n);
    for (int i = 0; i < n; ++i) {
      sp[i] = b->subs[i]->P.state;
      ep[i] = b->subs[i]->P.last_err;
    }
    if ((st = bupload(b, &b->state_p, sp)) || (st = bupload(b, &b->err_p, ep)) ||
        (st = balloc(b, &b->st_all, 4 * (size_t)n)) || (st = balloc(b, &b->err_all, n)))
      return bail(st);
  }
  // -- synthetic step of all problems: descriptors and block tables
  {
    SynthSet &S = b->S;
    std::vector<SynthDesc> D(n);
    int max_lc = 0;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
      const PlanDev &P = b->subs[i]->P;
      D[i] = make_synth_desc(P);
      max_lc = std::max(max_lc, D[i].lc);
      lds = std::max(lds, P.S.coarse_lds);
    }
    {
      char *d = nullptr;
      if ((st = balloc(b, &d, sizeof(SynthDesc) * n))) return bail(st);
      HIPCHK(ctx, hipMemcpy(d, D.data(), sizeof(SynthDesc) * n, hipMemcpyHostToDevice));
      S.desc = (SynthDesc *)d;
    }
    S.n = n;
    S.max_lc = max_lc;
    S.coarse_lds = lds;
    S.synth_max_iter = o->synth_max_iter;
    S.state0 = nullptr;
    auto nb = [](long long m) { return (int)((m + 255) / 256); };
    std::vector<int2> t;
    for (int i = 0; i < n; ++i)
      for (int lb = 0; lb < nb(D[i].N); ++lb) t.push_back(make_int2(i, lb));
    S.nb_cell = (int)t.size();
    if ((st = bupload(b, &S.bt_cell, t))) return bail(st);
    S.bt_tile.assign(max_lc, nullptr);
    S.nb_tile.assign(max_lc, 0);
    for (int l = 0; l < max_lc; ++l) {
      std::vector<int2> tt;
      for (int i = 0; i < n; ++i) {
        if (D[i].lc <= l) continue;
        for (int lb = 0; lb < tiles_of(D[i].lev[l].nx, D[i].lev[l].ny); ++lb)
          tt.push_back(make_int2(i, lb));
      }
      S.nb_tile[l] = (int)tt.size();
      if ((st = bupload(b, &S.bt_tile[l], tt))) return bail(st);
    }
    std::vector<int2> tfc;
    for (int i = 0; i < n; ++i)
      for (int f = 0; f < b->subs[i]->P.nbf; ++f) tfc.push_back(make_int2(i, f));
    b->nb_face = (int)tfc.size();
    if ((st = bupload(b, &b->bt_face, tfc))) return bail(st);
    prepare_synth(lds);
  }
  {
    void *h = nullptr;
    hipError_t e = hipHostMalloc(&h, 64, hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail(ctx, GSIS_E_OOM, "hipHostMalloc: %s", hipGetErrorString(e)));
    b->host_flag = (int32_t *)h;
  }
  // -- autotune the sweep launch: time every compiled configuration on this
  //    batch (the sweep reads the current iterate and rewrites the other
  //    buffer, so timing it changes no state)
  int cus = 0;
  HIPCHK(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  double best = 1e300;
  for (int c = 0; c < kNumBatchSweepConfigs; ++c) {
    const int per_cu = sweep_batch_blocks_per_cu(c, b->fp32);
    b->cfg_ms[c] = -1.0;
    if (per_cu <= 0) continue;
    const int grid = per_cu * cus;
    launch_sweep_batch(b->targs, b->items, b->n_items, b->counter, c, b->fp32, grid, b->stream);
    HIPCHK(ctx, hipEventRecord(e0, b->stream));
    for (int r = 0; r < 2; ++r)
      launch_sweep_batch(b->targs, b->items, b->n_items, b->counter, c, b->fp32, grid, b->stream);
    HIPCHK(ctx, hipEventRecord(e1, b->stream));
    HIPCHK(ctx, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
    b->cfg_ms[c] = ms / 2;
    if (ms / 2 < best) {
      best = ms / 2;
      b->cfg = c;
      b->grid = grid;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(ctx, hipGetLastError());
  if (best == 1e300) return bail(fail(ctx, GSIS_E_DEVICE, "no batched sweep configuration fits"));
  // -- CG iterations per outer iteration: the most any problem needed on
  //    one eager iteration (all problems run the full cap there), plus 2;
  //    then everything is reset
  if (b->method == GSIS_GSIS) {
    enqueue_iteration(b, false);
    double most = 0;
    for (gsis_plan *pl : b->subs) {
      double nit = 0;
      HIPCHK(ctx, hipMemcpyAsync(&nit, synth_iteration_counter(pl->P), sizeof nit,
                                 hipMemcpyDeviceToHost, b->stream));
      HIPCHK(ctx, hipStreamSynchronize(b->stream));
      most = std::max(most, nit);
    }
    b->cg_iters = std::max(4, std::min(o->synth_max_iter, (int)most + 2));
    b->S.synth_max_iter = b->cg_iters;
    if ((st = reset_all(b))) return bail(st);
  }
  // -- capture one outer iteration
  if (b->use_graph) {
    hipGraph_t g = nullptr;
    HIPCHK(ctx, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    enqueue_iteration(b, true);
    HIPCHK(ctx, hipStreamEndCapture(b->stream, &g));
    hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
      return bail(fail(ctx, GSIS_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e)));
  }
  *out = b;
  return GSIS_OK;
}

void gsis_batch_destroy(gsis_batch *b) { destroy(b); }

gsis_status gsis_batch_iterate(gsis_batch *b, int32_t n) {
  if (!b) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = b->ctx;
  if (n < 0) return fail(ctx, GSIS_E_INVALID_ARG, "n must be >= 0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  for (int i = 0; i < n; ++i) {
    if (b->gexec) HIPCHK(ctx, hipGraphLaunch(b->gexec, b->stream));
    else enqueue_iteration(b, false);
  }
  HIPCHK(ctx, hipGetLastError());
  return GSIS_OK;
}

gsis_status gsis_batch_status(gsis_batch *b, int32_t *n_iter, int32_t *converged,
                              double *last_err, int32_t *n_finished) {
  if (!b) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = b->ctx;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int n = b->n;
  hipLaunchKernelGGL(k_gather_status, dim3((n + 63) / 64), dim3(64), 0, b->stream, n,
                     (const int32_t *const *)b->state_p, (const double *const *)b->err_p, b->st_all,
                     b->err_all);
  std::vector<int32_t> st(4 * (size_t)n);
  std::vector<double> er(n);
  HIPCHK(ctx, hipMemcpyAsync(st.data(), b->st_all, st.size() * 4, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(ctx, hipMemcpyAsync(er.data(), b->err_all, er.size() * 8, hipMemcpyDeviceToHost, b->stream));
  HIPCHK(ctx, hipStreamSynchronize(b->stream));
  int fin = 0;
  for (int i = 0; i < n; ++i) {
    if (n_iter) n_iter[i] = st[4 * i];
    if (converged) converged[i] = st[4 * i + 1] == 1 ? 1 : (st[4 * i + 1] == -1 ? -1 : 0);
    if (last_err) last_err[i] = er[i];
    fin += st[4 * i + 1] != 0;
  }
  if (n_finished) *n_finished = fin;
  return GSIS_OK;
}

gsis_status gsis_batch_read(gsis_batch *b, int32_t i, gsis_result *r) {
  if (!b) return GSIS_E_INVALID_ARG;
  if (i < 0 || i >= b->n) return fail(b->ctx, GSIS_E_INVALID_ARG, "problem index %d out of range", i);
  return gsis_plan_read(b->subs[i], r);
}

gsis_status gsis_batch_reset(gsis_batch *b) {
  if (!b) return GSIS_E_INVALID_ARG;
  return reset_all(b);
}

gsis_status gsis_batch_get_tuning(gsis_batch *b, gsis_batch_tuning *t) {
  if (!b) return GSIS_E_INVALID_ARG;
  if (!t) return fail(b->ctx, GSIS_E_INVALID_ARG, "tuning is NULL");
  t->rows = kBatchSweepConfigs[b->cfg].rows;
  t->prefetch = kBatchSweepConfigs[b->cfg].pf;
  t->grid = b->grid;
  t->cg_iters = b->cg_iters;
  t->n_configs = kNumBatchSweepConfigs;
  for (int c = 0; c < kNumBatchSweepConfigs && c < 8; ++c) {
    t->config_rows[c] = kBatchSweepConfigs[c].rows;
    t->config_prefetch[c] = kBatchSweepConfigs[c].pf;
    t->config_ms[c] = b->cfg_ms[c];
  }
  return GSIS_OK;
}

gsis_status gsis_solve_batch(gsis_ctx *ctx, int32_t n, const gsis_problem *p,
                             const gsis_options *o, gsis_result *r) {
  if (!ctx) return fail(nullptr, GSIS_E_INVALID_ARG, "ctx is NULL");
  if (!r) return fail(ctx, GSIS_E_INVALID_ARG, "results is NULL");
  gsis_batch *b = nullptr;
  gsis_status st = gsis_batch_create(ctx, n, p, o, &b);
  if (st) return st;
  std::vector<int32_t> it(n);
  int32_t fin = 0;
  int done = 0;
  while (true) {
    const int todo = std::min(8, o->max_iter - done);
    if (todo <= 0) break;
    if ((st = gsis_batch_iterate(b, todo))) { destroy(b); return st; }
    done += todo;
    if ((st = gsis_batch_status(b, it.data(), nullptr, nullptr, &fin))) { destroy(b); return st; }
    if (fin == n) break;
  }
  gsis_status worst = GSIS_OK;
  for (int i = 0; i < n; ++i) {
    if ((st = gsis_batch_read(b, i, &r[i]))) { destroy(b); return st; }
    int32_t ni, conv;
    double le;
    gsis_plan_status(b->subs[i], &ni, &conv, &le);
    const gsis_status si = conv == 1 ? GSIS_OK : (conv == -1 ? GSIS_DIVERGED : GSIS_NOT_CONVERGED);
    if (si > worst) worst = si;
  }
  destroy(b);
  return worst;
}

}  // extern "C"
