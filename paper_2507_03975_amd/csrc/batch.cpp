// batch.cpp -- many independent problems of uneven size solved together.
//
// Every problem keeps its own plan (intensities, per-quadrant records,
// boundary data, multigrid hierarchy, CG scalars, state and convergence
// flag). One outer iteration of the batch is:
//   * the residual of every problem in one launch over items (problem,
//     tile, group of four ordinates), then one persistent recurrence launch
//     over the work items (problem, ordinate) of all problems, longest
//     first, with the rows per pass picked by timing every compiled
//     configuration on the batch itself (with the fused sweep selected, one
//     persistent fused launch instead);
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
// Problems that have finished turn their kernels into no-ops at once, and
// the next status query rebuilds the work tables without them (so a long
// tail of a few slow problems does not pay for launching the blocks of all
// the others). The whole iteration is captured in a hipGraph and replayed;
// the graph is captured again whenever the tables change.
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
  bool split = true;               // residual + recurrence (else the fused sweep)
  int4 *ritems = nullptr;          // residual items (problem, tile, group)
  int n_ritems = 0;
  int *counter = nullptr;
  int2 *bt_face = nullptr;         // (problem, boundary face)
  int nb_face = 0;
  int2 *bt_mtile = nullptr;        // (problem, moment tile or -1): each problem's
  int nb_mtile = 0;                // tiles in 8 runs, one per XCD (see the kernel)
  int32_t **state_p = nullptr;
  double **err_p = nullptr;
  int32_t *st_all = nullptr;
  double *err_all = nullptr;
  std::vector<void *> allocs;
  // tables of the problems still running (rebuilt when that set shrinks):
  // every table indexes problems by their place in `active`
  std::vector<int> active;
  std::vector<void *> tallocs;
  int32_t *host_flag = nullptr;    // pinned
  // tuning
  int cfg = 0, grid = 0, cg_iters = 0;
  int synth_cap = 50;              // options.synth_max_iter
  int cg_iters0 = 0;               // CG iterations chosen at creation
  double cfg_ms[8] = {};
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

template <typename T>
gsis_status tupload(gsis_batch *b, T **p, const std::vector<T> &h) {
  void *v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(h.size(), 1) * sizeof(T));
  if (e != hipSuccess)
    return fail(b->ctx, GSIS_E_OOM, "hipMalloc(%zu bytes): %s", h.size() * sizeof(T),
                hipGetErrorString(e));
  b->tallocs.push_back(v);
  *p = (T *)v;
  if (!h.empty())
    HIPCHK(b->ctx, hipMemcpy(v, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return GSIS_OK;
}

// Kernel arguments, work items, descriptors and block tables of the
// problems in act (in that order). Replaces the previous tables; the
// caller has synchronised the stream and dropped any graph using them.
gsis_status build_tables(gsis_batch *b, const std::vector<int> &act) {
  for (void *v : b->tallocs) (void)hipFree(v);
  b->tallocs.clear();
  b->active = act;
  const int n = (int)act.size();
  gsis_status st;
  // -- kernel arguments and the sweep work items, longest first
  const size_t tb = targs_bytes();
  std::vector<char> th(tb * std::max(n, 1));
  std::vector<std::pair<double, int2>> it;
  for (int a = 0; a < n; ++a) {
    const PlanDev &P = b->subs[act[a]]->P;
    fill_targs(P, th.data() + tb * a);
    const double cost = (double)P.ny * (P.nx + std::min(P.ny, 128));
    for (int kk = 0; kk < P.K; ++kk) it.push_back({cost, make_int2(a, kk)});
  }
  std::stable_sort(it.begin(), it.end(),
                   [](const std::pair<double, int2> &x, const std::pair<double, int2> &y) {
                     return x.first > y.first;
                   });
  std::vector<int2> items(it.size());
  for (size_t t = 0; t < it.size(); ++t) items[t] = it[t].second;
  b->n_items = (int)items.size();
  {
    char *d = nullptr;
    if ((st = tupload(b, &d, th))) return st;
    b->targs = d;
  }
  if ((st = tupload(b, &b->items, items))) return st;
  {
    std::vector<int4> ri;
    for (int a = 0; a < n; ++a) {
      const PlanDev &P = b->subs[act[a]]->P;
      int pairs = 0;
      for (int q = 0; q < 4; ++q) pairs += (P.qoff[q + 1] - P.qoff[q] + 1) / 2;
      const int groups = (pairs + kResidWaves - 1) / kResidWaves;
      for (int t = 0; t < P.n_rtiles; ++t)
        for (int g = 0; g < groups; ++g) ri.push_back(make_int4(a, t, g, 0));
    }
    b->n_ritems = (int)ri.size();
    if ((st = tupload(b, &b->ritems, ri))) return st;
  }
  // -- synthetic step: descriptors and block tables
  SynthSet &S = b->S;
  std::vector<SynthDesc> D(n);
  int max_lc = 0, min_lc = 1 << 30;
  bool any_sep = false;
  size_t lds = 0;
  for (int a = 0; a < n; ++a) {
    const PlanDev &P = b->subs[act[a]]->P;
    D[a] = make_synth_desc(P);
    D[a].n_tres = P.n_rtiles * residual_pairs(P);   // the batch's residual kernel's partials
    max_lc = std::max(max_lc, D[a].lc);
    min_lc = std::min(min_lc, D[a].lc);
    any_sep = any_sep || D[a].coef_sep != 0;
    lds = std::max(lds, P.S.coarse_lds);
  }
  {
    std::vector<char> dh(sizeof(SynthDesc) * std::max(n, 1));
    if (n) memcpy(dh.data(), D.data(), sizeof(SynthDesc) * n);
    char *d = nullptr;
    if ((st = tupload(b, &d, dh))) return st;
    S.desc = (SynthDesc *)d;
  }
  S.n = n;
  S.max_lc = max_lc;
  S.min_lc = n ? min_lc : 0;
  S.coarse_lds = lds;
  S.any_coef_sep = any_sep;
  S.state0 = nullptr;
  auto nb = [](long long m) { return (int)((m + 255) / 256); };
  std::vector<int2> t;
  for (int a = 0; a < n; ++a)
    for (int lb = 0; lb < nb(D[a].N); ++lb) t.push_back(make_int2(a, lb));
  S.nb_cell = (int)t.size();
  if ((st = tupload(b, &S.bt_cell, t))) return st;
  {
    std::vector<int2> ts;
    for (int a = 0; a < n; ++a)
      for (int lb = 0; lb < source_tiles_of(D[a].nx, D[a].ny); ++lb) ts.push_back(make_int2(a, lb));
    S.nb_src = (int)ts.size();
    if ((st = tupload(b, &S.bt_src, ts))) return st;
    // moment tiles: per problem 8 runs of tr = ceil(tiles / 8), entry p of
    // the problem's 8 tr (a multiple of 8, so p % 8 is the XCD) taking tile
    // (p % 8) tr + p / 8, or none
    std::vector<int2> tm;
    for (int a = 0; a < n; ++a) {
      const int nt = moment_tiles_of(D[a].nx, D[a].ny, moment_tile_size_batch());
      const int tr = (nt + 7) / 8;
      for (int p = 0; p < 8 * tr; ++p) {
        const int tl = (p % 8) * tr + p / 8;
        tm.push_back(make_int2(a, tl < nt ? tl : -1));
      }
    }
    b->nb_mtile = (int)tm.size();
    if ((st = tupload(b, &b->bt_mtile, tm))) return st;
  }
  S.bt_tile.assign(max_lc, nullptr);
  S.nb_tile.assign(max_lc, 0);
  for (int l = 0; l < max_lc; ++l) {
    std::vector<int2> tt;
    for (int a = 0; a < n; ++a) {
      if (D[a].lc <= l) continue;
      for (int lb = 0; lb < tiles_of(D[a].lev[l].nx, D[a].lev[l].ny); ++lb)
        tt.push_back(make_int2(a, lb));
    }
    S.nb_tile[l] = (int)tt.size();
    if ((st = tupload(b, &S.bt_tile[l], tt))) return st;
  }
  std::vector<int2> tfc;
  for (int a = 0; a < n; ++a)
    for (int f = 0; f < b->subs[act[a]]->P.nbf; ++f) tfc.push_back(make_int2(a, f));
  b->nb_face = (int)tfc.size();
  if ((st = tupload(b, &b->bt_face, tfc))) return st;
  prepare_synth(lds);
  return GSIS_OK;
}

void enqueue_iteration(gsis_batch *b, bool capture);

// (Re)capture one outer iteration of the current tables in a hipGraph.
gsis_status capture(gsis_batch *b) {
  gsis_ctx *ctx = b->ctx;
  if (b->gexec) {
    HIPCHK(ctx, hipStreamSynchronize(b->stream));
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  if (!b->use_graph || b->active.empty()) return GSIS_OK;
  hipGraph_t g = nullptr;
  HIPCHK(ctx, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  enqueue_iteration(b, true);
  HIPCHK(ctx, hipStreamEndCapture(b->stream, &g));
  hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(ctx, GSIS_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return GSIS_OK;
}

// Drop the problems that have finished from the tables (and the graph),
// so that later iterations launch no blocks for them.
gsis_status compact(gsis_batch *b, const std::vector<int32_t> &st4) {
  std::vector<int> act;
  for (int i : b->active)
    if (st4[4 * i + 1] == 0) act.push_back(i);
  if (act.size() == b->active.size()) return GSIS_OK;
  HIPCHK(b->ctx, hipStreamSynchronize(b->stream));
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  // CG iterations per outer iteration: the most a remaining problem used
  // in its last synthetic solve, plus 2
  if (b->method == GSIS_GSIS && !act.empty()) {
    double most = 0;
    for (int i : act) {
      double nit = 0;
      HIPCHK(b->ctx, hipMemcpy(&nit, synth_iteration_counter(b->subs[i]->P), sizeof nit,
                               hipMemcpyDeviceToHost));
      most = std::max(most, nit);
    }
    b->cg_iters = std::max(4, std::min(b->synth_cap, (int)most + 2));
    b->S.synth_max_iter = b->cg_iters;
  }
  gsis_status st = build_tables(b, act);
  if (st) return st;
  return capture(b);
}

std::vector<int> all_problems(int n) {
  std::vector<int> a(n);
  std::iota(a.begin(), a.end(), 0);
  return a;
}

// One outer iteration of the batch on b->stream. host_flag NULL: no host
// waits (graph capture).
void enqueue_iteration(gsis_batch *b, bool capture) {
  hipStream_t s = b->stream;
  (void)capture;
  if (b->active.empty()) return;
  if (b->split) {
    launch_resid_batch(b->targs, b->ritems, b->n_ritems, b->fp32, s);
    launch_chain_batch(b->targs, b->items, b->n_items, b->counter, b->cfg, b->fp32, b->grid, s);
  } else {
    launch_sweep_batch(b->targs, b->items, b->n_items, b->counter, b->cfg, b->fp32, b->grid, s);
  }
  launch_moments_batch(b->targs, b->S.bt_cell, b->S.nb_cell, b->bt_mtile, b->nb_mtile, b->fp32,
                       s);
  if (b->method == GSIS_GSIS) {
    launch_boundary_flux_batch(b->targs, b->bt_face, b->nb_face, s);
    launch_hot(b->S, s, false);
    launch_synth_solve(b->S, s, nullptr, 1);
  }
  launch_update(b->S, s);
}

gsis_status reset_all(gsis_batch *b) {
  gsis_status st;
  for (gsis_plan *pl : b->subs)
    if ((st = gsis_plan_reset(pl))) return st;
  if (b->cg_iters0 > 0) {
    b->cg_iters = b->cg_iters0;
    b->S.synth_max_iter = b->cg_iters0;
  }
  if ((int)b->active.size() != b->n) {
    HIPCHK(b->ctx, hipStreamSynchronize(b->stream));
    if (b->gexec) {
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    if ((st = build_tables(b, all_problems(b->n)))) return st;
    if ((st = capture(b))) return st;
  }
  return GSIS_OK;
}

void destroy(gsis_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (gsis_plan *pl : b->subs) gsis_plan_destroy(pl);
  for (void *v : b->allocs) (void)hipFree(v);
  for (void *v : b->tallocs) (void)hipFree(v);
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
  if (o->synth_form != 0)
    return fail(ctx, GSIS_E_UNSUPPORTED, "options.synth_form 1 is available for single plans only");
  if (o->method == GSIS_GSIS && o->hot_face != GSIS_HOT_CENTRAL)
    return fail(ctx, GSIS_E_UNSUPPORTED,
                "options.hot_face 1 (transport faces) is available for single plans only");
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
  // -- tables of all problems
  if ((st = balloc(b, &b->counter, 1))) return bail(st);
  b->split = b->subs[0]->P.sweep_impl == 0 || b->subs[0]->P.sweep_impl == 3;
  b->S.synth_max_iter = o->synth_max_iter;
  b->synth_cap = o->synth_max_iter;
  if ((st = build_tables(b, all_problems(n)))) return bail(st);
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
  const int ncfg = b->split ? kNumBatchChainConfigs : kNumBatchSweepConfigs;
  auto run = [&](int c, int grid) {
    if (b->split)
      launch_chain_batch(b->targs, b->items, b->n_items, b->counter, c, b->fp32, grid, b->stream);
    else
      launch_sweep_batch(b->targs, b->items, b->n_items, b->counter, c, b->fp32, grid, b->stream);
  };
  for (int c = 0; c < ncfg; ++c) {
    const int per_cu = b->split ? chain_batch_blocks_per_cu(c, b->fp32)
                                : sweep_batch_blocks_per_cu(c, b->fp32);
    b->cfg_ms[c] = -1.0;
    if (per_cu <= 0) continue;
    const int grid = per_cu * cus;
    // the recurrence rewrites the residual's output in place, so every
    // timed run starts from a fresh residual launch (outside the events)
    float ms = 0;
    for (int r = 0; r < 3; ++r) {
      if (b->split) launch_resid_batch(b->targs, b->ritems, b->n_ritems, b->fp32, b->stream);
      HIPCHK(ctx, hipEventRecord(e0, b->stream));
      run(c, grid);
      HIPCHK(ctx, hipEventRecord(e1, b->stream));
      HIPCHK(ctx, hipEventSynchronize(e1));
      float m1 = 0;
      HIPCHK(ctx, hipEventElapsedTime(&m1, e0, e1));
      if (r > 0) ms += m1;           // the first run warms up
    }
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
    b->cg_iters0 = b->cg_iters;
    if ((st = reset_all(b))) return bail(st);
  }
  // -- capture one outer iteration
  if ((st = capture(b))) return bail(st);
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
  // problems found finished leave the launches from now on
  return compact(b, st);
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
  const BatchSweepConfig *cf = b->split ? kBatchChainConfigs : kBatchSweepConfigs;
  const int ncfg = b->split ? kNumBatchChainConfigs : kNumBatchSweepConfigs;
  t->rows = cf[b->cfg].rows;
  t->prefetch = cf[b->cfg].pf;
  t->grid = b->grid;
  t->cg_iters = b->cg_iters;
  t->n_configs = ncfg;
  for (int c = 0; c < ncfg && c < 8; ++c) {
    t->config_rows[c] = cf[c].rows;
    t->config_prefetch[c] = cf[c].pf;
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
