// plan.h -- host-side state shared by the C-ABI translation units: the
// context and plan objects, error reporting, device allocation helpers and
// the synthetic-solve set-up.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "gsis_internal.h"

using namespace gsis;

struct gsis_ctx {
  int device = 0;
  std::string err;
};

struct gsis_plan {
  gsis_ctx *ctx = nullptr;
  PlanDev P;
  hipStream_t stream = nullptr;
  int device_ptrs = 0;
  int profile = 0;
  std::vector<int> perm;          // internal ordinate -> caller ordinate
  double swmu = 0, sweta = 0;     // sum_k w_k mu_k, sum_k w_k eta_k
  std::vector<double> I0_host;    // warm start in the internal layout (may be empty)
  std::vector<float> I0_host_f;   // FP32-mixed: I0 - phi0/(4 pi) in the internal layout
  std::vector<double> phi0_host;  // phi of the warm start
  std::vector<double> T0_host;    // time-dependent form: initial temperature
  std::vector<void *> allocs;
  double *host_scal = nullptr;    // pinned
  hipEvent_t spec_ev = nullptr;   // marks the synthetic solve's flag copy (see
                                  // launch_synth_solve); not in the allocation-free solve
  // profiling: per iteration GSIS_NUM_PHASES + 1 events bracketing the phases
  std::vector<hipEvent_t> events;
  int prof_iters = 0;
  int pseudo = 0;                 // a pseudo-time shift is on
  AdjointBuffers *adj = nullptr;  // adjoint state (first gsis_plan_adjoint)
  // device memory carved from a caller-free region instead of hipMalloc
  // (gsis_solve_noalloc): base, bytes used, capacity; the host flags then
  // live in host_flag_store instead of pinned memory
  char *arena = nullptr;
  size_t arena_used = 0, arena_cap = 0;
  double host_flag_store[8] = {};
};

extern thread_local std::string g_create_err;

inline gsis_status fail_impl(gsis_ctx *ctx, gsis_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  else g_create_err = buf;
  return st;
}
#define fail fail_impl

#define HIPCHK(ctx, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, GSIS_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)


template <typename T>
gsis_status dalloc(gsis_plan *pl, T **p, size_t n) {
  void *v = nullptr;
  if (pl->arena) {
    // 256-byte aligned pieces of the region, in allocation order
    const size_t bytes = (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
    if (bytes > pl->arena_cap - pl->arena_used)
      return fail(pl->ctx, GSIS_E_INVALID_ARG,
                  "the problem needs more device memory than the %zu-byte scratch region of "
                  "gsis_solve_noalloc (%zu bytes used when %zu more were asked for)",
                  pl->arena_cap, pl->arena_used, bytes);
    *p = (T *)(pl->arena + pl->arena_used);
    pl->arena_used += bytes;
    return GSIS_OK;
  }
  hipError_t e = hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess)
    return fail(pl->ctx, GSIS_E_OOM, "hipMalloc(%zu bytes): %s", n * sizeof(T),
                hipGetErrorString(e));
  pl->allocs.push_back(v);
  *p = (T *)v;
  return GSIS_OK;
}

template <typename T>
gsis_status upload(gsis_plan *pl, T **p, const std::vector<T> &h) {
  gsis_status st = dalloc(pl, p, h.size());
  if (st) return st;
  if (!h.empty()) HIPCHK(pl->ctx, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return GSIS_OK;
}

struct HostLevel {
  int nx, ny, fx = 1, fy = 1;
  std::vector<double> diag, ax, ay;
};

// Multigrid hierarchy of hl[0] and the device state of a synthetic solve on
// P (defined in capi.cpp).
gsis_status setup_synth(gsis_plan *pl, PlanDev &P, std::vector<HostLevel> &hl);
// P.S for the plan alone (descriptor upload, block counts).
gsis_status make_single_set(gsis_plan *pl);
// Frees the adjoint's host-side state (device memory goes with the plan).
void adjoint_release(gsis_plan *pl);
