// capi.cpp -- C-ABI of libgsis.so: argument checks, plan set-up (ordinate
// regrouping, least-squares / synthetic coefficients, multigrid hierarchy)
// and the outer-iteration driver. Every arithmetic step of an iteration runs
// in the HIP kernels; the host only sets up coefficients once per plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gsis.h"
#include "plan.h"

thread_local std::string g_create_err;

extern "C" {

const char *gsis_version(void) {
  return "libgsis (HIP, gfx950) FP64 wavefront sweep + CG/GMG synthetic solve";
}

gsis_status gsis_ctx_create(int32_t device, gsis_ctx **out) {
  if (!out) return fail(nullptr, GSIS_E_INVALID_ARG, "out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0)
    return fail(nullptr, GSIS_E_DEVICE, "no HIP device: %s", hipGetErrorString(e));
  if (device < 0 || device >= n)
    return fail(nullptr, GSIS_E_INVALID_ARG, "device %d out of range [0,%d)", device, n);
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, GSIS_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  gsis_ctx *c = new gsis_ctx;
  c->device = device;
  *out = c;
  return GSIS_OK;
}

void gsis_ctx_destroy(gsis_ctx *ctx) { delete ctx; }

const char *gsis_last_error(const gsis_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

gsis_status gsis_options_default(gsis_options *o) {
  if (!o) return GSIS_E_INVALID_ARG;
  std::memset(o, 0, sizeof *o);
  o->method = GSIS_GSIS;
  o->precision = GSIS_FP64;
  o->order = 2;
  o->limiter = 1;
  o->alsm = 1;
  o->hot_face = GSIS_HOT_CENTRAL;
  o->tol = 1e-6;
  o->max_iter = 1000;
  o->synth_rtol = 0.1;
  o->synth_max_iter = 50;
  o->cfl_p = 0.0;
  o->beta = 0.0;
  o->graph = 1;
  o->synth_form = 0;
  o->synth_sub = 4;
  return GSIS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ helpers
namespace {

// Copy n doubles from caller memory (host or device) to a host vector.
gsis_status fetch(gsis_ctx *ctx, const double *src, size_t n, int dev, std::vector<double> &dst,
                  const char *name) {
  if (!src) return fail(ctx, GSIS_E_INVALID_ARG, "%s is NULL", name);
  dst.resize(n);
  if (n == 0) return GSIS_OK;
  if (dev) {
    hipError_t e = hipMemcpy(dst.data(), src, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
      return fail(ctx, GSIS_E_DEVICE, "reading %s: %s", name, hipGetErrorString(e));
  } else {
    std::memcpy(dst.data(), src, n * sizeof(double));
  }
  return GSIS_OK;
}

gsis_status check_problem(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                          std::vector<double> &mu, std::vector<double> &eta,
                          std::vector<double> &w, std::vector<double> &sa,
                          std::vector<double> &ss, std::vector<double> &q,
                          std::vector<double> &bnd) {
  if (!p) return fail(ctx, GSIS_E_INVALID_ARG, "problem is NULL");
  if (!o) return fail(ctx, GSIS_E_INVALID_ARG, "options is NULL");
  if (p->nx < 1 || p->ny < 1)
    return fail(ctx, GSIS_E_INVALID_ARG, "nx, ny must be >= 1 (got %d, %d)", p->nx, p->ny);
  if ((long long)p->nx * p->ny > GSIS_MAX_CELLS)
    return fail(ctx, GSIS_E_INVALID_ARG, "nx*ny = %lld too large (at most %d cells)",
                (long long)p->nx * p->ny, GSIS_MAX_CELLS);
  if (!(p->dx > 0) || !(p->dy > 0) || !std::isfinite(p->dx) || !std::isfinite(p->dy))
    return fail(ctx, GSIS_E_INVALID_ARG, "dx, dy must be finite and > 0");
  if (p->K < 1) return fail(ctx, GSIS_E_INVALID_ARG, "K must be >= 1 (got %d)", p->K);
  if (o->method != GSIS_SI && o->method != GSIS_GSIS)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.method must be 0 or 1");
  if (o->precision != GSIS_FP64 && o->precision != GSIS_FP32_MIXED)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.precision must be 0 or 1");
  if (o->order != 1 && o->order != 2)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.order must be 1 or 2");
  if (o->hot_face != GSIS_HOT_CENTRAL && o->hot_face != GSIS_HOT_TRANSPORT)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.hot_face must be 0 or 1");
  if (o->max_iter < 1) return fail(ctx, GSIS_E_INVALID_ARG, "options.max_iter must be >= 1");
  if (!(o->tol >= 0) || std::isnan(o->tol))
    return fail(ctx, GSIS_E_INVALID_ARG, "options.tol must be >= 0");
  if (!(o->synth_rtol > 0)) return fail(ctx, GSIS_E_INVALID_ARG, "options.synth_rtol must be > 0");
  if (o->synth_max_iter < 1)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.synth_max_iter must be >= 1");
  if (!(o->cfl_p >= 0) || !std::isfinite(o->cfl_p))
    return fail(ctx, GSIS_E_INVALID_ARG, "options.cfl_p must be finite and >= 0");
  if (!(o->beta >= 0) || !std::isfinite(o->beta))
    return fail(ctx, GSIS_E_INVALID_ARG, "options.beta must be finite and >= 0");
  if (o->synth_form != 0 && o->synth_form != 1)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.synth_form must be 0 or 1");
  if (o->synth_form == 1 && o->synth_sub < 1)
    return fail(ctx, GSIS_E_INVALID_ARG, "options.synth_sub must be >= 1");
  const int dev = o->device_ptrs;
  const size_t N = (size_t)p->nx * p->ny, K = p->K;
  gsis_status st;
  if ((st = fetch(ctx, p->mu, K, dev, mu, "mu")) || (st = fetch(ctx, p->eta, K, dev, eta, "eta")) ||
      (st = fetch(ctx, p->w, K, dev, w, "w")) ||
      (st = fetch(ctx, p->sigma_a, N, dev, sa, "sigma_a")) ||
      (st = fetch(ctx, p->sigma_s, N, dev, ss, "sigma_s")) ||
      (st = fetch(ctx, p->q, N, dev, q, "q")))
    return st;
  double wsum = 0;
  for (size_t k = 0; k < K; ++k) {
    if (!std::isfinite(mu[k]) || !std::isfinite(eta[k]) || !std::isfinite(w[k]))
      return fail(ctx, GSIS_E_INVALID_ARG, "quadrature entry %zu is not finite", k);
    if (mu[k] * mu[k] + eta[k] * eta[k] > 1.0 + 1e-12)
      return fail(ctx, GSIS_E_INVALID_ARG, "mu[%zu]^2 + eta[%zu]^2 > 1", k, k);
    if (w[k] < 0) return fail(ctx, GSIS_E_INVALID_ARG, "w[%zu] < 0", k);
    wsum += w[k];
  }
  if (std::fabs(wsum - kFourPi) > 1e-12 * kFourPi)
    return fail(ctx, GSIS_E_INVALID_ARG, "sum(w) = %.17g, expected 4*pi", wsum);
  for (size_t c = 0; c < N; ++c) {
    if (!std::isfinite(sa[c]) || sa[c] < 0)
      return fail(ctx, GSIS_E_INVALID_ARG, "sigma_a[%zu] must be finite and >= 0", c);
    if (!std::isfinite(ss[c]) || ss[c] < 0)
      return fail(ctx, GSIS_E_INVALID_ARG, "sigma_s[%zu] must be finite and >= 0", c);
    if (!(sa[c] + ss[c] > 0))
      return fail(ctx, GSIS_E_INVALID_ARG, "sigma_a[%zu] + sigma_s[%zu] must be > 0", c, c);
    if (!std::isfinite(q[c])) return fail(ctx, GSIS_E_INVALID_ARG, "q[%zu] is not finite", c);
  }
  const size_t nbf = 2 * ((size_t)p->nx + p->ny);
  if (p->bnd_in) {
    if ((st = fetch(ctx, p->bnd_in, nbf * K, dev, bnd, "bnd_in"))) return st;
    for (size_t t = 0; t < nbf * K; ++t)
      if (!std::isfinite(bnd[t]))
        return fail(ctx, GSIS_E_INVALID_ARG, "bnd_in[%zu][%zu] is not finite", t / K, t % K);
  } else {
    bnd.assign(nbf * K, 0.0);
  }
  return GSIS_OK;
}

// One intensity buffer: N*K doubles, or N*K floats in FP32-mixed mode.
gsis_status alloc_intensity(gsis_plan *pl, int which, size_t nk, bool f32) {
  gsis_status st;
  if (f32) {
    float *p = nullptr;
    st = dalloc(pl, &p, nk);
    pl->P.I[which] = p;
  } else {
    double *p = nullptr;
    st = dalloc(pl, &p, nk);
    pl->P.I[which] = p;
  }
  return st;
}

// Dense SPD inverse by Cholesky (coarsest multigrid level, n <= a few hundred).
bool dense_spd_inverse(int n, std::vector<double> &A) {
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double s = L[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0)) return false;
    const double d = std::sqrt(s);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = L[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / d;
    }
  }
  // columns of A^{-1}: solve L L^T x = e_c
  std::vector<double> x(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * x[k];
      x[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = x[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * x[k];
      x[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) A[(size_t)i * n + c] = x[i];
  }
  return true;
}


}  // namespace

// Multigrid hierarchy of the level-0 synthetic operator hl[0] (Galerkin
// coarsening) and the device state of a synthetic solve on P: levels, dense
// coarsest inverse, CG vectors, block partials and scalars. P.N must be set.
gsis_status setup_synth(gsis_plan *pl, PlanDev &P, std::vector<HostLevel> &hl) {
  // Galerkin coarsening. Aggregates are 2x2, or 2x1 / 1x2 when the
  // couplings in one direction are much weaker than in the other (then
  // merging across the weak direction would leave error the point smoother
  // cannot reach).
  const int kCoarseMax = 64;   // dense inverse of the coarsest level: at most 64 x 64
  while ((long)hl.back().nx * hl.back().ny > kCoarseMax && (hl.back().nx > 1 || hl.back().ny > 1)) {
    HostLevel &F = hl.back();
    double lx = 0, ly = 0;
    long mx = 0, my = 0;
    for (int j = 0; j < F.ny; ++j)
      for (int i = 0; i < F.nx; ++i) {
        const int c = j * F.nx + i;
        if (i + 1 < F.nx) { lx += std::log(F.ax[c]); ++mx; }
        if (j + 1 < F.ny) { ly += std::log(F.ay[c]); ++my; }
      }
    const double gx = mx ? std::exp(lx / mx) : 0.0, gy = my ? std::exp(ly / my) : 0.0;
    F.fx = (F.nx > 1 && gx >= 0.25 * gy) ? 2 : 1;
    F.fy = (F.ny > 1 && gy >= 0.25 * gx) ? 2 : 1;
    HostLevel C;
    C.nx = (F.nx + F.fx - 1) / F.fx;
    C.ny = (F.ny + F.fy - 1) / F.fy;
    const int Nc = C.nx * C.ny;
    C.diag.assign(Nc, 0.0); C.ax.assign(Nc, 0.0); C.ay.assign(Nc, 0.0);
    for (int j = 0; j < F.ny; ++j)
      for (int i = 0; i < F.nx; ++i) {
        const int c = j * F.nx + i;
        const int Ci = i / F.fx, Cj = j / F.fy;
        const int Cc = Cj * C.nx + Ci;
        C.diag[Cc] += F.diag[c];
        if (i + 1 < F.nx) {
          const int Ci2 = (i + 1) / F.fx;
          if (Ci2 == Ci) C.diag[Cc] -= 2.0 * F.ax[c];
          else C.ax[Cc] += F.ax[c];
        }
        if (j + 1 < F.ny) {
          const int Cj2 = (j + 1) / F.fy;
          if (Cj2 == Cj) C.diag[Cc] -= 2.0 * F.ay[c];
          else C.ay[Cc] += F.ay[c];
        }
      }
    hl.push_back(std::move(C));
  }
  // dense inverse of the coarsest level
  const HostLevel &Lc = hl.back();
  const int nc = Lc.nx * Lc.ny;
  std::vector<double> dense((size_t)nc * nc, 0.0);
  for (int j = 0; j < Lc.ny; ++j)
    for (int i = 0; i < Lc.nx; ++i) {
      const int c = j * Lc.nx + i;
      dense[(size_t)c * nc + c] = Lc.diag[c];
      if (i + 1 < Lc.nx) {
        dense[(size_t)c * nc + c + 1] = -Lc.ax[c];
        dense[(size_t)(c + 1) * nc + c] = -Lc.ax[c];
      }
      if (j + 1 < Lc.ny) {
        dense[(size_t)c * nc + c + Lc.nx] = -Lc.ay[c];
        dense[(size_t)(c + Lc.nx) * nc + c] = -Lc.ay[c];
      }
    }
  if (!dense_spd_inverse(nc, dense))
    return fail(pl->ctx, GSIS_E_INVALID_ARG, "synthetic operator is not positive definite");

  gsis_status st;
  const int N = P.N;
  if ((st = dalloc(pl, &P.cg_r, N)) || (st = dalloc(pl, &P.cg_r2, N)) ||
      (st = dalloc(pl, &P.cg_z, N)) ||
      (st = dalloc(pl, &P.cg_p, N)) || (st = dalloc(pl, &P.cg_s0, N)) ||
      (st = dalloc(pl, &P.cg_s1, N)) || (st = dalloc(pl, &P.cg_w, N)) ||
      (st = dalloc(pl, &P.scal, 16)))
    return st;
  if (P.synth_form == 1 &&
      ((st = dalloc(pl, &P.wide_wx, N)) || (st = dalloc(pl, &P.wide_wy, N))))
    return st;
  // block partials: r.r and b.b (one per 256 cells each), then r.z, the
  // r.r of the level-0 tile kernel and z.Az (one per level-0 multigrid tile
  // each)
  P.red_blocks = (N + 255) / 256;
  const size_t ntp = std::max<size_t>(tiles_of(P.nx, P.ny), P.red_blocks);
  if ((st = dalloc(pl, &P.red, 2 * (size_t)P.red_blocks + 3 * ntp + 2))) return st;
  P.mg.resize(hl.size());
  for (size_t l = 0; l < hl.size(); ++l) {
    MGLevel &L = P.mg[l];
    L.nx = hl[l].nx; L.ny = hl[l].ny; L.fx = hl[l].fx; L.fy = hl[l].fy;
    const size_t n = (size_t)L.nx * L.ny;
    if ((st = upload(pl, &L.diag, hl[l].diag)) || (st = upload(pl, &L.ax, hl[l].ax)) ||
        (st = upload(pl, &L.ay, hl[l].ay)) || (st = dalloc(pl, &L.x, n)) ||
        (st = dalloc(pl, &L.b, n)) || (st = dalloc(pl, &L.r, n)))
      return st;
  }
  P.coarse_n = nc;
  if ((st = upload(pl, &P.coarse_inv, dense))) return st;
  return GSIS_OK;
}

// Launch set of a single plan: its synthetic-step descriptor on the device
// and block counts per level (no block tables). Needs every array of P.
gsis_status make_single_set(gsis_plan *pl) {
  PlanDev &P = pl->P;
  SynthSet &S = P.S;
  const SynthDesc D = make_synth_desc(P);
  gsis_status st;
  {
    char *d = nullptr;
    if ((st = dalloc(pl, &d, sizeof D))) return st;
    HIPCHK(pl->ctx, hipMemcpy(d, &D, sizeof D, hipMemcpyHostToDevice));
    S.desc = (SynthDesc *)d;
  }
  auto nb = [](int n) { return (n + 255) / 256; };
  S.n = 1;
  S.max_lc = D.lc;
  S.min_lc = D.lc;
  S.any_coef_sep = D.coef_sep != 0;
  P.lc = D.lc;
  S.coarse_lds = coarse_lds_bytes(P);
  S.synth_max_iter = P.synth_max_iter;
  S.nb_cell = nb(P.N);
  S.bt_cell = nullptr;
  S.nb_src = source_tiles_of(P.nx, P.ny);
  S.bt_src = nullptr;
  S.bt_tile.assign(D.lc, nullptr);
  S.nb_tile.resize(D.lc);
  for (int l = 0; l < D.lc; ++l) S.nb_tile[l] = tiles_of(P.mg[l].nx, P.mg[l].ny);
  S.state0 = P.state;
  prepare_synth(S.coarse_lds);
  return GSIS_OK;
}

// ------------------------------------------------------------------- plans
// A plan whose device memory comes from hipMalloc (arena NULL) or is carved
// from the arena_cap bytes at arena (no device or pinned allocation at all;
// profiling off).
// With mt, the time-dependent form (backward-Euler steps of size mt->dt).
// room for the partial sums of w r^2 of either residual kernel (a batch
// runs its own on a plan made for the pipelined step)
static size_t tres_slots(const PlanDev &P) {
  return std::max((size_t)P.n_tres, (size_t)P.n_rtiles * residual_pairs(P));
}

static gsis_status plan_create(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                               gsis_plan **out, char *arena, size_t arena_cap,
                               const gsis_material *mt = nullptr) {
  if (!ctx) return fail(nullptr, GSIS_E_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(ctx, GSIS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::vector<double> mu, eta, w, sa, ss, q, bnd;
  gsis_status st = check_problem(ctx, p, o, mu, eta, w, sa, ss, q, bnd);
  if (st) return st;
  std::vector<double> cvh, T0h;
  if (mt) {
    if (!(mt->c > 0) || !std::isfinite(mt->c))
      return fail(ctx, GSIS_E_INVALID_ARG, "material.c must be finite and > 0");
    if (!(mt->a >= 0) || !std::isfinite(mt->a))
      return fail(ctx, GSIS_E_INVALID_ARG, "material.a must be finite and >= 0");
    if (!(mt->dt > 0) || !std::isfinite(mt->dt) || !std::isfinite(1.0 / (mt->c * mt->dt)))
      return fail(ctx, GSIS_E_INVALID_ARG, "material.dt must be finite and > 0");
    if (mt->sub_iter < 1) return fail(ctx, GSIS_E_INVALID_ARG, "material.sub_iter must be >= 1");
    if (o->precision != GSIS_FP64)
      return fail(ctx, GSIS_E_UNSUPPORTED, "the time-dependent form runs in FP64 only");
    if (o->synth_form != 0)
      return fail(ctx, GSIS_E_UNSUPPORTED, "the time-dependent form needs options.synth_form 0");
    const size_t N = (size_t)p->nx * p->ny;
    if ((st = fetch(ctx, mt->cv, N, o->device_ptrs, cvh, "material.cv")) ||
        (st = fetch(ctx, mt->T0, N, o->device_ptrs, T0h, "material.T0")))
      return st;
    for (size_t c = 0; c < N; ++c) {
      if (!(cvh[c] > 0) || !std::isfinite(cvh[c]))
        return fail(ctx, GSIS_E_INVALID_ARG, "material.cv[%zu] must be finite and > 0", c);
      if (!(T0h[c] >= 0) || !std::isfinite(T0h[c]))
        return fail(ctx, GSIS_E_INVALID_ARG, "material.T0[%zu] must be finite and >= 0", c);
    }
  }
  if (o->method == GSIS_GSIS && o->hot_face == GSIS_HOT_TRANSPORT && o->synth_form != 0)
    return fail(ctx, GSIS_E_UNSUPPORTED,
                "options.synth_form 1 needs central HoT faces (options.hot_face 0)");
  HIPCHK(ctx, hipSetDevice(ctx->device));

  gsis_plan *pl = new gsis_plan;
  pl->ctx = ctx;
  pl->stream = (hipStream_t)o->stream;
  pl->device_ptrs = o->device_ptrs;
  pl->profile = arena ? 0 : o->profile;
  pl->arena = arena;
  pl->arena_cap = arena_cap;
  pl->pseudo = (o->cfl_p > 0 || o->beta > 0) ? 1 : 0;
  PlanDev &P = pl->P;
  const int nx = p->nx, ny = p->ny, N = nx * ny, K = p->K;
  P.nx = nx; P.ny = ny; P.N = N; P.K = K; P.nbf = 2 * (nx + ny);
  P.dx = p->dx; P.dy = p->dy; P.V = p->dx * p->dy;
  P.method = o->method; P.precision = o->precision; P.order = o->order;
  P.limiter = o->limiter ? 1 : 0; P.alsm = o->alsm ? 1 : 0; P.hot_face = o->hot_face;
  P.tol = o->tol; P.max_iter = o->max_iter; P.synth_rtol = o->synth_rtol;
  P.synth_max_iter = o->synth_max_iter;
  P.synth_form = o->method == GSIS_GSIS ? o->synth_form : 0;
  P.synth_sub = o->synth_sub;
  if (mt) {
    P.td = 1;
    P.sub_iter = mt->sub_iter;
    P.tdiag = 1.0 / (mt->c * mt->dt);
    P.ca = mt->a * mt->c;
    P.dt = mt->dt;
    pl->T0_host = T0h;
  }
  auto bail = [&](gsis_status s) {
    gsis_plan_destroy(pl);
    return s;
  };

  // -- regroup ordinates by quadrant (bit 0: mu < 0, bit 1: eta < 0)
  pl->perm.clear();
  for (int qd = 0; qd < 4; ++qd) {
    P.qoff[qd] = (int)pl->perm.size();
    for (int k = 0; k < K; ++k) {
      int qk = (mu[k] < 0 ? 1 : 0) | (eta[k] < 0 ? 2 : 0);
      if (qk == qd) pl->perm.push_back(k);
    }
    P.Kq[qd] = (int)pl->perm.size() - P.qoff[qd];
  }
  P.qoff[4] = K;
  std::vector<double> amu(K), aeta(K), wv(K), wmu(K), weta(K);
  pl->swmu = pl->sweta = 0;
  for (int kk = 0; kk < K; ++kk) {
    const int k = pl->perm[kk];
    amu[kk] = std::fabs(mu[k]) / p->dx;
    aeta[kk] = std::fabs(eta[k]) / p->dy;
    wv[kk] = w[k];
    wmu[kk] = w[k] * mu[k];
    weta[kk] = w[k] * eta[k];
    pl->swmu += wmu[kk];
    pl->sweta += weta[kk];
    P.sw += wv[kk];
  }
  P.swm = pl->swmu;
  P.swe = pl->sweta;
  const bool f32 = P.precision == GSIS_FP32_MIXED;

  // -- per-cell coefficients
  std::vector<double> st_(N), cE(N), cW(N), cN(N), cS(N);
  for (int c = 0; c < N; ++c) st_[c] = sa[c] + ss[c];
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      // distance from x_c to the (shifted) neighbour point along the normal
      // (Eq. shifted_j): half a cell to the face, then sigma_nb/sigma_c times
      // the half cell beyond it; plain least squares uses the centre.
      auto dist = [&](int nb, double h) {
        if (nb < 0) return 0.0;
        return P.alsm ? 0.5 * h + (st_[nb] / st_[c]) * (0.5 * h) : h;
      };
      const double dE = dist(i + 1 < nx ? c + 1 : -1, p->dx);
      const double dW = dist(i > 0 ? c - 1 : -1, p->dx);
      const double dN = dist(j + 1 < ny ? c + nx : -1, p->dy);
      const double dS = dist(j > 0 ? c - nx : -1, p->dy);
      const double mx = dE * dE + dW * dW, my = dN * dN + dS * dS;
      cE[c] = mx > 0 ? dE / mx : 0.0;
      cW[c] = mx > 0 ? dW / mx : 0.0;
      cN[c] = my > 0 ? dN / my : 0.0;
      cS[c] = my > 0 ? dS / my : 0.0;
    }
  // kappa per boundary face (Eqs. macro_bc_delta_flux, macro_bc_delta_flux2)
  std::vector<double> kap(P.nbf);
  for (int j = 0; j < ny; ++j) {
    kap[j] = 2.0 / (3.0 * st_[j * nx] * p->dx) + 0.25;
    kap[ny + j] = 2.0 / (3.0 * st_[j * nx + nx - 1] * p->dx) + 0.25;
  }
  for (int i = 0; i < nx; ++i) {
    kap[2 * ny + i] = 2.0 / (3.0 * st_[i] * p->dy) + 0.25;
    kap[2 * ny + nx + i] = 2.0 / (3.0 * st_[(ny - 1) * nx + i] * p->dy) + 0.25;
  }
  // D1 (Eqs. MSE_d_mtx1, elem_mtx_M, Gamma_ij_com2), multiplied by V
  std::vector<HostLevel> hl(1);
  hl[0].nx = nx; hl[0].ny = ny;
  hl[0].diag.assign(N, 0.0); hl[0].ax.assign(N, 0.0); hl[0].ay.assign(N, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      double d = P.V * sa[c];
      if (i + 1 < nx) {
        const double a = p->dy * 2.0 / (3.0 * (st_[c] * p->dx + st_[c + 1] * p->dx));
        hl[0].ax[c] = a;
      }
      if (j + 1 < ny) {
        const double a = p->dx * 2.0 / (3.0 * (st_[c] * p->dy + st_[c + nx] * p->dy));
        hl[0].ay[c] = a;
      }
      if (i + 1 < nx) d += hl[0].ax[c]; else d += p->dy * kap[ny + j];
      if (i > 0) d += hl[0].ax[c - 1]; else d += p->dy * kap[j];
      if (j + 1 < ny) d += hl[0].ay[c]; else d += p->dx * kap[2 * ny + nx + i];
      if (j > 0) d += hl[0].ay[c - nx]; else d += p->dx * kap[2 * ny + i];
      hl[0].diag[c] = d + P.V * P.tdiag;   // 1/(c dt) of Eq. elem_mtx_M (td form)
    }
  // -- pseudo-time shift of the increment-solve diagonal (Eqs. cfl_pse,
  // tau_pse, elem_main_shifted); |sigma_i r^L - sigma_j r^R| is
  // (sigma_i h + sigma_j h) / 2 for the face-normal width h
  std::vector<double> shift(N, 0.0);
  {
    const double dref = std::min(p->dx, p->dy);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int c = j * nx + i;
        double sh = o->cfl_p > 0 ? 1.0 / (o->cfl_p * dref) : 0.0;
        if (o->beta > 0) {
          double m = 0.0;
          if (i > 0) m = std::max(m, 0.5 * (st_[c] + st_[c - 1]) * p->dx);
          if (i + 1 < nx) m = std::max(m, 0.5 * (st_[c] + st_[c + 1]) * p->dx);
          if (j > 0) m = std::max(m, 0.5 * (st_[c] + st_[c - nx]) * p->dy);
          if (j + 1 < ny) m = std::max(m, 0.5 * (st_[c] + st_[c + nx]) * p->dy);
          sh += m / (o->beta * dref);
        }
        shift[c] = sh;
      }
  }

  // -- per-quadrant coefficient records in each quadrant's mirrored frame
  //    (cE, cW, cN, cS, sigma_t, sigma_t + pseudo-time shift)
  std::vector<double> cellq((size_t)4 * N * 6, 0.0), sdq((size_t)4 * N, 0.0);
  for (int qd = 0; qd < 4; ++qd)
    for (int yl = 0; yl < ny; ++yl)
      for (int xl = 0; xl < nx; ++xl) {
        const int i = (qd & 1) ? nx - 1 - xl : xl, j = (qd & 2) ? ny - 1 - yl : yl;
        const int c = j * nx + i;
        double *r = &cellq[((size_t)qd * N + dg_idx(xl, yl, nx, ny)) * 6];
        r[0] = (qd & 1) ? cW[c] : cE[c];
        r[1] = (qd & 1) ? cE[c] : cW[c];
        r[2] = (qd & 2) ? cS[c] : cN[c];
        r[3] = (qd & 2) ? cN[c] : cS[c];
        // the time-dependent form's 1/(c dt) joins sigma_t in the residual's
        // -sigma_t I term and in the increment solve's diagonal (Eqs.
        // RTE_d_res, elem_mtx)
        r[4] = st_[c] + P.tdiag;
        r[5] = st_[c] + P.tdiag + shift[c];
        sdq[(size_t)qd * N + dg_idx(xl, yl, nx, ny)] = r[5];
      }
  {
    // transport step: 0 residual kernel + recurrence, 3 pipelined (one
    // launch); 1 two-kernel reference and 2 fused wavefront sweep (tests
    // compare them); GSIS_SWEEP_REFERENCE=0..3 picks one. By default the
    // pipelined step runs FP64 problems of at least 2^26 cell-ordinates,
    // where enough rows run at once to hide its longer step (1024 x 1024 x
    // 128: 1.46 against 1.74 ms); on smaller grids the wavefront's length
    // decides and the split step is faster (256 x 256 x 128: 0.20 against
    // 0.13 ms), as it is in FP32-mixed form.
    const char *e = getenv("GSIS_SWEEP_REFERENCE");
    if (e && e[0] >= '0' && e[0] <= '3' && e[1] == 0)
      P.sweep_impl = e[0] - '0';
    else
      P.sweep_impl = (!f32 && (long long)N * K >= (1LL << 26)) ? 3 : 0;
    // the time terms live in the residual kernels of the split and
    // pipelined steps only
    if (P.td && P.sweep_impl != 3) P.sweep_impl = 0;
  }
  {
    // pipelined step: bands of 64 rows per workgroup (GSIS_PIPE_BANDS=1, 2
    // or 4 sets it), parts to cover the rows
    int nb = 2;
    const char *e = getenv("GSIS_PIPE_BANDS");
    if (e && (e[0] == '1' || e[0] == '2' || e[0] == '4') && e[1] == 0) nb = e[0] - '0';
    P.pipe_bands = nb;
    P.pipe_parts = P.sweep_impl == 3 ? (ny + 64 * nb - 1) / (64 * nb) : 1;
  }
  {
    // workgroups per ordinate in the recurrence (GSIS_CHAIN_PARTS=1..4 sets
    // it): a step costs a wave about the same whatever the rest of the chip
    // does, but waves sharing a SIMD take turns, so parts of about 256 rows
    // (one wave per SIMD); more parts while the ordinates fill fewer than
    // half the CUs; at most 4, each a multiple of 64 rows and at most 1024,
    // the top part not empty
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
        hipSuccess)
      cus = 0;
    int parts = std::min((ny + 255) / 256, 4);
    while (parts < 4 && 2 * K * parts < cus) parts *= 2;
    const char *e = getenv("GSIS_CHAIN_PARTS");
    if (e && e[0] >= '1' && e[0] <= '4' && e[1] == 0) parts = e[0] - '0';
    parts = std::max(1, std::min(parts, 4));
    int rows = 0;
    for (; parts > 1; --parts) {
      rows = ((ny + parts - 1) / parts + 63) / 64 * 64;
      if (rows <= 1024 && (parts - 1) * rows < ny) break;
    }
    if (P.sweep_impl == 1 || P.sweep_impl == 2) parts = 1;
    P.chain_parts = parts;
    P.chain_rows = parts > 1 ? rows : 0;
  }
  // residual tiles (GSIS_RESID_DIAGONALS=31 or 47 sets their length)
  P.resid_rd = residual_tile_diagonals((long long)N * K);
  {
    const char *e = getenv("GSIS_RESID_DIAGONALS");
    if (e && (!strcmp(e, "31") || !strcmp(e, "47"))) P.resid_rd = atoi(e);
  }
  const std::vector<int2> rtiles = residual_tiles(nx, ny, P.resid_rd);
  P.n_rtiles = (int)rtiles.size();
  // partial sums of w r^2: one per residual wave
  P.n_tres = P.sweep_impl == 3 ? K * P.pipe_parts * P.pipe_bands
                               : P.n_rtiles * residual_pairs(P);

  // -- boundary intensities in the internal ordinate order
  std::vector<double> bnd_int((size_t)P.nbf * K);
  for (int f = 0; f < P.nbf; ++f)
    for (int kk = 0; kk < K; ++kk) bnd_int[(size_t)f * K + kk] = bnd[(size_t)f * K + pl->perm[kk]];

  // -- warm start
  std::vector<double> phi0(N, 0.0);
  if (o->I0) {
    std::vector<double> I0;
    if ((st = fetch(ctx, o->I0, (size_t)N * K, o->device_ptrs, I0, "I0"))) return bail(st);
    pl->I0_host.assign((size_t)N * K, 0.0);
    for (int kk = 0; kk < K; ++kk) {
      const int k = pl->perm[kk];
      const int qd = (mu[k] < 0 ? 1 : 0) | (eta[k] < 0 ? 2 : 0);
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const int xl = (qd & 1) ? nx - 1 - i : i, yl = (qd & 2) ? ny - 1 - j : j;
          pl->I0_host[(size_t)kk * N + dg_idx(xl, yl, nx, ny)] = I0[(size_t)(j * nx + i) * K + k];
        }
    }
    for (int c = 0; c < N; ++c) {
      double s = 0;
      for (int k = 0; k < K; ++k) s += w[k] * I0[(size_t)c * K + k];
      phi0[c] = s;
    }
    if (f32) {
      // stored deviation from phi0/(4 pi); the first read adds base = phi0
      pl->I0_host_f.resize((size_t)N * K);
      for (int kk = 0; kk < K; ++kk) {
        const int k = pl->perm[kk];
        const int qd = (mu[k] < 0 ? 1 : 0) | (eta[k] < 0 ? 2 : 0);
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            const int xl = (qd & 1) ? nx - 1 - i : i, yl = (qd & 2) ? ny - 1 - j : j;
            const int c = j * nx + i;
            pl->I0_host_f[(size_t)kk * N + dg_idx(xl, yl, nx, ny)] =
                (float)(I0[(size_t)c * K + k] - phi0[c] / kFourPi);
          }
      }
      pl->I0_host.clear();
    }
  }
  pl->phi0_host = phi0;

  // -- device allocations and uploads
  if ((st = upload(pl, &P.amu, amu)) || (st = upload(pl, &P.aeta, aeta)) ||
      (st = upload(pl, &P.w, wv)) || (st = upload(pl, &P.wmu, wmu)) ||
      (st = upload(pl, &P.weta, weta)) || (st = alloc_intensity(pl, 0, (size_t)N * K, f32)) ||
      (st = alloc_intensity(pl, 1, (size_t)N * K, f32)) ||
      (st = dalloc(pl, &P.R, P.sweep_impl == 1 ? (size_t)N * K : 1)) ||
      (st = upload(pl, &P.cellq, cellq)) || (st = dalloc(pl, &P.dynq, (size_t)4 * N * 3)) ||
      (st = dalloc(pl, &P.rowbuf, (size_t)K * 3 * nx)) || (st = upload(pl, &P.sdq, sdq)) ||
      (st = upload(pl, &P.rtiles, rtiles)) || (st = upload(pl, &P.dso, diag_row0_table(nx, ny))) ||
      (st = upload(pl, &P.sig_t, st_)) || (st = upload(pl, &P.sig_a, sa)) ||
      (st = upload(pl, &P.sig_s, ss)) || (st = upload(pl, &P.q, q)) ||
      (st = upload(pl, &P.cE, cE)) || (st = upload(pl, &P.cW, cW)) ||
      (st = upload(pl, &P.cN, cN)) || (st = upload(pl, &P.cS, cS)) ||
      (st = dalloc(pl, &P.src, N)) || (st = dalloc(pl, &P.phi, N)) ||
      (st = dalloc(pl, &P.phih, N)) || (st = dalloc(pl, &P.Fx, N)) ||
      (st = dalloc(pl, &P.mom_part, (size_t)12 * N)) ||
      (st = dalloc(pl, &P.Fy, N)) || (st = dalloc(pl, &P.delta, N)) ||
      (st = dalloc(pl, &P.hx, N)) || (st = dalloc(pl, &P.hy, N)) ||
      (st = dalloc(pl, &P.rhs, N)) || (st = upload(pl, &P.bnd, bnd_int)) ||
      (st = dalloc(pl, &P.bflux, P.nbf)) || (st = upload(pl, &P.kappa, kap)) ||
      (st = dalloc(pl, &P.err_hist, o->max_iter)) ||
      (st = dalloc(pl, &P.tres_hist, o->max_iter)) ||
      (st = dalloc(pl, &P.tres_part, tres_slots(P))) ||
      (st = dalloc(pl, &P.src2_part, (size_t)(N + 255) / 256)) ||
      (st = dalloc(pl, &P.state, 5)) || (st = dalloc(pl, &P.last_err, 2)))
    return bail(st);
  if (std::max(P.chain_parts, P.pipe_parts) > 1 &&
      (st = dalloc(pl, &P.hand, (size_t)K * (std::max(P.chain_parts, P.pipe_parts) - 1) * nx)))
    return bail(st);
  if (f32) {
    std::vector<float> sdqf(sdq.begin(), sdq.end());
    if ((st = upload(pl, &P.sdq_f, sdqf))) return bail(st);
    // w, w mu, w eta in FP32 for the moment sums of the deviations
    std::vector<float> wf(3 * (size_t)K);
    for (int kk = 0; kk < K; ++kk) {
      wf[kk] = (float)wv[kk];
      wf[K + kk] = (float)wmu[kk];
      wf[2 * K + kk] = (float)weta[kk];
    }
    if ((st = upload(pl, &P.w_f, wf))) return bail(st);
  }
  if (P.method == GSIS_GSIS && P.hot_face == GSIS_HOT_TRANSPORT &&
      (st = dalloc(pl, &P.ftp, (size_t)8 * N)))
    return bail(st);
  if (P.td &&
      ((st = upload(pl, &P.cv, cvh)) || (st = dalloc(pl, &P.Tm, N)) || (st = dalloc(pl, &P.Tn, N)) ||
       (st = dalloc(pl, &P.Tsub0, N)) || (st = dalloc(pl, &P.Tsub1, N)) ||
       (st = dalloc(pl, &P.rho_n, N)) ||
       (st = dalloc(pl, &P.err_parts_T, 2 * (size_t)((N + 255) / 256) + 2)) ||
       (st = dalloc(pl, &P.In, (size_t)N * K))))
    return bail(st);
  if (f32) {
    if ((st = dalloc(pl, &P.base, N))) return bail(st);
  } else {
    P.base = P.delta;
  }
  if ((st = dalloc(pl, &P.err_parts, 2 * (size_t)((N + 255) / 256) + 2)) ||
      (st = setup_synth(pl, P, hl)))
    return bail(st);
  if (P.mg.size() > (size_t)kMaxLevels)
    return bail(fail(ctx, GSIS_E_INVALID_ARG, "multigrid hierarchy deeper than %d levels",
                     kMaxLevels));
  if ((st = make_single_set(pl))) return bail(st);
  if (arena) {
    // pageable host flags: the synthetic solve's copies of them are followed
    // by a stream synchronisation either way
    pl->host_scal = pl->host_flag_store;
  } else {
    // flags read back by the synthetic solve: [0, 3) state and [8] the CG
    // count of the last forward solve; [4, 7) and [12] the same for the
    // adjoint's solves
    void *h = nullptr;
    hipError_t e = hipHostMalloc(&h, 64, hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail(ctx, GSIS_E_OOM, "hipHostMalloc: %s", hipGetErrorString(e)));
    memset(h, 0, 64);
    pl->host_scal = (double *)h;
    if ((e = hipEventCreateWithFlags(&pl->spec_ev, hipEventDisableTiming)) != hipSuccess) {
      pl->spec_ev = nullptr;
      return bail(fail(ctx, GSIS_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e)));
    }
  }
  if ((st = gsis_plan_reset(pl))) return bail(st);
  *out = pl;
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_create(gsis_ctx *ctx, const gsis_problem *p,
                                        const gsis_options *o, gsis_plan **out) {
  return plan_create(ctx, p, o, out, nullptr, 0);
}

extern "C" void gsis_plan_destroy(gsis_plan *pl) {
  if (!pl) return;
  if (pl->stream) (void)hipStreamSynchronize(pl->stream);
  else (void)hipDeviceSynchronize();
  for (void *v : pl->allocs) (void)hipFree(v);
  for (hipEvent_t e : pl->events) (void)hipEventDestroy(e);
  if (pl->spec_ev) (void)hipEventDestroy(pl->spec_ev);
  adjoint_release(pl);
  if (pl->host_scal && !pl->arena) (void)hipHostFree(pl->host_scal);
  delete pl;
}

extern "C" gsis_status gsis_plan_reset(gsis_plan *pl) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  PlanDev &P = pl->P;
  const size_t NK = (size_t)P.N * P.K;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = pl->stream;
  const bool f32 = P.precision == GSIS_FP32_MIXED;
  if (f32 && !pl->I0_host_f.empty())
    HIPCHK(ctx, hipMemcpyAsync(P.I[0], pl->I0_host_f.data(), NK * sizeof(float),
                               hipMemcpyHostToDevice, s));
  else if (!f32 && !pl->I0_host.empty())
    HIPCHK(ctx, hipMemcpyAsync(P.I[0], pl->I0_host.data(), NK * sizeof(double),
                               hipMemcpyHostToDevice, s));
  else
    HIPCHK(ctx, hipMemsetAsync(P.I[0], 0, NK * (f32 ? sizeof(float) : sizeof(double)), s));
  HIPCHK(ctx, hipMemcpyAsync(P.phi, pl->phi0_host.data(), P.N * sizeof(double),
                             hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemsetAsync(P.delta, 0, P.N * sizeof(double), s));
  if (f32)   // I^0 = Itilde + phi0/(4 pi)
    HIPCHK(ctx, hipMemcpyAsync(P.base, pl->phi0_host.data(), P.N * sizeof(double),
                               hipMemcpyHostToDevice, s));
  if (P.td)   // T^0 (the source kernel below takes the emission of T^m)
    HIPCHK(ctx, hipMemcpyAsync(P.Tm, pl->T0_host.data(), P.N * sizeof(double),
                               hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemsetAsync(P.state, 0, 5 * sizeof(int32_t), s));
  launch_hand_reset(P, s);
  HIPCHK(ctx, hipMemsetAsync(P.err_hist, 0, P.max_iter * sizeof(double), s));
  HIPCHK(ctx, hipMemsetAsync(P.tres_hist, 0, P.max_iter * sizeof(double), s));
  HIPCHK(ctx, hipMemsetAsync(P.tres_part, 0, tres_slots(P) * sizeof(double), s));
  HIPCHK(ctx, hipMemsetAsync(synth_vcycle_total(P), 0, sizeof(double), s));
  {
    // Err of the last iteration and the smallest ||phi^{m+1} - phi^m||_V so
    // far (divergence test)
    static const double init[2] = {0.0, INFINITY};
    HIPCHK(ctx, hipMemcpyAsync(P.last_err, init, sizeof init, hipMemcpyHostToDevice, s));
  }
  launch_source(P.S, s);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipStreamSynchronize(s));
  pl->prof_iters = 0;
  return GSIS_OK;
}

static gsis_status record(gsis_plan *pl, int slot) {
  if (!pl->profile) return GSIS_OK;
  const size_t idx = (size_t)pl->prof_iters * (GSIS_NUM_PHASES + 1) + slot;
  while (pl->events.size() <= idx) {
    hipEvent_t e;
    HIPCHK(pl->ctx, hipEventCreate(&e));
    pl->events.push_back(e);
  }
  HIPCHK(pl->ctx, hipEventRecord(pl->events[idx], pl->stream));
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_iterate(gsis_plan *pl, int32_t n) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  if (n < 0) return fail(ctx, GSIS_E_INVALID_ARG, "n must be >= 0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  PlanDev &P = pl->P;
  hipStream_t s = pl->stream;
  gsis_status st;
  for (int it = 0; it < n; ++it) {
    if (pl->profile && pl->prof_iters >= 100000) pl->profile = 0;
    if ((st = record(pl, 0))) return st;
    launch_residual(P, s);
    if ((st = record(pl, 1))) return st;
    launch_sweep(P, s);
    if ((st = record(pl, 2))) return st;
    launch_moments(P, s, P.method == GSIS_GSIS);
    if ((st = record(pl, 3))) return st;
    if (P.method == GSIS_GSIS) {
      launch_hot(P.S, s, true);
    }
    if ((st = record(pl, 4))) return st;
    // the synthetic solve copies the device flags to the host once while it
    // runs (host_flag[0]: the outer iteration's done flag); cleared first,
    // so a nonzero value below was read during this iteration
    int32_t *host_flag = (int32_t *)pl->host_scal;
    host_flag[0] = 0;
    bool updated = false;
    if (P.td) {
      // time-dependent form: sub-iterations of the material equation and
      // (GSIS) the synthetic equation, each from the previous sub-iterate
      for (int sub = 0; sub < P.sub_iter; ++sub) {
        launch_material(P.S, s, sub);
        if (P.method == GSIS_GSIS) {
          launch_synth_solve(P.S, s, host_flag, sub == 0 ? 1 : 3, sub);
          if (host_flag[0] != 0) break;
        }
      }
    } else if (P.method == GSIS_GSIS && P.synth_form == 1) {
      // face-averaged balance: sub-iterations from phi^{m+1/2}
      for (int sub = 0; sub < P.synth_sub; ++sub) {
        launch_wide_grad(P.S, s, sub == 0);
        launch_synth_solve(P.S, s, host_flag, 2);
        if (host_flag[0] != 0) break;
      }
    } else if (P.method == GSIS_GSIS) {
      // (the phase-timed pass keeps the update after the wait)
      updated = launch_synth_solve(P.S, s, host_flag, 1, 0, pl->profile ? nullptr : pl->spec_ev);
    }
    if ((st = record(pl, 5))) return st;
    if (!updated) launch_update(P.S, s);
    if ((st = record(pl, 6))) return st;
    HIPCHK(ctx, hipGetLastError());
    if (pl->profile) pl->prof_iters++;
    // an earlier iteration ended the solve (converged, diverged or at the
    // iteration cap): the remaining ones would only launch kernels that exit
    if (host_flag[0] != 0) break;
  }
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_status(gsis_plan *pl, int32_t *n_iter, int32_t *converged,
                                        double *last_err) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int32_t stv[5];
  double le = 0;
  HIPCHK(ctx, hipMemcpyAsync(stv, pl->P.state, sizeof stv, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(ctx, hipMemcpyAsync(&le, pl->P.last_err, sizeof le, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(ctx, hipStreamSynchronize(pl->stream));
  if (stv[4] != 0)
    return fail(ctx, GSIS_E_DEVICE,
                "the recurrence's workgroups of one ordinate stopped waiting for each other; "
                "reset the plan");
  if (n_iter) *n_iter = stv[0];
  if (converged) *converged = stv[1] == 1 ? 1 : (stv[1] == -1 ? -1 : 0);
  if (last_err) *last_err = le;
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_read(gsis_plan *pl, gsis_result *r) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  if (!r) return fail(ctx, GSIS_E_INVALID_ARG, "result is NULL");
  if (!r->phi || !r->Fx || !r->Fy) return fail(ctx, GSIS_E_INVALID_ARG, "result.phi/Fx/Fy is NULL");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  PlanDev &P = pl->P;
  hipStream_t s = pl->stream;
  int32_t n_iter = 0, conv = 0;
  double le = 0;
  gsis_status st = gsis_plan_status(pl, &n_iter, &conv, &le);
  if (st) return st;
  const size_t bytes = P.N * sizeof(double);
  // F of the final iterate: F_half plus the pending correction's flux (hx, hy
  // are free here and serve as staging).
  launch_apply_delta_final(P, s, pl->swmu, pl->sweta, P.hx, P.hy);
  HIPCHK(ctx, hipGetLastError());
  const hipMemcpyKind k = pl->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(ctx, hipMemcpyAsync(r->phi, P.phi, bytes, k, s));
  HIPCHK(ctx, hipMemcpyAsync(r->Fx, P.hx, bytes, k, s));
  HIPCHK(ctx, hipMemcpyAsync(r->Fy, P.hy, bytes, k, s));
  if (r->err_hist && n_iter > 0)
    HIPCHK(ctx, hipMemcpyAsync(r->err_hist, P.err_hist, n_iter * sizeof(double), k, s));
  if (r->tres_hist && n_iter > 0)
    HIPCHK(ctx, hipMemcpyAsync(r->tres_hist, P.tres_hist, n_iter * sizeof(double), k, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  r->n_iter = n_iter;
  r->final_err = n_iter > 0 ? le : INFINITY;
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_transport_form(gsis_plan *pl, int32_t *form, int32_t *bands,
                                                int32_t *parts) {
  if (!pl) return GSIS_E_INVALID_ARG;
  if (!form) return fail(pl->ctx, GSIS_E_INVALID_ARG, "form is NULL");
  const PlanDev &P = pl->P;
  *form = P.sweep_impl;
  if (bands) *bands = P.sweep_impl == 3 ? P.pipe_bands : 0;
  if (parts) *parts = P.sweep_impl == 3 ? P.pipe_parts : P.chain_parts;
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_synth_vcycles(gsis_plan *pl, int64_t *vcycles) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  if (!vcycles) return fail(ctx, GSIS_E_INVALID_ARG, "vcycles is NULL");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double v = 0;
  HIPCHK(ctx, hipMemcpyAsync(&v, synth_vcycle_total(pl->P), sizeof v, hipMemcpyDeviceToHost,
                             pl->stream));
  HIPCHK(ctx, hipStreamSynchronize(pl->stream));
  *vcycles = (int64_t)v;
  return GSIS_OK;
}

extern "C" gsis_status gsis_plan_phase_times(gsis_plan *pl, double *ms, int32_t *n_iter) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  if (!ms) return fail(ctx, GSIS_E_INVALID_ARG, "ms is NULL");
  HIPCHK(ctx, hipStreamSynchronize(pl->stream));
  for (int ph = 0; ph < GSIS_NUM_PHASES; ++ph) ms[ph] = 0;
  for (int it = 0; it < pl->prof_iters; ++it)
    for (int ph = 0; ph < GSIS_NUM_PHASES; ++ph) {
      float t = 0;
      const size_t e0 = (size_t)it * (GSIS_NUM_PHASES + 1) + ph;
      HIPCHK(ctx, hipEventElapsedTime(&t, pl->events[e0], pl->events[e0 + 1]));
      ms[ph] += t;
    }
  if (n_iter) *n_iter = pl->prof_iters;
  pl->prof_iters = 0;
  return GSIS_OK;
}

// Plan, iterate until Err < tol, divergence or max_iter, read, destroy.
static gsis_status solve_with(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                              gsis_result *r, char *arena, size_t arena_cap) {
  if (!ctx) return fail(nullptr, GSIS_E_INVALID_ARG, "ctx is NULL");
  if (!r) return fail(ctx, GSIS_E_INVALID_ARG, "result is NULL");
  gsis_plan *pl = nullptr;
  gsis_status st = plan_create(ctx, p, o, &pl, arena, arena_cap);
  if (st) return st;
  int32_t n = 0, conv = 0;
  double le = 0;
  const int chunk = 8;
  while (true) {
    const int todo = std::min(chunk, o->max_iter - n);
    if ((st = gsis_plan_iterate(pl, todo))) break;
    if ((st = gsis_plan_status(pl, &n, &conv, &le))) break;
    if (conv != 0 || n >= o->max_iter) break;
  }
  if (st == GSIS_OK) st = gsis_plan_read(pl, r);
  gsis_plan_destroy(pl);
  if (st) return st;
  if (conv == -1) return GSIS_DIVERGED;
  if (conv == 0) return GSIS_NOT_CONVERGED;
  return GSIS_OK;
}

extern "C" gsis_status gsis_solve(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                                  gsis_result *r) {
  return solve_with(ctx, p, o, r, nullptr, 0);
}

// ------------------------------------------------------ solve without allocation
// The device state of gsis_solve_noalloc lives in this file-scope array (one
// copy per GPU, held until the process ends). In host code its name only
// stands in for the symbol: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this device's scratch copy (the context's device is
// current).
gsis_status scratch_address(gsis_ctx *ctx, char **out) {
  if (ctx->device < 0 || ctx->device >= kMaxScratchDevices)
    return fail(ctx, GSIS_E_UNSUPPORTED, "gsis_solve_noalloc: device %d beyond %d", ctx->device,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(ctx, GSIS_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[ctx->device] = ptr;
  }
  *out = (char *)g_scratch_ptr[ctx->device];
  return GSIS_OK;
}
}  // namespace

extern "C" gsis_status gsis_solve_noalloc(gsis_ctx *ctx, const gsis_problem *p,
                                          const gsis_options *o, gsis_result *r) {
  if (!ctx) return fail(nullptr, GSIS_E_INVALID_ARG, "ctx is NULL");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  char *base = nullptr;
  gsis_status st = scratch_address(ctx, &base);
  if (st) return st;
  return solve_with(ctx, p, o, r, base, kScratchBytes);
}

// ------------------------------------------------------- time-dependent form
extern "C" gsis_status gsis_td_create(gsis_ctx *ctx, const gsis_problem *p, const gsis_options *o,
                                      const gsis_material *mt, gsis_plan **out) {
  if (!mt) return fail(ctx, GSIS_E_INVALID_ARG, "material is NULL");
  return plan_create(ctx, p, o, out, nullptr, 0, mt);
}

extern "C" gsis_status gsis_td_advance(gsis_plan *pl, int32_t n_steps, int32_t *inner_iters,
                                       double *last_err) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  if (!pl->P.td) return fail(ctx, GSIS_E_INVALID_ARG, "not a time-dependent plan");
  if (n_steps < 0) return fail(ctx, GSIS_E_INVALID_ARG, "n_steps must be >= 0");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  gsis_status worst = GSIS_OK;
  for (int step = 0; step < n_steps; ++step) {
    launch_td_begin(pl->P, pl->stream);
    HIPCHK(ctx, hipGetLastError());
    int32_t n = 0, conv = 0;
    double le = 0;
    gsis_status st;
    while (true) {
      if ((st = gsis_plan_iterate(pl, std::min(8, pl->P.max_iter - n)))) return st;
      if ((st = gsis_plan_status(pl, &n, &conv, &le))) return st;
      if (conv != 0 || n >= pl->P.max_iter) break;
    }
    if (inner_iters) inner_iters[step] = n;
    if (last_err) last_err[step] = le;
    if (conv == -1) return GSIS_DIVERGED;
    if (conv == 0) worst = GSIS_NOT_CONVERGED;
  }
  return worst;
}

extern "C" gsis_status gsis_td_read(gsis_plan *pl, double *rho, double *T, double *Fx,
                                    double *Fy) {
  if (!pl) return GSIS_E_INVALID_ARG;
  gsis_ctx *ctx = pl->ctx;
  if (!pl->P.td) return fail(ctx, GSIS_E_INVALID_ARG, "not a time-dependent plan");
  if (!rho || !T || !Fx || !Fy) return fail(ctx, GSIS_E_INVALID_ARG, "an output is NULL");
  gsis_result r;
  std::memset(&r, 0, sizeof r);
  r.phi = rho; r.Fx = Fx; r.Fy = Fy;
  gsis_status st = gsis_plan_read(pl, &r);
  if (st) return st;
  const hipMemcpyKind k = pl->device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(ctx, hipMemcpyAsync(T, pl->P.Tm, pl->P.N * sizeof(double), k, pl->stream));
  HIPCHK(ctx, hipStreamSynchronize(pl->stream));
  return GSIS_OK;
}
