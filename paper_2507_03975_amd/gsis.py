"""ctypes binding of libgsis.so (the C-ABI declared in include/gsis.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels. Arrays may be numpy arrays (host memory) or torch CUDA tensors
(device memory; the plan then runs on torch's current stream). If the library
has not been built, every call raises ``GSISError``: there is no CPU
fallback.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsis.so")
_lib = None

GSIS_OK, GSIS_NOT_CONVERGED, GSIS_DIVERGED = 0, 1, 2
GSIS_E_INVALID_ARG, GSIS_E_DEVICE, GSIS_E_OOM, GSIS_E_UNSUPPORTED = -1, -2, -3, -4
GSIS_SI, GSIS_GSIS = 0, 1
GSIS_FP64, GSIS_FP32_MIXED = 0, 1
GSIS_HOT_CENTRAL, GSIS_HOT_TRANSPORT = 0, 1
GSIS_NUM_PHASES = 6
PHASES = ("residual", "sweep", "moments", "hot", "synth", "update")

_dp = ctypes.POINTER(ctypes.c_double)


class GSISError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("gsis status %d: %s" % (status, msg))
        self.status = status


class gsis_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("K", ctypes.c_int32),
                ("mu", ctypes.c_void_p), ("eta", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("sigma_a", ctypes.c_void_p), ("sigma_s", ctypes.c_void_p),
                ("q", ctypes.c_void_p), ("bnd_in", ctypes.c_void_p)]


class gsis_options(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("order", ctypes.c_int32), ("limiter", ctypes.c_int32),
                ("alsm", ctypes.c_int32), ("hot_face", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("synth_rtol", ctypes.c_double), ("synth_max_iter", ctypes.c_int32),
                ("I0", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("device_ptrs", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("cfl_p", ctypes.c_double), ("beta", ctypes.c_double),
                ("graph", ctypes.c_int32), ("synth_form", ctypes.c_int32),
                ("synth_sub", ctypes.c_int32)]


class gsis_batch_tuning(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("n_configs", ctypes.c_int32), ("config_rows", ctypes.c_int32 * 8),
                ("config_prefetch", ctypes.c_int32 * 8), ("config_ms", ctypes.c_double * 8)]


class gsis_adjoint_info(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int32), ("final_err", ctypes.c_double),
                ("forward_iter", ctypes.c_int32)]


class gsis_material(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("a", ctypes.c_double), ("dt", ctypes.c_double),
                ("cv", ctypes.c_void_p), ("T0", ctypes.c_void_p), ("sub_iter", ctypes.c_int32)]


class gsis_result(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("Fx", ctypes.c_void_p), ("Fy", ctypes.c_void_p),
                ("err_hist", ctypes.c_void_p), ("tres_hist", ctypes.c_void_p),
                ("n_iter", ctypes.c_int32), ("final_err", ctypes.c_double)]


EXPORTS = ("gsis_ctx_create", "gsis_ctx_destroy", "gsis_last_error", "gsis_options_default",
           "gsis_solve", "gsis_plan_create", "gsis_plan_destroy", "gsis_plan_iterate",
           "gsis_plan_status", "gsis_plan_read", "gsis_plan_reset", "gsis_plan_phase_times",
           "gsis_batch_create", "gsis_batch_destroy", "gsis_batch_iterate", "gsis_batch_status",
           "gsis_batch_read", "gsis_batch_reset", "gsis_batch_get_tuning", "gsis_solve_batch",
           "gsis_plan_adjoint", "gsis_adjoint", "gsis_version", "gsis_solve_noalloc",
           "gsis_plan_synth_vcycles", "gsis_td_create", "gsis_td_advance", "gsis_td_read",
           "gsis_plan_transport_form")


def load():
    """Open libgsis.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GSISError(GSIS_E_DEVICE, "libgsis.so is not built (run paper_2507_03975_amd.build)")
    try:
        import torch  # noqa: F401  (loads the HIP runtime torch uses)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, i32 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32
    lib.gsis_ctx_create.argtypes = [i32, ctypes.POINTER(vp)]
    lib.gsis_ctx_destroy.argtypes = [vp]
    lib.gsis_ctx_destroy.restype = None
    lib.gsis_last_error.argtypes = [vp]
    lib.gsis_last_error.restype = ctypes.c_char_p
    lib.gsis_options_default.argtypes = [ctypes.POINTER(gsis_options)]
    lib.gsis_solve.argtypes = [vp, ctypes.POINTER(gsis_problem), ctypes.POINTER(gsis_options),
                               ctypes.POINTER(gsis_result)]
    lib.gsis_solve_noalloc.argtypes = lib.gsis_solve.argtypes
    lib.gsis_plan_create.argtypes = [vp, ctypes.POINTER(gsis_problem),
                                     ctypes.POINTER(gsis_options), ctypes.POINTER(vp)]
    lib.gsis_plan_destroy.argtypes = [vp]
    lib.gsis_plan_destroy.restype = None
    lib.gsis_plan_iterate.argtypes = [vp, i32]
    lib.gsis_plan_status.argtypes = [vp, ip, ip, _dp]
    lib.gsis_plan_read.argtypes = [vp, ctypes.POINTER(gsis_result)]
    lib.gsis_plan_reset.argtypes = [vp]
    lib.gsis_plan_phase_times.argtypes = [vp, _dp, ip]
    lib.gsis_plan_synth_vcycles.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.gsis_plan_transport_form.argtypes = [vp, ip, ip, ip]
    lib.gsis_batch_create.argtypes = [vp, i32, ctypes.POINTER(gsis_problem),
                                      ctypes.POINTER(gsis_options), ctypes.POINTER(vp)]
    lib.gsis_batch_destroy.argtypes = [vp]
    lib.gsis_batch_destroy.restype = None
    lib.gsis_batch_iterate.argtypes = [vp, i32]
    lib.gsis_batch_status.argtypes = [vp, ip, ip, _dp, ip]
    lib.gsis_batch_read.argtypes = [vp, i32, ctypes.POINTER(gsis_result)]
    lib.gsis_batch_reset.argtypes = [vp]
    lib.gsis_batch_get_tuning.argtypes = [vp, ctypes.POINTER(gsis_batch_tuning)]
    lib.gsis_solve_batch.argtypes = [vp, i32, ctypes.POINTER(gsis_problem),
                                     ctypes.POINTER(gsis_options), ctypes.POINTER(gsis_result)]
    lib.gsis_plan_adjoint.argtypes = [vp, vp, vp, vp, ctypes.c_double, i32, vp, vp, vp,
                                      ctypes.POINTER(gsis_adjoint_info)]
    lib.gsis_adjoint.argtypes = [vp, ctypes.POINTER(gsis_problem), ctypes.POINTER(gsis_options),
                                 vp, vp, vp, vp, vp, vp, ctypes.POINTER(gsis_result),
                                 ctypes.POINTER(gsis_adjoint_info)]
    lib.gsis_td_create.argtypes = [vp, ctypes.POINTER(gsis_problem), ctypes.POINTER(gsis_options),
                                   ctypes.POINTER(gsis_material), ctypes.POINTER(vp)]
    lib.gsis_td_advance.argtypes = [vp, i32, ip, _dp]
    lib.gsis_td_read.argtypes = [vp, vp, vp, vp, vp]
    lib.gsis_version.argtypes = []
    lib.gsis_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("gsis_ctx_destroy", "gsis_plan_destroy", "gsis_batch_destroy",
                        "gsis_last_error", "gsis_version"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def gsis_version():
    return load().gsis_version().decode()


def gsis_last_error(ctx=None):
    return load().gsis_last_error(ctx.handle if ctx is not None else None).decode()


def _check(st, ctx=None, allow=(GSIS_OK,)):
    if st not in allow:
        raise GSISError(st, gsis_last_error(ctx))
    return st


class Context:
    """gsis_ctx_create / gsis_ctx_destroy."""

    def __init__(self, device=0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.gsis_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load().gsis_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Args:
    """Pointers for one call; keeps host copies alive."""

    def __init__(self, prob, I0=None):
        keys = ("mu", "eta", "w", "sigma_a", "sigma_s", "q")
        vals = [prob[k] for k in keys]
        self.device = any(_is_torch(v) and v.is_cuda for v in vals)
        self.keep = []
        ptr = {}
        for k, v in zip(keys, vals):
            ptr[k] = self._ptr(v)
        b = prob.get("bnd_in")
        ptr["bnd_in"] = None if b is None else self._ptr(b)
        self.I0 = None if I0 is None else self._ptr(I0)
        K = int(len(prob["mu"]))
        self.nx, self.ny, self.K = int(prob["nx"]), int(prob["ny"]), K
        self.s = gsis_problem(self.nx, self.ny, float(prob["dx"]), float(prob["dy"]), K,
                              ptr["mu"], ptr["eta"], ptr["w"], ptr["sigma_a"],
                              ptr["sigma_s"], ptr["q"], ptr["bnd_in"])

    def _ptr(self, a):
        if _is_torch(a):
            import torch
            if a.is_cuda != self.device:
                raise ValueError("mix of host and device arrays")
            a = a.detach().to(torch.float64).contiguous()
            self.keep.append(a)
            return a.data_ptr()
        if self.device:
            raise ValueError("mix of host and device arrays")
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.keep.append(a)
        return a.ctypes.data


def make_options(method=GSIS_GSIS, precision=GSIS_FP64, order=2, limiter=1, alsm=1,
                 hot_face=GSIS_HOT_CENTRAL, tol=1e-6, max_iter=1000, synth_rtol=0.1,
                 synth_max_iter=50, profile=0, cfl_p=0.0, beta=0.0, graph=1, synth_form=0,
                 synth_sub=4):
    o = gsis_options()
    load().gsis_options_default(ctypes.byref(o))
    o.method, o.precision, o.order, o.limiter = int(method), int(precision), int(order), int(limiter)
    o.alsm, o.hot_face, o.tol, o.max_iter = int(alsm), int(hot_face), float(tol), int(max_iter)
    o.synth_rtol, o.synth_max_iter, o.profile = float(synth_rtol), int(synth_max_iter), int(profile)
    o.cfl_p, o.beta, o.graph = float(cfl_p), float(beta), int(graph)
    o.synth_form, o.synth_sub = int(synth_form), int(synth_sub)
    return o


def _stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """gsis_plan_create / iterate / status / read / reset / phase_times / destroy."""

    def __init__(self, ctx, prob, I0=None, **opts):
        lib = load()
        self.ctx = ctx
        self.args = _Args(prob, I0)
        o = make_options(**opts)
        o.I0 = self.args.I0
        o.device_ptrs = 1 if self.args.device else 0
        o.stream = _stream_handle() if self.args.device else None
        self.opts = o
        h = ctypes.c_void_p()
        _check(lib.gsis_plan_create(ctx.handle, ctypes.byref(self.args.s), ctypes.byref(o),
                                    ctypes.byref(h)), ctx)
        self.handle = h
        self.N = self.args.nx * self.args.ny

    def iterate(self, n):
        _check(load().gsis_plan_iterate(self.handle, int(n)), self.ctx)

    def status(self):
        n, c, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(load().gsis_plan_status(self.handle, ctypes.byref(n), ctypes.byref(c),
                                       ctypes.byref(e)), self.ctx)
        return n.value, c.value, e.value

    def reset(self):
        _check(load().gsis_plan_reset(self.handle), self.ctx)

    def read(self, out=None):
        """Return dict(phi, Fx, Fy, err_hist, n_iter, final_err); arrays are
        numpy (host plans) or torch tensors on the plan's device."""
        N, maxit = self.N, self.opts.max_iter
        (phi, fx, fy, hist, thist), r = _result_buffers(self.args, maxit)
        _check(load().gsis_plan_read(self.handle, ctypes.byref(r)), self.ctx)
        return dict(phi=phi, Fx=fx, Fy=fy, err_hist=hist[:r.n_iter], tres_hist=thist[:r.n_iter],
                    n_iter=r.n_iter, final_err=r.final_err)

    def synth_vcycles(self):
        """Multigrid V-cycles of all synthetic solves since creation or reset."""
        v = ctypes.c_int64()
        _check(load().gsis_plan_synth_vcycles(self.handle, ctypes.byref(v)), self.ctx)
        return v.value

    def transport_form(self):
        """(form, bands, parts) of the plan's transport step: form 0 split
        (residual launch, then the recurrence), 3 pipelined (one launch)."""
        f, b, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().gsis_plan_transport_form(self.handle, ctypes.byref(f), ctypes.byref(b),
                                               ctypes.byref(p)), self.ctx)
        return f.value, b.value, p.value

    def phase_times(self):
        ms = (ctypes.c_double * GSIS_NUM_PHASES)()
        n = ctypes.c_int32()
        _check(load().gsis_plan_phase_times(self.handle, ms, ctypes.byref(n)), self.ctx)
        return {k: ms[i] for i, k in enumerate(PHASES)}, n.value

    def adjoint(self, g_phi=None, g_Fx=None, g_Fy=None, tol=1e-10, max_iter=1000):
        """gsis_plan_adjoint on the converged plan: returns (dJ/dsigma_a,
        dJ/dsigma_s, dJ/dq, info dict) for J = <g_phi, phi> + <g_F, F>."""
        N = self.args.nx * self.args.ny
        keep = []

        def cot(g):
            if g is None:
                return None
            if self.args.device:
                import torch
                t = g.detach().to(torch.float64).contiguous()
                keep.append(t)
                return t.data_ptr()
            a = np.ascontiguousarray(g, dtype=np.float64).ravel()
            keep.append(a)
            return a.ctypes.data
        if self.args.device:
            import torch
            dev = self.args.keep[0].device
            outs = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(3)]
            ptr = lambda t: t.data_ptr()
        else:
            outs = [np.empty(N) for _ in range(3)]
            ptr = lambda a: a.ctypes.data
        info = gsis_adjoint_info()
        st = load().gsis_plan_adjoint(self.handle, cot(g_phi), cot(g_Fx), cot(g_Fy), float(tol),
                                      int(max_iter), ptr(outs[0]), ptr(outs[1]), ptr(outs[2]),
                                      ctypes.byref(info))
        _check(st, self.ctx, allow=(GSIS_OK, GSIS_NOT_CONVERGED))
        return outs[0], outs[1], outs[2], dict(n_iter=info.n_iter, final_err=info.final_err,
                                               forward_iter=info.forward_iter, status=st)

    def close(self):
        if getattr(self, "handle", None):
            load().gsis_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gsis_solve(ctx, prob, I0=None, noalloc=False, **opts):
    """One-shot solve (gsis_solve, or gsis_solve_noalloc with noalloc=True).
    Returns the result dict plus ``status``."""
    lib = load()
    entry = lib.gsis_solve_noalloc if noalloc else lib.gsis_solve
    a = _Args(prob, I0)
    o = make_options(**opts)
    o.I0 = a.I0
    o.device_ptrs = 1 if a.device else 0
    o.stream = _stream_handle() if a.device else None
    (phi, fx, fy, hist, thist), r = _result_buffers(a, o.max_iter)
    st = entry(ctx.handle, ctypes.byref(a.s), ctypes.byref(o), ctypes.byref(r))
    _check(st, ctx, allow=(GSIS_OK, GSIS_NOT_CONVERGED, GSIS_DIVERGED))
    return dict(phi=phi, Fx=fx, Fy=fy, err_hist=hist[:r.n_iter], tres_hist=thist[:r.n_iter],
                n_iter=r.n_iter, final_err=r.final_err, status=st)


_default_ctx = None


def solve(prob, I0=None, device=0, **opts):
    """Convenience: gsis_solve on a per-process default context."""
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(device)
    return gsis_solve(_default_ctx, prob, I0, **opts)


def _result_buffers(a, max_iter):
    """Output arrays of one problem (torch tensors on the problem's device, or
    numpy arrays) and the gsis_result pointing at them."""
    N = a.nx * a.ny
    if a.device:
        import torch
        dev = a.keep[0].device
        phi = torch.empty(N, dtype=torch.float64, device=dev)
        fx, fy = torch.empty_like(phi), torch.empty_like(phi)
        hist = torch.zeros(max_iter, dtype=torch.float64, device=dev)
        thist = torch.zeros_like(hist)
        p = lambda t: t.data_ptr()
    else:
        phi, fx, fy = np.empty(N), np.empty(N), np.empty(N)
        hist, thist = np.zeros(max_iter), np.zeros(max_iter)
        p = lambda x: x.ctypes.data
    return (phi, fx, fy, hist, thist), gsis_result(p(phi), p(fx), p(fy), p(hist), p(thist),
                                                   0, 0.0)


class Batch:
    """gsis_batch_create / iterate / status / read / reset / get_tuning /
    destroy for a list of problem dicts (all host arrays or all device
    tensors) sharing one set of options."""

    def __init__(self, ctx, probs, **opts):
        lib = load()
        self.ctx = ctx
        self.args = [_Args(p) for p in probs]
        dev = {a.device for a in self.args}
        if len(dev) != 1:
            raise ValueError("mix of host and device problems")
        self.device = dev.pop()
        self.n = len(probs)
        o = make_options(**opts)
        o.device_ptrs = 1 if self.device else 0
        o.stream = None
        self.opts = o
        arr = (gsis_problem * self.n)(*[a.s for a in self.args])
        h = ctypes.c_void_p()
        _check(lib.gsis_batch_create(ctx.handle, self.n, arr, ctypes.byref(o), ctypes.byref(h)),
               ctx)
        self.handle = h

    def iterate(self, n=1):
        _check(load().gsis_batch_iterate(self.handle, int(n)), self.ctx)

    def status(self):
        n = self.n
        it, cv, er = (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)(), (ctypes.c_double * n)()
        fin = ctypes.c_int32()
        _check(load().gsis_batch_status(self.handle, it, cv, er, ctypes.byref(fin)), self.ctx)
        return list(it), list(cv), list(er), fin.value

    def read(self, i):
        bufs, r = _result_buffers(self.args[i], self.opts.max_iter)
        _check(load().gsis_batch_read(self.handle, int(i), ctypes.byref(r)), self.ctx)
        phi, fx, fy, hist, thist = bufs
        return dict(phi=phi, Fx=fx, Fy=fy, err_hist=hist[:r.n_iter], tres_hist=thist[:r.n_iter],
                    n_iter=r.n_iter, final_err=r.final_err)

    def reset(self):
        _check(load().gsis_batch_reset(self.handle), self.ctx)

    def tuning(self):
        t = gsis_batch_tuning()
        _check(load().gsis_batch_get_tuning(self.handle, ctypes.byref(t)), self.ctx)
        cfgs = [dict(rows=t.config_rows[c], prefetch=t.config_prefetch[c], ms=t.config_ms[c])
                for c in range(t.n_configs)]
        return dict(rows=t.rows, prefetch=t.prefetch, grid=t.grid, cg_iters=t.cg_iters,
                    configs=cfgs)

    def close(self):
        if getattr(self, "handle", None):
            load().gsis_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gsis_solve_batch(ctx, probs, **opts):
    """One-shot batched solve (gsis_solve_batch); returns (results, status)."""
    lib = load()
    args = [_Args(p) for p in probs]
    dev = {a.device for a in args}
    if len(dev) != 1:
        raise ValueError("mix of host and device problems")
    device = dev.pop()
    o = make_options(**opts)
    o.device_ptrs = 1 if device else 0
    o.stream = None
    n = len(probs)
    bufs, res = [], (gsis_result * n)()
    for i, a in enumerate(args):
        b, r = _result_buffers(a, o.max_iter)
        bufs.append(b)
        res[i] = r
    arr = (gsis_problem * n)(*[a.s for a in args])
    st = lib.gsis_solve_batch(ctx.handle, n, arr, ctypes.byref(o), res)
    _check(st, ctx, allow=(GSIS_OK, GSIS_NOT_CONVERGED, GSIS_DIVERGED))
    out = []
    for i in range(n):
        phi, fx, fy, hist, thist = bufs[i]
        out.append(dict(phi=phi, Fx=fx, Fy=fy, err_hist=hist[:res[i].n_iter],
                        tres_hist=thist[:res[i].n_iter], n_iter=res[i].n_iter,
                        final_err=res[i].final_err))
    return out, st


class TDPlan(Plan):
    """gsis_td_create / gsis_td_advance / gsis_td_read: the time-dependent
    form. c, a, dt scalars; cv and T0 per cell (arrays like the problem's,
    or scalars); I0 the initial intensity [N, K] or None."""

    def __init__(self, ctx, prob, T0, c=1.0, a=1.0, dt=1.0, cv=1.0, sub_iter=4, I0=None, **opts):
        lib = load()
        self.ctx = ctx
        self.args = _Args(prob, I0)
        N = self.args.nx * self.args.ny
        self.N = N

        def per_cell(v):
            if _is_torch(v) or isinstance(v, np.ndarray):
                return self.args._ptr(v)
            if self.args.device:
                import torch
                t = torch.full((N,), float(v), dtype=torch.float64,
                               device=self.args.keep[0].device)
                self.args.keep.append(t)
                return t.data_ptr()
            return self.args._ptr(np.full(N, float(v)))
        mat = gsis_material(float(c), float(a), float(dt), per_cell(cv), per_cell(T0),
                            int(sub_iter))
        o = make_options(**opts)
        o.I0 = self.args.I0
        o.device_ptrs = 1 if self.args.device else 0
        o.stream = _stream_handle() if self.args.device else None
        self.opts = o
        h = ctypes.c_void_p()
        _check(lib.gsis_td_create(ctx.handle, ctypes.byref(self.args.s), ctypes.byref(o),
                                  ctypes.byref(mat), ctypes.byref(h)), ctx)
        self.handle = h

    def advance(self, n_steps):
        """Run n_steps time steps; returns (status, inner iterations per step,
        final Err per step)."""
        its = (ctypes.c_int32 * max(n_steps, 1))()
        errs = (ctypes.c_double * max(n_steps, 1))()
        st = load().gsis_td_advance(self.handle, int(n_steps), its, errs)
        _check(st, self.ctx, allow=(GSIS_OK, GSIS_NOT_CONVERGED, GSIS_DIVERGED))
        return st, list(its)[:n_steps], list(errs)[:n_steps]

    def read_td(self):
        """dict(rho, T, Fx, Fy) of the current state."""
        N = self.N
        if self.args.device:
            import torch
            dev = self.args.keep[0].device
            outs = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(4)]
            p = lambda t: t.data_ptr()
        else:
            outs = [np.empty(N) for _ in range(4)]
            p = lambda a: a.ctypes.data
        _check(load().gsis_td_read(self.handle, *[p(x) for x in outs]), self.ctx)
        return dict(rho=outs[0], T=outs[1], Fx=outs[2], Fy=outs[3])
