"""Plain FP64 CPU oracle of steady gray SI / GSIS (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code: this module loads ``liboracle.so`` built from ``gsis_oracle.c`` by gcc.

Every function takes a problem dict with keys ``nx, ny, dx, dy, mu, eta, w,
sigma_a, sigma_s, q, bnd_in`` (``bnd_in`` is ``None`` for vacuum or a
``[2*(nx+ny), K]`` array of incoming intensities, sides W, E, S, N).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsis_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("K", ctypes.c_int),
        ("mu", _dp), ("eta", _dp), ("w", _dp),
        ("sig_a", _dp), ("sig_s", _dp), ("q", _dp),
        ("bnd_in", _dp),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int), ("order", ctypes.c_int),
        ("limiter", ctypes.c_int), ("alsm", ctypes.c_int),
        ("hot_face", ctypes.c_int), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int), ("cfl_p", ctypes.c_double),
        ("beta", ctypes.c_double), ("synth_form", ctypes.c_int),
        ("synth_sub", ctypes.c_int),
    ]


class _Material(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("a", ctypes.c_double), ("dt", ctypes.c_double),
                ("cv", _dp), ("sub_iter", ctypes.c_int)]


def build(force=True):
    """Compile the oracle with gcc (plain -O2, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call([
        "gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
        "-std=c11", "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P, O = ctypes.POINTER(_Problem), ctypes.POINTER(_Options)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.ora_gradient.argtypes = [P, ctypes.c_int, _dp, _dp, _dp]
        lib.ora_bj_limiter.argtypes = [P, _dp, _dp, _dp, _dp]
        lib.ora_face_coeffs.argtypes = [P, _dp, _dp, _dp]
        lib.ora_plant_kappa.argtypes = [ctypes.c_int]
        lib.ora_residual.argtypes = [P, O, _dp, _dp]
        lib.ora_sweep.argtypes = [P, O, _dp, _dp]
        lib.ora_pseudo_shift.argtypes = [P, O, ctypes.c_int]
        lib.ora_pseudo_shift.restype = ctypes.c_double
        lib.ora_iterate.argtypes = [P, O, _dp, _dp, _dp]
        lib.ora_iterate.restype = ctypes.c_int
        lib.ora_solve.argtypes = [P, O, _dp, _dp, _dp, _dp, _dp, _dp, ip, _dp, _dp]
        lib.ora_solve.restype = ctypes.c_int
        lib.ora_synthetic_solve.argtypes = [P, _dp, _dp]
        lib.ora_synthetic_solve.restype = ctypes.c_int
        lib.ora_synthetic_apply.argtypes = [P, _dp, _dp]
        lib.ora_wide_correction.argtypes = [P, ctypes.c_int, _dp, _dp]
        lib.ora_synthetic_wide.argtypes = [P, ctypes.c_int, _dp, ctypes.c_int, _dp]
        lib.ora_synthetic_wide.restype = ctypes.c_int
        lib.ora_td_solve.argtypes = [P, O, ctypes.POINTER(_Material), _dp, _dp, ctypes.c_int,
                                     _dp, _dp, _dp, _dp, _dp, ip, _dp]
        lib.ora_td_solve.restype = ctypes.c_int
        lib.ora_adjoint.argtypes = [P, O, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                    _dp, _dp, _dp, _dp, ip, _dp]
        lib.ora_adjoint.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class _Marshal:
    """Keeps contiguous float64 copies alive while a C call runs."""

    def __init__(self, prob):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.mu, self.eta, self.w = f(prob["mu"]), f(prob["eta"]), f(prob["w"])
        self.sa, self.ss, self.q = f(prob["sigma_a"]), f(prob["sigma_s"]), f(prob["q"])
        b = prob.get("bnd_in")
        self.bnd = None if b is None else f(b)
        self.nx, self.ny, self.K = int(prob["nx"]), int(prob["ny"]), len(self.mu)
        self.s = _Problem(self.nx, self.ny, float(prob["dx"]), float(prob["dy"]), self.K,
                          _ptr(self.mu), _ptr(self.eta), _ptr(self.w),
                          _ptr(self.sa.ravel()), _ptr(self.ss.ravel()), _ptr(self.q.ravel()),
                          _ptr(self.bnd))


def _opts(method=1, order=2, limiter=1, alsm=1, hot_face=0, tol=1e-8, max_iter=1000,
          cfl_p=0.0, beta=0.0, synth_form=0, synth_sub=1):
    return _Options(int(method), int(order), int(limiter), int(alsm), int(hot_face),
                    float(tol), int(max_iter), float(cfl_p), float(beta), int(synth_form),
                    int(synth_sub))


def gradient(prob, U, alsm=1):
    m = _Marshal(prob)
    U = np.ascontiguousarray(U, dtype=np.float64).ravel()
    gx, gy = np.empty_like(U), np.empty_like(U)
    _load().ora_gradient(ctypes.byref(m.s), int(alsm), _ptr(U), _ptr(gx), _ptr(gy))
    return gx, gy


def bj_limiter(prob, U, gx, gy):
    m = _Marshal(prob)
    U = np.ascontiguousarray(U, dtype=np.float64).ravel()
    gx = np.ascontiguousarray(gx, dtype=np.float64)
    gy = np.ascontiguousarray(gy, dtype=np.float64)
    psi = np.empty_like(U)
    _load().ora_bj_limiter(ctypes.byref(m.s), _ptr(U), _ptr(gx), _ptr(gy), _ptr(psi))
    return psi


def wide_correction(prob, x, alsm=1):
    """corr(x) of the face-averaged synthetic balance D1 x = b + corr(x)
    (Eq. Fij_d against the compact Gamma flux)."""
    m = _Marshal(prob)
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.empty_like(x)
    _load().ora_wide_correction(ctypes.byref(m.s), int(alsm), _ptr(x), _ptr(out))
    return out


def synthetic_wide(prob, b, x0, n_sub, alsm=1):
    """n_sub defect-correction sub-iterations x <- D1^{-1} (b + corr(x))."""
    m = _Marshal(prob)
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    x = np.array(x0, dtype=np.float64).ravel()
    st = _load().ora_synthetic_wide(ctypes.byref(m.s), int(alsm), _ptr(b), int(n_sub), _ptr(x))
    assert st == 0, st
    return x


def plant_kappa(mode):
    """Test hook: replace the wall coefficient kappa by a misreading of Eq.
    macro_bc_delta_flux (1 escape term only, 2 diffusion term only, 3 the two
    in series, 4 none); 0 restores the paper's sum."""
    _load().ora_plant_kappa(int(mode))


def face_coeffs(prob):
    m = _Marshal(prob)
    nx, ny = m.nx, m.ny
    gx = np.zeros(max((nx - 1) * ny, 1))
    gy = np.zeros(max(nx * (ny - 1), 1))
    kap = np.zeros(2 * (nx + ny))
    _load().ora_face_coeffs(ctypes.byref(m.s), _ptr(gx), _ptr(gy), _ptr(kap))
    return gx[:(nx - 1) * ny], gy[:nx * (ny - 1)], kap


def residual(prob, I, **opts):
    m = _Marshal(prob)
    I = np.ascontiguousarray(I, dtype=np.float64)
    r = np.empty_like(I)
    o = _opts(**opts)
    _load().ora_residual(ctypes.byref(m.s), ctypes.byref(o), _ptr(I), _ptr(r))
    return r


def sweep(prob, r, **opts):
    """Exact increment solve; ``cfl_p`` / ``beta`` add the pseudo-time shift."""
    m = _Marshal(prob)
    r = np.ascontiguousarray(r, dtype=np.float64)
    dI = np.empty_like(r)
    o = _opts(**opts)
    _load().ora_sweep(ctypes.byref(m.s), ctypes.byref(o), _ptr(r), _ptr(dI))
    return dI


def pseudo_shift(prob, **opts):
    """Per-cell pseudo-time shift of the increment-solve diagonal."""
    m = _Marshal(prob)
    o = _opts(**opts)
    lib = _load()
    return np.array([lib.ora_pseudo_shift(ctypes.byref(m.s), ctypes.byref(o), c)
                     for c in range(m.nx * m.ny)])


def iterate(prob, I, **opts):
    """One outer iteration from I [N, K]; returns (I_next, phi_next)."""
    m = _Marshal(prob)
    I = np.ascontiguousarray(I, dtype=np.float64)
    Io = np.empty_like(I)
    phi = np.empty(m.nx * m.ny)
    o = _opts(**opts)
    e = _load().ora_iterate(ctypes.byref(m.s), ctypes.byref(o), _ptr(I), _ptr(Io), _ptr(phi))
    if e:
        raise RuntimeError("ora_iterate failed: %d" % e)
    return Io, phi


def synthetic_solve(prob, b):
    m = _Marshal(prob)
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    x = np.empty_like(b)
    e = _load().ora_synthetic_solve(ctypes.byref(m.s), _ptr(b), _ptr(x))
    if e:
        raise RuntimeError("ora_synthetic_solve failed: %d" % e)
    return x


def synthetic_apply(prob, x):
    m = _Marshal(prob)
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.empty_like(x)
    _load().ora_synthetic_apply(ctypes.byref(m.s), _ptr(x), _ptr(y))
    return y


def solve(prob, I0=None, return_I=False, **opts):
    """Iterate to Err(phi) < tol (Eq. Err_W) or max_iter.

    Returns a dict: phi, Fx, Fy [N], err_hist [n_iter], tres_hist [n_iter]
    (relative transport residual of the iterate each iteration starts from),
    n_iter, final_err, status (0 converged, 1 not converged, 2 diverged,
    <0 error) and optionally I [N, K].
    """
    m = _Marshal(prob)
    o = _opts(**opts)
    N, K = m.nx * m.ny, m.K
    phi, fx, fy = np.zeros(N), np.zeros(N), np.zeros(N)
    hist = np.zeros(max(o.max_iter, 1))
    thist = np.zeros(max(o.max_iter, 1))
    n_iter = ctypes.c_int(0)
    ferr = ctypes.c_double(0)
    If = np.empty((N, K)) if return_I else None
    I0c = None if I0 is None else np.ascontiguousarray(I0, dtype=np.float64)
    st = _load().ora_solve(ctypes.byref(m.s), ctypes.byref(o), _ptr(I0c), _ptr(phi),
                           _ptr(fx), _ptr(fy), _ptr(hist), _ptr(thist), ctypes.byref(n_iter),
                           ctypes.byref(ferr), _ptr(If))
    out = dict(phi=phi, Fx=fx, Fy=fy, err_hist=hist[:n_iter.value],
               tres_hist=thist[:n_iter.value], n_iter=n_iter.value,
               final_err=ferr.value, status=st)
    if return_I:
        out["I"] = If
    return out


def adjoint(prob, I_star, g_phi=None, g_Fx=None, g_Fy=None, tol=1e-12, max_iter=2000,
            return_lambda=False, **opts):
    """Adjoint of the fixed point I_star [N, K] (limiter off): lambda and
    dJ/dsigma_a, dJ/dsigma_s, dJ/dq for J = <g_phi, phi*> + <g_F, F*>."""
    m = _Marshal(prob)
    N, K = m.nx * m.ny, m.K
    o = _opts(**dict(opts, limiter=opts.get("limiter", 0)))
    I_star = np.ascontiguousarray(I_star, dtype=np.float64)
    f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
    gp, gx, gy = f(g_phi), f(g_Fx), f(g_Fy)
    ga, gs, gq = np.zeros(N), np.zeros(N), np.zeros(N)
    lam = np.zeros((N, K)) if return_lambda else None
    hist = np.zeros(max(max_iter, 1))
    n = ctypes.c_int(0)
    st = _load().ora_adjoint(ctypes.byref(m.s), ctypes.byref(o), _ptr(I_star), _ptr(gp),
                             _ptr(gx), _ptr(gy), float(tol), int(max_iter), _ptr(ga), _ptr(gs),
                             _ptr(gq), _ptr(lam), ctypes.byref(n), _ptr(hist))
    out = dict(g_sigma_a=ga, g_sigma_s=gs, g_q=gq, n_iter=n.value, status=st,
               err_hist=hist[:n.value])
    if return_lambda:
        out["lambda"] = lam
    return out


def td_solve(prob, T0, n_steps, c=1.0, a=1.0, dt=1.0, cv=1.0, sub_iter=4, I0=None,
             return_I=False, **opts):
    """Time-dependent gray RTE with the material energy equation: n_steps
    backward-Euler steps of size dt from I0 [N, K] (None = 0) and T0 [N],
    each iterated (SI or GSIS, opts as in solve) until max(Err(rho), Err(T))
    < tol or max_iter. cv is the volume specific heat (scalar or [N]).
    Returns dict(rho, T, Fx, Fy, inner_iters [n_steps], err_last [n_steps],
    status, and I [N, K] with return_I)."""
    m = _Marshal(prob)
    o = _opts(**opts)
    N, K = m.nx * m.ny, m.K
    cvv = np.ascontiguousarray(np.broadcast_to(np.asarray(cv, dtype=np.float64), (N,)))
    mat = _Material(float(c), float(a), float(dt), _ptr(cvv), int(sub_iter))
    T0c = np.ascontiguousarray(np.broadcast_to(np.asarray(T0, dtype=np.float64), (N,)))
    I0c = None if I0 is None else np.ascontiguousarray(I0, dtype=np.float64)
    Io = np.empty((N, K)) if return_I else None
    T, rho, fx, fy = np.zeros(N), np.zeros(N), np.zeros(N), np.zeros(N)
    its = (ctypes.c_int * max(n_steps, 1))()
    errs = np.zeros(max(n_steps, 1))
    st = _load().ora_td_solve(ctypes.byref(m.s), ctypes.byref(o), ctypes.byref(mat), _ptr(I0c),
                              _ptr(T0c), int(n_steps), _ptr(Io), _ptr(T), _ptr(rho), _ptr(fx),
                              _ptr(fy), its, _ptr(errs))
    out = dict(rho=rho, T=T, Fx=fx, Fy=fy, inner_iters=list(its)[:n_steps],
               err_last=errs[:n_steps], status=st)
    if return_I:
        out["I"] = Io
    return out
