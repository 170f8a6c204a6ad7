"""The pipelined transport step (residual and recurrence in one launch, the
recurrence's right-hand side passed through LDS) against the split step
(residual kernel, then the recurrence): the same iterates bit for bit, for
every band count, on ragged, tall, wide and single-cell grids, FP64 and
FP32-mixed, first and second order, with and without the limiter, with
inflow on every side, and in the time-dependent form. The transport
residual history is a sum in another order and agrees to rounding."""
import sys

import numpy as np
import pytest

from paper_2507_03975_amd import gsis, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gsis.Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _np(a):
    return a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)


def _impl(monkeypatch, impl, bands=None):
    monkeypatch.setenv("GSIS_SWEEP_REFERENCE", impl)
    if bands is None:
        monkeypatch.delenv("GSIS_PIPE_BANDS", raising=False)
    else:
        monkeypatch.setenv("GSIS_PIPE_BANDS", bands)


def _same(a, b, keys):
    for k in keys:
        assert np.array_equal(_np(a[k]), _np(b[k])), k


SHAPES = [((37, 70), (2, 4)), ((256, 256), (4, 8)), ((5, 1300), (2, 4)), ((1300, 5), (2, 4)),
          ((200, 65), (2, 8)), ((64, 128), (3, 6)), ((1, 1), (2, 4)), ((1, 200), (2, 4)),
          ((129, 1), (2, 4))]


@pytest.mark.parametrize("shape,quad", SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
def test_pipe_bitwise(ctx, shape, quad, prec, monkeypatch):
    """SI and GSIS, three outer iterations: phi, F and the Err history of
    the pipelined step equal the split step's bit for bit, with 1, 2 and 4
    bands of 64 rows per workgroup (1300 rows: 21, 11 and 6 parts)."""
    nx, ny = shape
    p = inputs.random_problem(nx, ny, quad=inputs.quad_product(*quad), seed=nx + 7 * ny,
                              sigma_range=(0.05, 50.0))
    for method in (0, 1):
        kw = dict(method=method, tol=0.0, max_iter=3, precision=prec, synth_rtol=1e-13,
                  synth_max_iter=200)
        _impl(monkeypatch, "0")
        _say("pipe bitwise %s K=%d prec=%d method=%d split" % (shape, quad[0] * quad[1], prec,
                                                                method))
        ref = gsis.gsis_solve(ctx, p, **kw)
        for bands in ("1", "2", "4"):
            _impl(monkeypatch, "3", bands)
            _say("  pipelined, %s bands" % bands)
            out = gsis.gsis_solve(ctx, p, **kw)
            assert out["n_iter"] == 3
            _same(ref, out, ("phi", "Fx", "Fy", "err_hist"))
            t0, t1 = np.asarray(ref["tres_hist"]), np.asarray(out["tres_hist"])
            assert np.all(np.abs(t0 - t1) <= 1e-12 * np.abs(t0)), (t0, t1)


@pytest.mark.parametrize("kw", [dict(order=1, limiter=0), dict(order=2, limiter=0),
                                dict(order=2, limiter=1, alsm=0),
                                dict(order=2, limiter=1, hot_face=1)])
def test_pipe_bitwise_options(ctx, kw, monkeypatch):
    """First order, limiter off, plain least squares and the transport-face
    HoT: the same bits as the split step (GSIS, three iterations)."""
    p = inputs.random_problem(90, 150, quad=inputs.quad_product(2, 8), seed=5,
                              sigma_range=(0.05, 50.0))
    kw = dict(method=1, tol=0.0, max_iter=3, synth_rtol=1e-13, synth_max_iter=200, **kw)
    _impl(monkeypatch, "0")
    _say("pipe options %s" % kw)
    ref = gsis.gsis_solve(ctx, p, **kw)
    _impl(monkeypatch, "3", "2")
    out = gsis.gsis_solve(ctx, p, **kw)
    _same(ref, out, ("phi", "Fx", "Fy", "err_hist"))


def test_pipe_bitwise_converged(ctx, monkeypatch):
    """The headline thick square converged to Err < 1e-6 with the library
    defaults: the same iteration count and bits."""
    p = inputs.thick_square(256)
    _impl(monkeypatch, "0")
    _say("pipe converged thick square, split")
    ref = gsis.gsis_solve(ctx, p, tol=1e-6, max_iter=200)
    _impl(monkeypatch, "3")
    _say("pipe converged thick square, pipelined")
    out = gsis.gsis_solve(ctx, p, tol=1e-6, max_iter=200)
    assert ref["status"] == gsis.GSIS_OK and out["n_iter"] == ref["n_iter"]
    _same(ref, out, ("phi", "Fx", "Fy", "err_hist"))


@pytest.mark.parametrize("shape", [(13, 9), (70, 140)])
def test_pipe_bitwise_time_dependent(ctx, shape, monkeypatch):
    """The time-dependent form (I^n / (c dt) in the residual): two steps of
    the pipelined step equal the split step's bits."""
    p = inputs.random_problem(shape[0], shape[1], seed=shape[1], sigma_range=(0.05, 50.0))
    N = shape[0] * shape[1]
    rng = np.random.Generator(np.random.PCG64(shape[0]))
    cv, T0 = rng.uniform(0.5, 2.0, N), rng.uniform(0.2, 1.2, N)
    out = {}
    for impl in ("0", "3"):
        _impl(monkeypatch, impl, "1" if impl == "3" else None)
        _say("pipe time-dependent %s impl=%s" % (shape, impl))
        pl = gsis.TDPlan(ctx, p, T0, cv=cv, c=2.0, a=0.7, dt=0.05, sub_iter=2, tol=0.0,
                         max_iter=3, synth_rtol=1e-13, synth_max_iter=200)
        st, its, _ = pl.advance(2)
        out[impl] = pl.read_td()
        pl.close()
        assert its == [3, 3]
    _same(out["0"], out["3"], ("rho", "T", "Fx", "Fy"))


def test_pipe_default_selection(ctx, monkeypatch):
    """The transport step a plan runs by default: split for the 256x256x128
    thick square and in FP32-mixed form, pipelined with 2 bands of 64 rows for
    FP64 problems of 2^26 cell-ordinates and more; the environment variable
    overrides either way."""
    monkeypatch.delenv("GSIS_SWEEP_REFERENCE", raising=False)
    monkeypatch.delenv("GSIS_PIPE_BANDS", raising=False)
    small = inputs.thick_square(256)
    big = inputs.random_problem(512, 1024, quad=inputs.quad_product(4, 32), seed=3, inflow=False)
    cases = [(small, {}, None, (0, 0)), (big, {}, None, (3, 2)),
             (big, dict(precision=1), None, (0, 0)), (small, {}, "3", (3, 2)),
             (big, {}, "0", (0, 0))]
    for p, kw, env, want in cases:
        if env is None:
            monkeypatch.delenv("GSIS_SWEEP_REFERENCE", raising=False)
        else:
            monkeypatch.setenv("GSIS_SWEEP_REFERENCE", env)
        _say("transport form %dx%d %s env=%s" % (p["nx"], p["ny"], kw, env))
        pl = gsis.Plan(ctx, p, **kw)
        form, bands, parts = pl.transport_form()
        pl.close()
        assert (form, bands) == want, (form, bands, parts)
        if form == 3:
            assert parts == -(-p["ny"] // 128)
