"""The synthetic solve's host check with the next CG step already in the
stream (the device keeps working while the host reads the convergence
flags) against a plain wait for the stream: the same iterates, histories,
iteration and V-cycle counts, bit for bit. After the flags show convergence
that step's kernels must return before touching anything."""
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


def _run_plan(ctx, p, iters, **kw):
    pl = gsis.Plan(ctx, p, **kw)
    pl.iterate(iters)
    out = pl.read()
    out["status_tuple"] = pl.status()
    out["vcycles"] = pl.synth_vcycles()
    pl.close()
    return out


CASES = [
    ("thick square, defaults", lambda: inputs.thick_square(256),
     dict(tol=1e-6, max_iter=200), 200),
    ("random, tight CG, cap 7", lambda: inputs.random_problem(70, 67, seed=3, sigma_range=(0.05, 50.0)),
     dict(tol=0.0, max_iter=6, synth_rtol=1e-15, synth_max_iter=7), 6),
    ("block medium FP32-mixed", lambda: inputs.checkerboard_blocks(128),
     dict(tol=1e-6, max_iter=300, precision=1, beta=10.0, limiter=0), 300),
    ("random, rtol 0.3", lambda: inputs.random_problem(40, 90, seed=9, sigma_range=(0.5, 500.0)),
     dict(tol=1e-8, max_iter=300, synth_rtol=0.3), 300),
]


@pytest.mark.parametrize("name,make,kw,iters", CASES, ids=[c[0] for c in CASES])
def test_speculative_step_changes_nothing(ctx, name, make, kw, iters, monkeypatch):
    p = make()
    out = {}
    for spec in ("1", "0"):
        monkeypatch.setenv("GSIS_SYNTH_SPECULATE", spec)
        _say("speculate=%s %s" % (spec, name))
        out[spec] = _run_plan(ctx, p, iters, **kw)
    a, b = out["1"], out["0"]
    assert a["status_tuple"][:2] == b["status_tuple"][:2]
    assert a["vcycles"] == b["vcycles"]
    for k in ("phi", "Fx", "Fy", "err_hist", "tres_hist"):
        assert np.array_equal(_np(a[k]), _np(b[k])), k


def test_speculative_step_time_dependent(ctx, monkeypatch):
    """Time steps (several synthetic solves per inner iteration) with and
    without the speculative CG step: the same bits."""
    p = inputs.random_problem(48, 40, seed=12, sigma_range=(0.1, 80.0))
    N = 48 * 40
    rng = np.random.Generator(np.random.PCG64(12))
    cv, T0 = rng.uniform(0.5, 2.0, N), rng.uniform(0.2, 1.2, N)
    out = {}
    for spec in ("1", "0"):
        monkeypatch.setenv("GSIS_SYNTH_SPECULATE", spec)
        _say("speculate=%s time-dependent" % spec)
        pl = gsis.TDPlan(ctx, p, T0, cv=cv, c=1.0, a=0.5, dt=0.2, sub_iter=3, tol=1e-8,
                         max_iter=200)
        st, its, errs = pl.advance(3)
        out[spec] = (st, its, errs, pl.read_td())
        pl.close()
    assert out["1"][:3] == out["0"][:3]
    for k in ("rho", "T", "Fx", "Fy"):
        assert np.array_equal(_np(out["1"][3][k]), _np(out["0"][3][k])), k
