"""Batched form: many problems of uneven size in one plan (persistent sweep
launch over (problem, ordinate) items, one block-diagonal synthetic solve,
hipGraph-captured iterations), through the C-ABI, against the oracle."""
import sys

import numpy as np
import pytest

import oracle
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


def _rel(a, b):
    a = _np(a)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _mixed():
    """Uneven shapes and quadratures: one cell, a strip needing two sweep
    passes at every launch configuration, ragged sizes, K = 12 / 32 / 64."""
    return [inputs.random_problem(1, 1, seed=1),
            inputs.random_problem(37, 21, seed=2, sigma_range=(0.05, 50.0)),
            inputs.random_problem(5, 600, seed=3, sigma_range=(0.1, 5.0)),
            dict(inputs.random_problem(64, 48, seed=4, sigma_range=(0.05, 50.0)),
                 **{k: v for k, v in zip(("mu", "eta", "w"), inputs.quad_product(2, 16))},
                 bnd_in=None),
            dict(inputs.random_problem(90, 130, seed=5, sigma_range=(0.5, 500.0)),
                 **{k: v for k, v in zip(("mu", "eta", "w"), inputs.quad_product(4, 16))},
                 bnd_in=None)]


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("method", [0, 1])
def test_batch_iterates_match_oracle(ctx, graph, method):
    probs = _mixed()
    _say("batch iterates graph=%d method=%d" % (graph, method))
    b = gsis.Batch(ctx, probs, method=method, tol=0.0, max_iter=3, synth_rtol=1e-15,
                   synth_max_iter=300, graph=graph)
    b.iterate(3)
    it, conv, err, fin = b.status()
    assert it == [3] * len(probs) and fin == len(probs)
    tun = b.tuning()
    _say("  tuning %s" % tun)
    assert tun["rows"] in (64, 128, 256, 512)
    for i, p in enumerate(probs):
        g = b.read(i)
        o = oracle.solve(p, method=method, tol=0.0, max_iter=3)
        tol = 1e-12 if method == 0 else 1e-10
        assert _rel(g["phi"], o["phi"]) < tol, i
        assert _rel(g["Fx"], o["Fx"]) < 10 * tol and _rel(g["Fy"], o["Fy"]) < 10 * tol, i
        np.testing.assert_allclose(g["err_hist"], o["err_hist"], rtol=1e-8)
    b.reset()
    assert b.status()[0] == [0] * len(probs)
    b.close()


def test_batch_fp32_iterates(ctx):
    probs = _mixed()[1:]
    b = gsis.Batch(ctx, probs, precision=gsis.GSIS_FP32_MIXED, tol=0.0, max_iter=3,
                   synth_rtol=1e-15, synth_max_iter=300)
    b.iterate(3)
    for i, p in enumerate(probs):
        g = b.read(i)
        o = oracle.solve(p, tol=0.0, max_iter=3)
        assert _rel(g["phi"], o["phi"]) < 1e-6 and _rel(g["Fx"], o["Fx"]) < 1e-6, i
    b.close()


def test_batch_converges_each_problem(ctx):
    """Each problem stops on its own Err < tol; the converged fields agree
    with the oracle's fixed points."""
    probs = [inputs.small_s4_32(), inputs.random_problem(24, 40, seed=9, sigma_range=(0.5, 5.0)),
             inputs.random_problem(33, 17, seed=3, sigma_range=(0.5, 20.0))]
    out, st = gsis.gsis_solve_batch(ctx, probs, tol=1e-11, max_iter=400, limiter=0,
                                    synth_rtol=1e-12, synth_max_iter=100)
    assert st == gsis.GSIS_OK
    for p, g in zip(probs, out):
        o = oracle.solve(p, tol=1e-11, max_iter=400, limiter=0)
        assert o["status"] == 0
        assert g["final_err"] < 1e-11 and abs(g["n_iter"] - o["n_iter"]) <= 2
        assert _rel(g["phi"], o["phi"]) < 1e-9


def test_batch_matches_single_plans(ctx):
    """A problem gets the same iterates in a batch as alone (same kernels,
    its own CG scalars); with the CG converging inside the fixed count the
    fields agree to rounding."""
    probs = _mixed()[1:]
    b = gsis.Batch(ctx, probs, tol=0.0, max_iter=4, synth_rtol=1e-13, synth_max_iter=300)
    b.iterate(4)
    for i, p in enumerate(probs):
        g = b.read(i)
        s = gsis.gsis_solve(ctx, p, tol=0.0, max_iter=4, synth_rtol=1e-13, synth_max_iter=300)
        assert _rel(g["phi"], s["phi"]) < 1e-12, i
    b.close()


def test_batch_mixed_coarse_starts(ctx):
    """Problems whose one-workgroup coarse cycle starts on level 0, 1, 2 and
    3 (37 x 21, 90 x 130, 200 x 180, 400 x 300) in one batch: the CG update
    runs in the per-cell kernel for the first and in the level-0 tile kernel
    for the others, side by side in the same launches; each matches its
    single plan."""
    probs = [inputs.random_problem(37, 21, seed=2, sigma_range=(0.05, 50.0)),
             inputs.random_problem(90, 130, seed=5, sigma_range=(0.5, 500.0)),
             inputs.random_problem(200, 180, seed=6, sigma_range=(0.1, 50.0)),
             inputs.random_problem(400, 300, seed=7, sigma_range=(0.1, 50.0))]
    _say("batch of mixed coarse starts")
    b = gsis.Batch(ctx, probs, tol=0.0, max_iter=3, synth_rtol=1e-13, synth_max_iter=300)
    b.iterate(3)
    for i, p in enumerate(probs):
        g = b.read(i)
        s = gsis.gsis_solve(ctx, p, tol=0.0, max_iter=3, synth_rtol=1e-13, synth_max_iter=300)
        assert _rel(g["phi"], s["phi"]) < 1e-12, i
        assert _rel(g["Fx"], s["Fx"]) < 1e-11, i
    b.close()


def test_batch_sweep_forms_agree(ctx, monkeypatch):
    """The batch's split transport step (residual items, then the
    persistent recurrence) and its fused persistent sweep give the same
    iterates; the tuning reports the configuration table of the form used."""
    probs = _mixed()
    out = {}
    for ref in ("0", "2"):
        monkeypatch.setenv("GSIS_SWEEP_REFERENCE", ref)
        _say("batch sweep form %s" % ref)
        b = gsis.Batch(ctx, probs, tol=0.0, max_iter=3, synth_rtol=1e-15, synth_max_iter=300)
        b.iterate(3)
        tun = b.tuning()
        _say("  tuning %s" % tun)
        assert len(tun["configs"]) == (4 if ref == "0" else 6)
        assert all(c["ms"] > 0 for c in tun["configs"])
        out[ref] = [b.read(i) for i in range(len(probs))]
        b.close()
    for i in range(len(probs)):
        a, c = out["0"][i], out["2"][i]
        cp = c["phi"].cpu().numpy() if hasattr(c["phi"], "cpu") else np.asarray(c["phi"])
        assert _rel(a["phi"], cp) < 1e-10, i


@pytest.mark.timeout(1500)
def test_full_batch_sampled(ctx):
    """The 64-problem batch (grids 64..512, 32..128 ordinates, 8 x 8 random
    blocks) at full size, with the graph: after two iterations the first
    problem of every (nx, ny, K) class present (33 classes, from 64 x 64 x 32
    to 512 x 512 x 128) matches the oracle element by element; every
    problem's history is finite."""
    probs = inputs.batch_problems()
    _say("full batch: %d problems" % len(probs))
    b = gsis.Batch(ctx, probs, tol=0.0, max_iter=2, beta=20.0, synth_rtol=1e-14,
                   synth_max_iter=400, graph=1)
    b.iterate(2)
    it, conv, err, fin = b.status()
    assert it == [2] * len(probs) and all(np.isfinite(err))
    _say("  tuning %s" % b.tuning())
    seen = {}
    for i, p in enumerate(probs):
        seen.setdefault((p["nx"], p["ny"], len(p["mu"])), i)
    assert (512, 512, 128) in seen and len(seen) >= 16
    for cls, i in sorted(seen.items(), key=lambda t: t[1]):
        p = probs[i]
        g = b.read(i)
        _say("  problem %d %s" % (i, cls))
        o = oracle.solve(p, tol=0.0, max_iter=2, beta=20.0)
        assert _rel(g["phi"], o["phi"]) < 1e-9, i
        assert _rel(g["Fx"], o["Fx"]) < 1e-8 and _rel(g["Fy"], o["Fy"]) < 1e-8, i
        np.testing.assert_allclose(_np(g["tres_hist"]), o["tres_hist"], rtol=1e-8)
    b.close()
