"""FP32-mixed form: FP32 storage of the angular intensity (as a deviation
from the FP64 scalar flux) and an FP32 wavefront recurrence; FP64 residual,
moments, synthetic solve and Err. Compared with the FP64 oracle; the stated
bound for converged results is 1e-5 relative (max norm over the field,
relative to its max)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2507_03975_amd import gsis, inputs

pytestmark = pytest.mark.gpu

FP32_BOUND = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gsis.Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = b.cpu().numpy() if hasattr(b, "cpu") else np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("kw", [dict(method=0, limiter=1), dict(method=1, limiter=1),
                                dict(method=1, limiter=0, beta=3.0),
                                dict(method=1, limiter=1, synth_form=1, synth_sub=2)])
def test_fp32_iterates(ctx, kw):
    """At fixed m the only difference is the FP32 rounding of the stored
    deviation, about 6e-8 of |I - phi/(4 pi)| per iteration."""
    p = inputs.random_problem(41, 23, seed=17, sigma_range=(0.05, 200.0))
    _say("fp32 iterates %s" % kw)
    g = gsis.gsis_solve(ctx, p, precision=gsis.GSIS_FP32_MIXED, tol=0.0, max_iter=3,
                        synth_rtol=1e-15, synth_max_iter=200, **kw)
    o = oracle.solve(p, tol=0.0, max_iter=3, **kw)
    assert _rel(g["phi"], o["phi"]) < 1e-6
    assert _rel(g["Fx"], o["Fx"]) < 1e-6 and _rel(g["Fy"], o["Fy"]) < 1e-6


@pytest.mark.parametrize("case", ["s4", "thick128", "blocks64"])
def test_fp32_fixed_point(ctx, case):
    if case == "s4":
        p, kw = inputs.small_s4_32(), dict(limiter=0)
    elif case == "thick128":
        p, kw = inputs.thick_square(128, inputs.quad_product(2, 16)), dict(limiter=0)
    else:
        p, kw = inputs.checkerboard_blocks(64, inputs.quad_product(2, 16)), dict(limiter=0,
                                                                                 beta=10.0)
    _say("fp32 fixed point %s" % case)
    # In a thin medium the stored deviation is as large as I itself and the
    # FP32 recurrence rounds it at every step of a chain, so Err levels off
    # near 1e-8 (the FP32 floor); 600 iterations reach it.
    g = gsis.gsis_solve(ctx, p, precision=gsis.GSIS_FP32_MIXED, tol=1e-10, max_iter=600,
                        synth_rtol=1e-12, synth_max_iter=300, **kw)
    o = oracle.solve(p, tol=1e-12, max_iter=3000, **kw)
    assert o["status"] == 0
    assert g["status"] in (gsis.GSIS_OK, gsis.GSIS_NOT_CONVERGED) and g["final_err"] < 1e-7
    errs = [_rel(g[f], o[f]) for f in ("phi", "Fx", "Fy")]
    _say("  fp32 vs oracle: phi %.2e Fx %.2e Fy %.2e" % tuple(errs))
    assert max(errs) < FP32_BOUND


def test_fp32_block_medium_full_size(ctx):
    """1024 x 1024 x 128 block medium (local pseudo time beta = 10, limiter
    off): FP32-mixed against the FP64 GPU path, which the other tests tie to
    the oracle; both converged to Err < 1e-9."""
    import torch
    p = inputs.checkerboard_blocks(1024)
    pd = {k: (torch.from_numpy(v).cuda() if isinstance(v, np.ndarray) else v)
          for k, v in p.items()}
    out = {}
    for prec in (gsis.GSIS_FP64, gsis.GSIS_FP32_MIXED):
        _say("block medium 1024 precision %d" % prec)
        out[prec] = gsis.gsis_solve(ctx, pd, precision=prec, tol=1e-9, max_iter=400, limiter=0,
                                    beta=10.0, synth_rtol=1e-8)
        assert out[prec]["status"] == 0
    a, b = out[gsis.GSIS_FP32_MIXED], out[gsis.GSIS_FP64]
    errs = [_rel(a[f], b[f]) for f in ("phi", "Fx", "Fy")]
    _say("  fp32 vs fp64: phi %.2e Fx %.2e Fy %.2e" % tuple(errs))
    assert max(errs) < FP32_BOUND
