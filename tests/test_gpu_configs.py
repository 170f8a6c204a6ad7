"""Parity of the HIP path with the oracle on the remaining workloads and
outputs: the 1024 x 1024 x 128 block medium at full size, its FP32-mixed
fixed point at 256 x 256 x 128, the diffusion limit, long fixed-m runs, the
transport-residual history, the divergence guard, the size limit and GSIS
with transport face fluxes in the synthetic equation.

Every case prints its name before it runs (flushed), so that a run that
ends early names it.
"""
import math
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
    return np.abs(_np(a) - b).max() / max(np.abs(b).max(), 1e-300)


# ------------------------------------------------ transport-residual history
@pytest.mark.parametrize("kw", [dict(method=0, limiter=1), dict(method=1, limiter=1),
                                dict(method=1, limiter=0, alsm=0),
                                dict(method=1, limiter=0, precision=1)])
def test_tres_history_matches_oracle(ctx, kw):
    """||r(I^m)||_V / ||(sigma_s phi^m + q)/(4 pi)||_V per iteration, against
    the oracle's on the same iterates (two tile rows, ragged edges, inflow)."""
    p = inputs.random_problem(70, 67, seed=70, sigma_range=(0.05, 50.0))
    _say("tres history %s" % kw)
    kw = dict(kw)
    prec = kw.pop("precision", 0)
    g = gsis.gsis_solve(ctx, p, tol=0.0, max_iter=5, synth_rtol=1e-15, synth_max_iter=200,
                        precision=prec, **kw)
    o = oracle.solve(p, tol=0.0, max_iter=5, **kw)
    np.testing.assert_allclose(_np(g["tres_hist"]), o["tres_hist"], rtol=1e-9 if prec == 0 else 1e-5)


def test_tres_limits(ctx):
    """From I = 0 in vacuum the relative residual is 1; at the converged SI
    fixed point it vanishes, at the converged central-face GSIS fixed point
    it does not (F1), and the GPU's final value matches the oracle's."""
    p = dict(inputs.random_problem(10, 8, seed=5, sigma_range=(0.2, 20.0)), bnd_in=None)
    _say("tres limits 10x8")
    si = gsis.gsis_solve(ctx, p, method=0, limiter=0, tol=1e-13, max_iter=5000)
    gc = gsis.gsis_solve(ctx, p, method=1, limiter=0, tol=1e-13, max_iter=5000,
                         synth_rtol=1e-15, synth_max_iter=200)
    oc = oracle.solve(p, method=1, limiter=0, tol=1e-13, max_iter=5000)
    for r in (si, gc):
        assert r["status"] == gsis.GSIS_OK
        assert abs(_np(r["tres_hist"])[0] - 1.0) < 1e-13
    assert _np(si["tres_hist"])[-1] < 1e-10
    t = _np(gc["tres_hist"])[-1]
    assert t > 1e-4 and abs(t - oc["tres_hist"][-1]) < 1e-8 * t


def test_tres_history_batch(ctx):
    """The batch records the same history per problem as the oracle."""
    probs = [inputs.random_problem(37, 21, seed=2, sigma_range=(0.05, 50.0)),
             inputs.random_problem(5, 300, seed=3, sigma_range=(0.1, 5.0))]
    _say("tres history batch")
    b = gsis.Batch(ctx, probs, tol=0.0, max_iter=3, synth_rtol=1e-15, synth_max_iter=300)
    b.iterate(3)
    for i, p in enumerate(probs):
        g = b.read(i)
        o = oracle.solve(p, tol=0.0, max_iter=3)
        np.testing.assert_allclose(_np(g["tres_hist"]), o["tres_hist"], rtol=1e-9)
    b.close()


# --------------------------------------------------------- guard and limits
def test_divergence_guard(ctx):
    """GSIS without the pseudo-time shift on the 7 x 7 block medium at 64 x 64
    blows up geometrically; the GPU stops it as DIVERGED at the same
    iteration as the oracle's guard."""
    p = inputs.checkerboard_blocks(64, inputs.quad_product(2, 16))
    _say("divergence guard 64x64 blocks")
    g = gsis.gsis_solve(ctx, p, method=1, limiter=0, tol=1e-6, max_iter=40, synth_rtol=1e-12,
                        synth_max_iter=200)
    o = oracle.solve(p, method=1, limiter=0, tol=1e-6, max_iter=40)
    assert o["status"] == 2
    assert g["status"] == gsis.GSIS_DIVERGED and g["n_iter"] == o["n_iter"] < 40
    ok = oracle.solve(p, method=1, limiter=0, tol=1e-6, max_iter=200, beta=10.0)
    gk = gsis.gsis_solve(ctx, p, method=1, limiter=0, tol=1e-6, max_iter=200, beta=10.0,
                         synth_rtol=1e-12, synth_max_iter=200)
    assert gk["status"] == gsis.GSIS_OK and abs(gk["n_iter"] - ok["n_iter"]) <= 1


def test_cell_count_limit(ctx):
    """nx*ny one above GSIS_MAX_CELLS (48-byte records addressed with 32-bit
    offsets) is refused before any array is read or allocated."""
    n_max = 89478485
    nx = 9460
    ny = n_max // nx + 1
    assert nx * ny > n_max
    tiny = np.ones(1)
    mu, eta, w = inputs.quad_s4()
    p = dict(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, mu=mu, eta=eta, w=w,
             sigma_a=tiny, sigma_s=tiny, q=tiny, bnd_in=None)
    _say("cell limit %d x %d" % (nx, ny))
    with pytest.raises(gsis.GSISError) as e:
        gsis.Plan(ctx, p)
    assert e.value.status == gsis.GSIS_E_INVALID_ARG and "too large" in str(e.value)


# ------------------------------------------------------------ long fixed m
@pytest.mark.parametrize("method", [0, 1])
def test_fixed_m_long_small_s4(ctx, method):
    """Iterates at m = 10 and m = 100 (limiter on) on the 32 x 32 S4 medium."""
    p = inputs.small_s4_32()
    for m in (10, 100):
        _say("fixed m=%d small_s4 method=%d" % (m, method))
        g = gsis.gsis_solve(ctx, p, method=method, tol=0.0, max_iter=m, synth_rtol=1e-15,
                            synth_max_iter=200)
        o = oracle.solve(p, method=method, tol=0.0, max_iter=m)
        assert g["n_iter"] == m == o["n_iter"]
        assert _rel(g["phi"], o["phi"]) < 1e-12
        assert _rel(g["Fx"], o["Fx"]) < 1e-11 and _rel(g["Fy"], o["Fy"]) < 1e-11


def test_fixed_m10_thick_square(ctx):
    """m = 10 GSIS iterates of the two-region medium at 64 x 64 x 32."""
    p = inputs.thick_square(64, inputs.quad_product(2, 16))
    _say("fixed m=10 thick square 64")
    g = gsis.gsis_solve(ctx, p, tol=0.0, max_iter=10, limiter=0, beta=10.0, synth_rtol=1e-15,
                        synth_max_iter=300)
    o = oracle.solve(p, tol=0.0, max_iter=10, limiter=0, beta=10.0)
    assert _rel(g["phi"], o["phi"]) < 1e-10
    assert _rel(g["Fx"], o["Fx"]) < 1e-9


# --------------------------------------------------------- diffusion limit
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_diffusion_limit(ctx, eps, n, prec):
    """sigma_s = 1/eps, sigma_a = 0, q = eps (App. A in 2D), converged GSIS
    against the oracle's converged GSIS: FP64 to 1e-9, FP32-mixed to the
    stated 1e-5; iteration counts within 2."""
    p = inputs.diffusion_limit(n, eps)
    _say("diffusion limit eps=%g n=%d precision=%d" % (eps, n, prec))
    o = oracle.solve(p, method=1, limiter=0, tol=1e-10, max_iter=300)
    g = gsis.gsis_solve(ctx, p, method=1, limiter=0, tol=1e-10, max_iter=300, precision=prec,
                        synth_rtol=1e-14, synth_max_iter=300)
    assert o["status"] == 0
    if prec == 0:
        assert g["status"] == gsis.GSIS_OK and abs(g["n_iter"] - o["n_iter"]) <= 2
        assert _rel(g["phi"], o["phi"]) < 1e-9
        assert _rel(g["Fx"], o["Fx"]) < 1e-7 and _rel(g["Fy"], o["Fy"]) < 1e-7
    else:
        assert g["status"] in (gsis.GSIS_OK, gsis.GSIS_NOT_CONVERGED)
        assert abs(g["n_iter"] - o["n_iter"]) <= 2 or g["final_err"] < 1e-8
        assert _rel(g["phi"], o["phi"]) < 1e-5
        assert _rel(g["Fx"], o["Fx"]) < 1e-5 and _rel(g["Fy"], o["Fy"]) < 1e-5


# ------------------------------------------- block medium (1024^2 x 128)
@pytest.mark.timeout(1500)
def test_block_medium_full_iterates(ctx):
    """The 7 x 7 block medium at full size, 1024 x 1024 x 128 (four-part
    split recurrence, deep multigrid hierarchy), beta = 10, limiter off:
    SI and GSIS iterates at m = 2 element by element against the oracle
    (whose synthetic solve is a banded Cholesky factorisation of the
    10^6-cell system)."""
    p = inputs.checkerboard_blocks(1024)
    for method, tol in ((0, 1e-12), (1, 1e-10)):
        _say("block medium 1024x1024x128 method=%d m=2" % method)
        g = gsis.gsis_solve(ctx, p, method=method, tol=0.0, max_iter=2, beta=10.0, limiter=0,
                            synth_rtol=1e-15, synth_max_iter=400)
        gphi, gfx, gfy = _np(g["phi"]), _np(g["Fx"]), _np(g["Fy"])
        gt = _np(g["tres_hist"])
        del g
        _say("  oracle")
        o = oracle.solve(p, method=method, tol=0.0, max_iter=2, beta=10.0, limiter=0)
        assert o["n_iter"] == 2
        e = (_rel(gphi, o["phi"]), _rel(gfx, o["Fx"]), _rel(gfy, o["Fy"]))
        _say("  rel diff phi %.3e Fx %.3e Fy %.3e" % e)
        assert e[0] < tol and e[1] < 10 * tol and e[2] < 10 * tol
        np.testing.assert_allclose(gt, o["tres_hist"], rtol=1e-9)


@pytest.mark.timeout(900)
def test_block_medium_fp32_fixed_point(ctx):
    """FP32-mixed and FP64 GSIS converged on the block medium at 256 x 256 x
    128 (beta = 10, limiter off) against the oracle's FP64 fixed point: FP64
    to 1e-8, FP32-mixed per field to the stated 1e-5."""
    p = inputs.checkerboard_blocks(256)
    _say("block medium 256x256x128 fixed point")
    o = oracle.solve(p, method=1, tol=1e-10, max_iter=300, beta=10.0, limiter=0)
    assert o["status"] == 0
    for prec in (0, 1):
        g = gsis.gsis_solve(ctx, p, method=1, tol=1e-10, max_iter=300, beta=10.0, limiter=0,
                            precision=prec, synth_rtol=1e-13, synth_max_iter=300)
        e = (_rel(g["phi"], o["phi"]), _rel(g["Fx"], o["Fx"]), _rel(g["Fy"], o["Fy"]))
        _say("  precision %d: %d iterations (oracle %d), rel diff phi %.3e Fx %.3e Fy %.3e"
             % ((prec, g["n_iter"], o["n_iter"]) + e))
        if prec == 0:
            assert g["status"] == gsis.GSIS_OK
            assert e[0] < 1e-8 and e[1] < 1e-7 and e[2] < 1e-7
        else:
            assert g["final_err"] < 1e-8
            assert max(e) < 1e-5


# ------------------------------------------- transport-face HoT (Alcouffe)
@pytest.mark.parametrize("kw", [dict(limiter=1), dict(limiter=0, alsm=0), dict(order=1),
                                dict(limiter=0, precision=1)])
@pytest.mark.parametrize("shape", [(13, 9), (70, 67)])
def test_transport_face_iterates(ctx, kw, shape):
    """GSIS with the transport face fluxes in the synthetic equation (Sec.
    3.1, Eq. DSA_Alcouffe): iterates at fixed m against the oracle."""
    p = inputs.random_problem(shape[0], shape[1], seed=shape[0] + 3, sigma_range=(0.05, 50.0))
    kw = dict(kw)
    prec = kw.pop("precision", 0)
    for m in (1, 4):
        _say("transport faces %s %s m=%d precision=%d" % (shape, kw, m, prec))
        g = gsis.gsis_solve(ctx, p, method=1, hot_face=1, tol=0.0, max_iter=m, precision=prec,
                            synth_rtol=1e-15, synth_max_iter=200, **kw)
        o = oracle.solve(p, method=1, hot_face=1, tol=0.0, max_iter=m, **kw)
        tol = 1e-10 if prec == 0 else 1e-6
        assert _rel(g["phi"], o["phi"]) < tol
        assert _rel(g["Fx"], o["Fx"]) < 10 * tol and _rel(g["Fy"], o["Fy"]) < 10 * tol


def test_transport_face_reaches_si_fixed_point(ctx):
    """P7: with transport face fluxes the GSIS fixed point is the SI fixed
    point (32 x 32, S4, limiter off), to 1e-10; it matches the oracle's."""
    p = inputs.small_s4_32()
    _say("transport faces fixed point small_s4")
    t = gsis.gsis_solve(ctx, p, method=1, hot_face=1, limiter=0, tol=1e-13, max_iter=2000,
                        synth_rtol=1e-15, synth_max_iter=200)
    si = gsis.gsis_solve(ctx, p, method=0, limiter=0, tol=1e-14, max_iter=5000)
    o = oracle.solve(p, method=1, hot_face=1, limiter=0, tol=1e-13, max_iter=2000)
    assert t["status"] == gsis.GSIS_OK and o["status"] == 0
    assert abs(t["n_iter"] - o["n_iter"]) <= 2
    assert _rel(t["phi"], _np(si["phi"])) < 1e-10
    assert _rel(t["phi"], o["phi"]) < 1e-10
    assert _np(t["tres_hist"])[-1] < 1e-10


def test_transport_face_rejections(ctx):
    p = inputs.random_problem(6, 5, seed=2)
    with pytest.raises(gsis.GSISError) as e:
        gsis.Batch(ctx, [p, p], hot_face=1)
    assert e.value.status == gsis.GSIS_E_UNSUPPORTED
    with pytest.raises(gsis.GSISError) as e:
        gsis.gsis_solve(ctx, p, hot_face=1, synth_form=1)
    assert e.value.status == gsis.GSIS_E_UNSUPPORTED
    plan = gsis.Plan(ctx, p, tol=1e-10, max_iter=500, limiter=0, hot_face=1)
    plan.iterate(500)
    assert plan.status()[1] == 1
    with pytest.raises(gsis.GSISError) as e:
        plan.adjoint(np.ones(30))
    assert e.value.status == gsis.GSIS_E_UNSUPPORTED
    plan.close()
