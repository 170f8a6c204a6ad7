"""Adjoint through the C-ABI: gradients of the GSIS / SI fixed point against
the FP64 oracle's adjoint (element by element) and against central
differences of the GPU forward solve, and the torch.autograd.Function."""
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


def _rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _cot(N, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0, 1, N), rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)


def _gpu_adjoint(ctx, p, g, adj_tol=1e-13, **kw):
    plan = gsis.Plan(ctx, p, tol=1e-13, max_iter=3000, synth_rtol=1e-13, synth_max_iter=200,
                     limiter=0, **kw)
    plan.iterate(3000)
    n, conv, err = plan.status()
    assert conv == 1
    out = plan.adjoint(*g, tol=adj_tol, max_iter=3000)
    plan.close()
    return out


@pytest.mark.parametrize("kw", [dict(method=1), dict(method=0), dict(method=1, alsm=0),
                                dict(method=1, order=1)])
@pytest.mark.parametrize("shape", [(4, 5), (23, 17)])
def test_adjoint_matches_oracle(ctx, kw, shape):
    p = inputs.random_problem(shape[0], shape[1], seed=shape[0] + 1, sigma_range=(0.5, 5.0))
    g = _cot(shape[0] * shape[1], 7)
    _say("adjoint %s %s" % (shape, kw))
    ga, gs, gq, info = _gpu_adjoint(ctx, p, g, **kw)
    assert info["status"] == gsis.GSIS_OK
    r = oracle.solve(p, tol=1e-14, max_iter=5000, limiter=0, return_I=True, **kw)
    o = oracle.adjoint(p, r["I"], *g, tol=1e-14, limiter=0, **kw)
    assert o["status"] == 0
    assert _rel(ga, o["g_sigma_a"]) < 1e-9
    assert _rel(gs, o["g_sigma_s"]) < 1e-9
    assert _rel(gq, o["g_q"]) < 1e-9


@pytest.mark.parametrize("parts", ["1", None])
def test_adjoint_tall_strip_against_oracle(ctx, parts, monkeypatch):
    """A 3 x 1100 strip: more than 1024 rows per ordinate, so with one
    workgroup per ordinate the adjoint sweep takes its two-pass form; by
    default its rows are spread over four workgroups. The adjoint iteration
    of this strip levels off near 1e-13, so both sides stop at 1e-12."""
    if parts is None:
        monkeypatch.delenv("GSIS_CHAIN_PARTS", raising=False)
    else:
        monkeypatch.setenv("GSIS_CHAIN_PARTS", parts)
    p = inputs.random_problem(3, 1100, seed=4, sigma_range=(0.5, 5.0))
    g = _cot(3 * 1100, 7)
    _say("adjoint strip 3 x 1100 parts=%s" % parts)
    ga, gs, gq, info = _gpu_adjoint(ctx, p, g, adj_tol=1e-12, method=1)
    assert info["status"] == gsis.GSIS_OK
    r = oracle.solve(p, tol=1e-14, max_iter=5000, limiter=0, return_I=True, method=1)
    o = oracle.adjoint(p, r["I"], *g, tol=1e-12, max_iter=5000, limiter=0, method=1)
    assert o["status"] == 0
    assert _rel(ga, o["g_sigma_a"]) < 1e-8
    assert _rel(gs, o["g_sigma_s"]) < 1e-8
    assert _rel(gq, o["g_q"]) < 1e-8


def test_adjoint_two_region_against_oracle(ctx):
    """The noisy two-region medium at 128 x 128, K = 32 (resolved enough for
    plain GSIS to converge), with the detector objective
    J = sum_W V sigma_a phi (cotangent V sigma_a on W)."""
    p = inputs.noisy_thick_square(128, inputs.quad_product(2, 16))
    W = inputs.detector_window(128)
    V = p["dx"] * p["dy"]
    gphi = np.where(W, V * p["sigma_a"], 0.0)
    _say("adjoint two-region 64")
    ga, gs, gq, info = _gpu_adjoint(ctx, p, (gphi, None, None))
    r = oracle.solve(p, tol=1e-14, max_iter=5000, limiter=0, return_I=True)
    o = oracle.adjoint(p, r["I"], gphi, tol=1e-14, limiter=0)
    assert _rel(ga, o["g_sigma_a"]) < 1e-9 and _rel(gs, o["g_sigma_s"]) < 1e-9


def test_adjoint_full_size_against_central_differences(ctx):
    """512 x 512 x 128 noisy two-region medium, detector objective:
    dJ/dsigma at 16 sampled cells (4 in the window, 4 on the thick square's
    east edge, 4 between, 4 anywhere; seed 55) against central differences of
    GPU forward solves converged to Err < 1e-14 (h = 1e-3 relative), to 1e-6
    of the gradient's largest value. The differences carry the forward
    solves' rounding over h, about 1e-8 of J per unit relative step, which
    sets their floor (measured: at most 1.8e-7 of the largest gradient over
    the 32 values; the window cells agree to 1e-8 of themselves, while a cell
    whose gradient is 1e-5 of the largest can only be checked against that
    floor)."""
    import torch
    n = 512
    p = inputs.noisy_thick_square(n)
    W = inputs.detector_window(n)
    V = p["dx"] * p["dy"]
    dev = torch.device("cuda:0")
    pd = {k: (torch.from_numpy(v).to(dev) if isinstance(v, np.ndarray) else v)
          for k, v in p.items()}
    Wt = torch.from_numpy(W).to(dev)

    def J(sa, ss):
        q = dict(pd, sigma_a=sa, sigma_s=ss)
        r = gsis.gsis_solve(ctx, q, tol=1e-14, max_iter=3000, limiter=0, synth_rtol=1e-12)
        assert r["status"] == 0
        return float((V * sa * r["phi"] * Wt).sum())
    gphi = torch.where(Wt, V * pd["sigma_a"], torch.zeros_like(pd["sigma_a"]))
    _say("full-size adjoint")
    plan = gsis.Plan(ctx, pd, tol=1e-14, max_iter=3000, limiter=0, synth_rtol=1e-12)
    plan.iterate(3000)
    assert plan.status()[1] == 1
    phi = plan.read()["phi"]
    ga, gs, gq, info = plan.adjoint(gphi, tol=1e-13, max_iter=3000)
    plan.close()
    ga = ga + torch.where(Wt, V * phi, torch.zeros_like(phi))   # explicit part of J
    cells = inputs.adjoint_fd_cells(n)
    _say("  sampled cells %s" % list(cells))
    for name, grad in (("sigma_a", ga), ("sigma_s", gs)):
        for c in cells:
            h = 1e-3 * float(pd[name][c])
            plus = pd[name].clone(); plus[c] += h
            minus = pd[name].clone(); minus[c] -= h
            args_p = (plus, pd["sigma_s"]) if name == "sigma_a" else (pd["sigma_a"], plus)
            args_m = (minus, pd["sigma_s"]) if name == "sigma_a" else (pd["sigma_a"], minus)
            fd = (J(*args_p) - J(*args_m)) / (2 * h)
            g = float(grad[c])
            _say("  %s cell %d fd %.9e adjoint %.9e" % (name, c, fd, g))
            assert abs(fd - g) <= 1e-6 * float(grad.abs().max())


def test_autograd_function(ctx):
    import torch
    from paper_2507_03975_amd.autograd import gsis_fixed_point
    p = inputs.random_problem(12, 9, seed=5, sigma_range=(0.5, 5.0))
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    static = dict(nx=p["nx"], ny=p["ny"], dx=p["dx"], dy=p["dy"], mu=t(p["mu"]), eta=t(p["eta"]),
                  w=t(p["w"]), bnd_in=t(p["bnd_in"]),
                  options=dict(tol=1e-13, synth_rtol=1e-13, synth_max_iter=200))
    sa = t(p["sigma_a"]).requires_grad_(True)
    ss = t(p["sigma_s"]).requires_grad_(True)
    q = t(p["q"]).requires_grad_(True)
    phi, fx, fy = gsis_fixed_point(sa, ss, q, static)
    loss = (sa * phi).sum() + (fx ** 2).sum()       # explicit sa dependence stays in torch
    loss.backward()
    r = oracle.solve(p, tol=1e-14, max_iter=5000, limiter=0, return_I=True)
    o = oracle.adjoint(p, r["I"], p["sigma_a"], 2 * r["Fx"], None, tol=1e-14, limiter=0)
    want_sa = o["g_sigma_a"] + r["phi"]
    assert _rel(sa.grad, want_sa) < 1e-8
    assert _rel(ss.grad, o["g_sigma_s"]) < 1e-8
    assert _rel(q.grad, o["g_q"]) < 1e-8


def test_adjoint_split_sweep_bitwise(ctx, monkeypatch):
    """The downstream-first sweep with an ordinate's rows spread over 2, 3
    or 4 workgroups gives the same gradients, bit for bit, as one workgroup
    per ordinate (40 x 300 cells, 16 ordinates: 192/108, 128/128/44 and
    128/128/44 rows, 4 parts falling back to 3)."""
    p = inputs.random_problem(40, 300, quad=inputs.quad_product(2, 8), seed=9,
                              sigma_range=(0.5, 5.0))
    g = _cot(40 * 300, 3)
    out = {}
    for parts in ("1", "2", "3", "4"):
        monkeypatch.setenv("GSIS_CHAIN_PARTS", parts)
        _say("adjoint split sweep parts=%s" % parts)
        out[parts] = _gpu_adjoint(ctx, p, g, adj_tol=1e-10, method=1)
        assert out[parts][3]["status"] == gsis.GSIS_OK
    for parts in ("2", "3", "4"):
        for t in range(3):
            assert np.array_equal(np.asarray(out["1"][t]), np.asarray(out[parts][t])), (parts, t)
