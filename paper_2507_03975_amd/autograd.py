"""torch.autograd.Function over the GSIS fixed point.

``GSISFunction.apply(sigma_a, sigma_s, q, static)`` runs the HIP forward
solve on the tensors' device (a plan, iterated until Err < tol) and returns
(phi, Fx, Fy); ``backward`` calls the hand-written adjoint of that plan
(gsis_plan_adjoint) with the incoming cotangents and returns dL/dsigma_a,
dL/dsigma_s, dL/dq. ``static`` holds the rest of the problem (nx, ny, dx,
dy, mu, eta, w, optional bnd_in as CUDA tensors) and the solver options
(limiter must be 0). Any explicit dependence of a loss on the parameters
stays with torch autograd.
"""
import torch

from . import gsis

__all__ = ["GSISFunction", "gsis_fixed_point"]

_ctx = {}


def _context(device):
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _ctx:
        _ctx[idx] = gsis.Context(idx)
    return _ctx[idx]


class GSISFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma_a, sigma_s, q, static):
        opts = dict(static.get("options", {}))
        opts.setdefault("limiter", 0)
        opts.setdefault("tol", 1e-10)
        opts.setdefault("max_iter", 2000)
        adj_tol = opts.pop("adjoint_tol", opts["tol"])
        prob = {k: static[k] for k in ("nx", "ny", "dx", "dy", "mu", "eta", "w")}
        prob["bnd_in"] = static.get("bnd_in")
        prob["sigma_a"], prob["sigma_s"], prob["q"] = (t.detach() for t in (sigma_a, sigma_s, q))
        plan = gsis.Plan(_context(sigma_a.device), prob, **opts)
        done = 0
        while True:
            plan.iterate(16)
            n, conv, err = plan.status()
            if conv != 0 or n >= opts["max_iter"]:
                break
        if conv != 1:
            plan.close()
            raise gsis.GSISError(gsis.GSIS_NOT_CONVERGED,
                                 "forward solve stopped at Err %.3g after %d iterations"
                                 % (err, n))
        r = plan.read()
        ctx.plan = plan
        ctx.adj = (adj_tol, opts["max_iter"])
        return r["phi"], r["Fx"], r["Fy"]

    @staticmethod
    def backward(ctx, g_phi, g_Fx, g_Fy):
        plan = ctx.plan
        tol, max_iter = ctx.adj
        ga, gs, gq, info = plan.adjoint(g_phi, g_Fx, g_Fy, tol=tol, max_iter=max_iter)
        plan.close()
        ctx.plan = None
        return ga, gs, gq, None


def gsis_fixed_point(sigma_a, sigma_s, q, static):
    """Differentiable (phi, Fx, Fy) of the GSIS fixed point."""
    return GSISFunction.apply(sigma_a, sigma_s, q, static)
