"""-2lnL as a differentiable torch function, and a batched L-BFGS fit.

The forward and the backward both come from the library's kernels: one call
computes -2lnL and its gradient (the adjoint of the fold); the gradient is
kept for ``backward``.  Nothing here computes any part of the likelihood.
"""
from __future__ import annotations

import torch

from . import Context, eval_nll_multi_dev


FORMS = ("batched", "plain", "templates")


def _form(form) -> str:
    """True / False select the batched / plain form (the older boolean
    switch); the names of FORMS select themselves."""
    if form is True:
        return "batched"
    if form is False:
        return "plain"
    if form not in FORMS:
        raise ValueError(f"form must be one of {FORMS}, got {form!r}")
    return form


def _buffers(context: Context, P: int, dev, form: str):
    """Fixed input/output buffers per (context, P, form): the library then
    replays one cached graph for every call of a fit."""
    cache = context.__dict__.setdefault("_autograd_bufs", {})
    key = (P, str(dev), form)
    b = cache.get(key)
    if b is None:
        D = context.n_theta
        b = (torch.empty(P, D, dtype=torch.float64, device=dev),
             torch.empty(P, dtype=torch.float64, device=dev),
             torch.empty(P, D, dtype=torch.float64, device=dev))
        cache[key] = b
    return b


class NllFunction(torch.autograd.Function):
    """nll[p] = -2lnL(theta[p]) for theta [P, n_theta] float64 on the
    context's device (n_theta = 7, or 5 + K + B for a multi-component
    context, which only the template form takes).  ``form``: "batched" (the GEMM form, many points at once; also
    True), "plain" (P single-point evaluations; also False) or "templates"
    (the folded-template form)."""

    @staticmethod
    def forward(fctx, theta: torch.Tensor, context: Context, form="batched"):
        form = _form(form)
        P = theta.shape[0]
        th, nll, grad = _buffers(context, P, theta.device, form)
        th.copy_(theta.detach())
        stream = torch.cuda.current_stream(th.device)
        if form == "batched":
            eval_nll_multi_dev([context], [th], [nll], [grad], stream=stream)
        elif form == "templates":
            context.eval_nll_templates_dev(th, nll, grad, stream=stream)
        else:
            context.eval_nll_dev(th, nll, grad, stream=stream)
        out, g = nll.clone(), grad.clone()
        fctx.save_for_backward(g)
        return out

    @staticmethod
    def backward(fctx, g):
        (grad,) = fctx.saved_tensors
        return g[:, None].to(grad.dtype) * grad, None, None


def nll(theta: torch.Tensor, context: Context, form="batched"):
    return NllFunction.apply(theta, context, form)


def lbfgs_fit(context: Context, theta0: torch.Tensor, iters: int = 100,
              history: int = 10, gtol: float = 1e-5, form="batched",
              free=None):
    """Independent L-BFGS minimisations of -2lnL from every row of theta0
    ([S, 7]), advanced together: one batched likelihood+gradient call per
    line-search trial for all starts.  Two-loop recursion per start and a
    backtracking Armijo line search per start, whose sufficient-decrease
    test allows for the FP64 rounding noise of -2lnL (1e-12 |f|).  ``free``: the indices of the
    parameters that move (default all seven); the others keep the values
    theta0 gives them.  ``form``: as for ``nll``.

    Returns (theta_min [S, 7], nll_min [S], grad_norm [S], n_calls); the
    gradient norm is over the free parameters.
    """
    form = _form(form)
    x = theta0.detach().to(torch.float64).clone()
    S, D = x.shape
    dev = x.device
    mask = torch.ones(D, dtype=torch.float64, device=dev)
    if free is not None:
        mask.zero_()
        mask[list(free)] = 1.0

    def fg(th):
        t = th.detach().clone().requires_grad_(True)
        v = nll(t, context, form)
        v.sum().backward()
        return v.detach(), t.grad.detach() * mask

    f, g = fg(x)
    calls = 1
    s_hist = torch.zeros(history, S, D, dtype=torch.float64, device=dev)
    y_hist = torch.zeros_like(s_hist)
    rho = torch.zeros(history, S, dtype=torch.float64, device=dev)
    valid = torch.zeros(history, S, dtype=torch.bool, device=dev)
    head = 0
    done = g.norm(dim=1) <= gtol
    for _ in range(iters):
        if bool(done.all()):
            break
        # two-loop recursion, per start
        q = g.clone()
        alpha = torch.zeros(history, S, dtype=torch.float64, device=dev)
        order = [(head - 1 - i) % history for i in range(history)]
        for k in order:
            a = rho[k] * (s_hist[k] * q).sum(1)
            a = torch.where(valid[k], a, torch.zeros_like(a))
            alpha[k] = a
            q = q - a[:, None] * y_hist[k]
        last = (head - 1) % history
        sy = (s_hist[last] * y_hist[last]).sum(1)
        yy = (y_hist[last] * y_hist[last]).sum(1)
        gamma = torch.where(valid[last] & (yy > 0), sy / yy.clamp_min(1e-300),
                            torch.ones_like(sy))
        r = gamma[:, None] * q
        for k in reversed(order):
            b = rho[k] * (y_hist[k] * r).sum(1)
            b = torch.where(valid[k], b, torch.zeros_like(b))
            r = r + (alpha[k] - b)[:, None] * s_hist[k]
        d = -r
        slope = (d * g).sum(1)
        bad = ~(slope < 0)
        d = torch.where(bad[:, None], -g, d)
        slope = torch.where(bad, -(g * g).sum(1), slope)
        # first iteration without curvature: a unit-length step at most
        step = torch.ones(S, dtype=torch.float64, device=dev)
        first = ~valid.any(0)
        dn = d.norm(dim=1).clamp_min(1e-300)
        step = torch.where(first, torch.clamp(1e-2 / dn, max=1.0), step)
        accepted = done.clone()
        x_new, f_new, g_new = x.clone(), f.clone(), g.clone()
        for _ls in range(30):
            trial = x + (step * (~accepted))[:, None] * d
            ft, gt = fg(torch.where(accepted[:, None], x_new, trial))
            calls += 1
            # sufficient decrease, up to the rounding noise of -2lnL itself
            # (about 1e-13 |f| in FP64 over thousands of bins): near a
            # minimum the decrease the test asks for falls below that
            # noise, and without the allowance line searches fail by chance
            ok = ((ft <= f + 1e-4 * step * slope + 1e-12 * f.abs().clamp_min(1.0))
                  & torch.isfinite(ft) & ~accepted)
            x_new = torch.where(ok[:, None], trial, x_new)
            f_new = torch.where(ok, ft, f_new)
            g_new = torch.where(ok[:, None], gt, g_new)
            accepted = accepted | ok
            if bool(accepted.all()):
                break
            step = torch.where(accepted, step, step * 0.5)
        moved = accepted & ~done
        s = x_new - x
        yv = g_new - g
        sy = (s * yv).sum(1)
        keep = moved & (sy > 1e-12 * s.norm(dim=1) * yv.norm(dim=1))
        s_hist[head] = torch.where(keep[:, None], s, torch.zeros_like(s))
        y_hist[head] = torch.where(keep[:, None], yv, torch.zeros_like(yv))
        rho[head] = torch.where(keep, 1.0 / sy.clamp_min(1e-300),
                                torch.zeros_like(sy))
        valid[head] = keep
        head = (head + 1) % history
        x, f, g = x_new, f_new, g_new
        stalled = ~accepted
        done = done | (g.norm(dim=1) <= gtol) | stalled
    return x, f, g.norm(dim=1), calls
