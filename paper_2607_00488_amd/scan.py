"""Profile-likelihood scans with injected signals (the paper's Asimov
demonstration, Sec. VI.B): a parameter of interest is stepped over a grid,
the nuisance parameters are minimised at every grid value by the batched
L-BFGS driver (all grid values advance together, one batched likelihood and
gradient call per line-search trial), and the profile Delta(-2lnL) is read
against the chi-square quantile of the requested confidence level.  Only
buffers and calls: every likelihood and gradient comes from the library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Context
from .autograd import lbfgs_fit

# 90 % quantile of the chi-square distribution with one degree of freedom
CHI2_1DOF_90 = 2.705543454095404


def profile_scan(context: Context, index: int, values, base,
                 free=(5, 6), iters: int = 200, gtol: float = 1e-6,
                 lower=None, form="batched"):
    """-2lnL profiled over the parameters ``free`` at every value of
    parameter ``index`` (the others stay at ``base``).  ``lower`` optionally
    clamps the grid from below (a physical boundary such as m2 >= 0).
    ``form``: the likelihood form the fits call ("batched", "plain",
    "templates").

    Returns a dict with the grid, the profiled -2lnL, Delta(-2lnL) from the
    grid minimum, the fitted nuisances and the gradient norms."""
    values = np.asarray(values, dtype=np.float64)
    if lower is not None:
        values = np.maximum(values, lower)
    th0 = np.repeat(np.asarray(base, dtype=np.float64)[None], len(values), 0)
    th0[:, index] = values
    dev = torch.device(f"cuda:{context.device}")
    x, f, gn, calls = lbfgs_fit(context, torch.tensor(th0, device=dev),
                                iters=iters, gtol=gtol, free=free, form=form)
    f = f.cpu().numpy()
    d = f - f.min()
    return dict(values=values, nll=f, delta=d, theta=x.cpu().numpy(),
                grad_norm=gn.cpu().numpy(), calls=calls)


def interval(values, delta, level=CHI2_1DOF_90):
    """The set {v : Delta(v) <= level} of a scan as [lo, hi], with the
    crossings linearly interpolated between grid values; an end of the grid
    that stays below the level is returned as that end."""
    v = np.asarray(values, dtype=np.float64)
    d = np.asarray(delta, dtype=np.float64)
    i0 = int(np.argmin(d))
    lo, hi = v[0], v[-1]
    for i in range(i0, 0, -1):
        if d[i - 1] > level >= d[i]:
            t = (level - d[i]) / (d[i - 1] - d[i])
            lo = v[i] + t * (v[i - 1] - v[i])
            break
    for i in range(i0, len(v) - 1):
        if d[i + 1] > level >= d[i]:
            t = (level - d[i]) / (d[i + 1] - d[i])
            hi = v[i] + t * (v[i + 1] - v[i])
            break
    return float(lo), float(hi)
