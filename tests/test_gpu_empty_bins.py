"""Gradients at empty bins (Sec. III.C, Eq. (logL)).

A bin with n_j = 0 contributes 2 mu_j to -2lnL, so d(-2lnL)/d mu_j = 2 there
whatever mu_j is; with an empty response column and no background mu_j = 0
as well, and a form that writes the derivative as 2 (1 - n_j / mu_j) gets
0/0.  The plain, batched and template forms are compared element by element
with the FP64 oracle (its gradient is pinned against central differences on
such a problem) on a response with empty columns, zero background and zero
counts there, beside ordinary n_j = 0 bins."""
import sys

import numpy as np
import pytest

import oracle
import synth
from problems import inputs, parity_thetas

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def grad_close(got, ref):
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return np.abs(got - ref) <= 1e-4 * scale + 1e-6


@pytest.fixture(scope="module")
def empty_cols():
    import paper_2607_00488_amd as nr
    p = inputs(333, 77, 37, 200_000, 91, 92)
    R = p["R"].copy()
    cols = [0, 5, 38, 76]
    R[:, cols] = 0.0
    b = p["b"].copy()
    b[cols] = 0.0
    n = p["n"].copy()
    n[cols] = 0.0
    n[[7, 40]] = 0.0          # ordinary empty bins (mu_j > 0)
    pm = np.array([0, 0, 0, 0, 0, 1.0, 1.0])
    ps = np.array([0, 0, 0, 0, 0, 0.1, 0.1])
    o = oracle.Oracle()
    o.set_sources(p["src"], p["n_t"], 0.0, p["t_hi"])
    o.set_response(R, n_sig=p["n_sig"])
    o.set_data(n, b, pm, ps)
    ctx = nr.Context(0)
    ctx.set_sources(p["src"], p["n_t"], 0.0, p["t_hi"])
    ctx.set_response(R, n_sig=p["n_sig"])
    ctx.set_data(n, b, pm, ps)
    yield o, ctx, cols
    ctx.close()
    o.close()


def test_gradient_forms_at_empty_bins(empty_cols):
    o, ctx, cols = empty_cols
    th = parity_thetas(0, 24)
    th[:, 5:7] = synth.rng(31).uniform(0.8, 1.2, (len(th), 2))
    log(f"[gpu] empty bins {cols}: plain, batched and template gradients "
        f"over {len(th)} points")
    mu0 = o.mu(th[1])
    assert np.all(mu0[cols] == 0.0)
    nll_p, g_p = ctx.eval_nll_grad(th)
    nll_b, g_b = ctx.eval_nll_grad_batched(th)
    ctx.build_templates()
    nll_t, g_t = ctx.eval_nll_templates(th, grad=True)
    for name, v, g in (("plain", nll_p, g_p), ("batched", nll_b, g_b),
                       ("templates", nll_t, g_t)):
        assert np.all(np.isfinite(v)) and np.all(np.isfinite(g)), name
    worst = 0.0
    for i in range(len(th)):
        v, rg = o.nll_grad(th[i])
        assert np.all(np.isfinite(rg))
        for name, nl, g in (("plain", nll_p, g_p), ("batched", nll_b, g_b),
                            ("templates", nll_t, g_t)):
            assert abs(nl[i] - v) <= 1e-3, (name, i, nl[i], v)
            assert grad_close(g[i], rg).all(), (name, i, g[i], rg)
            worst = max(worst, float(np.max(np.abs(g[i] - rg))))
    log(f"[gpu] empty bins: max |d grad| {worst:.2e} over the three forms")
