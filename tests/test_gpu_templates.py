"""Parity of the template form (basis templates folded once through R, then
21 products and a logarithm per bin and point) with the FP64 oracle: spectra,
-2lnL and gradients at the parity sizes, ragged shapes and point counts,
empty bins and mu <= 0, invalidation by set_data / set_response and graph
replay (the multi-component form is tested with the other multi-component
paths)."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from problems import config_inputs, gpu_context, inputs, parity_thetas

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mu_close(got, ref):
    tol = 1e-5 * np.abs(ref) + 1e-9 * np.abs(ref).max()
    return np.abs(got - ref) <= tol


def grad_close(got, ref):
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return np.abs(got - ref) <= 1e-4 * scale + 1e-6


PULLS = ([0, 0, 0, 0, 0, 1.0, 1.0], [0, 0, 0, 0, 0, 0.1, 0.1])


@pytest.fixture(scope="module")
def cfg0():
    """Config-0 analysis with nuisance pulls, on the GPU and on an oracle of
    its own (the shared one keeps its pull-free data)."""
    p = config_inputs(0)
    o = oracle.Oracle()
    o.set_sources(p["src"], p["n_t"])
    o.set_response(p["R"], n_sig=p["n_sig"])
    o.set_data(p["n"], p["b"], *PULLS)
    yield dict(p, oracle=o), gpu_context(p, pulls=PULLS)
    o.close()


def test_templates_config0_against_oracle(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    th = parity_thetas(0, 1024)
    th[:, 5:7] = synth.rng(21).uniform(0.8, 1.2, (len(th), 2))
    log(f"[gpu] templates config-0 over {len(th)} points")
    ctx.build_templates()
    nll = ctx.eval_nll_templates(th)
    nll_g, g = ctx.eval_nll_templates(th, grad=True)
    assert np.array_equal(nll, nll_g)
    mu = ctx.eval_mu_templates(th[::16])
    worst = worst_mu = 0.0
    for i in range(len(th)):
        ref = o.nll(th[i])
        assert abs(nll[i] - ref) <= 1e-3, (i, nll[i], ref)
        worst = max(worst, abs(nll[i] - ref))
    for k, i in enumerate(range(0, len(th), 16)):
        ref_mu = o.mu(th[i])
        ok = mu_close(mu[k], ref_mu)
        assert ok.all(), (i, int(np.argmin(ok)))
        worst_mu = max(worst_mu, float(np.max(np.abs(mu[k] - ref_mu) / ref_mu)))
    for i in range(0, len(th), 32):
        v, rg = o.nll_grad(th[i])
        assert grad_close(g[i], rg).all(), (i, g[i], rg)
    # the same quantities as the plain and batched forms
    assert np.max(np.abs(nll - ctx.eval_nll(th))) <= 1e-3
    assert np.max(np.abs(nll - ctx.eval_nll_batched(th))) <= 1e-3
    log(f"[gpu] templates max |dnll| {worst:.3e}, max rel dmu {worst_mu:.3e}")


@pytest.mark.parametrize("n_t,n_reco,n_e", [(333, 77, 37), (64, 5, 8),
                                            (1000, 1023, 100), (7, 3, 3),
                                            (600, 2000, 24)])
def test_templates_ragged_shapes(n_t, n_reco, n_e):
    """Row counts that are not multiples of the template slab, bin counts
    that are not multiples of the column slices, rows beyond every
    kinematic reach (w := 1)."""
    log(f"[gpu] templates ragged {n_t}x{n_reco} N_E={n_e}")
    p = inputs(n_t, n_reco, n_e, 200_000, 91, 92)
    ctx = gpu_context(p)
    o = p["oracle"]
    th = parity_thetas(0, 16)
    mu = ctx.eval_mu_templates(th)
    nll, g = ctx.eval_nll_templates(th, grad=True)
    for i in range(len(th)):
        assert mu_close(mu[i], o.mu(th[i])).all(), i
        v, rg = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        assert grad_close(g[i], rg).all(), i


@pytest.mark.parametrize("n_pts", [1, 63, 65, 1000, 5000])
def test_templates_point_counts(cfg0, n_pts):
    """Point counts around the 64-lane work-group and across the choice of
    column slices."""
    p, ctx = cfg0
    th = synth.theta_prior(n_pts, 700 + n_pts, f_range=(0.8, 1.2))
    nll, g = ctx.eval_nll_templates(th, grad=True)
    assert np.all(np.isfinite(nll)) and np.all(np.isfinite(g))
    o = p["oracle"]
    for i in sorted({0, n_pts // 2, n_pts - 1}):
        v, rg = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        assert grad_close(g[i], rg).all()


def test_templates_zero_counts_infinite_and_invalidation():
    """n_j = 0 bins contribute mu_j, mu_j <= 0 under n_j > 0 gives +inf,
    and new data or a new response is picked up (templates refolded)."""
    p = inputs(128, 64, 32, 100_000, 5, 6)
    ctx = gpu_context(p)
    th = parity_thetas(0, 4)
    first = ctx.eval_nll_templates(th)
    n = p["n"].copy()
    n[::3] = 0.0
    ctx.set_data(n, p["b"])
    o = oracle.Oracle()
    o.set_sources(p["src"], p["n_t"])
    o.set_response(p["R"], n_sig=p["n_sig"])
    o.set_data(n, p["b"])
    got = ctx.eval_nll_templates(th)
    assert not np.allclose(got, first)
    for i in range(len(th)):
        assert abs(got[i] - o.nll(th[i])) <= 1e-3
    bad = synth.theta_sm().copy()
    bad[6] = -100.0
    assert ctx.eval_nll_templates(bad)[0] == math.inf
    # a different response: the templates follow it
    R2 = p["R"][:, ::-1].copy()
    ctx.set_response(R2, n_sig=p["n_sig"])
    o.set_response(R2, n_sig=p["n_sig"])
    got = ctx.eval_nll_templates(th)
    for i in range(len(th)):
        assert abs(got[i] - o.nll(th[i])) <= 1e-3


def test_templates_device_path_and_graph_replay(cfg0):
    """The device-pointer entry on a torch stream, eagerly and captured in
    a torch CUDA graph replayed with eager work in between; every replay
    bitwise equal to the host entry."""
    import torch
    p, ctx = cfg0
    dev = torch.device("cuda:0")
    th = synth.theta_prior(300, 811, f_range=(0.8, 1.2))
    ref, gref = ctx.eval_nll_templates(th, grad=True)
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    out = torch.empty(len(th), dtype=torch.float64, device=dev)
    gr = torch.empty(len(th), 7, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    ctx.build_templates()
    ctx.eval_nll_templates_dev(tt, out, gr, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(gr.cpu().numpy(), gref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ctx.eval_nll_templates_dev(tt, out, gr, stream=s)
    for rep in range(3):
        out.zero_()
        gr.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
        assert np.array_equal(gr.cpu().numpy(), gref), rep
        x = torch.randn(1 << 20, device=dev)
        (x * 2).sum().item()
