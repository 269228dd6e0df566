"""Parity of the single-point HIP path (E-integral, weights, fold,
likelihood, adjoint gradient) with the FP64 oracle, through the C ABI.

Tolerances: weights are computed in FP64 on the device (1e-12 relative);
mu_j within 1e-5 relative per bin (+1e-9 of the largest bin);
|Delta(-2lnL)| <= 1e-3; gradients within 1e-4 of the larger of |g| and the
sum of the absolute per-bin contributions times 1e-3.
"""
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


@pytest.fixture(scope="module")
def cfg0():
    log("[gpu] building config-0 (512 x 256) inputs")
    p = config_inputs(0)
    ctx = gpu_context(p)
    return p, ctx


def test_sm_reference_and_row_factors(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    s_sm, m = ctx.reference()
    ref_m = o.row_factors()
    assert np.allclose(m, ref_m, rtol=1e-12, atol=1e-12 * ref_m.max())
    # the device S_SM is in its own units; its shape matches the oracle's
    so = o.spectrum(oracle.THETA_SM)
    nz = so > 0
    assert np.array_equal(s_sm > 0, nz)
    r = s_sm[nz] / so[nz]
    assert np.allclose(r, r[0], rtol=1e-12)


def test_weights_fp64_parity(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    th = parity_thetas(0, 64)
    w = ctx.eval_weights(th)
    assert np.all(w[0] == 1.0)  # theta_SM: exactly one, by construction
    for i in range(len(th)):
        ref = o.weights(th[i])
        assert np.allclose(w[i], ref, rtol=1e-12, atol=0), i


def test_mu_and_nll_parity_config0(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    th = parity_thetas(0, 1024)
    log(f"[gpu] config-0 parity over {len(th)} points")
    mu = ctx.eval_mu(th)
    nll = ctx.eval_nll(th)
    worst_mu, worst_nll = 0.0, 0.0
    for i in range(len(th)):
        ref_mu = o.mu(th[i])
        ok = mu_close(mu[i], ref_mu)
        assert ok.all(), (i, np.argmin(ok))
        worst_mu = max(worst_mu, float(np.max(np.abs(mu[i] - ref_mu) / ref_mu)))
        ref = o.nll(th[i])
        assert abs(nll[i] - ref) <= 1e-3, (i, nll[i], ref)
        worst_nll = max(worst_nll, abs(nll[i] - ref))
    log(f"[gpu] max rel dmu {worst_mu:.3e}  max |dnll| {worst_nll:.3e}")


def test_gradient_parity_config0(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    th = parity_thetas(0, 48)
    th[:, 5:7] = synth.rng(77).uniform(0.8, 1.2, (len(th), 2))
    nll, g = ctx.eval_nll_grad(th)
    for i in range(len(th)):
        v, ref = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        assert np.all(np.abs(g[i] - ref) <= 1e-4 * scale + 1e-6), (i, g[i], ref)


def test_pulls_and_grad(cfg0):
    p, _ = cfg0
    pm = np.array([0, 0, 0, 0, 0, 1.0, 1.0])
    ps = np.array([0, 0, 0, 0, 0, 0.1, 0.1])
    ctx = gpu_context(p, pulls=(pm, ps))
    o = oracle.Oracle()
    o.set_sources(p["src"], p["n_t"])
    o.set_response(p["R"], n_sig=p["n_sig"])
    o.set_data(p["n"], p["b"], pm, ps)
    th = parity_thetas(0, 8)
    th[:, 5:7] = [1.07, 0.93]
    nll, g = ctx.eval_nll_grad(th)
    for i in range(len(th)):
        v, ref = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        assert np.all(np.abs(g[i] - ref) <= 1e-4 * scale + 1e-6)


@pytest.mark.parametrize("n_t,n_reco,n_e", [(333, 77, 37), (64, 5, 8),
                                            (1000, 1023, 100), (7, 3, 3)])
def test_ragged_shapes(n_t, n_reco, n_e):
    """Sizes that are not multiples of the tiles: partial row blocks,
    column padding to 16 bytes, units with fewer than 64 nodes."""
    log(f"[gpu] ragged {n_t}x{n_reco} N_E={n_e}")
    p = inputs(n_t, n_reco, n_e, 200_000, 91, 92)
    ctx = gpu_context(p)
    o = p["oracle"]
    th = parity_thetas(0, 16)
    mu = ctx.eval_mu(th)
    nll, g = ctx.eval_nll_grad(th)
    for i in range(len(th)):
        ref_mu = o.mu(th[i])
        assert mu_close(mu[i], ref_mu).all(), i
        v, rg = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        scale = np.maximum(np.abs(rg), 1e-3 * np.abs(rg).max())
        assert np.all(np.abs(g[i] - rg) <= 1e-4 * scale + 1e-6), i


def test_zero_counts_and_infinite_nll():
    """n_j = 0 bins contribute mu_j; mu_j <= 0 under n_j > 0 gives +inf."""
    p = inputs(128, 64, 32, 100_000, 5, 6)
    n = p["n"].copy()
    n[::3] = 0.0
    import paper_2607_00488_amd as nr
    ctx = gpu_context(p)
    ctx.set_data(n, p["b"])
    o = oracle.Oracle()
    o.set_sources(p["src"], p["n_t"])
    o.set_response(p["R"], n_sig=p["n_sig"])
    o.set_data(n, p["b"])
    th = parity_thetas(0, 4)
    got = ctx.eval_nll(th)
    for i in range(len(th)):
        assert abs(got[i] - o.nll(th[i])) <= 1e-3
    bad = synth.theta_sm().copy()
    bad[6] = -100.0
    assert ctx.eval_nll(bad)[0] == math.inf
    assert o.nll(bad) == math.inf


def test_deterministic_and_graph_replay(cfg0):
    """Repeated evaluations are bitwise equal (no float atomics), also when
    a cached HIP graph is replayed with eager work in between."""
    import torch
    p, ctx = cfg0
    th = parity_thetas(0, 32)
    a = ctx.eval_nll(th)
    b = ctx.eval_nll(th)
    assert np.array_equal(a, b)
    dev = torch.device("cuda:0")
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    out = torch.empty(len(th), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    ref = None
    for rep in range(4):
        ctx.eval_nll_dev(tt, out, stream=s)
        s.synchronize()
        got = out.cpu().numpy().copy()
        if ref is None:
            ref = got
            assert np.array_equal(got, a)
        assert np.array_equal(got, ref), rep
        x = torch.randn(1 << 20, device=dev)
        (x * 2).sum().item()  # unrelated eager work between replays


def test_error_codes(cfg0):
    import paper_2607_00488_amd as nr
    p, ctx = cfg0
    bad = synth.theta_sm().copy()
    bad[0] = float("nan")
    with pytest.raises(nr.NrError) as e:
        ctx.eval_nll(bad)
    assert e.value.code == nr.NR_EINVAL
    fresh = nr.Context(0)
    with pytest.raises(nr.NrError) as e:
        fresh.eval_nll(synth.theta_sm())
    assert e.value.code == nr.NR_ESTATE
    with pytest.raises(nr.NrError) as e:
        fresh.set_response(p["R"])  # m = NULL needs the sources first
    assert e.value.code == nr.NR_ESTATE
    fresh.set_sources(p["src"], p["n_t"])
    with pytest.raises(nr.NrError) as e:
        fresh.set_response(p["R"][:-1])  # n_t mismatch
    assert e.value.code == nr.NR_EINVAL
    fresh.set_response(p["R"])
    neg = p["n"].copy()
    neg[3] = -1
    with pytest.raises(nr.NrError) as e:
        fresh.set_data(neg, p["b"])
    assert e.value.code == nr.NR_EINVAL
    with pytest.raises(nr.NrError) as e:
        fresh.set_data(p["n"][:-2], p["b"][:-2])
    assert e.value.code == nr.NR_EINVAL
    # set_* copies: the caller's arrays may change afterwards
    n = p["n"].copy()
    fresh.set_data(n, p["b"])
    v0 = fresh.eval_nll(synth.theta_sm())[0]
    n[:] = 0
    assert fresh.eval_nll(synth.theta_sm())[0] == v0


def test_user_row_factors(cfg0):
    """A caller-given m (joint-histogram style response) is used as is."""
    p, _ = cfg0
    m = synth.rng(4).uniform(0.5, 2.0, p["n_t"])
    import paper_2607_00488_amd as nr
    ctx = nr.Context(0)
    ctx.set_sources(p["src"], p["n_t"])
    ctx.set_response(p["R"], m=m)
    ctx.set_data(p["n"], p["b"])
    o = oracle.Oracle()
    o.set_sources(p["src"], p["n_t"])
    o.set_response(p["R"], m=m)
    o.set_data(p["n"], p["b"])
    th = parity_thetas(0, 8)
    mu = ctx.eval_mu(th)
    for i in range(len(th)):
        assert mu_close(mu[i], o.mu(th[i])).all()
