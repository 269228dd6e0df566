"""Parity of the batched (FP64-MFMA GEMM) path with the FP64 oracle and with
the single-point path: one analysis, several analyses of uneven binning in
one grouped launch (also at the largest shapes of the 64-dataset scan), the
batched gradient, and graph replays."""
import sys

import numpy as np
import pytest

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
    p = config_inputs(0)
    return p, gpu_context(p)


def test_batched_mu_and_nll_config0(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    th = parity_thetas(0, 1024)
    log(f"[gpu] batched config-0 over {len(th)} points")
    mu = ctx.eval_mu_batched(th)
    nll = ctx.eval_nll_batched(th)
    plain = ctx.eval_nll(th)
    worst_mu = worst = 0.0
    for i in range(len(th)):
        ref_mu = o.mu(th[i])
        ok = mu_close(mu[i], ref_mu)
        assert ok.all(), (i, int(np.argmin(ok)))
        worst_mu = max(worst_mu, float(np.max(np.abs(mu[i] - ref_mu) / ref_mu)))
        ref = o.nll(th[i])
        assert abs(nll[i] - ref) <= 1e-3, (i, nll[i], ref)
        worst = max(worst, abs(nll[i] - ref))
    assert np.max(np.abs(nll - plain)) <= 1e-3
    log(f"[gpu] batched max rel dmu {worst_mu:.3e}, max |dnll| {worst:.3e}")


def test_batched_gradient_config0(cfg0):
    p, ctx = cfg0
    o = p["oracle"]
    th = parity_thetas(0, 64)
    th[:, 5:7] = synth.rng(3).uniform(0.8, 1.2, (len(th), 2))
    nll, g = ctx.eval_nll_grad_batched(th)
    for i in range(len(th)):
        v, ref = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        assert np.all(np.abs(g[i] - ref) <= 1e-4 * scale + 1e-6), (i, g[i], ref)


@pytest.mark.parametrize("n_t", [2047, 3001, 3002])
def test_gradient_contraction_chunks(n_t):
    """The gradient's contraction over response rows runs in chunks of 1024
    rows once there are at least 2048, the last chunk taking the remainder:
    2047 rows finish in one chunk, 3001 in two (1024 and 1977 rows, not a
    multiple of the 16-row steps).  With an even row count (3002) the rows
    are read in 16-byte pairs, and the last chunk ends in part of a group
    of four rows, which is read row by row.  Against the oracle's analytic
    gradient, and against the single-point path's adjoint (other code) on
    every point."""
    p = inputs(n_t, 200, 48, 300_000, 7401 + n_t, 7402 + n_t)
    ctx = gpu_context(p)
    o = p["oracle"]
    th = synth.theta_prior(37, 7403)
    th[:, 5:7] = synth.rng(7404).uniform(0.8, 1.2, (len(th), 2))
    log(f"[gpu] batched gradient contraction, {n_t} rows")
    nll, g = ctx.eval_nll_grad_batched(th)
    for i in (0, 13, 36):
        v, ref = o.nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        assert np.all(np.abs(g[i] - ref) <= 1e-4 * scale + 1e-6), (i, g[i], ref)
    _, gp = ctx.eval_nll_grad(th)
    scale = np.maximum(np.abs(gp), 1e-6 * np.abs(gp).max())
    assert np.all(np.abs(g - gp) <= 1e-9 * scale), np.max(np.abs(g - gp) / scale)
    ctx.close()


SHAPES = [  # n_t, n_reco, n_e, n_pts: tile edges in every dimension
    (256, 128, 64, 128),
    (300, 77, 40, 131),
    (512, 256, 32, 64),
    (130, 300, 16, 7),
    (2048, 512, 48, 257),
    (64, 1, 8, 3),
]


@pytest.fixture(scope="module")
def multi():
    probs, ctxs, ths = [], [], []
    for d, (n_t, n_reco, n_e, P) in enumerate(SHAPES):
        p = inputs(n_t, n_reco, n_e, 100_000, 500 + d, 600 + d)
        probs.append(p)
        ctxs.append(gpu_context(p))
        ths.append(synth.theta_prior(P, 700 + d))
    return probs, ctxs, ths


def test_grouped_uneven_datasets(multi):
    import paper_2607_00488_amd as nr
    probs, ctxs, ths = multi
    log(f"[gpu] grouped launch over {len(ctxs)} datasets")
    outs = nr.eval_nll_multi(ctxs, ths)
    for d, (p, th, out) in enumerate(zip(probs, ths, outs)):
        o = p["oracle"]
        for i in range(0, len(th), max(1, len(th) // 16)):
            ref = o.nll(th[i])
            assert abs(out[i] - ref) <= 1e-3, (d, i, out[i], ref)
        single = ctxs[d].eval_nll_batched(th)
        assert np.max(np.abs(single - out)) <= 1e-9 * np.abs(out).max()


def test_grouped_graph_replay_and_grad(multi):
    """Device-pointer grouped launch, replayed as a cached graph with eager
    work in between; every replay equals the first; gradients match."""
    import torch
    import paper_2607_00488_amd as nr
    probs, ctxs, ths = multi
    dev = torch.device("cuda:0")
    tt = [torch.tensor(t, dtype=torch.float64, device=dev) for t in ths]
    nl = [torch.empty(len(t), dtype=torch.float64, device=dev) for t in ths]
    gr = [torch.empty(len(t), 7, dtype=torch.float64, device=dev) for t in ths]
    s = torch.cuda.Stream(device=dev)
    ref = None
    for rep in range(3):
        nr.eval_nll_multi_dev(ctxs, tt, nl, gr, stream=s)
        s.synchronize()
        got = [x.cpu().numpy().copy() for x in nl] + [x.cpu().numpy().copy() for x in gr]
        if ref is None:
            ref = got
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
        (torch.randn(1 << 18, device=dev) ** 2).sum().item()
    for d, p in enumerate(probs):
        o = p["oracle"]
        g = ref[len(probs) + d]
        for i in range(0, len(ths[d]), max(1, len(ths[d]) // 4)):
            v, rg = o.nll_grad(ths[d][i])
            assert abs(ref[d][i] - v) <= 1e-3
            scale = np.maximum(np.abs(rg), 1e-3 * np.abs(rg).max())
            assert np.all(np.abs(g[i] - rg) <= 1e-4 * scale + 1e-6), (d, i)


# Shapes of the 64-dataset scan (N_T in {2048..16384}, N_reco in
# {512..4096}, 1e6 MC events, N_E = 256, up to 4096 points per dataset) in
# one grouped launch beside small ragged analyses: n_t, n_reco, n_pts, grid
SCAN_SHAPES = [(16384, 4096, 1024, True), (2048, 4096, 512, True),
               (8192, 1024, 4096, True), (300, 77, 131, False),
               (64, 1, 3, False)]


def test_grouped_scan_shapes():
    import torch
    import paper_2607_00488_amd as nr
    probs, ctxs, ths = [], [], []
    for d, (n_t, n_reco, P, grid) in enumerate(SCAN_SHAPES):
        log(f"[gpu] scan-shape dataset {d}: {n_t} x {n_reco}, {P} points")
        p = inputs(n_t, n_reco, 256 if grid else 32, 10 ** 6, 2000 + d, 4000 + d)
        probs.append(p)
        ctxs.append(gpu_context(p))
        ths.append(synth.theta_grid_scan(P, 6000 + d) if grid
                   else synth.theta_prior(P, 6000 + d))
    dev = torch.device("cuda:0")
    tt = [torch.tensor(t, dtype=torch.float64, device=dev) for t in ths]
    nl = [torch.empty(len(t), dtype=torch.float64, device=dev) for t in ths]
    gr = [torch.empty(len(t), 7, dtype=torch.float64, device=dev) for t in ths]
    s = torch.cuda.Stream(device=dev)
    log("[gpu] grouped launch over the scan shapes (likelihood and gradient)")
    nr.eval_nll_multi_dev(ctxs, tt, nl, gr, stream=s)
    s.synchronize()
    outs = nr.eval_nll_multi(ctxs, ths)
    worst = worst_g = worst_mu = 0.0
    for d, p in enumerate(probs):
        o = p["oracle"]
        th, nll_d, g_d = ths[d], nl[d].cpu().numpy(), gr[d].cpu().numpy()
        # the likelihood-only call and the call with the gradient are tuned
        # separately and may run different tile shapes, whose column-tile
        # partial sums group the deviance differently: equal up to rounding
        assert np.allclose(nll_d, outs[d], rtol=1e-12, atol=0.0), \
            (d, float(np.max(np.abs(nll_d - outs[d]))))
        P = len(th)
        for i in sorted({0, P // 3, P - 1}):
            v, rg = o.nll_grad(th[i])
            assert abs(nll_d[i] - v) <= 1e-3, (d, i, nll_d[i], v)
            scale = np.maximum(np.abs(rg), 1e-3 * np.abs(rg).max())
            assert np.all(np.abs(g_d[i] - rg) <= 1e-4 * scale + 1e-6), (d, i)
            worst = max(worst, abs(nll_d[i] - v))
            worst_g = max(worst_g, float(np.max(np.abs(g_d[i] - rg) / scale)))
        # the same points through the single-dataset launch, and spectra
        k = [0, P - 1]
        single = ctxs[d].eval_nll_batched(th[k])
        assert np.max(np.abs(single - nll_d[k])) <= 1e-9 * np.abs(single).max()
        mu = ctxs[d].eval_mu_batched(th[k])
        for r, i in enumerate(k):
            ref = o.mu(th[i])
            tol = 1e-5 * np.abs(ref) + 1e-9 * np.abs(ref).max()
            ok = np.abs(mu[r] - ref) <= tol
            assert ok.all(), (d, i, int(np.argmin(ok)))
            worst_mu = max(worst_mu, float(np.max(np.abs(mu[r] - ref) /
                                                  np.maximum(np.abs(ref), 1e-300))))
    for c in ctxs:
        c.close()
    log(f"[gpu] scan shapes: max |d(-2lnL)| {worst:.2e}, max rel d grad "
        f"{worst_g:.2e}, max rel d mu {worst_mu:.2e}")


@pytest.mark.parametrize("cfg", [str(c) for c in range(4)])
def test_every_tile_configuration(cfg, monkeypatch):
    """Each GEMM tile shape the autotuner may pick gives the same
    likelihoods and gradients (tile edges in M, N and K included)."""
    import paper_2607_00488_amd as nr
    monkeypatch.setenv("NR_GEMM_CONFIG", cfg)
    probs, ctxs, ths = [], [], []
    for d, (n_t, n_reco, n_e, P) in enumerate(SHAPES[:4]):
        p = inputs(n_t, n_reco, n_e, 100_000, 500 + d, 600 + d)
        probs.append(p)
        ctxs.append(gpu_context(p))
        ths.append(synth.theta_prior(P, 700 + d))
    outs = nr.eval_nll_multi(ctxs, ths)
    for d, (p, th, out) in enumerate(zip(probs, ths, outs)):
        for i in range(0, len(th), max(1, len(th) // 8)):
            assert abs(out[i] - p["oracle"].nll(th[i])) <= 1e-3, (cfg, d, i)
    # the adjoint product on the same configuration
    th = ths[1][:24]
    nll, g = ctxs[1].eval_nll_grad_batched(th)
    for i in range(0, len(th), 6):
        v, rg = probs[1]["oracle"].nll_grad(th[i])
        assert abs(nll[i] - v) <= 1e-3
        scale = np.maximum(np.abs(rg), 1e-3 * np.abs(rg).max())
        assert np.all(np.abs(g[i] - rg) <= 1e-4 * scale + 1e-6), (cfg, i)
    for c in ctxs:
        c.close()


def test_autotuner_cache(tmp_path, monkeypatch):
    """The autotuner writes its choice to the cache file; a corrupt file is
    ignored (the shape class is tuned again)."""
    import json
    import paper_2607_00488_amd as nr
    cache = tmp_path / "tune.json"
    cache.write_text("{ this is not json")
    monkeypatch.setenv("NR_AUTOTUNE_CACHE", str(cache))
    monkeypatch.delenv("NR_GEMM_CONFIG", raising=False)
    p = inputs(*SHAPES[0][:3], 100_000, 500, 600)
    ctx = gpu_context(p)
    th = synth.theta_prior(SHAPES[0][3], 700)
    out = ctx.eval_nll_batched(th)
    assert abs(out[0] - p["oracle"].nll(th[0])) <= 1e-3
    saved = json.loads(cache.read_text())
    assert len(saved) == 1
    (key, cfg), = saved.items()
    assert key.startswith("nll|") and cfg in (0, 1, 2, 3)
    ctx.close()


def test_mfma_probe_runs():
    """The matrix-core probe the batched GEMM rate is read against returns
    a finite, plausible rate (between 1 TFLOP/s and the data-sheet peak)."""
    import paper_2607_00488_amd as nr
    r = nr.nr_probe_mfma_f64(0, 1024, 50)
    log(f"[gpu] FP64 MFMA probe (1024 work-groups, short): {r:.1f} TFLOP/s")
    assert 1.0 < r < 80.0
    g = nr.nr_probe_hbm_read(0, 256 << 20, 4)
    log(f"[gpu] HBM read probe (256 MiB): {g:.0f} GB/s")
    assert 100.0 < g < 20000.0
    for flags in (nr.NR_PROBE_CACHED, nr.NR_PROBE_ALTERNATE,
                  nr.NR_PROBE_CACHED | nr.NR_PROBE_ALTERNATE):
        g = nr.nr_probe_read(0, (1 << 20) + 16 * 1001, 3, flags)  # ragged tail
        assert 1.0 < g < 50000.0, flags
