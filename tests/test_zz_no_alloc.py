"""The allocation-free entry point nr_eval_nll_dev_noalloc against
nr_eval_nll_dev, through the C ABI: two calls in a row on the same device
workspace, the second with a smaller input (fewer points, a smaller
response), each with and without the gradient, and the size check of the
static workspace.  Both entry points run the same kernels in the same
order, so the results are compared for equality (the parity bar,
|d(-2lnL)| <= 1e-3, is implied)."""
import sys

import numpy as np
import pytest

import synth
from problems import config_inputs, gpu_context, inputs

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(ctx, th, grad, torch, dev):
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    out = {}
    for name, fn in (("dev", ctx.eval_nll_dev), ("noalloc", ctx.eval_nll_dev_noalloc)):
        nl = torch.full((len(th),), float("nan"), dtype=torch.float64, device=dev)
        gr = (torch.full((len(th), 7), float("nan"), dtype=torch.float64, device=dev)
              if grad else None)
        fn(tt, nl, gr, stream=s)
        s.synchronize()
        out[name] = (nl.cpu().numpy(), None if gr is None else gr.cpu().numpy())
    return out["dev"], out["noalloc"]


def check(ctx, th, torch, dev, what):
    for grad in (False, True):
        log(f"[gpu] noalloc vs dev: {what}, {len(th)} points, grad={grad}")
        (n0, g0), (n1, g1) = both(ctx, th, grad, torch, dev)
        assert np.all(np.isfinite(n0))
        assert np.max(np.abs(n1 - n0)) <= 1e-3
        assert np.array_equal(n0, n1), (what, np.max(np.abs(n1 - n0)))
        if grad:
            assert np.all(np.isfinite(g0))
            assert np.array_equal(g0, g1), (what, np.max(np.abs(g1 - g0)))


def test_noalloc_matches_dev_entry_point():
    import torch
    dev = torch.device("cuda:0")
    log("[gpu] noalloc: building a 4096 x 2048 analysis")
    big = inputs(4096, 2048, 512, 2_000_000, 7101, 7102)
    small = config_inputs(0)
    c_big = gpu_context(big)
    c_small = gpu_context(small)
    try:
        th_big = np.vstack([synth.theta_sm()[None],
                            synth.theta_prior(36, 7103, f_range=(0.8, 1.2))])
        check(c_big, th_big, torch, dev, "4096 x 2048")
        # second call: a smaller response and fewer points on the same
        # workspace, which still holds the first call's values
        th_small = synth.theta_prior(5, 7104, f_range=(0.8, 1.2))
        check(c_small, th_small, torch, dev, "512 x 256")
    finally:
        c_big.close()
        c_small.close()


def test_noalloc_rejects_shapes_beyond_the_workspace():
    import torch
    import paper_2607_00488_amd as nr
    dev = torch.device("cuda:0")
    g = synth.rng(7105)
    n_t, n_reco = 16384, 512
    R = (g.random((n_t, n_reco), dtype=np.float32) / n_reco).astype(np.float32)
    ctx = nr.Context(0)
    try:
        ctx.set_sources(synth.source_nodes(256), n_t)
        ctx.set_response(R, n_sig=1.0e4)
        b = np.full(n_reco, 10.0)
        ctx.set_data(b, b)
        # 8-row fold tiles: 2 x 2048 x 512 partial sums (16.8 MB) exceed the
        # 16 MiB workspace
        nr.nr_set_fold_tiling(ctx.h, 8, 1)
        tt = torch.tensor(synth.theta_prior(3, 7106), dtype=torch.float64, device=dev)
        nl = torch.empty(3, dtype=torch.float64, device=dev)
        log("[gpu] noalloc: workspace size check")
        rc = nr.load().nr_eval_nll_dev_noalloc(ctx.h, nr.C.c_void_p(tt.data_ptr()), 3,
                                              nr.C.c_void_p(nl.data_ptr()), None, None)
        assert rc == nr.NR_EINVAL
        assert "workspace" in nr.load().nr_last_error().decode()
        # the context's own entry point still serves the same call
        log("[gpu] noalloc: the context's entry point on the same context")
        ctx.eval_nll_dev(tt, nl)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(nl.cpu().numpy()))
    finally:
        ctx.close()
