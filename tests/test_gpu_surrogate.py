"""The learned surrogate: its BF16 matrix-core forward and backward kernels
against a plain numpy reference with the same weights, training on spectra
from the batched method, and the fallback to the exact method."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import mlp as ref
from problems import config_inputs, gpu_context

pytestmark = pytest.mark.gpu


def exp_bound(mu, lm):
    """How far the fused likelihood kernel's -2lnL may lie from the host's,
    given the same FP32 ln mu_j on both sides: the kernel takes mu_j =
    2^(ln mu_j log2 e) in FP32 (the FP32 constant, off by 2^-26 relative,
    and the rounded product change mu_j by at most 1.25 2^-24 |ln mu_j|
    relative; the exponential adds about an ulp, 2^-23) and sums the mu_j
    of four bins in FP32 (at most 3 2^-24 of their sum) where the host takes
    FP64 exponentials.  Only mu_j is off, not ln mu_j, so the deviance term
    mu_j - n_j ln mu_j moves by mu_j times the relative error:
    |d(-2lnL)| <= 2 sum_j mu_j (1.25 2^-24 |ln mu_j| + 2^-23 + 3 2^-24),
    here with more than a factor two of margin."""
    return 2.0 * np.sum(mu * (np.abs(lm) * 2.0 ** -22 + 2.0 ** -20), axis=1)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


@pytest.mark.parametrize("B,N", [(128, 256), (2048, 256), (1024, 1024)])
def test_backward_kernels_match_reference(torch_dev, B, N):
    """Long reductions are split over work-groups (slabs summed in order):
    at B = 2048 and 1024 the weight gradients' batch sums, at N = 1024 the
    first backward product's sum over the outputs (with its SiLU'
    epilogue in the summing kernel); at B = 128, N = 256 nothing is."""
    torch, dev = torch_dev
    from paper_2607_00488_amd.surrogate import Surrogate, init_params
    lo, hi = synth.theta_box()
    H = 256
    s = Surrogate(N, lo, hi, hidden=H, seed=11)
    params = init_params(H, N, 12, out_scale=1.0)
    s.set_params(params)
    from paper_2607_00488_amd import nr_mlp_set_output_norm, nr_mlp_train_step_dev
    nr_mlp_set_output_norm(s.h, np.zeros(N, np.float32), np.ones(N, np.float32))
    g = synth.rng(13)
    th = g.uniform(lo, hi, (B, 7))
    tg = g.standard_normal((B, N)).astype(np.float32)
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    tgt = torch.tensor(tg, device=dev)
    loss = nr_mlp_train_step_dev(s.h, tt.data_ptr(), tgt.data_ptr(), B, 0.0, True)
    got = s.grads().astype(np.float64)
    rl, rg, mag = ref.mse_grad(params.astype(np.float64), th,
                               tg.astype(np.float64), lo, hi, H, N, bf16=True,
                               magnitude=True)
    # Element by element.  Both sides round the same quantities to bfloat16
    # (8 significant bits, neighbours 2^-7 apart relative); the values being
    # rounded differ only by the order of FP32 accumulation (relative to
    # their sum of absolute terms about K 2^-24), so a quantity near a
    # rounding boundary can land on neighbouring values.  A gradient element
    # is a sum of products of one back-propagated error and one activation,
    # each possibly one neighbour away: the difference of an element is then
    # within 2^-6 of its terms' absolute sum (the magnitude from the
    # reference), plus K 2^-24 of it for the accumulation.  Elements with no
    # terms (the parameter layout's padding) are exactly zero on both sides.
    live = mag > 0
    assert np.all(got[~live] == 0.0)
    ratio = np.abs(got - rg)[live] / mag[live]
    bound = 2.0 ** -6 + max(B, N) * 2.0 ** -24
    log(f"[gpu] mlp gradient B={B} N={N}: max |diff|/magnitude "
        f"{ratio.max():.2e} (bound {bound:.2e}), loss rel diff "
        f"{abs(loss - rl) / rl:.2e}")
    assert ratio.max() <= bound, int(np.argmax(ratio))
    # the loss: FP64 sum of FP32 squared residuals; a residual differs by
    # the FP32 accumulation of its output (K 2^-24 of its terms)
    assert loss == pytest.approx(rl, rel=1e-4)
    # forward (log mu with mean 0, std 1 is the raw output)
    y = s.logmu(tt).cpu().numpy()
    ry, acts, _ = ref.forward(params.astype(np.float64), th, lo, hi, H, N,
                              bf16=True)
    w_out = np.abs(params.astype(np.float64)[-N * (H + 8):].reshape(N, H + 8)
                   [:, :H + 1])
    ymag = np.abs(acts[3]) @ ref.bf16_round(w_out).T
    yr = np.abs(y - ry) / ymag
    log(f"[gpu] mlp forward: max |diff|/magnitude {yr.max():.2e}")
    assert yr.max() <= 2.0 ** -6
    s.close()


@pytest.fixture(scope="module")
def trained(torch_dev):
    torch, dev = torch_dev
    from paper_2607_00488_amd.surrogate import Surrogate
    p = config_inputs(0)
    ctx = gpu_context(p)
    lo, hi = synth.theta_box()
    s = Surrogate(p["n_reco"], lo, hi, hidden=256, seed=4001)
    th_train = s.sample_box(1 << 14, 4001)
    t0 = time.time()
    targets = s.make_targets(ctx, th_train)
    info = s.train(th_train, targets, epochs=60, batch=1024, log_every=200)
    log(f"[gpu] surrogate trained: {info['steps']} steps in {info['seconds']:.1f}s "
        f"(data+train {time.time() - t0:.1f}s); losses {info['losses'][-3:]}")
    return p, ctx, s


def test_surrogate_accuracy_and_fallback(trained, torch_dev):
    torch, dev = torch_dev
    import paper_2607_00488_amd as nr
    p, ctx, s = trained
    o = p["oracle"]
    th_val = s.sample_box(1 << 11, 4002)
    nll_s, outside = s.nll(ctx, th_val)
    exact = torch.empty_like(nll_s)
    nr.eval_nll_multi_dev([ctx], [th_val], [exact])
    torch.cuda.synchronize()
    d = (nll_s - exact).abs().cpu().numpy()
    assert not outside.any()
    log(f"[gpu] surrogate |d(-2lnL)| on validation: median {np.median(d):.3g}, "
        f"90% {np.quantile(d, 0.9):.3g}, max {d.max():.3g}; "
        f"within 0.1: {np.mean(d <= 0.1):.3f}")
    # the fused output layer + likelihood kernel against -2lnL formed on the
    # host from the network's own log mu (no pulls on this context)
    import math
    nobs = p["n"]
    cdata = float(np.sum(nobs - np.where(nobs > 0, nobs * np.log(np.where(nobs > 0, nobs, 1)), 0)
                         + np.array([math.lgamma(x + 1.0) for x in nobs])))
    lm = s.logmu(th_val[:256]).cpu().numpy().astype(np.float64)
    mu_h = np.exp(lm)
    dvs = np.sum(mu_h - nobs + np.where(nobs > 0, nobs * (np.log(np.where(nobs > 0, nobs, 1)) - lm), 0.0), axis=1)
    ref = 2.0 * (dvs + cdata)
    fused = nll_s[:256].cpu().numpy()
    bound = exp_bound(mu_h, lm)
    assert np.all(np.abs(fused - ref) <= bound + 1e-9 * np.abs(ref) + 1e-6), \
        np.max(np.abs(fused - ref) - bound)
    # the exact reference itself against the oracle on a few points
    ev = exact.cpu().numpy()
    tv = th_val.cpu().numpy()
    for i in range(0, len(tv), 512):
        assert abs(ev[i] - o.nll(tv[i])) <= 1e-3
    # fallback 1: a failing spot check sends the whole batch to the exact path
    out, info = s.evaluate(ctx, th_val, force_fail=True)
    assert info["fallback"] == "batch"
    assert torch.equal(out, exact)
    # fallback 2: points outside the training box always take the exact path
    th_mix = th_val[:256].clone()
    th_mix[::4, 4] = 40.0          # mu_nu beyond the box
    th_mix[1::4, 0] = -0.9         # eps_eL beyond the box
    exact_mix = torch.empty(256, dtype=torch.float64, device=dev)
    nr.eval_nll_multi_dev([ctx], [th_mix.contiguous()], [exact_mix])
    out, info = s.evaluate(ctx, th_mix, tol=1e30)  # spot checks always pass
    ob = torch.zeros(256, dtype=torch.bool, device=dev)
    ob[::4] = True
    ob[1::4] = True
    assert info["fallback"] == "outside"
    assert torch.equal(out[ob], exact_mix[ob])
    assert info["fallback_fraction"] == pytest.approx(0.5)


def test_surrogate_gain(trained, torch_dev):
    """What the trained network gains over the exact batched method, with
    spot checks and fallback counted: reported, not assumed."""
    torch, dev = torch_dev
    import paper_2607_00488_amd as nr
    p, ctx, s = trained
    th = s.sample_box(1 << 14, 4005)
    exact = torch.empty(len(th), dtype=torch.float64, device=dev)
    nr.eval_nll_multi_dev([ctx], [th], [exact])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        nr.eval_nll_multi_dev([ctx], [th], [exact])
    torch.cuda.synchronize()
    t_exact = (time.perf_counter() - t0) / 3
    out, info = s.evaluate(ctx, th)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(3):
        out, info = s.evaluate(ctx, th, seed=k)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / 3
    d = (out - exact).abs()
    log(f"[gpu] surrogate gain {t_exact / t_sur:.2f}x over exact batched "
        f"({len(th) / t_sur:.0f} vs {len(th) / t_exact:.0f} evals/s), "
        f"fallback {info['fallback']} ({info['fallback_fraction']:.2f}), "
        f"spot worst {info['spot_worst']:.3g}, max |d| returned {d.max().item():.3g}")
    if info["fallback"] == "batch":
        assert torch.equal(out, exact)


def test_network_seeded_fits(trained, torch_dev):
    """What the trained network gains where its values are never returned:
    it ranks 16384 points of the box, and exact L-BFGS fits (template form)
    started from the 32 best need fewer exact likelihood-and-gradient calls
    than fits from 32 uniform starts, and reach the same minimum."""
    torch, dev = torch_dev
    from paper_2607_00488_amd.autograd import lbfgs_fit
    p, ctx, s = trained
    lo, hi = synth.theta_box()
    ctx.build_templates()
    S = 32
    g = np.random.Generator(np.random.PCG64(5001))
    starts = torch.tensor(g.uniform(lo, hi, (S, 7)), dtype=torch.float64, device=dev)
    _, f1, gn1, c1 = lbfgs_fit(ctx, starts, iters=300, gtol=1e-3, form="templates")
    cand = s.sample_box(1 << 14, 6001)
    nl, _ = s.nll(ctx, cand)
    best = cand[torch.argsort(nl)[:S]].contiguous()
    _, f2, gn2, c2 = lbfgs_fit(ctx, best, iters=300, gtol=1e-3, form="templates")
    b1, b2 = float(f1.min()), float(f2.min())
    log(f"[gpu] seeded fits: {c1} exact calls from uniform starts, {c2} from "
        f"network-ranked starts (gain {c1 / c2:.2f}); minima {b1:.6f} / {b2:.6f}")
    # the network's starts find the exact minimum the uniform starts find
    assert abs(b2 - b1) <= 1e-6 * abs(b1) + 1e-6
    assert c2 < c1


@pytest.mark.parametrize("H,N", [(256, None), (128, None), (256, 4000), (128, 4000)])
def test_network_likelihood_ragged_batches(torch_dev, H, N):
    """The network's -2lnL at batch sizes that are not multiples of the
    kernels' 128-point tiles, for the whole-network kernel (256 hidden
    units: hidden layers formed in LDS) and for the layer-by-layer path
    (other widths), against -2lnL formed on the host from the network's
    own log mu, with the bound of the FP32 exponential (no pulls here).
    At the parity binning (256 bins) and at 4000 bins, which ends in part
    of a 256-bin step: there the last waves' bins lie past the end and one
    wave has none at all."""
    torch, dev = torch_dev
    import math
    from paper_2607_00488_amd.surrogate import Surrogate, init_params
    import paper_2607_00488_amd as nr
    if N is None:
        p = config_inputs(0)
        ctx = gpu_context(p)
        N = p["n_reco"]
    else:
        g = synth.rng(4100)
        R = (g.random((64, N), dtype=np.float32) / N).astype(np.float32)
        p = {"n": g.poisson(10.0, N).astype(np.float64)}
        ctx = nr.Context(0)
        ctx.set_sources(synth.source_nodes(64), 64)
        ctx.set_response(R, n_sig=1e4)
        ctx.set_data(p["n"], np.full(N, 10.0))
    lo, hi = synth.theta_box()
    s = Surrogate(N, lo, hi, hidden=H, seed=4101)
    s.set_params(init_params(H, N, 4102, out_scale=1.0))
    nr.nr_mlp_set_output_norm(s.h, np.full(N, 2.0, np.float32), np.full(N, 0.3, np.float32))
    nobs = p["n"]
    cdata = float(np.sum(nobs - np.where(nobs > 0, nobs * np.log(np.where(nobs > 0, nobs, 1)), 0)
                         + np.array([math.lgamma(x + 1.0) for x in nobs])))
    for B in (8, 136, 1000):
        th = s.sample_box(B, 4103 + B)
        got, outside = s.nll(ctx, th)
        lm = s.logmu(th).cpu().numpy().astype(np.float64)
        mu_h = np.exp(lm)
        dvs = np.sum(mu_h - nobs + np.where(nobs > 0, nobs * (np.log(np.where(nobs > 0, nobs, 1)) - lm), 0.0), axis=1)
        ref = 2.0 * (dvs + cdata)
        bound = exp_bound(mu_h, lm)
        d = np.abs(got.cpu().numpy() - ref)
        log(f"[gpu] network -2lnL, {H} hidden, {N} bins, B = {B}: max |d| {d.max():.3g}")
        assert not outside.any()
        assert np.all(d <= bound + 1e-9 * np.abs(ref) + 1e-6), np.max(d - bound)
    s.close()
    ctx.close()


def test_network_likelihood_full_batch(torch_dev):
    """The whole-network likelihood kernel at the surrogate form's
    inference shape and launch (65 536 points, 4096 bins: one group of bins
    per work-group, all 16 steps of 256 bins), on 96 sampled points against
    -2lnL formed on the host from the network's own log mu."""
    torch, dev = torch_dev
    import math
    from paper_2607_00488_amd.surrogate import Surrogate, init_params
    import paper_2607_00488_amd as nr
    N, B = 4096, 1 << 16
    g = synth.rng(4201)
    R = (g.random((256, N), dtype=np.float32) / N).astype(np.float32)
    nobs = g.poisson(30.0, N).astype(np.float64)
    ctx = nr.Context(0)
    ctx.set_sources(synth.source_nodes(64), 256)
    ctx.set_response(R, n_sig=1e4)
    ctx.set_data(nobs, np.full(N, 10.0))
    lo, hi = synth.theta_box()
    s = Surrogate(N, lo, hi, hidden=256, seed=4202)
    s.set_params(init_params(256, N, 4203, out_scale=1.0))
    nr.nr_mlp_set_output_norm(s.h, np.full(N, 3.0, np.float32), np.full(N, 0.2, np.float32))
    th = s.sample_box(B, 4204)
    log(f"[gpu] network -2lnL at {B} points x {N} bins")
    got, outside = s.nll(ctx, th)
    got = got.cpu().numpy()
    assert not outside.cpu().numpy().any()
    idx = np.sort(synth.rng(4205).choice(B, 96, replace=False))
    lm = s.logmu(th[torch.as_tensor(idx, device=dev)]).cpu().numpy().astype(np.float64)
    mu_h = np.exp(lm)
    cdata = float(np.sum(nobs - np.where(nobs > 0, nobs * np.log(np.where(nobs > 0, nobs, 1)), 0)
                         + np.array([math.lgamma(x + 1.0) for x in nobs])))
    dvs = np.sum(mu_h - nobs + np.where(nobs > 0, nobs * (np.log(np.where(nobs > 0, nobs, 1)) - lm), 0.0),
                 axis=1)
    ref = 2.0 * (dvs + cdata)
    d = np.abs(got[idx] - ref)
    bound = exp_bound(mu_h, lm)
    log(f"[gpu] full batch: max |d| {d.max():.3g}, max d / bound {np.max(d / bound):.3g}")
    assert np.all(d <= bound + 1e-9 * np.abs(ref) + 1e-6), np.max(d - bound)
    s.close()
    ctx.close()
