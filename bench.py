"""Benchmark: likelihood evaluations per second on one MI355X.

A step is one batch of parameter points (100 by default, a row of a
likelihood scan), each put through the whole plain single-point path
(device E-integral, weights, HBM-streaming fold of the 16384 x 4096 FP32
response, Poisson -2lnL), with every input resident in HBM.  The K timed
steps are one HIP-graph replay of K x 100 evaluations; the value is
evaluations per second.

Prints one JSON line: the plain rate as `value`, the roofline of the step
kernel, the batched and gradient forms and the CPU oracle timed beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("likelihood evals/s at |Δ(−2lnL)|≤1e-3 vs FP64: "
          "plain vs batched/grad/surrogate")
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(n_t, n_reco):
    """Bytes one evaluation must move at least once: the FP32 response, the
    two FP64 per-row inputs of the weights (S_SM and m) and the FP64 data
    and background per observed bin."""
    return 4 * n_t * n_reco + 16 * n_t + 16 * n_reco


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles",
                               "k_step_plain_16384x4096_hbm_traffic.md")
# the step kernel and the host code that picks its tiling
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2607_00488_amd", "csrc", f)
                  for f in ("plain.hip", "common.h", "api.hip")]


def measured_traffic():
    """HBM bytes per k_step launch from the committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        txt = open(TRAFFIC_PROFILE).read()
        src = b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)
    except OSError:
        return None
    vals = dict(ln.split(": ", 1) for ln in txt.splitlines()
                if ln.startswith(("traffic_bytes_per_launch:",
                                  "kernel_source_sha256:")))
    if vals.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return int(vals["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_plain(cfg_id=1):
    import synth
    import paper_2607_00488_amd as nr
    c = synth.CONFIGS[cfg_id]
    s = c.seeds(0)
    t0 = time.time()
    src = synth.source_nodes(c.n_e)
    rsp = synth.response_mc(c.n_t, c.n_reco, c.n_mc, seed=s["response"],
                            keep_counts=False)
    log(f"[bench] response MC {c.n_mc:.0e} events in {time.time() - t0:.1f}s")
    b = np.full(c.n_reco, c.bkg)
    ctx = nr.Context(0)
    ctx.set_sources(src, c.n_t)
    ctx.set_response(rsp.R, n_sig=c.n_sig)
    # toy data drawn from the library's own SM expectation
    ctx.set_data(b, b)
    mu_sm = ctx.eval_mu(synth.theta_sm())[0]
    n = synth.poisson_data(mu_sm, s["data"])
    ctx.set_data(n, b)
    return dict(cfg=c, seeds=s, src=src, R=rsp.R, b=b, n=n, ctx=ctx,
                row_events=rsp.row_events)


def build_batched(n_datasets=64):
    """The uneven-binning scan: 64 analyses, 16 shape classes."""
    import synth
    import paper_2607_00488_amd as nr
    t0 = time.time()
    ctxs, ths, flops = [], [], 0.0
    src = synth.source_nodes(256)
    for sd in synth.batched_schedule(n_datasets):
        rsp = synth.response_mc(sd["n_t"], sd["n_reco"], sd["n_mc"],
                                seed=sd["seed_response"], keep_counts=False)
        b = np.full(sd["n_reco"], 10.0)
        ctx = nr.Context(0)
        ctx.set_sources(src, sd["n_t"])
        ctx.set_response(rsp.R, n_sig=1.0e4)
        ctx.set_data(b, b)
        mu_sm = ctx.eval_mu(synth.theta_sm())[0]
        ctx.set_data(synth.poisson_data(mu_sm, sd["seed_data"]), b)
        ctxs.append(ctx)
        ths.append(synth.theta_grid_scan(sd["n_pts"], sd["seed_theta"]))
        flops += 2.0 * sd["n_pts"] * sd["n_t"] * sd["n_reco"]
    log(f"[bench] batched inputs ({n_datasets} datasets) in {time.time() - t0:.1f}s")
    return ctxs, ths, flops


def time_batched(ctxs, ths, reps=3, grad=False):
    import torch
    import paper_2607_00488_amd as nr
    dev = torch.device("cuda:0")
    tt = [torch.tensor(t, dtype=torch.float64, device=dev) for t in ths]
    nl = [torch.empty(len(t), dtype=torch.float64, device=dev) for t in ths]
    gr = ([torch.empty(len(t), 7, dtype=torch.float64, device=dev) for t in ths]
          if grad else None)
    s = torch.cuda.Stream(device=dev)
    nr.eval_nll_multi_dev(ctxs, tt, nl, gr, stream=s)  # capture + run
    s.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        nr.eval_nll_multi_dev(ctxs, tt, nl, gr, stream=s)
    s.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return dt, [x.cpu().numpy() for x in nl], (None if gr is None else
                                                [g.cpu().numpy() for g in gr])


def plain_config0_form(n_pts=4096, reps=5):
    """The plain single-point path at the parity configuration (512 recoil x
    256 reco bins, N_E = 256, 1e6 MC events): the response is 512 KiB and
    stays in L2, so the chain of step launches is latency-bound.  One graph
    replay of n_pts evaluations at prior points, timed with events."""
    import torch
    import synth
    p = build_plain(0)
    ctx = p["ctx"]
    dev = torch.device("cuda:0")
    th = torch.tensor(synth.theta_prior(n_pts, p["seeds"]["theta"] + 11),
                      dtype=torch.float64, device=dev)
    out = torch.empty(n_pts, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    ctx.eval_nll_dev(th, out, stream=s)
    s.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ctx.eval_nll_dev(th, out, stream=s)
    e1.record(s)
    s.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ctx.close()
    return dict(evals_per_s=round(n_pts / (ms * 1e-3), 1), points=n_pts,
                us_per_eval=round(ms * 1e3 / n_pts, 3),
                what="plain single-point path at 512 x 256 (N_E = 256): the "
                     "512 KiB response stays in L2; one graph replay of "
                     f"{n_pts} evaluations ({n_pts + 4} step launches)")


def templates_form(ctx, seed, n_pts=65536, reps=5):
    """The template form at the paper-scale shapes: the 20 basis templates
    and the S_SM = 0 rows folded once through R (one FP64 pass), then 21
    products and one logarithm per (point, reco bin).  Timed with events on
    the stream the kernels run on; a few points checked against the plain
    (single-point streaming) method."""
    import torch
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.build_templates()
    build_ms = (time.perf_counter() - t0) * 1e3
    th = synth.theta_prior(n_pts, seed, f_range=(0.8, 1.2))
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    nl = torch.empty(n_pts, dtype=torch.float64, device=dev)
    gr = torch.empty(n_pts, 7, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    ms = {}
    for mode, g in (("nll", None), ("nll_grad", gr)):
        ctx.eval_nll_templates_dev(tt, nl, g, stream=s)
        s.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            ctx.eval_nll_templates_dev(tt, nl, g, stream=s)
        e1.record(s)
        s.synchronize()
        ms[mode] = e0.elapsed_time(e1) / reps
    got = nl.cpu().numpy()
    k = 16
    plain = ctx.eval_nll(th[:k])
    bins = float(n_pts) * ctx.n_reco
    return dict(
        evals_per_s=round(n_pts / (ms["nll"] * 1e-3), 1),
        grad_evals_per_s=round(n_pts / (ms["nll_grad"] * 1e-3), 1),
        points=n_pts, ms=round(ms["nll"], 3), grad_ms=round(ms["nll_grad"], 3),
        ns_per_point_bin=round(ms["nll"] * 1e6 / bins, 4),
        template_fold_ms=round(build_ms, 2),
        max_abs_dnll_vs_plain=float(np.max(np.abs(got[:k] - plain))),
        bound="alu",
        what="exact template form: mu_j = f_bkg b_j + G0_j + sum_b c_b(theta) "
             "G_bj with the 20 basis templates folded once through R; per "
             "(point, bin) 21 FP64 products and one FP64 logarithm")


def asimov_scan_form(p):
    """The paper's injection-recovery demonstration at the paper-scale
    binning: Asimov data at eps_eL = 0.05, a 31-value scan of eps_eL over
    [-0.1, 0.2] with f_8B and f_bkg profiled (pulls 1 +- 0.1) by the batched
    L-BFGS driver, end to end (all fits, every likelihood and gradient call),
    once with the batched GEMM form and once with the template form.  The
    context's data are restored afterwards."""
    import torch
    import synth
    from paper_2607_00488_amd.scan import interval, profile_scan
    ctx = p["ctx"]
    th_inj = synth.theta_sm().copy()
    th_inj[0] = 0.05
    asimov = ctx.eval_mu_templates(th_inj)[0]
    pm = [0, 0, 0, 0, 0, 1.0, 1.0]
    ps = [0, 0, 0, 0, 0, 0.1, 0.1]
    ctx.set_data(asimov, p["b"], pm, ps)
    grid = np.linspace(-0.1, 0.2, 31)
    out = {}
    for form in ("batched", "templates"):
        dts = []
        for _ in range(2):   # the first run also tunes, captures and allocates
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sc = profile_scan(ctx, 0, grid, synth.theta_sm(), free=(5, 6), form=form)
            torch.cuda.synchronize()
            dts.append(time.perf_counter() - t0)
        lo, hi = interval(sc["values"], sc["delta"])
        k = int(np.argmin(sc["delta"]))
        out[form] = dict(seconds=round(dts[1], 3), first_seconds=round(dts[0], 3),
                         calls=sc["calls"],
                         minimum_at=float(sc["values"][k]),
                         interval_90=[round(lo, 5), round(hi, 5)],
                         max_grad_norm=float(sc["grad_norm"].max()))
    ctx.set_data(p["n"], p["b"])
    out["what"] = ("Asimov eps_eL = 0.05 at 16384 x 4096: 31-value scan, "
                   "f_8B and f_bkg profiled by batched L-BFGS (31 fits "
                   "advanced together), 90% CL interval at 2.706")
    return out


def ess_form(ctx, row_events, seed, n_pts=40):
    """The effective-sample-size diagnostic at the benchmark's shapes: per
    point the node table and weights, then one non-temporal pass over R
    forming both sums per observed bin.  Host-timed call of n_pts points
    (the spectra come back to the host), after one warm call."""
    import synth
    ctx.set_mc_events(np.asarray(row_events, dtype=np.float64))
    th = synth.theta_prior(n_pts, seed)
    ctx.eval_ess(th[:2])
    t0 = time.perf_counter()
    ess = ctx.eval_ess(th)
    dt = time.perf_counter() - t0
    n_t, n_reco = ctx.n_t, ctx.n_reco
    alg = 4 * n_t * n_reco + 16 * n_t + 8 * n_reco   # R, n w and n w^2, ESS out
    return dict(evals_per_s=round(n_pts / dt, 1), points=n_pts,
                us_per_eval=round(dt / n_pts * 1e6, 2),
                gbs=round(alg * n_pts / dt / 1e9, 1),
                frac_hbm=round(alg * n_pts / dt / 1e9 / 8000.0, 3),
                finite=bool(np.all(np.isfinite(ess))),
                what="ESS_j = (sum_l N_lj w_l)^2 / sum_l N_lj w_l^2 per observed bin "
                     "(N_lj = R_lj n_l), one streaming pass over R per point; "
                     "host-timed, copies and the final synchronisation included")


def banded_form(ctx, R, tt, dense_out, stream):
    """The same scan with band skipping on: the fold and the adjoint read
    only the column bands of R that hold non-zero responses.  The results
    are compared bit for bit with the dense scan just timed; the bytes a
    banded fold must read at least are each row's non-zero band (in 16-byte
    column groups) plus the per-row and per-bin inputs."""
    import torch
    nz = R != 0
    any_nz = nz.any(axis=1)
    n_reco = R.shape[1]
    lo = np.where(any_nz, np.argmax(nz, axis=1), 0)
    hi = np.where(any_nz, n_reco - np.argmax(nz[:, ::-1], axis=1), 0)
    band_bytes = int(np.sum(np.where(any_nz, ((hi + 3) // 4 - lo // 4) * 16, 0)))
    alg = band_bytes + 16 * R.shape[0] + 16 * n_reco
    ctx.set_band_skipping(True)
    out = torch.empty_like(dense_out)
    ctx.eval_nll_dev(tt, out, stream=stream)          # capture + run
    stream.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    ctx.eval_nll_dev(tt, out, stream=stream)
    ev1.record(stream)
    stream.synchronize()
    dt = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    ctx.set_band_skipping(False)
    n = tt.shape[0]
    us = dev_ms * 1e3 / n
    return dict(evals_per_s=round(n / dt, 1), points=n, us_per_eval=round(us, 2),
                bitwise_equal_to_dense=bool(torch.equal(out, dense_out)),
                band_fraction=round(band_bytes / (4.0 * R.size), 4),
                band_bytes_per_eval=alg,
                band_gbs=round(alg / (us * 1e-6) / 1e9, 1),
                what="the headline scan with band skipping: each fold tile reads "
                     "only the columns where its rows' responses are non-zero "
                     "(exact zeros elsewhere); results bitwise those of the "
                     "dense read")


def seeded_fit_study(ctx, sur, S=64, gtols=(1e-2, 1e-4)):
    """Where the network helps without its values being returned: it ranks
    65 536 points of the box and the S best start exact L-BFGS fits (the
    template form), against S uniform starts.  Every returned minimum is
    exact; the gain is in exact likelihood calls."""
    import torch
    import synth
    from paper_2607_00488_amd.autograd import lbfgs_fit
    lo, hi = synth.theta_box()
    ctx.build_templates()
    out = {}
    for gtol in gtols:
        g = np.random.Generator(np.random.PCG64(5000))
        starts = torch.tensor(g.uniform(lo, hi, (S, 7)), dtype=torch.float64,
                              device=sur.dev)
        _, f1, gn1, c1 = lbfgs_fit(ctx, starts, iters=300, gtol=gtol, form="templates")
        cand = sur.sample_box(1 << 16, 6000)
        nl, _ = sur.nll(ctx, cand)
        best = cand[torch.argsort(nl)[:S]].contiguous()
        _, f2, gn2, c2 = lbfgs_fit(ctx, best, iters=300, gtol=gtol, form="templates")
        fmin = float(min(f1.min().item(), f2.min().item()))
        out[f"gtol_{gtol:g}"] = dict(
            uniform_starts_calls=c1, network_starts_calls=c2,
            call_gain=round(c1 / c2, 3),
            best_uniform=float(f1.min().item()), best_network=float(f2.min().item()),
            at_best_uniform=float((f1 <= fmin + 0.01).double().mean().item()),
            at_best_network=float((f2 <= fmin + 0.01).double().mean().item()))
    out["what"] = (f"{S} exact L-BFGS fits (template form) from uniform box starts "
                   f"against the {S} best of 65536 box points ranked by the network")
    return out


def mlp_flop_per_point(n_out, hidden=256):
    """Matrix flop per point of the 7-H-H-H-n_out network: each layer's
    inputs plus the bias column (K = 8, H + 1, H + 1, H + 1), no K padding
    (2.37 MFLOP at H = 256, n_out = 4096)."""
    return 2 * (8 * hidden + 2 * (hidden + 1) * hidden + (hidden + 1) * n_out)


def surrogate_ceiling(ctx, sur, n_data, th_val, ks=(16, 32, 64)):
    """How far the trained network's -2lnL is from the exact one, and how
    far first-order corrections from exact linear functionals of mu would
    take it (measurement only, FP64 torch on the device).  Writing
    d_j = ln mu^_j - ln mu_j, the error is 2 sum_j (mu^_j - mu_j) - 2 sum_j
    n_j d_j.  The first sum is a linear functional of mu, exact for any
    point from the 21 folded templates; the second is to first order
    2 sum_j (n_j / mu^_j)(mu_j - mu^_j), which exact functionals
    L_k = sum_j V_kj mu_j remove along the span of V (the leading K right
    singular vectors of n / mu over 8192 other points of the box)."""
    import torch
    import paper_2607_00488_amd as nr
    dev = th_val.device
    s = torch.cuda.current_stream(dev)

    def exact_mu(th):
        mu = torch.empty(th.shape[0], ctx.n_reco, dtype=torch.float64, device=dev)
        for c0 in range(0, th.shape[0], 4096):
            k = min(4096, th.shape[0] - c0)
            nr.nr_eval_mu_batched_dev(ctx.h, th[c0:c0 + k].contiguous().data_ptr(),
                                      k, mu[c0:c0 + k].data_ptr(), s.cuda_stream)
        return mu

    nt = torch.tensor(n_data, dtype=torch.float64, device=dev)

    def dev2(m):
        return 2.0 * torch.where(nt > 0, m - nt + nt * torch.log(nt / m), m).sum(1)

    r = nt / exact_mu(sur.sample_box(8192, 4006))
    V = torch.linalg.svd(r, full_matrices=False)[2]
    del r
    mu = exact_mu(th_val)
    lmh = sur.logmu(th_val).double()
    muh = torch.exp(lmh)
    d_ex = dev2(mu)
    raw = dev2(muh) - d_ex
    summ = raw - 2.0 * (muh.sum(1) - mu.sum(1))
    rh = nt / muh
    far = d_ex - d_ex.min()

    def q(x):
        a = x.abs()
        return dict(median=float(a.median()), q90=float(a.quantile(0.9)),
                    max=float(a.max()), frac_le_0p1=float((a <= 0.1).double().mean()))

    out = dict(dln_mu_rms=float((lmh - torch.log(mu)).pow(2).mean().sqrt()),
               raw=q(raw), exact_sum_mu=q(summ))
    for k in ks:
        Vk = V[:k]
        corr = 2.0 * ((rh @ Vk.T) * (mu @ Vk.T - muh @ Vk.T)).sum(1)
        dk = summ - corr
        out[f"functionals_{k}"] = q(dk)
        for lim in (100.0, 1.0e3, 1.0e4):
            m = far <= lim
            if int(m.sum()) >= 8:
                out[f"functionals_{k}_within_dchi2_{int(lim)}"] = dict(
                    q(dk[m]), fraction_of_box=float(m.double().mean()))
    out["what"] = ("validation points: |d(-2lnL)| of the network as is, with "
                   "the exact sum of mu, and with first-order corrections "
                   "from K exact linear functionals of mu")
    return out


def surrogate_form(ctx, train_seconds=20.0, n_data=None):
    """The learned surrogate at the paper-scale binning: 7 -> 256 -> 256 ->
    256 -> 4096 SiLU MLP trained on 2^18 spectra from the batched method
    (prior box), validated on 2^14 held-out points against the exact
    batched -2lnL, then timed on a batch of 65 536 points with 1 % spot
    checks and fallback, beside the exact batched method on the same batch."""
    import torch
    import synth
    import paper_2607_00488_amd as nr
    from paper_2607_00488_amd.surrogate import Surrogate
    dev = torch.device("cuda:0")
    lo, hi = synth.theta_box()
    sur = Surrogate(ctx.n_reco, lo, hi, hidden=256, seed=4001)
    t0 = time.perf_counter()
    th_tr = sur.sample_box(1 << 18, 4001)
    tg = sur.make_targets(ctx, th_tr)
    t_data = time.perf_counter() - t0
    info = sur.train(th_tr, tg, epochs=10000, batch=2048, lr_max=1e-3,
                     log_every=1000, time_limit=train_seconds)
    del tg
    th_val = sur.sample_box(1 << 14, 4002)
    ex_val = torch.empty(1 << 14, dtype=torch.float64, device=dev)
    nr.eval_nll_multi_dev([ctx], [th_val], [ex_val])
    nl_val, _ = sur.nll(ctx, th_val)
    d = (nl_val - ex_val).abs().cpu().numpy()
    ceiling = (surrogate_ceiling(ctx, sur, n_data, th_val)
               if n_data is not None else None)
    B = 1 << 16
    th = sur.sample_box(B, 4005)
    ex = torch.empty(B, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream(dev)
    nr.eval_nll_multi_dev([ctx], [th], [ex], stream=s)   # capture + run
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nr.eval_nll_multi_dev([ctx], [th], [ex], stream=s)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t1
    sur.nll(ctx, th)
    torch.cuda.synchronize()
    reps = 10                     # back-to-back calls, as a scan issues them
    t1 = time.perf_counter()
    for _ in range(reps):
        sur.nll(ctx, th)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t1) / reps
    seeded = seeded_fit_study(ctx, sur)
    out, ev = sur.evaluate(ctx, th, seed=1)              # warm the spot graph
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out, ev = sur.evaluate(ctx, th, seed=2)
    torch.cuda.synchronize()
    t_eval = time.perf_counter() - t1
    worst_returned = float((out - ex).abs().max().item())
    sur.close()
    q = lambda x: float(np.quantile(d, x))
    return dict(
        evals_per_s=round(B / t_eval, 1), points=B,
        ms=round(t_eval * 1e3, 3), fallback=ev["fallback"],
        fallback_fraction=ev["fallback_fraction"],
        spot_checks=ev["spot"], spot_worst=ev["spot_worst"],
        max_abs_dnll_returned=worst_returned,
        exact_batched_evals_per_s=round(B / t_exact, 1),
        gain_vs_exact_batched=round(t_exact / t_eval, 3),
        network_only_evals_per_s=round(B / t_net, 1),
        network_tflops_bf16=round(B * mlp_flop_per_point(ctx.n_reco) / t_net / 1e12, 2),
        val_abs_dnll=dict(median=q(0.5), q90=q(0.9), max=float(d.max()),
                          frac_le_0p1=float(np.mean(d <= 0.1)),
                          frac_le_1=float(np.mean(d <= 1.0))),
        train=dict(samples=1 << 18, steps=info["steps"],
                   seconds=round(info["seconds"], 2),
                   data_seconds=round(t_data, 2),
                   final_loss=info["losses"][-1][1] if info["losses"] else None),
        ceiling=ceiling,
        seeded_fit=seeded,
        what="MLP 7-256-256-256-4096 SiLU on BF16 matrix cores; -2lnL "
             "with 1% exact spot checks, fallback to the exact batched "
             "method when a check misses by more than 0.1")


def components_form(n_pts=400):
    """The multi-component form at the paper-scale binning: five signal
    components (one per solar source) with their own 16384 x 4096 responses
    stacked row-wise (1.25 GiB of FP32 read per evaluation), two background
    templates, masks; single-point evaluations through the step-kernel
    pipeline, timed as one graph replay."""
    import torch
    import synth
    import paper_2607_00488_amd as nr
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    src = synth.source_nodes(2048)
    d = synth.component_inputs(16384, 4096, 20_000_000, 8001, shared_mc=True)
    ctx = nr.Context(0)
    ctx.set_sources(src, 16384, 0.0, 16.0)
    ctx.set_components(d["comp_of_source"], d["hist"], d["scale"], d["rate_sm"],
                       bkg_pdf=d["bkg_pdf"], bkg_rate=d["bkg_rate"],
                       comp_mask=d["comp_mask"], mask=d["mask"],
                       exposure=d["exposure"])
    K = len(d["scale"])
    del d
    g = synth.rng(8002)
    n_theta = ctx.n_theta
    ctx.set_data(np.full(4096, 20.0), None)
    th = np.concatenate([g.uniform(-0.5, 0.5, (n_pts, 4)), g.uniform(0, 25, (n_pts, 1)),
                         g.uniform(0.8, 1.2, (n_pts, n_theta - 5))], axis=1)
    t_setup = time.perf_counter() - t0
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    out = torch.empty(n_pts, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)
    ctx.eval_nll_dev(tt, out, stream=s)
    s.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t1 = time.perf_counter()
    ev0.record(s)
    ctx.eval_nll_dev(tt, out, stream=s)
    ev1.record(s)
    s.synchronize()
    dt = time.perf_counter() - t1
    step_ms = ev0.elapsed_time(ev1) / n_pts
    alg = 4 * K * 16384 * 4096 + 16 * K * 16384 + 16 * 4096
    # the template form of the same likelihood: 65 536 points per call
    t2 = time.perf_counter()
    ctx.build_templates()
    t_fold = time.perf_counter() - t2
    P = 65536
    tht = np.concatenate([g.uniform(-0.5, 0.5, (P, 4)), g.uniform(0, 25, (P, 1)),
                          g.uniform(0.8, 1.2, (P, n_theta - 5))], axis=1)
    ttt = torch.tensor(tht, dtype=torch.float64, device=dev)
    nl = torch.empty(P, dtype=torch.float64, device=dev)
    gr = torch.empty(P, n_theta, dtype=torch.float64, device=dev)
    tms = {}
    for mode, gg in (("nll", None), ("grad", gr)):
        ctx.eval_nll_templates_dev(ttt, nl, gg, stream=s)
        s.synchronize()
        ev0.record(s)
        for _ in range(3):
            ctx.eval_nll_templates_dev(ttt, nl, gg, stream=s)
        ev1.record(s)
        s.synchronize()
        tms[mode] = ev0.elapsed_time(ev1) / 3
    ctx.eval_nll_templates_dev(tt, out, None, stream=s)   # the streaming path's points
    s.synchronize()
    stream_nll = ctx.eval_nll(th[:16])
    d_vs_stream = float(np.max(np.abs(out.cpu().numpy()[:16] - stream_nll)))
    ctx.close()
    return dict(evals_per_s=round(n_pts / dt, 1), points=n_pts,
                templates=dict(evals_per_s=round(P / (tms["nll"] * 1e-3), 1),
                               grad_evals_per_s=round(P / (tms["grad"] * 1e-3), 1),
                               points=P, ms=round(tms["nll"], 3),
                               grad_ms=round(tms["grad"], 3),
                               template_fold_ms=round(t_fold * 1e3, 1),
                               max_abs_dnll_vs_streaming=d_vs_stream),
                us_per_eval=round(dt / n_pts * 1e6, 2), components=K,
                backgrounds=2, n_theta=n_theta, algorithmic_bytes=alg,
                step_kernel_us=round(step_ms * 1e3, 2),
                achieved_gbs=round(alg / (step_ms * 1e-3) / 1e9, 1),
                frac_hbm=round(alg / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                setup_seconds=round(t_setup, 1),
                what="Eqs. (Rij), (fNp_reweight), (mu_total): 5 components x "
                     "16384 x 4096 FP32 responses stacked, one R stream per "
                     "evaluation through the step kernel")


def gemm_counter_pass():
    """The batched likelihood GEMM alone, for hardware counters: 1024 points
    on a 4096 x 4096 dataset (one of the 64-dataset scan's shapes; 256
    tiles of 128 x 128, one per compute unit), eight calls after the tuner
    has picked its tile."""
    import torch
    import synth
    import paper_2607_00488_amd as nr
    dev = torch.device("cuda:0")
    src = synth.source_nodes(256)
    rsp = synth.response_mc(4096, 4096, 1_000_000, seed=2001, keep_counts=False)
    ctx = nr.Context(0)
    ctx.set_sources(src, 4096)
    ctx.set_response(rsp.R, n_sig=1.0e4)
    b = np.full(4096, 10.0)
    ctx.set_data(b, b)
    th = synth.theta_prior(1024, 2002)
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    nl = torch.empty(1024, dtype=torch.float64, device=dev)
    nr.eval_nll_multi_dev([ctx], [tt], [nl])       # tunes and captures
    torch.cuda.synchronize()
    for _ in range(8):
        nr.eval_nll_multi_dev([ctx], [tt], [nl])
    torch.cuda.synchronize()
    ctx.close()
    log("[bench] GEMM counter pass done: 8 calls of 2 x 1024 x 4096 x 4096 flop")


def grad_counter_pass():
    """The batched likelihood and gradient alone, for hardware counters:
    1024 points on the 16384 x 4096 shapes of the single-point benchmark
    (the dense products read every entry, so a response histogrammed from
    fewer events does the same work), eight calls after the tuner has
    picked its tiles: the weights, the forward product with its Poisson
    epilogue, the adjoint product and the gradient contraction."""
    import torch
    import synth
    import paper_2607_00488_amd as nr
    dev = torch.device("cuda:0")
    src = synth.source_nodes(2048)
    rsp = synth.response_mc(16384, 4096, 4_000_000, seed=2301, keep_counts=False)
    ctx = nr.Context(0)
    ctx.set_sources(src, 16384)
    ctx.set_response(rsp.R, n_sig=1.0e4)
    b = np.full(4096, 10.0)
    ctx.set_data(b, b)
    th = synth.theta_prior(1024, 2302)
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    nl = torch.empty(1024, dtype=torch.float64, device=dev)
    gr = torch.empty(1024, 7, dtype=torch.float64, device=dev)
    nr.eval_nll_multi_dev([ctx], [tt], [nl], [gr])   # tunes and captures
    torch.cuda.synchronize()
    for _ in range(8):
        nr.eval_nll_multi_dev([ctx], [tt], [nl], [gr])
    torch.cuda.synchronize()
    ctx.close()
    log("[bench] gradient counter pass done: 8 calls of 1024 points at 16384 x 4096, "
        "2 x 2 x 1024 x 16384 x 4096 flop in the two products")


def mlp_counter_pass():
    """The surrogate network's kernels alone, for matrix-core counters: a
    7-256-256-256-4096 network (random weights; the work does not depend
    on them), 8 training steps of 2048 points, then 8 inference calls of
    65536 points through the fused network-and-likelihood kernel.  Data
    and response are 4096 bins of a 512-row synthetic analysis (the network
    never reads the response)."""
    import torch
    import synth
    import paper_2607_00488_amd as nr
    from paper_2607_00488_amd.surrogate import Surrogate, init_params
    dev = torch.device("cuda:0")
    g = synth.rng(2201)
    n_t, n_reco = 512, 4096
    R = (g.random((n_t, n_reco), dtype=np.float32) / n_reco).astype(np.float32)
    ctx = nr.Context(0)
    ctx.set_sources(synth.source_nodes(256), n_t)
    ctx.set_response(R, n_sig=1.0e4)
    ctx.set_data(g.poisson(10.0, n_reco).astype(np.float64), np.full(n_reco, 10.0))
    lo, hi = synth.theta_box()
    sur = Surrogate(n_reco, lo, hi, hidden=256, seed=2202)
    sur.set_params(init_params(256, n_reco, 2203, out_scale=1.0))
    nr.nr_mlp_set_output_norm(sur.h, np.full(n_reco, 2.0, np.float32),
                              np.full(n_reco, 0.3, np.float32))
    th = sur.sample_box(2048, 2204)
    tg = torch.randn(2048, n_reco, dtype=torch.float32, device=dev,
                     generator=torch.Generator(device=dev).manual_seed(2205))
    s = torch.cuda.current_stream(dev)
    for _ in range(8):
        nr.nr_mlp_train_step_dev(sur.h, th.data_ptr(), tg.data_ptr(), 2048, 1e-4,
                                 False, s.cuda_stream)
    thi = sur.sample_box(1 << 16, 2206)
    for _ in range(8):
        sur.nll(ctx, thi)
    torch.cuda.synchronize()
    sur.close()
    ctx.close()
    log("[bench] MLP counter pass done: 8 training steps of 2048, 8 inference "
        "calls of 65536 points")


def tmpl_counter_pass():
    """The template form's evaluation kernels alone, for instruction
    counters: 65536 points over 4096 observed bins (the per-point cost does
    not depend on N_T, so a 4096-row response keeps the set-up short), one
    untimed call of each variant, then 8 likelihood calls and 8 calls with
    the gradient."""
    import torch
    import synth
    import paper_2607_00488_amd as nr
    dev = torch.device("cuda:0")
    src = synth.source_nodes(256)
    rsp = synth.response_mc(4096, 4096, 1_000_000, seed=2101, keep_counts=False)
    ctx = nr.Context(0)
    ctx.set_sources(src, 4096)
    ctx.set_response(rsp.R, n_sig=1.0e4)
    b = np.full(4096, 10.0)
    ctx.set_data(synth.poisson_data(b + 30.0, 2102), b)
    P = 65536
    tt = torch.tensor(synth.theta_prior(P, 2103, f_range=(0.8, 1.2)),
                      dtype=torch.float64, device=dev)
    nl = torch.empty(P, dtype=torch.float64, device=dev)
    gr = torch.empty(P, 7, dtype=torch.float64, device=dev)
    ctx.build_templates()
    ctx.eval_nll_templates_dev(tt, nl)
    ctx.eval_nll_templates_dev(tt, nl, gr)
    torch.cuda.synchronize()
    for _ in range(8):
        ctx.eval_nll_templates_dev(tt, nl)
    for _ in range(8):
        ctx.eval_nll_templates_dev(tt, nl, gr)
    torch.cuda.synchronize()
    ctx.close()
    log("[bench] template counter pass done: 8 + 8 calls of 65536 points x 4096 bins")


def cpu_baseline(p, n_eval, gpu_ctx):
    """The FP64 oracle on the host cores for a bounded sample of points, and
    the GPU's -2lnL on the same inputs for the |Delta| column."""
    import oracle
    import synth
    c = p["cfg"]
    o = oracle.Oracle()
    o.set_sources(p["src"], c.n_t)
    o.set_response(p["R"], n_sig=c.n_sig)
    sig = o.mu(oracle.THETA_SM)
    n = synth.poisson_data(sig + p["b"], p["seeds"]["data"])
    o.set_data(n, p["b"])
    th = synth.theta_prior(n_eval, p["seeds"]["theta"] + 17)
    o.nll(th[0])  # warm-up (page-in of the response)
    t0 = time.perf_counter()
    ref = [o.nll(t) for t in th]
    dt = time.perf_counter() - t0
    cores = oracle.get_threads()
    # the paper's protocol (ten consecutive evaluations, the first dropped,
    # mean and spread of the other nine), with all threads and with one
    def protocol(threads, n=10):
        oracle.set_threads(threads)
        ts = []
        for t in th[:n]:
            t1 = time.perf_counter()
            o.nll(t)
            ts.append(time.perf_counter() - t1)
        oracle.set_threads(cores)
        ts = np.array(ts[1:]) * 1e3
        return [round(float(ts.mean()), 2), round(float(ts.std()), 2)]
    all_threads = protocol(cores)
    one_thread = protocol(1, n=4)
    gpu_ctx.set_data(n, p["b"])
    got = gpu_ctx.eval_nll(th)
    gpu_ctx.set_data(p["n"], p["b"])
    return dict(value=n_eval / dt, unit="evals/s", cores=cores,
                kind="oracle",
                sample=f"{n_eval} plain evaluations at the same 16384x4096 "
                       f"workload (prior-box points), FP64, OpenMP over bins",
                seconds=dt,
                paper_protocol_ms=dict(threads=cores, mean_std=all_threads),
                one_thread_ms=dict(evals=3, mean_std=one_thread)), \
        float(np.max(np.abs(np.array(got) - ref)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points-per-step", type=int, default=100,
                    help="parameter points per step (one scan row)")
    ap.add_argument("--cpu-evals", type=int, default=96,
                    help="oracle evaluations timed for cpu_baseline (~10 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-components", action="store_true")
    ap.add_argument("--no-banded", action="store_true",
                    help="skip the band-skipping forms (a trace of the dense "
                         "step kernel alone)")
    ap.add_argument("--surrogate-seconds", type=float, default=20.0)
    ap.add_argument("--gemm-counter-pass", action="store_true",
                    help="short run for matrix-core counters: the batched "
                         "likelihood GEMM of 1024 points on a 4096 x 4096 "
                         "dataset (a shape of the 64-dataset scan), 8 calls")
    ap.add_argument("--grad-counter-pass", action="store_true",
                    help="short run for matrix-core counters of the batched "
                         "gradient: 8 calls of 1024 points at 16384 x 4096")
    ap.add_argument("--mlp-counter-pass", action="store_true",
                    help="short run for matrix-core counters of the surrogate "
                         "network: 8 training steps of 2048 points, 8 fused "
                         "inference calls of 65536 points")
    ap.add_argument("--tmpl-counter-pass", action="store_true",
                    help="short run for instruction counters: the template "
                         "form's evaluation on 65536 points x 4096 bins, "
                         "8 calls without and 8 with the gradient")
    ap.add_argument("--counter-pass", action="store_true",
                    help="short run for hardware-counter collection: 20 "
                         "single-point evaluations, then 20 plain 256 MiB "
                         "device copies as the byte-count reference")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no "
              "multi-GPU path (a parameter scan would shard by points and "
              "needs no collective)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    dev = torch.device("cuda:0")
    if args.gemm_counter_pass:
        gemm_counter_pass()
        return
    if args.tmpl_counter_pass:
        tmpl_counter_pass()
        return
    if args.mlp_counter_pass:
        mlp_counter_pass()
        return
    if args.grad_counter_pass:
        grad_counter_pass()
        return
    p = build_plain(1)
    ctx, c = p["ctx"], p["cfg"]
    if args.counter_pass:
        th = torch.tensor(synth.theta_prior(20, 99), dtype=torch.float64,
                          device=dev)
        out = torch.empty(20, dtype=torch.float64, device=dev)
        ctx.set_fold_tiling(0, 0)           # eager launches, one per kernel
        ctx.eval_nll_dev(th, out)
        torch.cuda.synchronize()
        a = torch.empty(1 << 26, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(20):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] counter pass done")
        return
    K, W, PPS = args.steps, args.warmup, args.points_per_step
    NE = K * PPS                      # evaluations in the timed region
    th = synth.theta_prior(NE, p["seeds"]["theta"])
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    out = torch.empty(NE, dtype=torch.float64, device=dev)
    thw = torch.tensor(synth.theta_prior(max(W, 1) * PPS, p["seeds"]["theta"] + 1),
                       dtype=torch.float64, device=dev)
    outw = torch.empty(max(W, 1) * PPS, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    # warm-up: captures the timed and the warm-up graphs and runs them once
    ctx.eval_nll_dev(thw, outw, stream=stream)
    ctx.eval_nll_dev(tt, out, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    ctx.eval_nll_dev(tt, out, stream=stream)
    ev1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # device time of the timed region on the stream the step kernels run
    # on: NE + 4 launches, NE - 4 of them the steady-state k_step
    dev_ms = ev0.elapsed_time(ev1)
    ms_step = dt * 1e3 / K
    evals_s = NE / dt
    log(f"[bench] plain: {ms_step * 1e3:.2f} us/eval, {evals_s:.0f} evals/s")

    # host-visible synchronous latency (paper protocol: 10 calls, drop 1st)
    lat = []
    for i in range(10):
        t1 = time.perf_counter()
        ctx.eval_nll(th[i])
        lat.append(time.perf_counter() - t1)
    lat = np.array(lat[1:]) * 1e3

    # roofline of the dominant kernel, the step kernel as the pipeline runs
    # it: device time of the timed region (HIP events on its stream) per
    # evaluation, which charges the 8 shorter fill/drain launches to the
    # NE - 4 steady-state ones (a conservative average); the steady-state
    # launch alone back to back, the fold role alone and the other stages
    # for the breakdown
    step_ms = dev_ms / NE
    step_bb_ms = ctx.time_stage(5, 200)
    # the same launch after 512 MiB of other data have been read through the
    # device's caches (the 256 MB Infinity Cache included): the cold-cache
    # figure (a read, so no dirty lines are left to write back)
    flush = torch.ones(1 << 27, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    cold, warm = [], []
    for i in range(20):
        flush.sum()
        torch.cuda.synchronize()
        cold.append(ctx.time_stage(5, 1))
        warm.append(ctx.time_stage(5, 1))   # the same single launch, warm
    del flush
    step_cold_ms = float(np.mean(cold))
    step_warm1_ms = float(np.mean(warm))
    fold_ms = ctx.time_stage(4, 200)
    fold_lik_ms = ctx.time_stage(2, 200)
    eint_ms = ctx.time_stage(1, 200)
    alg_bytes = algorithmic_bytes(c.n_t, c.n_reco)
    achieved = alg_bytes / (step_ms * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=measured_traffic(), kernel="k_step",
                avg_kernel_us=round(step_ms * 1e3, 2),
                algorithmic_bytes=alg_bytes,
                note="effective rate: the algorithmic bytes of a launch over "
                     "its time, whether HBM or the Infinity Cache served "
                     "them (consecutive points walk R in opposite "
                     "directions and reuse what the last one left cached); "
                     "one launch after a 512 MiB cache flush: "
                     "detail.step_after_cache_flush_us")
    res = dict(metric=METRIC, value=round(evals_s, 1), unit="evals/s",
               n_gpus=1, steps=K, warmup=W, ms_per_step=round(ms_step, 5),
               points_per_step=PPS,
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f64", data="synthetic",
               config=dict(workload="plain single-point eval: N_T=16384 "
                           "recoil bins, N_reco=4096, N_E=2048 per continuum "
                           "(5 solar sources), dense FP32 response 256 MiB "
                           "from 1e8 seeded MC events",
                           n_t=c.n_t, n_reco=c.n_reco, n_e=c.n_e),
               roofline=roof,
               detail=dict(sync_latency_ms_mean=round(float(lat.mean()), 4),
                           sync_latency_ms_std=round(float(lat.std()), 4),
                           eint_weights_us=round(eint_ms * 1e3, 2),
                           step_back_to_back_us=round(step_bb_ms * 1e3, 2),
                           step_single_launch_us=round(step_warm1_ms * 1e3, 2),
                           step_after_cache_flush_us=round(step_cold_ms * 1e3, 2),
                           fold_alone_us=round(fold_ms * 1e3, 2),
                           fold_plus_likelihood_us=round(fold_lik_ms * 1e3, 2)))
    forms = {}
    if not args.no_banded:
        forms["plain_banded"] = banded_form(ctx, p["R"], tt, out, stream)
        log(f"[bench] plain with band skipping: "
            f"{forms['plain_banded']['evals_per_s']:.0f} evals/s, bitwise equal: "
            f"{forms['plain_banded']['bitwise_equal_to_dense']}")
    # the FP64 matrix-core rate the chip sustains on register operands: the
    # practical ceiling of the batched GEMM beside the data-sheet 78.6
    import paper_2607_00488_amd as nr
    probe = nr.nr_probe_mfma_f64(0, 8192, 16)
    res["detail"]["fp64_mfma_probe_tflops"] = round(probe, 2)
    # and the HBM read rate of a plain stream (2 GiB, far beyond the caches)
    rd = nr.nr_probe_hbm_read(0, 2 << 30, 10)
    res["detail"]["hbm_read_probe_gbs"] = round(rd, 1)
    res["detail"]["step_frac_of_read_probe"] = round(roof["achieved"] / rd, 4)
    # the same stream over a buffer of R's size with ordinary loads and
    # passes alternating in direction, as consecutive fold passes read R:
    # HBM plus what L2 and the Infinity Cache keep between passes
    r_bytes = 4 * c.n_t * ((c.n_reco + 3) // 4 * 4)
    rc_ = nr.nr_probe_read(0, r_bytes, 40, nr.NR_PROBE_CACHED | nr.NR_PROBE_ALTERNATE)
    res["detail"]["cache_read_probe_gbs"] = round(rc_, 1)
    res["detail"]["step_frac_of_cache_read_probe"] = round(roof["achieved"] / rc_, 4)
    log(f"[bench] probes: FP64 MFMA {probe:.1f} TFLOP/s, HBM read {rd:.0f} GB/s, "
        f"R-sized alternating cached read {rc_:.0f} GB/s")
    # gradient form: 1024 points at the same shapes, -2lnL + 7 derivatives
    # per point through the FP64-MFMA forward and adjoint products
    thg = synth.theta_prior(1024, p["seeds"]["theta"] + 5, f_range=(0.8, 1.2))
    dtg, _, _ = time_batched([ctx], [thg], reps=3, grad=True)
    forms["grad_batched"] = dict(
        evals_per_s=round(1024 / dtg, 1), points=1024, ms=round(dtg * 1e3, 3),
        flop=2 * 2.0 * 1024 * c.n_t * c.n_reco,
        tflops=round(2 * 2.0 * 1024 * c.n_t * c.n_reco / dtg / 1e12, 2),
        peak_tflops=78.6,
        frac_of_probe=round(2 * 2.0 * 1024 * c.n_t * c.n_reco / dtg / 1e12 / probe, 3),
        what="nll + gradient, forward and adjoint GEMMs")
    dtb, _, _ = time_batched([ctx], [thg], reps=3, grad=False)
    forms["nll_batched_same_shapes"] = dict(
        evals_per_s=round(1024 / dtb, 1), points=1024, ms=round(dtb * 1e3, 3),
        tflops=round(2.0 * 1024 * c.n_t * c.n_reco / dtb / 1e12, 2),
        frac_of_probe=round(2.0 * 1024 * c.n_t * c.n_reco / dtb / 1e12 / probe, 3))
    log(f"[bench] grad batched: {1024 / dtg:.0f} evals/s; nll batched "
        f"{1024 / dtb:.0f} evals/s")
    if not args.no_banded:
        # the same two with band skipping: every GEMM tile reduces only over the
        # K-steps where its response entries are not all zero (results equal to
        # rounding: the tuner may pick another tile shape, bitwise equality at a
        # fixed shape is tested)
        _, nl_d, g_d = time_batched([ctx], [thg], reps=1, grad=True)
        ctx.set_band_skipping(True)
        dtgb, nl_b, g_b = time_batched([ctx], [thg], reps=3, grad=True)
        dtbb, _, _ = time_batched([ctx], [thg], reps=3, grad=False)
        ctx.set_band_skipping(False)
        forms["batched_banded"] = dict(
            evals_per_s=round(1024 / dtbb, 1), grad_evals_per_s=round(1024 / dtgb, 1),
            points=1024, ms=round(dtbb * 1e3, 3), grad_ms=round(dtgb * 1e3, 3),
            max_abs_dnll_vs_dense=float(np.max(np.abs(nl_b[0] - nl_d[0]))),
            max_rel_dgrad_vs_dense=float(np.max(np.abs(g_b[0] - g_d[0])) /
                                         np.max(np.abs(g_d[0]))),
            what="the batched likelihood and gradient with band skipping: each "
                 "tile of the forward and adjoint GEMMs reduces only over the "
                 "K-steps of 16 where its response entries are not all zero")
        log(f"[bench] batched with band skipping: {1024 / dtbb:.0f} evals/s, "
            f"{1024 / dtgb:.0f} with gradient")
    forms["plain_config0"] = pc = plain_config0_form()
    log(f"[bench] plain at 512 x 256: {pc['evals_per_s']:.0f} evals/s "
        f"({pc['us_per_eval']:.2f} us/eval)")
    forms["templates"] = tf = templates_form(ctx, p["seeds"]["theta"] + 7)
    log(f"[bench] templates: {tf['evals_per_s']:.0f} evals/s "
        f"({tf['grad_evals_per_s']:.0f} with gradient), fold "
        f"{tf['template_fold_ms']:.1f} ms once, max |d| vs plain "
        f"{tf['max_abs_dnll_vs_plain']:.2e}")
    forms["ess"] = ef = ess_form(ctx, p["row_events"], p["seeds"]["theta"] + 9)
    log(f"[bench] ESS diagnostic: {ef['evals_per_s']:.0f} evals/s "
        f"({ef['us_per_eval']:.1f} us/eval, {ef['gbs']:.0f} GB/s)")
    forms["asimov_scan"] = sc = asimov_scan_form(p)
    log(f"[bench] Asimov scan (31 values, nuisances profiled): batched "
        f"{sc['batched']['seconds']:.3f} s warm / {sc['batched']['first_seconds']:.2f} s "
        f"first ({sc['batched']['calls']} calls), templates "
        f"{sc['templates']['seconds']:.3f} s / {sc['templates']['first_seconds']:.3f} s; "
        f"interval {sc['templates']['interval_90']}")
    if not args.no_batched:
        ctxs, ths, flops = build_batched()
        dt2, nls, _ = time_batched(ctxs, ths, reps=2)
        npts = sum(len(t) for t in ths)
        # agreement with the single-point path: the first and last point of
        # each of the 16 shape classes (datasets 0-15)
        dscan = 0.0
        for d in range(min(16, len(ctxs))):
            k = [0, len(ths[d]) - 1]
            pl = ctxs[d].eval_nll(ths[d][k])
            dscan = max(dscan, float(np.max(np.abs(pl - nls[d][k]))))
        forms["batched_scan_64_datasets"] = dict(
            evals_per_s=round(npts / dt2, 1), points=npts,
            ms=round(dt2 * 1e3, 3), flop=flops,
            tflops=round(flops / dt2 / 1e12, 2), peak_tflops=78.6,
            frac_of_probe=round(flops / dt2 / 1e12 / probe, 3),
            max_abs_dnll_vs_plain=dscan,
            checked="first and last point of each of the 16 shape classes "
                    "against the single-point path",
            what="64 datasets, N_T 2048-16384, N_reco 512-4096, one grouped "
                 "persistent FP64-MFMA launch per scan (graph replay)")
        log(f"[bench] batched scan: {npts / dt2:.0f} evals/s, "
            f"{flops / dt2 / 1e12:.1f} TFLOP/s, max |d| vs plain {dscan:.2e}")
        for cx in ctxs:
            cx.close()
    if not args.no_surrogate:
        forms["surrogate"] = sf = surrogate_form(ctx, args.surrogate_seconds,
                                                 n_data=p["n"])
        log(f"[bench] surrogate: {sf['evals_per_s']:.0f} evals/s with "
            f"fallback {sf['fallback']} ({sf['fallback_fraction']:.2f}); "
            f"network alone {sf['network_only_evals_per_s']:.0f} evals/s; "
            f"gain {sf['gain_vs_exact_batched']}x; median |d| "
            f"{sf['val_abs_dnll']['median']:.3g}")
    if not args.no_components:
        forms["multi_component"] = mc = components_form()
        log(f"[bench] multi-component: {mc['evals_per_s']:.0f} evals/s, "
            f"{mc['achieved_gbs']:.0f} GB/s ({mc['frac_hbm']:.3f} of peak); "
            f"templates {mc['templates']['evals_per_s']:.0f} evals/s "
            f"({mc['templates']['grad_evals_per_s']:.0f} with gradient), "
            f"max |d| vs streaming {mc['templates']['max_abs_dnll_vs_streaming']:.1e}")
    res["forms"] = forms
    if not args.no_cpu_baseline:
        cb, dmax = cpu_baseline(p, args.cpu_evals, ctx)
        res["cpu_baseline"] = cb
        res["detail"]["max_abs_dnll_vs_oracle"] = dmax
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
