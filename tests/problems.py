"""Matched analyses for the parity tests: the same seeded inputs handed to
the FP64 oracle and (when a GPU is present) to the HIP library."""
from __future__ import annotations

import functools

import numpy as np

import oracle
import synth


@functools.lru_cache(maxsize=4)
def inputs(n_t, n_reco, n_e, n_mc, seed_rsp, seed_data, n_sig=1.0e4,
           bkg=10.0, t_hi=16.0):
    src = synth.source_nodes(n_e)
    rsp = synth.response_mc(n_t, n_reco, n_mc, seed=seed_rsp, keep_counts=False)
    o = oracle.Oracle()
    o.set_sources(src, n_t, 0.0, t_hi)
    o.set_response(rsp.R, n_sig=n_sig)
    b = np.full(n_reco, bkg)
    # before set_data the oracle's mu holds the signal only
    sig_sm = o.mu(oracle.THETA_SM)
    n = synth.poisson_data(sig_sm + b, seed_data)
    o.set_data(n, b)
    return dict(src=src, R=rsp.R, b=b, n=n, oracle=o, n_t=n_t, n_reco=n_reco,
                n_sig=n_sig, t_hi=t_hi, row_events=rsp.row_events)


def config_inputs(cfg: int):
    c = synth.CONFIGS[cfg]
    s = c.seeds(0)
    return inputs(c.n_t, c.n_reco, c.n_e, c.n_mc, s["response"], s["data"],
                  c.n_sig, c.bkg)


def gpu_context(p, device=0, pulls=None):
    import paper_2607_00488_amd as nr
    ctx = nr.Context(device)
    ctx.set_sources(p["src"], p["n_t"], 0.0, p["t_hi"])
    ctx.set_response(p["R"], n_sig=p["n_sig"])
    if pulls is None:
        ctx.set_data(p["n"], p["b"])
    else:
        ctx.set_data(p["n"], p["b"], *pulls)
    return ctx


def parity_thetas(cfg: int, n: int = 1024):
    s = synth.CONFIGS[cfg].seeds(0)
    return np.vstack([synth.theta_sm()[None], synth.theta_corners(),
                      synth.theta_prior(n, s["theta"])])
