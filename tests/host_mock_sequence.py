"""Call sequences for tests/test_host_mock.py: run as a child process with
the library built host-only against the CPU stand-in of the HIP runtime
and AddressSanitizer preloaded.  The results are meaningless (no kernel
runs); the run checks that the host code of every call stays in bounds.
Usage: host_mock_sequence.py LIBRARY {broad|paper}."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, ".."))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import paper_2607_00488_amd as nr  # noqa: E402
import synth  # noqa: E402
from problems import config_inputs, gpu_context, inputs  # noqa: E402

nr._LIB_PATH = sys.argv[1]
which = sys.argv[2]


def step(name, f, *a):
    out = f(*a)
    print(f"[mock] {name}", flush=True)
    return out


pm = np.array([0, 0, 0, 0, 0, 1.0, 1.0])
ps = np.array([0, 0, 0, 0, 0, 0.1, 0.1])
th = np.vstack([synth.theta_sm()[None], synth.theta_corners()[[0, 31]],
                synth.theta_prior(64, 3001, f_range=(0.8, 1.2))])
if which == "paper":
    # the sequence of the skipped paper-scale test: 67 likelihoods, then
    # the spectra of the first 4 points, on the 16384 x 4096 context
    p = config_inputs(1)
    ctx = gpu_context(p, pulls=(pm, ps))
    step("eval_nll 67", ctx.eval_nll, th)
    step("eval_mu 4", ctx.eval_mu, th[:4])
    step("eval_mu 1", ctx.eval_mu, th[:1])
    step("eval_nll_grad 2", ctx.eval_nll_grad, th[:2])
    step("eval_nll 1", ctx.eval_nll, th[:1])
    ctx.close()
else:
    p = config_inputs(0)
    ctx = gpu_context(p, pulls=(pm, ps))
    step("eval_nll 67", ctx.eval_nll, th)
    step("eval_mu 4", ctx.eval_mu, th[:4])
    step("eval_weights 3", ctx.eval_weights, th[:3])
    step("eval_nll_grad 5", ctx.eval_nll_grad, th[:5])
    step("eval_mu 67", ctx.eval_mu, th)
    step("eval_nll 2", ctx.eval_nll, th[:2])
    step("set_mc_events", ctx.set_mc_events, p["row_events"].astype(np.float64))
    step("eval_ess 3", ctx.eval_ess, th[:3])
    step("reference", ctx.reference)
    step("band skipping on", ctx.set_band_skipping, True)
    step("eval_nll 9 (bands)", ctx.eval_nll, th[:9])
    step("eval_nll_grad 2 (bands)", ctx.eval_nll_grad, th[:2])
    step("band skipping off", ctx.set_band_skipping, False)
    step("fold tiling 16", ctx.set_fold_tiling, 16)
    step("eval_nll 5 (16-row tiles)", ctx.eval_nll, th[:5])
    step("eval_nll_batched 67", ctx.eval_nll_batched, th)
    step("eval_nll_grad_batched 33", ctx.eval_nll_grad_batched, th[:33])
    step("eval_mu_batched 10", ctx.eval_mu_batched, th[:10])
    step("build_templates", ctx.build_templates)
    step("eval_nll_templates 30", ctx.eval_nll_templates, th[:30])
    step("eval_mu_templates 3", ctx.eval_mu_templates, th[:3])
    step("eval_nll_templates 5 (gradient)", ctx.eval_nll_templates, th[:5], True)
    step("set_data again", ctx.set_data, p["n"], p["b"])
    step("eval_nll 3 (new data)", ctx.eval_nll, th[:3])
    step("set_response again", lambda: ctx.set_response(0.5 * p["R"], n_sig=p["n_sig"]))
    step("eval_nll 4 (new response)", ctx.eval_nll, th[:4])
    step("eval_mu 4 (new response)", ctx.eval_mu, th[:4])
    ctx.close()
    # a second context of ragged shapes
    q = inputs(333, 77, 37, 200_000, 91, 92)
    c2 = gpu_context(q)
    step("333 x 77: eval_nll 67", c2.eval_nll, th)
    step("333 x 77: eval_mu 4", c2.eval_mu, th[:4])
    step("333 x 77: eval_nll_grad 3", c2.eval_nll_grad, th[:3])
    step("333 x 77: eval_nll_batched 67", c2.eval_nll_batched, th)
    step("333 x 77: eval_nll_templates 9", lambda: (c2.build_templates(),
                                                   c2.eval_nll_templates(th[:9])))
    c2.close()
print("mock sequence done", flush=True)
