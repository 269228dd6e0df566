"""The effective-sample-size diagnostic on the GPU against the oracle's
definition, at the parity workload and a ragged shape."""
import sys

import numpy as np
import pytest

import synth
from oracle.diagnostics import ess
from problems import config_inputs, gpu_context, inputs, parity_thetas

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape", ["config0", "ragged"])
def test_ess_parity(shape):
    import paper_2607_00488_amd as nr
    if shape == "config0":
        p = config_inputs(0)
        th = parity_thetas(0, 64)
    else:
        p = inputs(333, 77, 37, 200_000, 901, 902)
        th = parity_thetas(0, 16)
    ctx = gpu_context(p)
    with pytest.raises(nr.NrError):
        ctx.eval_ess(th[:1])                  # before set_mc_events
    ctx.set_mc_events(p["row_events"].astype(np.float64))
    got = ctx.eval_ess(th)
    o = p["oracle"]
    w = np.vstack([o.weights(t) for t in th])
    ref = ess(p["R"], p["row_events"], w)
    scale = np.maximum(ref, 1e-6 * ref.max())
    worst = float(np.max(np.abs(got - ref) / scale))
    log(f"[gpu] ESS {shape}: {len(th)} points, max rel diff {worst:.2e}")
    assert worst <= 1e-9
    # at theta_SM the weights are one: ESS is the raw MC histogram
    raw = ess(p["R"], p["row_events"], np.ones(p["n_t"]))[0]
    assert np.allclose(got[0], raw, rtol=1e-12, atol=0)
    ctx.close()


def test_ess_magnetic_moment_low_recoil():
    """A large magnetic moment weights the low-recoil MC up (1/T): the
    effective sample of the lowest observed bins falls below the raw count,
    while the SM point keeps every bin at its raw count."""
    p = config_inputs(0)
    ctx = gpu_context(p)
    ctx.set_mc_events(p["row_events"].astype(np.float64))
    th = np.vstack([synth.theta_sm(), synth.theta_sm()])
    th[1, 4] = 25.0                           # mu_nu = 5e-11 mu_B
    e = ctx.eval_ess(th)
    raw = e[0]
    ok = raw > 0
    ratio = e[1][ok] / raw[ok]
    log(f"[gpu] ESS/raw at m2 = 25: min {ratio.min():.3f} (bin "
        f"{int(np.flatnonzero(ok)[np.argmin(ratio)])}), median {np.median(ratio):.3f}")
    assert ratio.min() < 0.95
    assert np.all(ratio <= 1.0 + 1e-12)
    ctx.close()
