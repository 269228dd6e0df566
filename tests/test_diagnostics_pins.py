"""Pins of the oracle's effective-sample-size definition (no GPU): a worked
example by hand, the unweighted limit (ESS = the raw MC histogram), scale
invariance, and the Cauchy-Schwarz bound."""
import numpy as np
import pytest

import oracle
import synth
from oracle.diagnostics import ess


def test_hand_example():
    # two true bins of 10 events, half of each in the one observed bin,
    # weights 1 and 3: (5 + 15)^2 / (5 + 45) = 8
    R = np.array([[0.5], [0.5]], dtype=np.float32)
    assert ess(R, [10, 10], [1.0, 3.0])[0, 0] == pytest.approx(8.0, rel=1e-15)
    # a bin nothing reaches
    R0 = np.zeros((2, 1), dtype=np.float32)
    assert ess(R0, [10, 10], [1.0, 3.0])[0, 0] == 0.0


@pytest.fixture(scope="module")
def mc():
    rsp = synth.response_mc(256, 128, 200_000, seed=7, keep_counts=True)
    return rsp


def test_unweighted_is_raw_histogram(mc):
    raw = mc.counts.sum(0).astype(np.float64)
    e = ess(mc.R, mc.row_events, np.ones(256))[0]
    # R is float32 counts / events: N_lj = R_lj n_l to float32 rounding
    assert np.allclose(e, raw, rtol=1e-6, atol=1e-6)
    # a constant weight changes nothing
    assert np.allclose(ess(mc.R, mc.row_events, np.full(256, 3.7))[0], e,
                       rtol=1e-12)


def test_bound_and_weights_from_oracle(mc):
    g = synth.rng(11)
    w = g.uniform(0.1, 5.0, (4, 256))
    e = ess(mc.R, mc.row_events, w)
    raw = ess(mc.R, mc.row_events, np.ones(256))[0]
    assert np.all(e <= raw * (1 + 1e-12))
    assert np.all(e[:, raw > 0] > 0)
    # at theta_SM the oracle's weights are exactly one
    src = synth.source_nodes(64)
    o = oracle.Oracle()
    o.set_sources(src, 256, 0.0, 16.0)
    o.set_response(mc.R, n_sig=1e4)
    w_sm = o.weights(oracle.THETA_SM)
    assert np.all(w_sm == 1.0)
    assert np.array_equal(ess(mc.R, mc.row_events, w_sm)[0], raw)
