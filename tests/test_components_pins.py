"""Pins of the multi-component oracle (no GPU).  It is checked against what
does not depend on its own formulation: the single-component oracle it must
reduce to, the closed form at the SM point (every weight one), the
normalisation of Eq. (Rij), scale invariance under a uniform mask, and
linearity in the component rates."""
import numpy as np
import pytest

import oracle
import synth
from oracle.components import ComponentOracle

N_T, N_RECO = 128, 64


@pytest.fixture(scope="module")
def single():
    src = synth.source_nodes(64)
    rsp = synth.response_mc(N_T, N_RECO, 200_000, seed=31, keep_counts=False)
    o = oracle.Oracle()
    o.set_sources(src, N_T)
    o.set_response(rsp.R, n_sig=1e4)
    b = np.full(N_RECO, 10.0)
    o.set_data(np.zeros(N_RECO), b)
    return src, rsp.R, o, b


def test_reduces_to_single_component(single):
    """One component holding every source, histogram = the single form's
    joint SM histogram m_l R_lj, the background b as one template: the
    prediction is the single-component oracle's at f_8B = 1."""
    src, R, o, b = single
    m = o.row_factors()
    joint = (m[:, None] * R.astype(np.float64))[None]
    tot = joint.sum()
    co = ComponentOracle(src, np.zeros(len(src), int), N_T, joint.astype(np.float32),
                         scale=[1.0], rate_sm=[tot], bkg_pdf=[b / b.sum()],
                         bkg_rate=[b.sum()])
    for th in [synth.theta_sm(), *synth.theta_prior(6, 41)]:
        th = th.copy()
        th[5] = 1.0
        multi = np.concatenate([th[:5], [1.0, th[6]]])
        ref = o.mu(th)
        got = co.mu(multi)
        # the joint histogram passes through FP32 storage once more
        assert np.allclose(got, ref, rtol=2e-6, atol=1e-9 * ref.max())
    co.close()


@pytest.fixture(scope="module")
def comp():
    src = synth.source_nodes(64)
    d = synth.component_inputs(N_T, N_RECO, 100_000, 51)
    co = ComponentOracle(src, d["comp_of_source"], N_T, d["hist"], d["scale"],
                         d["rate_sm"], d["bkg_pdf"], d["bkg_rate"],
                         d["comp_mask"], d["mask"], d["exposure"])
    return src, d, co


def test_sm_closed_form(comp):
    src, d, co = comp
    K = len(d["scale"])
    th = np.concatenate([np.zeros(5), np.ones(K + 2)])
    closed = np.zeros(N_RECO)
    for k in range(K):
        NM = d["hist"][k] / d["comp_mask"][k][None, :]
        Rk = (NM / NM.sum() * d["scale"][k]).astype(np.float32).astype(np.float64)
        closed += d["rate_sm"][k] * Rk.sum(0)
    closed += (d["bkg_pdf"] * d["bkg_rate"][:, None]).sum(0)
    closed *= d["exposure"] * d["mask"]
    assert np.allclose(co.mu(th), closed, rtol=1e-12, atol=0)


def test_response_normalisation_and_mask_invariance(comp):
    src, d, co = comp
    for k, Rk in enumerate(co.R):
        assert Rk.sum() == pytest.approx(d["scale"][k], rel=1e-6)
    # a uniform component mask leaves R^(k) unchanged
    co2 = ComponentOracle(src, d["comp_of_source"], N_T, d["hist"], d["scale"],
                          d["rate_sm"], d["bkg_pdf"], d["bkg_rate"],
                          np.full_like(d["comp_mask"], 0.7), d["mask"], d["exposure"])
    co3 = ComponentOracle(src, d["comp_of_source"], N_T, d["hist"], d["scale"],
                          d["rate_sm"], d["bkg_pdf"], d["bkg_rate"],
                          None, d["mask"], d["exposure"])
    for a, b in zip(co2.R, co3.R):
        assert np.allclose(a, b, rtol=1e-6, atol=0)
    co2.close()
    co3.close()


def test_linear_in_rates(comp):
    src, d, co = comp
    K = len(d["scale"])
    g = synth.rng(5)
    th = np.concatenate([g.uniform(-0.3, 0.3, 4), [4.0], g.uniform(0.8, 1.2, K + 2)])
    base = co.mu(th)
    for k in range(K + 2):
        t2 = th.copy()
        t2[5 + k] *= 2.0
        t0 = th.copy()
        t0[5 + k] = 0.0
        # mu is affine in each rate: doubling adds what zeroing removes
        assert np.allclose(co.mu(t2) - base, base - co.mu(t0), rtol=1e-9,
                           atol=1e-12 * base.max())
