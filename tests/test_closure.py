"""The paper's closure test of the bin-level reweighting (Sec. VI.A): the
oracle's cross sections and the reweighting rule against a direct
continuum fold, pinned to the values the paper prints."""
import json
import os

import numpy as np
import pytest

from oracle import closure

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "closure.json")))
NSI = np.array(GOLD["nsi_theta"], dtype=float)
MM = np.array([0, 0, 0, 0, GOLD["mm_mu_nu_over_1e-11"] ** 2, 1, 1.0])


@pytest.fixture(scope="module")
def table():
    out = {}
    for n in (25, 50, 100, 200):
        out[n] = (closure.closure(NSI, n), closure.closure(MM, n))
    return out


def test_printed_25_bin_deviations(table):
    tol = GOLD["rel_tol_25_bins"]
    nsi, mm = table[25]
    assert nsi[1] == pytest.approx(GOLD["at_25_bins_integral_deviation"]["nsi"], rel=tol)
    assert mm[1] == pytest.approx(GOLD["at_25_bins_integral_deviation"]["mm"], rel=tol)
    ratio = mm[1] / nsi[1]
    assert 0.5 * GOLD["mm_over_nsi_at_fixed_binning"] < ratio < 2 * GOLD["mm_over_nsi_at_fixed_binning"]


def test_midpoint_scaling(table):
    for k in (0, 1):
        dev = [table[n][k][1] for n in (25, 50, 100, 200)]
        slope = np.polyfit(np.log([25, 50, 100, 200]), np.log(dev), 1)[0]
        assert slope == pytest.approx(-2.0, abs=0.05)


def test_framework_grid_bounds():
    b = closure.closure(MM, 2000)
    assert b[1] < GOLD["at_2000_bins"]["integral_deviation_below"]
    assert b[0] < GOLD["at_2000_bins"]["bin_residual_below"]


def test_sm_point_closes_exactly():
    """At theta_SM every weight is one: the two predictions coincide."""
    sm = np.array([0, 0, 0, 0, 0, 1, 1.0])
    edges = np.arange(0.0, 451.0)
    d, r = closure.predictions(sm, 40, edges)
    assert np.allclose(d, r, rtol=1e-13, atol=0)


def _signed_deviation(theta, n_t, weights_at=0.5):
    """(reweighted - direct) / direct over 50 < N_p < 400, with the weight of
    each recoil bin taken at fraction `weights_at` of the bin (0.5: centre,
    as the method does)."""
    edges = np.arange(0.0, 451.0)
    sel = (edges[:-1] >= 50) & (edges[1:] <= 400)
    if weights_at == 0.5:
        d, r = closure.predictions(theta, n_t, edges)
    else:  # the same assembly with the weights read off-centre
        d, _ = closure.predictions(theta, n_t, edges)
        Rjoint, pee, tmax = closure.binned_response(n_t, edges)
        o = closure.Oracle()
        at = (np.arange(n_t) + weights_at) * tmax / n_t
        sm = np.array([0, 0, 0, 0, 0, 1, 1.0])
        w = (closure.spectrum(o, closure.BE7, at, theta, pee)
             / closure.spectrum(o, closure.BE7, at, sm, pee))
        r = (Rjoint * w[:, None]).sum(0)
    return (r[sel].sum() - d[sel].sum()) / d[sel].sum()


def _midpoint_coefficient(theta, n_grid=8001):
    """Leading term of the closure deviation from a Taylor expansion of the
    weight about each bin centre: with w = S_theta / S_SM and g(T) = S_SM(T)
    times the probability that T lands in the N_p window, bin i contributes
    -(h^3 / 12) (g' w' + g w'' / 2) at its centre, so the deviation is
    -(h^2 / 12) int (g' w' + g w'' / 2) dT / int g w dT + O(h^4).  Returned
    as the coefficient of n_T^-2 (h = T_max / n_T); derivatives by finite
    differences on a fine grid, independent of the binned assembly."""
    from scipy import special
    o = closure.Oracle()
    E = closure.BE7
    pee = 0.32 + 0.23 / (1 + (E / 2) ** 2)
    tmax = closure.line_tmax(E)
    T = np.linspace(tmax * 1e-4, tmax * (1 - 1e-9), n_grid)
    sm = np.array([0, 0, 0, 0, 0, 1, 1.0])
    s_sm = closure.spectrum(o, E, T, sm, pee)
    w = closure.spectrum(o, E, T, theta, pee) / s_sm
    nb = closure.mean_pe(T)
    g = s_sm * (special.ndtr((400 - nb) / np.sqrt(nb)) - special.ndtr((50 - nb) / np.sqrt(nb)))
    dT = T[1] - T[0]
    gp = np.gradient(g, dT, edge_order=2)
    wp = np.gradient(w, dT, edge_order=2)
    wpp = np.gradient(wp, dT, edge_order=2)
    num = np.trapezoid(gp * wp + 0.5 * g * wpp, T)
    return -num / np.trapezoid(g * w, T) * tmax ** 2 / 12.0


@pytest.mark.parametrize("theta", [NSI, MM], ids=["nsi", "mm"])
def test_closure_matches_midpoint_expansion(theta):
    """The closure deviation itself (not only its slope) against the
    second-order expansion of the bin-centre weight: a pin that holds for
    any quenching function, so it does not lean on the reading chosen to
    reproduce the printed 25-bin values.  A weight read anywhere but the
    bin centre leaves an O(h) term and fails it by orders of magnitude."""
    c = _midpoint_coefficient(theta)
    for n in (100, 200):
        assert _signed_deviation(theta, n) * n * n / c == pytest.approx(1.0, abs=1e-3)
    off = _signed_deviation(theta, 100, weights_at=0.25) * 100 * 100 / c
    assert abs(off - 1.0) > 10.0
