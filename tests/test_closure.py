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
