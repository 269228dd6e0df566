"""Host-side helpers of the profile scans (no GPU)."""
import numpy as np
import pytest


def test_scan_interval_helper():
    """The confidence-interval reader of a profile scan on a parabola with a
    known half-width sigma * sqrt(q) around its minimum."""
    from paper_2607_00488_amd.scan import CHI2_1DOF_90, interval
    v = np.linspace(-1.0, 1.0, 2001)
    sig = 0.2
    d = ((v - 0.05) / sig) ** 2
    lo, hi = interval(v, d)
    half = sig * np.sqrt(CHI2_1DOF_90)
    assert lo == pytest.approx(0.05 - half, abs=1e-6)
    assert hi == pytest.approx(0.05 + half, abs=1e-6)
    # a side that never crosses the level ends at the grid
    lo, hi = interval(v[v > 0.0], ((v[v > 0.0] - 0.05) / sig) ** 2)
    assert lo == pytest.approx(v[v > 0.0][0])
    from scipy import stats
    assert CHI2_1DOF_90 == pytest.approx(stats.chi2.ppf(0.9, 1), rel=1e-12)


def test_form_names():
    from paper_2607_00488_amd.autograd import FORMS, _form
    assert _form(True) == "batched" and _form(False) == "plain"
    for f in FORMS:
        assert _form(f) == f
    with pytest.raises(ValueError):
        _form("surrogate")
