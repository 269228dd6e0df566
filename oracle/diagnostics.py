"""Effective sample size of reweighted Monte Carlo (test infrastructure
only; shares nothing with the library).

The prediction of an observed bin j is a weighted sum over the MC events
that land there; with N_lj events from true recoil bin l, each carrying the
weight w_l of its bin, the Kish effective sample size is
ESS_j = (sum_l N_lj w_l)^2 / sum_l N_lj w_l^2 -- the plain definition,
written out.  The weights come from the oracle (Eqs. (fT_norm),
(reweight_factor)); N_lj = R_lj n_l from the response and the events
generated per row.
"""
import numpy as np


def ess(R, n_events, w):
    """ESS_j for weights w [n_t] (or [P, n_t]); R [n_t][n_reco]."""
    N = np.asarray(R, dtype=np.float64) * np.asarray(n_events, dtype=np.float64)[:, None]
    w = np.atleast_2d(np.asarray(w, dtype=np.float64))
    s1 = w @ N
    s2 = (w * w) @ N
    out = np.zeros_like(s1)
    np.divide(s1 * s1, s2, out=out, where=s2 > 0)
    return out
